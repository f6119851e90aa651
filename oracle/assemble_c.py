"""The oracle's tangent of a structured box assembled into CSR by the C/OpenMP
code of ``oracle/csr_assemble.c`` (the same definition as
``Problem.assemble_tangent``, for meshes where the numpy assembly is too slow:
the assembled-matrix baseline of the benchmark).

TEST AND BASELINE INFRASTRUCTURE ONLY (see the package docstring).
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from .mesh import BoxMesh

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libcsr_assemble.so")


def _lib():
    if not os.path.exists(_LIB):
        from . import build_c
        build_c.build()
    lib = ctypes.CDLL(_LIB)
    lib.csr_pattern_box.restype = ctypes.c_int64
    lib.csr_pattern_box.argtypes = [ctypes.c_int] * 4 + [ctypes.c_void_p]
    lib.csr_assemble_box.restype = ctypes.c_int
    lib.csr_assemble_box.argtypes = ([ctypes.c_int] * 5 + [ctypes.c_void_p] * 2 + [ctypes.c_double] * 2 +
                                     [ctypes.c_void_p] * 6)
    return lib


def assemble_tangent_box(mesh: BoxMesh, mu: float, lam: float, u):
    """(indptr int64, indices int32, data float64, threads) of K(u) on ``mesh``
    (uniform material, no constraints), columns sorted within each row."""
    lib = _lib()
    n = mesh.n_dofs
    indptr = np.zeros(n + 1, dtype=np.int64)
    nnz = lib.csr_pattern_box(mesh.nx, mesh.ny, mesh.nz, mesh.degree, indptr.ctypes.data)
    indices = np.empty(nnz, dtype=np.int32)
    data = np.empty(nnz, dtype=np.float64)
    verts = np.ascontiguousarray(mesh.vertices, dtype=np.float64)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    qw = np.ascontiguousarray(mesh.basis.weights, dtype=np.float64)
    tg = np.ascontiguousarray(mesh._tri_grads, dtype=np.float64)
    bg = np.ascontiguousarray(mesh.basis.grads, dtype=np.float64)
    threads = lib.csr_assemble_box(mesh.nx, mesh.ny, mesh.nz, mesh.degree, qw.size, verts.ctypes.data,
                                   uu.ctypes.data, float(mu), float(lam), qw.ctypes.data, tg.ctypes.data,
                                   bg.ctypes.data, indptr.ctypes.data, indices.ctypes.data, data.ctypes.data)
    if threads < 0:
        raise ValueError("det J_g <= 0 or det F <= 0 at some quadrature point")
    return indptr, indices, data, threads
