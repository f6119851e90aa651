"""The oracle's OpenMP CSR product (the assembled-matrix baseline of the
benchmark's CPU leg) against scipy's own CSR product on the oracle's assembled
tangent and on a random sparse matrix with empty rows."""

import ctypes
import os

import numpy as np
import pytest
import scipy.sparse as sp

import synthetic
from oracle.fem import Problem
from oracle.mesh import BoxMesh

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "libcsr_spmv.so")


def _spmv(A, x):
    if not os.path.exists(LIB):
        import oracle.build_c
        oracle.build_c.build()
    lib = ctypes.CDLL(LIB)
    lib.csr_spmv.restype = ctypes.c_int
    lib.csr_spmv.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 5
    A = A.tocsr()
    indptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
    indices = np.ascontiguousarray(A.indices, dtype=np.int32)
    data = np.ascontiguousarray(A.data, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.full(A.shape[0], np.nan)
    threads = lib.csr_spmv(A.shape[0], indptr.ctypes.data, indices.ctypes.data, data.ctypes.data, x.ctypes.data,
                           y.ctypes.data)
    assert threads >= 1
    return y


def test_csr_product_on_assembled_tangent():
    nx, ny, nz = 3, 2, 2
    v = synthetic.box_vertices(nx, ny, nz, (1, 1, 1), 0.1, np.random.default_rng(1))
    u = synthetic.sine_displacement(nx, ny, nz, 2, 0.02, np.random.default_rng(2))
    K = Problem(BoxMesh(nx, ny, nz, 2, v), 1.0, 10.0).assemble_tangent(u)
    x = np.random.default_rng(3).standard_normal(K.shape[0])
    ref = K @ x
    assert np.linalg.norm(_spmv(K, x) - ref) <= 1e-14 * np.linalg.norm(ref)


@pytest.mark.parametrize("n,density", [(1, 1.0), (37, 0.1), (500, 0.01)])
def test_csr_product_random(n, density):
    A = sp.random(n, n, density=density, format="csr", random_state=np.random.default_rng(n))
    x = np.random.default_rng(n + 1).standard_normal(n)
    y = _spmv(A, x)
    assert np.allclose(y, A @ x, rtol=1e-14, atol=1e-14)   # empty rows give 0


@pytest.mark.parametrize("nx,ny,nz,p,jit", [(4, 4, 4, 2, 0.0), (3, 2, 2, 2, 0.15), (3, 3, 2, 1, 0.15),
                                           (2, 2, 1, 3, 0.1)])
def test_c_assembly_matches_numpy_assembly(nx, ny, nz, p, jit):
    """The C/OpenMP assembly (the benchmark's full-size CSR baseline) against
    the numpy assembly of the same definition, entry by entry, including the
    4^3 Q2 cube of the parity workload."""
    from oracle.assemble_c import assemble_tangent_box
    rng = np.random.default_rng(nx + 10 * p)
    v = synthetic.box_vertices(nx, ny, nz, (1.0, 0.9, 0.8), jit, rng)
    mesh = BoxMesh(nx, ny, nz, p, v)
    u = synthetic.sine_displacement(nx, ny, nz, p, 0.03, np.random.default_rng(p))
    K = Problem(mesh, 1.0, 10.0).assemble_tangent(u).tocsr()
    K.sort_indices()
    indptr, indices, data, threads = assemble_tangent_box(mesh, 1.0, 10.0, u)
    assert threads >= 1
    Kc = sp.csr_matrix((data, indices, indptr), shape=K.shape)
    # the analytic pattern: every pair of dofs of nodes that share a cell
    assert np.array_equal(Kc.indptr, K.indptr) and np.array_equal(Kc.indices, K.indices)
    assert np.max(np.abs(Kc.data - K.data)) <= 1e-13 * np.max(np.abs(K.data))
    x = np.random.default_rng(4).standard_normal(K.shape[0])
    assert np.linalg.norm(_spmv(Kc, x) - K @ x) <= 1e-13 * np.linalg.norm(K @ x)
