"""Python binding of libmfe (matrix-free finite-strain tangent on MI355X).

Thin ctypes layer over the C ABI declared in ``include/mfe.h``: the module
level functions have the same names and arguments as the C entry points
(device buffers and streams are passed as integer addresses), and
:class:`Operator` wraps a context for use with torch tensors.  Every step of
the computation runs in the HIP kernels of ``libmfe.so``; this module only
marshals arguments.  Importing it raises if the library has not been built.
"""

from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmfe.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "mfe.h")

# status codes
MFE_OK, MFE_EINVAL, MFE_EHIP, MFE_ENOMEM, MFE_EJACOBIAN, MFE_ESTATE, MFE_ENOTCONV, MFE_EUNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6, -7)
STATUS_NAMES = {0: "MFE_OK", -1: "MFE_EINVAL", -2: "MFE_EHIP", -3: "MFE_ENOMEM", -4: "MFE_EJACOBIAN",
                -5: "MFE_ESTATE", -6: "MFE_ENOTCONV", -7: "MFE_EUNSUPPORTED"}
# strategies
MFE_OTF, MFE_OTF_GEOM, MFE_T2, MFE_T4, MFE_OTF_AD = 0, 1, 2, 3, 4
STRATEGIES = {"otf": MFE_OTF, "otf_geom": MFE_OTF_GEOM, "t2": MFE_T2, "t4": MFE_T4, "otf_ad": MFE_OTF_AD}
# sweep precisions
MFE_FP64, MFE_SF_FP32, MFE_SF_BF16, MFE_SF_BF16X3 = 0, 1, 2, 3
PRECISIONS = {"fp64": MFE_FP64, "fp32": MFE_SF_FP32, "bf16": MFE_SF_BF16, "bf16x3": MFE_SF_BF16X3}
# preconditioners of the Newton-CG solver
MFE_PC_NONE, MFE_PC_JACOBI, MFE_PC_GMG, MFE_PC_GMG_NET = 0, 1, 2, 3
PRECONDITIONERS = {"none": MFE_PC_NONE, "jacobi": MFE_PC_JACOBI, "gmg": MFE_PC_GMG, "gmg_net": MFE_PC_GMG_NET}
MFE_NET_PARAMS = 35491
MFE_NET_RELU, MFE_NET_LINEAR = 0, 1
NET_VARIANTS = {"relu": MFE_NET_RELU, "linear": MFE_NET_LINEAR}
MFE_HISTORY = 64

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it first (python paper_2505_15535_amd/build.py)")

# torch owns the process's HIP runtime; loading it first makes libmfe bind to
# that same runtime (matching soname) instead of a second copy from /opt/rocm,
# which would put two HIP/HSA runtimes in one process.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)
_vp, _i, _i64, _d = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double


class SolveOpts(ctypes.Structure):
    """struct mfe_solve_opts"""
    _fields_ = [("strategy", _i), ("preconditioner", _i), ("max_newton", _i), ("max_cg", _i),
                ("newton_atol", _d), ("cg_rtol", _d), ("mg_levels", _i), ("cheb_degree", _i),
                ("cheb_range", _d), ("coarse_degree", _i), ("coarse_range", _d), ("mg_precision", _i),
                ("mg_graph", _i), ("coarse_direct", _i), ("forcing", _d), ("mg_lag", _i)]


class SolveReport(ctypes.Structure):
    """struct mfe_solve_report"""
    _fields_ = [("converged", _i), ("newton_iterations", _i), ("cg_iterations", _i), ("backtracks", _i),
                ("pc_fallbacks", _i), ("net_fallbacks", _i), ("initial_residual", _d), ("final_residual", _d),
                ("residual_history", _d * MFE_HISTORY)]

    def as_dict(self):
        n = min(self.newton_iterations + 1, MFE_HISTORY)
        return {"converged": bool(self.converged), "newton_iterations": self.newton_iterations,
                "cg_iterations": self.cg_iterations, "backtracks": self.backtracks,
                "pc_fallbacks": self.pc_fallbacks, "net_fallbacks": self.net_fallbacks,
                "initial_residual": self.initial_residual,
                "final_residual": self.final_residual, "residual_history": list(self.residual_history[:n])}


class PathState(ctypes.Structure):
    """struct mfe_path_state"""
    _fields_ = [("t", _d), ("h", _d), ("h_cap", _d), ("prev_h", _d)]


class PathReport(ctypes.Structure):
    """struct mfe_path_report"""
    _fields_ = [("t", _d), ("h", _d), ("failed", _i), ("status", _i), ("solve", SolveReport)]


LOAD_FN = ctypes.CFUNCTYPE(_i, _d, ctypes.POINTER(_d), _i64, _vp)
STEP_FN = ctypes.CFUNCTYPE(_i, ctypes.POINTER(PathState), _vp, _vp, _vp)

_SIGS = {
    "mfe_create": (_i, [ctypes.POINTER(_vp), _i]),
    "mfe_destroy": (None, [_vp]),
    "mfe_last_error": (ctypes.c_char_p, [_vp]),
    "mfe_mesh_box": (_i, [_vp, _i, _i, _i, _i, _vp]),
    "mfe_mesh_hex": (_i, [_vp, _i64, _vp, _i64, _vp, _i]),
    "mfe_node_coordinates": (_i, [_vp, _vp]),
    "mfe_hex_numbering": (_i, [_i64, _i64, _vp, _i, _vp, ctypes.POINTER(_i64)]),
    "mfe_n_dofs": (_i64, [_vp]),
    "mfe_n_cells": (_i64, [_vp]),
    "mfe_n_qpoints": (_i64, [_vp]),
    "mfe_set_material": (_i, [_vp, _d, _d, _vp]),
    "mfe_set_constraints": (_i, [_vp, _i64, _vp]),
    "mfe_set_model": (_i, [_vp, _i]),
    "mfe_set_state": (_i, [_vp, _vp, _vp]),
    "mfe_build_cache": (_i, [_vp, _i, _vp]),
    "mfe_build_cache_fp32": (_i, [_vp, _i, _vp]),
    "mfe_cache_bytes": (_i64, [_vp, _i]),
    "mfe_apply_tangent": (_i, [_vp, _vp, _vp, _i, _i, _vp]),
    "mfe_residual": (_i, [_vp, _vp, _vp, _vp]),
    "mfe_energy": (_i, [_vp, _vp, ctypes.POINTER(_d), _vp]),
    "mfe_energy_noalloc": (_i, [_vp, _vp, _vp, _vp]),
    "mfe_set_timing": (_i, [_vp, _i]),
    "mfe_set_deterministic": (_i, [_vp, _i]),
    "mfe_newton_solve": (_i, [_vp, ctypes.POINTER(SolveOpts), _vp, _vp, ctypes.POINTER(SolveReport), _vp]),
    "mfe_cg_solve": (_i, [_vp, ctypes.POINTER(SolveOpts), _vp, _vp, ctypes.POINTER(_i), ctypes.POINTER(_d), _vp]),
    "mfe_solve_load_path": (_i, [_vp, ctypes.POINTER(SolveOpts), _vp, _vp, _i, _d, _i, ctypes.POINTER(PathState),
                                 LOAD_FN, _vp, STEP_FN, _vp, ctypes.POINTER(PathReport), _i, ctypes.POINTER(_i),
                                 _vp]),
    "mfe_diagonal": (_i, [_vp, _vp, _vp]),
    "mfe_gmg_setup": (_i, [_vp, ctypes.POINTER(SolveOpts), _vp]),
    "mfe_set_network": (_i, [_vp, _vp, _i]),
    "mfe_patch_count": (_i64, [_vp]),
    "mfe_patch_features": (_i, [_vp, _vp, _vp, _vp, _i, _vp]),
    "mfe_patch_targets": (_i, [_vp, _vp, _vp, _vp, _vp]),
    "mfe_patch_scatter": (_i, [_vp, _vp, _vp, _d, _vp, _vp]),
    "mfe_patch_adjoint": (_i, [_vp, _vp, _vp, _d, _vp, _vp]),
    "mfe_net_forward": (_i, [_vp, _vp, _i, _i, _vp, _vp, _vp]),
    "mfe_net_backward": (_i, [_vp, _vp, _vp, _vp, _i, _i, _vp, _vp, _vp]),
    "mfe_net_loss": (_i, [_vp, _vp, _i64, _vp, _vp, ctypes.POINTER(_d), _vp]),
    "mfe_net_adam": (_i, [_vp, _vp, _vp, _vp, _i, ctypes.c_float, _vp]),
    "mfe_gmg_apply": (_i, [_vp, ctypes.POINTER(SolveOpts), _vp, _vp, _vp]),
    "mfe_axpby": (_i, [_vp, _d, _vp, _d, _vp, _vp]),
    "mfe_dot": (_i, [_vp, _vp, _vp, ctypes.POINTER(_d), _vp]),
    "mfe_zero_constrained": (_i, [_vp, _vp, _vp]),
    "mfe_apply_kernel_ms": (_d, [_vp, ctypes.POINTER(_i)]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def header_symbols(path: str = HEADER_PATH) -> list[str]:
    """Names of the functions declared in the C header."""
    with open(path) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mfe_[a-z0-9_]+)\s*\(", text)))


class MfeError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {message}")
        self.code = code


# ----------------------------------------------------------------- raw ABI
def mfe_create(hip_device: int = 0) -> int:
    h = _vp()
    rc = _lib.mfe_create(ctypes.byref(h), int(hip_device))
    if rc != MFE_OK:
        raise MfeError(rc, f"mfe_create(device={hip_device}) failed")
    return h.value


def mfe_destroy(ctx: int) -> None:
    _lib.mfe_destroy(ctx)


def mfe_last_error(ctx: int | None) -> str:
    return (_lib.mfe_last_error(ctx) or b"").decode()


def _check(ctx, rc):
    if rc != MFE_OK:
        raise MfeError(rc, mfe_last_error(ctx))
    return rc


def mfe_mesh_box(ctx, nx, ny, nz, degree, vertex_xyz_host_ptr):
    return _check(ctx, _lib.mfe_mesh_box(ctx, nx, ny, nz, degree, vertex_xyz_host_ptr))


def mfe_mesh_hex(ctx, n_vertices, vertex_xyz_host_ptr, n_cells, cell_vertices_host_ptr, degree):
    return _check(ctx, _lib.mfe_mesh_hex(ctx, int(n_vertices), vertex_xyz_host_ptr, int(n_cells),
                                         cell_vertices_host_ptr, int(degree)))


def mfe_hex_numbering(cells, degree, n_vertices):
    """(cell_nodes [n_cells, (degree+1)^3] int32, n_nodes) of the canonical
    numbering of a general hexahedral mesh (host only, no device needed)."""
    import numpy as np
    cv = np.ascontiguousarray(np.asarray(cells, dtype=np.int32).reshape(-1, 8))
    out = np.empty((cv.shape[0], (int(degree) + 1) ** 3), dtype=np.int32)
    n_nodes = _i64(0)
    rc = _lib.mfe_hex_numbering(int(n_vertices), cv.shape[0], cv.ctypes.data, int(degree), out.ctypes.data,
                                ctypes.byref(n_nodes))
    if rc != MFE_OK:
        raise MfeError(rc, "invalid hexahedral mesh")
    return out, int(n_nodes.value)


def mfe_node_coordinates(ctx, xyz_host_ptr):
    return _check(ctx, _lib.mfe_node_coordinates(ctx, xyz_host_ptr))


def mfe_n_dofs(ctx) -> int:
    return int(_lib.mfe_n_dofs(ctx))


def mfe_n_cells(ctx) -> int:
    return int(_lib.mfe_n_cells(ctx))


def mfe_n_qpoints(ctx) -> int:
    return int(_lib.mfe_n_qpoints(ctx))


def mfe_set_material(ctx, mu, lam, per_cell_host_ptr=None):
    return _check(ctx, _lib.mfe_set_material(ctx, float(mu), float(lam), per_cell_host_ptr))


def mfe_set_constraints(ctx, n, dofs_host_ptr):
    return _check(ctx, _lib.mfe_set_constraints(ctx, int(n), dofs_host_ptr))


def mfe_set_state(ctx, u_dev_ptr, stream=None):
    return _check(ctx, _lib.mfe_set_state(ctx, u_dev_ptr, stream))


def mfe_build_cache(ctx, strategy, stream=None):
    return _check(ctx, _lib.mfe_build_cache(ctx, int(strategy), stream))


def mfe_energy(ctx, u_dev_ptr, stream=None) -> float:
    e = _d()
    _check(ctx, _lib.mfe_energy(ctx, u_dev_ptr, ctypes.byref(e), stream))
    return e.value


def mfe_energy_noalloc(ctx, u_dev_ptr, energy_dev_ptr, stream=None):
    return _check(ctx, _lib.mfe_energy_noalloc(ctx, u_dev_ptr, energy_dev_ptr, stream))


def mfe_build_cache_fp32(ctx, strategy, stream=None):
    return _check(ctx, _lib.mfe_build_cache_fp32(ctx, int(strategy), stream))


def mfe_cache_bytes(ctx, strategy) -> int:
    return int(_lib.mfe_cache_bytes(ctx, int(strategy)))


def mfe_apply_tangent(ctx, w_dev_ptr, v_dev_ptr, strategy, precision=MFE_FP64, stream=None):
    return _check(ctx, _lib.mfe_apply_tangent(ctx, w_dev_ptr, v_dev_ptr, int(strategy), int(precision), stream))


def mfe_residual(ctx, u_dev_ptr, r_dev_ptr, stream=None):
    return _check(ctx, _lib.mfe_residual(ctx, u_dev_ptr, r_dev_ptr, stream))


def mfe_newton_solve(ctx, opts: SolveOpts, u_dev_ptr, g_dev_ptr=None, stream=None):
    """Returns (status, SolveReport); raises MfeError unless the status is
    MFE_OK or MFE_ENOTCONV (not converged within the iteration limits)."""
    rep = SolveReport()
    rc = _lib.mfe_newton_solve(ctx, ctypes.byref(opts), u_dev_ptr, g_dev_ptr, ctypes.byref(rep), stream)
    if rc not in (MFE_OK, MFE_ENOTCONV):
        raise MfeError(rc, mfe_last_error(ctx))
    return rc, rep


def mfe_solve_load_path(ctx, opts: SolveOpts, u_dev_ptr, prev_dev_ptr, n_steps, min_fraction, extrapolate,
                        state: PathState, load, on_step=None, max_reports=4096, stream=None):
    """Run the library's load-path driver.  load(t) -> values at the
    constrained dofs (ascending dof order); on_step(state, u_ptr, prev_ptr)
    -> truthy to stop.  Exceptions raised in the callbacks stop the path and
    are raised again here.  Returns (status, [PathReport]); raises MfeError
    unless the status is MFE_OK or MFE_ENOTCONV."""
    import numpy as np
    caught = []

    def _load(t, values, n, user):
        try:
            vals = np.asarray(load(t), dtype=np.float64).reshape(-1)
            if vals.size != n:
                raise ValueError(f"load callback returned {vals.size} values for {n} constrained dofs")
            ctypes.memmove(values, vals.ctypes.data, n * 8)
            return 0
        except BaseException as e:  # noqa: BLE001 -- re-raised after the C call returns
            caught.append(e)
            return 1

    def _step(st, u_ptr, prev_ptr, user):
        try:
            return 1 if (on_step is not None and on_step(st.contents, u_ptr, prev_ptr)) else 0
        except BaseException as e:  # noqa: BLE001
            caught.append(e)
            return 1

    load_cb, step_cb = LOAD_FN(_load), STEP_FN(_step)
    reports = (PathReport * max_reports)()
    n_rep = _i(0)
    rc = _lib.mfe_solve_load_path(ctx, ctypes.byref(opts), u_dev_ptr, prev_dev_ptr, int(n_steps),
                                  float(min_fraction), int(bool(extrapolate)), ctypes.byref(state), load_cb,
                                  None, step_cb, None, reports, max_reports, ctypes.byref(n_rep), stream)
    if caught:
        raise caught[0]
    if rc not in (MFE_OK, MFE_ENOTCONV):
        raise MfeError(rc, mfe_last_error(ctx))
    return rc, list(reports[:n_rep.value])


def mfe_gmg_setup(ctx, opts: SolveOpts, stream=None):
    return _check(ctx, _lib.mfe_gmg_setup(ctx, ctypes.byref(opts), stream))


def mfe_gmg_apply(ctx, opts: SolveOpts, r_dev_ptr, z_dev_ptr, stream=None):
    return _check(ctx, _lib.mfe_gmg_apply(ctx, ctypes.byref(opts), r_dev_ptr, z_dev_ptr, stream))


MFE_MODEL_NH, MFE_MODEL_SPLIT = 0, 1
MODELS = {"nh": MFE_MODEL_NH, "split": MFE_MODEL_SPLIT}


def mfe_set_model(ctx, model):
    return _check(ctx, _lib.mfe_set_model(ctx, int(model)))


def mfe_set_network(ctx, params_host_ptr, variant=MFE_NET_RELU):
    return _check(ctx, _lib.mfe_set_network(ctx, params_host_ptr, int(variant)))


def mfe_patch_count(ctx) -> int:
    return int(_lib.mfe_patch_count(ctx))


def mfe_patch_features(ctx, r_dev_ptr, feat_dev_ptr, scale_dev_ptr, variant=MFE_NET_RELU, stream=None):
    return _check(ctx, _lib.mfe_patch_features(ctx, r_dev_ptr, feat_dev_ptr, scale_dev_ptr, int(variant), stream))


def mfe_patch_targets(ctx, e_dev_ptr, scale_dev_ptr, t_dev_ptr, stream=None):
    return _check(ctx, _lib.mfe_patch_targets(ctx, e_dev_ptr, scale_dev_ptr, t_dev_ptr, stream))


def mfe_patch_scatter(ctx, y_dev_ptr, scale_dev_ptr, alpha, z_dev_ptr, stream=None):
    return _check(ctx, _lib.mfe_patch_scatter(ctx, y_dev_ptr, scale_dev_ptr, float(alpha), z_dev_ptr, stream))


def mfe_patch_adjoint(ctx, g_dev_ptr, scale_dev_ptr, alpha, dy_dev_ptr, stream=None):
    return _check(ctx, _lib.mfe_patch_adjoint(ctx, g_dev_ptr, scale_dev_ptr, float(alpha), dy_dev_ptr, stream))


def _check_free(rc, what):
    if rc != MFE_OK:
        raise MfeError(rc, what)
    return rc


def mfe_net_forward(params_ptr, x_ptr, n_patches, act_ptr, y_ptr, variant=MFE_NET_RELU, stream=None):
    return _check_free(_lib.mfe_net_forward(params_ptr, x_ptr, int(n_patches), int(variant), act_ptr, y_ptr, stream),
                       "mfe_net_forward")


def mfe_net_backward(params_ptr, x_ptr, act_ptr, dy_ptr, n_patches, work_ptr, grad_ptr, variant=MFE_NET_RELU,
                     stream=None):
    return _check_free(_lib.mfe_net_backward(params_ptr, x_ptr, act_ptr, dy_ptr, int(n_patches), int(variant),
                                             work_ptr, grad_ptr, stream), "mfe_net_backward")


def mfe_net_loss(y_ptr, t_ptr, n, dy_ptr, scratch_ptr, stream=None) -> float:
    loss = _d()
    _check_free(_lib.mfe_net_loss(y_ptr, t_ptr, int(n), dy_ptr, scratch_ptr, ctypes.byref(loss), stream),
                "mfe_net_loss")
    return loss.value


def mfe_net_adam(params_ptr, grad_ptr, m_ptr, v_ptr, step, lr, stream=None):
    return _check_free(_lib.mfe_net_adam(params_ptr, grad_ptr, m_ptr, v_ptr, int(step), float(lr), stream),
                       "mfe_net_adam")


def mfe_cg_solve(ctx, opts: SolveOpts, b_dev_ptr, x_dev_ptr, stream=None):
    """Returns (status, iterations, relative residual); raises MfeError unless
    the status is MFE_OK or MFE_ENOTCONV."""
    it, rel = _i(0), _d(0.0)
    rc = _lib.mfe_cg_solve(ctx, ctypes.byref(opts), b_dev_ptr, x_dev_ptr, ctypes.byref(it), ctypes.byref(rel), stream)
    if rc not in (MFE_OK, MFE_ENOTCONV):
        raise MfeError(rc, mfe_last_error(ctx))
    return rc, int(it.value), float(rel.value)


def mfe_axpby(ctx, a, x_dev_ptr, b, y_dev_ptr, stream=None):
    return _check(ctx, _lib.mfe_axpby(ctx, float(a), x_dev_ptr, float(b), y_dev_ptr, stream))


def mfe_dot(ctx, x_dev_ptr, y_dev_ptr, stream=None) -> float:
    r = _d()
    _check(ctx, _lib.mfe_dot(ctx, x_dev_ptr, y_dev_ptr, ctypes.byref(r), stream))
    return r.value


def mfe_zero_constrained(ctx, v_dev_ptr, stream=None):
    return _check(ctx, _lib.mfe_zero_constrained(ctx, v_dev_ptr, stream))


def mfe_diagonal(ctx, d_dev_ptr, stream=None):
    return _check(ctx, _lib.mfe_diagonal(ctx, d_dev_ptr, stream))


def mfe_set_timing(ctx, every):
    return _check(ctx, _lib.mfe_set_timing(ctx, int(every)))


def mfe_set_deterministic(ctx, on):
    return _check(ctx, _lib.mfe_set_deterministic(ctx, int(bool(on))))


def mfe_apply_kernel_ms(ctx):
    n = _i(0)
    ms = _lib.mfe_apply_kernel_ms(ctx, ctypes.byref(n))
    return float(ms), int(n.value)


# ----------------------------------------------------------------- torch helper
def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev_tensor(t, n, name, dtype):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of {n} entries")
    return t.data_ptr()


def _dev_f64(t, n, name):
    import torch
    return _dev_tensor(t, n, name, torch.float64)


def save_checkpoint(path, u, prev, t, h, h_cap, prev_h, n_steps):
    """State of the load-path driver after a converged step, as an .npz file
    (written to a temporary name and renamed, so an interruption leaves the
    previous checkpoint intact)."""
    import numpy as np
    tmp = str(path) + ".tmp.npz"
    np.savez(tmp, u=u.detach().cpu().numpy(), prev=prev.detach().cpu().numpy(), t=float(t), h=float(h),
             h_cap=float(h_cap), prev_h=float("nan") if prev_h is None else float(prev_h), n_steps=int(n_steps))
    os.replace(tmp, str(path))


def load_checkpoint(path):
    """The arrays saved by save_checkpoint (no pickled objects are loaded)."""
    import numpy as np
    with np.load(str(path), allow_pickle=False) as f:
        return {k: f[k] for k in f.files}


class Operator:
    """A context holding one mesh, material, constraints, state and caches.

    ``Operator(nx, ny, nz, degree, vertices, mu, lam)`` builds a box mesh,
    ``Operator.from_hex(vertices, cells, degree, mu, lam)`` a general
    hexahedral one; ``set_state(u)``, ``build_cache(strategy)``,
    ``apply(w, out, strategy)`` and ``residual(u, out)`` queue work on torch's
    current stream.
    """

    def __init__(self, nx, ny, nz, degree, vertices, mu=1.0, lam=1.0, per_cell=None, device=None):
        import numpy as np
        verts = np.ascontiguousarray(np.asarray(vertices, dtype=np.float64).reshape(-1))
        self._open(device)
        mfe_mesh_box(self.ctx, nx, ny, nz, degree, verts.ctypes.data)
        self._finish(mu, lam, per_cell)

    @classmethod
    def from_hex(cls, vertices, cells, degree, mu=1.0, lam=1.0, per_cell=None, device=None):
        """General hexahedral mesh: vertices [nv, 3], cells [ne, 8] vertex ids
        in lexicographic local order; nodes in the canonical numbering."""
        import numpy as np
        verts = np.ascontiguousarray(np.asarray(vertices, dtype=np.float64).reshape(-1, 3))
        cv = np.ascontiguousarray(np.asarray(cells).reshape(-1, 8))
        if cv.size and (cv.min() < 0 or cv.max() >= 2 ** 31):
            raise ValueError("cell vertex ids must fit in int32 and be >= 0")
        cv = cv.astype(np.int32)
        self = cls.__new__(cls)
        self._open(device)
        mfe_mesh_hex(self.ctx, verts.shape[0], verts.ctypes.data, cv.shape[0], cv.ctypes.data, degree)
        self._finish(mu, lam, per_cell)
        return self

    def _open(self, device):
        import torch
        dev = torch.cuda.current_device() if device is None else int(device)
        self.device = torch.device("cuda", dev)
        self.ctx = mfe_create(dev)

    def _finish(self, mu, lam, per_cell):
        self.n_dofs = mfe_n_dofs(self.ctx)
        self.n_cells = mfe_n_cells(self.ctx)
        self.n_qpoints = mfe_n_qpoints(self.ctx)
        self.set_material(mu, lam, per_cell)

    def node_coordinates(self):
        """Reference coordinates [n_nodes, 3] (numpy float64) of the nodes."""
        import numpy as np
        out = np.empty(self.n_dofs, dtype=np.float64)
        mfe_node_coordinates(self.ctx, out.ctypes.data)
        return out.reshape(-1, 3)

    def close(self):
        if getattr(self, "ctx", None):
            mfe_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_model(self, model):
        """Stored-energy law: "nh" (eq. hypref, (mu, lambda)) or "split" (eq. hypcomplex, (mu, kappa))."""
        mfe_set_model(self.ctx, MODELS.get(model, model))

    def set_material(self, mu, lam, per_cell=None):
        import numpy as np
        if per_cell is None:
            mfe_set_material(self.ctx, mu, lam, None)
        else:
            pc = np.ascontiguousarray(np.asarray(per_cell, dtype=np.float64).reshape(-1))
            if pc.size != 2 * self.n_cells:
                raise ValueError("per_cell must hold (mu, lambda) for every cell")
            mfe_set_material(self.ctx, mu, lam, pc.ctypes.data)

    def set_constraints(self, dofs):
        import numpy as np
        d = np.ascontiguousarray(np.asarray(dofs, dtype=np.int64).reshape(-1))
        mfe_set_constraints(self.ctx, d.size, d.ctypes.data if d.size else None)
        self._cidx = np.unique(d)   # the library's order of the constrained dofs

    def set_state(self, u, stream=None):
        mfe_set_state(self.ctx, _dev_f64(u, self.n_dofs, "u"), _stream_handle(stream))

    def build_cache(self, strategy, stream=None, precision="fp64"):
        """Per-point data of `strategy` for applies of `precision` ("fp64", or
        "fp32" / "bf16" / "bf16x3", which read the FP32 cache)."""
        prec = PRECISIONS.get(precision, precision)
        build = mfe_build_cache_fp32 if prec in (MFE_SF_FP32, MFE_SF_BF16, MFE_SF_BF16X3) else mfe_build_cache
        build(self.ctx, STRATEGIES.get(strategy, strategy), _stream_handle(stream))

    def cache_bytes(self, strategy):
        return mfe_cache_bytes(self.ctx, STRATEGIES.get(strategy, strategy))

    def apply(self, w, out=None, strategy="otf", precision=MFE_FP64, stream=None):
        """out = K(u) w.  precision "fp64" (float64 tensors), or "fp32", "bf16",
        "bf16x3" (float32 tensors: FP32 caches and vectors, the sweeps of w on
        the vector ALUs in FP32 or on the matrix cores, see mfe_precision)."""
        import torch
        prec = PRECISIONS.get(precision, precision)
        if out is None:
            out = torch.empty_like(w)
        if prec in (MFE_SF_FP32, MFE_SF_BF16, MFE_SF_BF16X3):
            wp, op = _dev_tensor(w, self.n_dofs, "w", torch.float32), _dev_tensor(out, self.n_dofs, "out", torch.float32)
        else:
            wp, op = _dev_f64(w, self.n_dofs, "w"), _dev_f64(out, self.n_dofs, "out")
        mfe_apply_tangent(self.ctx, wp, op, STRATEGIES.get(strategy, strategy), prec, _stream_handle(stream))
        return out

    def energy(self, u, stream=None):
        """Stored energy at displacement u (float64 device tensor)."""
        return mfe_energy(self.ctx, _dev_f64(u, self.n_dofs, "u"), _stream_handle(stream))

    def residual(self, u, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty_like(u)
        mfe_residual(self.ctx, _dev_f64(u, self.n_dofs, "u"), _dev_f64(out, self.n_dofs, "out"),
                     _stream_handle(stream))
        return out

    @staticmethod
    def solve_opts(strategy="t2", preconditioner="jacobi", max_newton=20, max_cg=5000, newton_atol=1e-8,
                   cg_rtol=1e-6, mg_levels=0, cheb_degree=4, cheb_range=15.0, coarse_degree=15,
                   coarse_range=200.0, mg_precision="fp64", mg_graph=1, coarse_direct=1, forcing=0.0, mg_lag=0):
        return SolveOpts(STRATEGIES.get(strategy, strategy), PRECONDITIONERS.get(preconditioner, preconditioner),
                         int(max_newton), int(max_cg), float(newton_atol), float(cg_rtol), int(mg_levels),
                         int(cheb_degree), float(cheb_range), int(coarse_degree), float(coarse_range),
                         PRECISIONS.get(mg_precision, mg_precision), int(mg_graph), int(coarse_direct),
                         float(forcing), int(mg_lag))

    def newton_solve(self, u, g=None, stream=None, **opts):
        """Solve R(u) = 0 in place; g (optional tensor) holds new Dirichlet values at the
        constrained dofs.  Returns the report as a dict."""
        gp = None if g is None else _dev_f64(g, self.n_dofs, "g")
        rc, rep = mfe_newton_solve(self.ctx, self.solve_opts(**opts), _dev_f64(u, self.n_dofs, "u"), gp,
                                   _stream_handle(stream))
        out = rep.as_dict()
        out["status"] = STATUS_NAMES.get(rc, rc)
        if rc != MFE_OK:
            out["message"] = mfe_last_error(self.ctx)
        return out

    def cg_solve(self, b, x=None, stream=None, **opts):
        """x = K(u)^-1 b at the current state; returns (x, iterations, relative residual, status)."""
        import torch
        if x is None:
            x = torch.empty_like(b)
        rc, it, rel = mfe_cg_solve(self.ctx, self.solve_opts(**opts), _dev_f64(b, self.n_dofs, "b"),
                                   _dev_f64(x, self.n_dofs, "x"), _stream_handle(stream))
        return x, it, rel, STATUS_NAMES.get(rc, rc)

    # ---------------------------------------------------------- learned correction
    def set_network(self, params, variant="relu"):
        """Network parameters for the "gmg_net" preconditioner (MFE_NET_PARAMS floats, host or device; None
        clears) and its variant ("relu" or "linear")."""
        import numpy as np
        var = NET_VARIANTS.get(variant, variant)
        if params is None:
            mfe_set_network(self.ctx, None, var)
            return
        if hasattr(params, "detach"):
            params = params.detach().cpu().numpy()
        h = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
        if h.size != MFE_NET_PARAMS:
            raise ValueError(f"expected {MFE_NET_PARAMS} parameters")
        mfe_set_network(self.ctx, h.ctypes.data, var)

    @property
    def n_patches(self):
        return mfe_patch_count(self.ctx)

    def patch_features(self, r, variant="relu", stream=None):
        """(feat [P,6,729] float32, scale [P] float32) of a residual r at the current state."""
        import torch
        P = self.n_patches
        feat = torch.empty((P, 6, 729), dtype=torch.float32, device=r.device)
        scale = torch.empty(P, dtype=torch.float32, device=r.device)
        mfe_patch_features(self.ctx, _dev_f64(r, self.n_dofs, "r"), feat.data_ptr(), scale.data_ptr(),
                           NET_VARIANTS.get(variant, variant), _stream_handle(stream))
        return feat, scale

    def patch_targets(self, e, scale, stream=None):
        import torch
        t = torch.empty((self.n_patches, 3, 729), dtype=torch.float32, device=e.device)
        mfe_patch_targets(self.ctx, _dev_f64(e, self.n_dofs, "e"), scale.data_ptr(), t.data_ptr(),
                          _stream_handle(stream))
        return t

    def patch_scatter(self, y, scale, z, alpha=1.0, stream=None):
        mfe_patch_scatter(self.ctx, y.data_ptr(), scale.data_ptr(), alpha, _dev_f64(z, self.n_dofs, "z"),
                          _stream_handle(stream))
        return z

    def patch_adjoint(self, g, scale, dy, alpha=1.0, stream=None):
        mfe_patch_adjoint(self.ctx, _dev_f64(g, self.n_dofs, "g"), scale.data_ptr(), alpha, dy.data_ptr(),
                          _stream_handle(stream))
        return dy

    def gmg_setup(self, stream=None, **opts):
        """Set up the multigrid level data at the current state (as a GMG CG solve does)."""
        mfe_gmg_setup(self.ctx, self.solve_opts(preconditioner="gmg", **opts), _stream_handle(stream))

    def gmg_apply(self, r, out=None, stream=None, net=False, **opts):
        """out = B r, one application of the GMG preconditioner (after gmg_setup with the same options);
        net=True: with the learned step in the finest post-smoother (set_network first)."""
        import torch
        if out is None:
            out = torch.empty_like(r)
        pc = "gmg_net" if net else "gmg"
        mfe_gmg_apply(self.ctx, self.solve_opts(preconditioner=pc, **opts), _dev_f64(r, self.n_dofs, "r"),
                      _dev_f64(out, self.n_dofs, "out"), _stream_handle(stream))
        return out

    def diagonal(self, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.n_dofs, dtype=torch.float64, device=self.device)
        mfe_diagonal(self.ctx, _dev_f64(out, self.n_dofs, "out"), _stream_handle(stream))
        return out

    def axpby(self, a, x, b, y, stream=None):
        """y = a x + b y (in place on y)."""
        mfe_axpby(self.ctx, a, _dev_f64(x, self.n_dofs, "x"), b, _dev_f64(y, self.n_dofs, "y"),
                  _stream_handle(stream))
        return y

    def dot(self, x, y, stream=None):
        """x . y (float64 device tensors), summed in a fixed order on the device."""
        return mfe_dot(self.ctx, _dev_f64(x, self.n_dofs, "x"), _dev_f64(y, self.n_dofs, "y"), _stream_handle(stream))

    def zero_constrained(self, v, stream=None):
        """v = 0 at the constrained dofs (in place)."""
        mfe_zero_constrained(self.ctx, _dev_f64(v, self.n_dofs, "v"), _stream_handle(stream))
        return v

    def solve_load_path(self, u, boundary_values, n_steps, min_fraction=1.0 / 256, on_step=None,
                        extrapolate=True, checkpoint=None, resume=False, stream=None, **opts):
        """Follow a load path t in (0, 1] with Newton-CG (Sec. 2.2, load stepping)
        through the library's driver (mfe_solve_load_path).

        boundary_values(t) -> (dofs, values): prescribed values at load t on the
        constrained dofs (constrained dofs it leaves out get 0).  Steps of
        1/n_steps; a step whose Newton solve fails is retried from the last
        converged state instead of the extrapolated one, then with half the
        increment (down to min_fraction), and later steps stay below 0.9 times
        the smallest increment that failed; the increment grows again by 1.25x
        after each converged step (up to those limits); each step starts from
        the linear extrapolation of the two previous converged states
        (extrapolate=True) or from the last converged state.
        u (device tensor) holds the state at t = 0 on entry and at t = 1 on return.
        on_step(t, u), if given, is called after every converged step.
        checkpoint: path of an .npz file rewritten after every converged step
        with everything the driver needs to go on (state, previous state, t,
        next increment and its limits); resume=True starts from that file
        instead of t = 0 (u is overwritten with its state), so a resumed path
        takes the same steps as an uninterrupted one.
        Returns a list of per-attempt reports (dicts with t, h, failed for the
        attempts that did not converge, and the Newton report); raises
        MfeError(MFE_ENOTCONV) when the increment falls below min_fraction.
        """
        import numpy as np
        import torch
        n = self.n_dofs
        _dev_f64(u, n, "u")
        prev = u.clone()
        st = PathState(0.0, 0.0, 0.0, 0.0)
        if resume:
            ck = load_checkpoint(checkpoint)
            if int(ck["n_steps"]) != n_steps or ck["u"].size != n:
                raise ValueError("checkpoint is of another path or mesh")
            u.copy_(torch.from_numpy(ck["u"]))
            prev.copy_(torch.from_numpy(ck["prev"]))
            prev_h = float(ck["prev_h"])
            st = PathState(float(ck["t"]), float(ck["h"]), float(ck["h_cap"]), 0.0 if np.isnan(prev_h) else prev_h)
        cidx = getattr(self, "_cidx", np.zeros(0, dtype=np.int64))

        def load(t):
            dofs, vals = boundary_values(t)
            g = np.zeros(n)
            g[np.asarray(dofs)] = vals
            return g[cidx]

        def step(state, u_ptr, prev_ptr):
            if checkpoint is not None:
                save_checkpoint(checkpoint, u=u, prev=prev, t=state.t, h=state.h, h_cap=state.h_cap,
                                prev_h=state.prev_h if state.prev_h > 0.0 else None, n_steps=n_steps)
            if on_step is not None:
                on_step(state.t, u)
            return False

        rc, reps = mfe_solve_load_path(self.ctx, self.solve_opts(**opts), u.data_ptr(), prev.data_ptr(), n_steps,
                                       min_fraction, extrapolate, st, load, step, stream=_stream_handle(stream))
        out = []
        for r in reps:
            d = dict(t=r.t, h=r.h)
            if r.failed:
                d["failed"] = True
            d.update(r.solve.as_dict())
            d["status"] = STATUS_NAMES.get(r.status, r.status)
            out.append(d)
        if rc != MFE_OK:
            raise MfeError(rc, mfe_last_error(self.ctx))
        return out

    def last_error(self):
        """Message of the last failed call on this operator ('' if none)."""
        return mfe_last_error(self.ctx)

    def set_timing(self, every=1):
        """Record the apply kernel of every `every`-th apply (True/1: each, 0/False: off)."""
        mfe_set_timing(self.ctx, int(every))

    def set_deterministic(self, on=True):
        """Coloured, bitwise reproducible summation of the applies (Q2 boxes)."""
        mfe_set_deterministic(self.ctx, on)

    def apply_kernel_ms(self):
        return mfe_apply_kernel_ms(self.ctx)
