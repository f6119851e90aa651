"""The allocation-free energy entry point through the C ABI: its result
against mfe_energy (the existing entry point, same kernels) and the oracle,
on two calls in a row on one GPU, the second on a smaller mesh, so the
second reads nothing the first left in the shared device array."""

import ctypes

import numpy as np
import pytest

import synthetic
from oracle.fem import Problem
from oracle.mesh import BoxMesh

pytestmark = pytest.mark.gpu


def _energy_pair(mfe, torch, nx, ny, nz, p, seed):
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(seed)
    verts = synthetic.box_vertices(nx, ny, nz, (1.0, 0.8, 0.9), 0.1, rng)
    u = synthetic.sine_displacement(nx, ny, nz, p, 0.03, np.random.default_rng(seed + 1))
    ctx = mfe.mfe_create(0)
    try:
        mfe.mfe_mesh_box(ctx, nx, ny, nz, p, np.ascontiguousarray(verts).ctypes.data)
        mfe.mfe_set_material(ctx, 1.0, 10.0)
        ud = torch.from_numpy(u).to(dev)
        out = torch.full((1,), np.nan, dtype=torch.float64, device=dev)
        stream = torch.cuda.current_stream().cuda_stream
        mfe.mfe_energy_noalloc(ctx, ctypes.c_void_p(ud.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                               ctypes.c_void_p(stream))
        torch.cuda.synchronize()
        e_noalloc = float(out.item())
        e_ref = mfe.mfe_energy(ctx, ctypes.c_void_p(ud.data_ptr()), ctypes.c_void_p(stream))
    finally:
        mfe.mfe_destroy(ctx)
    e_oracle = Problem(BoxMesh(nx, ny, nz, p, verts), 1.0, 10.0).energy(u)
    return e_noalloc, e_ref, e_oracle


def test_energy_noalloc_two_calls_smaller_second():
    import torch
    import paper_2505_15535_amd as mfe
    assert torch.cuda.is_available()
    cases = [(12, 10, 9, 2, 31), (3, 2, 2, 2, 41)]   # 12*10*9 cells first, then 12
    for nx, ny, nz, p, seed in cases:
        print(f"case noalloc energy {nx}x{ny}x{nz} Q{p}", flush=True)
        e_na, e_ref, e_or = _energy_pair(mfe, torch, nx, ny, nz, p, seed)
        assert np.isfinite(e_na)
        assert abs(e_na - e_ref) <= 1e-14 * abs(e_ref), (e_na, e_ref)
        assert abs(e_na - e_or) <= 1e-12 * abs(e_or), (e_na, e_or)


def test_energy_noalloc_refuses_null_and_oversize():
    """Null pointers, and a mesh with more bricks of cells (Q6: one cell per
    brick) than the fixed array holds, are refused before any launch."""
    import torch
    import paper_2505_15535_amd as mfe
    dev = torch.device("cuda", 0)
    ctx = mfe.mfe_create(0)
    try:
        verts = synthetic.box_vertices(1, 1, 1)
        mfe.mfe_mesh_box(ctx, 1, 1, 1, 2, np.ascontiguousarray(verts).ctypes.data)
        with pytest.raises(mfe.MfeError) as e:
            mfe.mfe_energy_noalloc(ctx, None, None, None)
        assert e.value.code == mfe.MFE_EINVAL
        nx, ny, nz = 66, 64, 63                       # 266,112 cells > 2^18
        big = synthetic.box_vertices(nx, ny, nz)
        mfe.mfe_mesh_box(ctx, nx, ny, nz, 6, np.ascontiguousarray(big).ctypes.data)
        u = torch.zeros(mfe.mfe_n_dofs(ctx), dtype=torch.float64, device=dev)
        out = torch.zeros(1, dtype=torch.float64, device=dev)
        with pytest.raises(mfe.MfeError) as e:
            mfe.mfe_energy_noalloc(ctx, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(out.data_ptr()), None)
        assert e.value.code == mfe.MFE_EINVAL
        assert "at most" in str(e.value)
        assert float(out.item()) == 0.0               # nothing was written
    finally:
        mfe.mfe_destroy(ctx)
