"""The split neo-Hookean law (eq. hypcomplex) through the model-independent
strategies: dual-number on-the-fly apply and the fourth-order cache filled
from dual-number derivatives, against the FP64 oracle (material_split)."""

import numpy as np
import pytest

import synthetic
from oracle.fem import Problem
from oracle.mesh import BoxMesh

pytestmark = pytest.mark.gpu

TOL = 1e-12
SPLIT = ["otf_ad", "t4"]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda", 0)


def _to(torch_dev, x, dtype=None):
    torch, dev = torch_dev
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dtype or np.float64)).to(dev)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _op(nx, ny, nz, p, verts, mu, kappa, per_cell=None):
    import paper_2505_15535_amd as mfe
    op = mfe.Operator(nx, ny, nz, p, verts, mu, kappa, device=0)
    op.set_model("split")
    if per_cell is not None:
        op.set_material(mu, kappa, per_cell=per_cell)
    return op


@pytest.mark.parametrize("p,shape", [(1, (3, 2, 2)), (2, (4, 4, 4)), (3, (3, 2, 1)), (4, (2, 2, 1))])
def test_split_apply_parity(torch_dev, p, shape):
    nx, ny, nz = shape
    verts = synthetic.box_vertices(nx, ny, nz, (1.0, 0.8, 0.9), 0.1, np.random.default_rng(40 + p))
    u = synthetic.sine_displacement(nx, ny, nz, p, 0.03, np.random.default_rng(50 + p))
    mu, kappa = 1.0, 25.0
    P = Problem(BoxMesh(nx, ny, nz, p, verts), mu, kappa, model="split")
    assert P.min_jacobian(u) > 0.1
    W = np.random.default_rng(60 + p).normal(size=(2, P.mesh.n_dofs))
    ref = np.stack([P.apply_naive(u, w) for w in W])
    op = _op(nx, ny, nz, p, verts, mu, kappa)
    op.set_state(_to(torch_dev, u))
    for s in SPLIT:
        op.build_cache(s)
        for k in range(2):
            v = op.apply(_to(torch_dev, W[k]), strategy=s).cpu().numpy()
            assert _rel(v, ref[k]) <= TOL, (s, p, k, _rel(v, ref[k]))
        op.build_cache(s, precision="fp32")
        v32 = op.apply(_to(torch_dev, W[0], np.float32), strategy=s, precision="fp32").cpu().numpy()
        ref32 = P.apply_naive(u, W[0].astype(np.float32).astype(np.float64))
        assert _rel(v32.astype(np.float64), ref32) <= 1e-5, (s, p)
        # the matrix-core sweeps read the same FP32 cache (bounds derived in test_gpu_bf16)
        for prec, lo, hi in (("bf16x3", 0.0, 1e-5), ("bf16", 1e-4, 3e-2)):
            vb = op.apply(_to(torch_dev, W[0], np.float32), strategy=s, precision=prec).cpu().numpy()
            e = _rel(vb.astype(np.float64), ref32)
            assert lo < e <= hi, (s, p, prec, e)
    # residual and energy of the split law
    r = op.residual(_to(torch_dev, u)).cpu().numpy()
    assert _rel(r, P.residual(u)) <= TOL
    assert abs(op.energy(_to(torch_dev, u)) - P.energy(u)) <= 1e-12 * abs(P.energy(u))


def test_split_per_cell_constraints_and_unsupported(torch_dev):
    import paper_2505_15535_amd as mfe
    cfg = synthetic.get_config("cube4_q2_jit")
    verts, u, w = cfg.vertices(), cfg.displacement(), cfg.test_vector(0)
    mesh = BoxMesh(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts)
    ml = np.tile([1.0, 15.0], (cfg.n_elems, 1))
    ml[::4] *= 30.0
    left = np.where(mesh.node_positions()[:, 0] < 1e-12)[0]
    cdofs = (3 * left[:, None] + np.arange(3)).ravel()
    P = Problem(mesh, 0.0, 0.0, elem_mu_lam=ml, constrained_dofs=cdofs, model="split")
    op = _op(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts, 1.0, 1.0, per_cell=ml)
    op.set_constraints(cdofs)
    op.set_state(_to(torch_dev, u))
    ref = P.apply_naive(u, w)
    for s in SPLIT:
        op.build_cache(s)
        v = op.apply(_to(torch_dev, w), strategy=s).cpu().numpy()
        assert _rel(v, ref) <= TOL, s
        assert np.array_equal(v[cdofs], w[cdofs])
    for s in ("otf", "otf_geom", "t2"):
        with pytest.raises(mfe.MfeError) as e:
            op.build_cache(s)
            op.apply(_to(torch_dev, w), strategy=s)
        assert e.value.code == mfe.MFE_EUNSUPPORTED, s
    with pytest.raises(mfe.MfeError) as e:
        op.cg_solve(_to(torch_dev, w), preconditioner="jacobi")
    assert e.value.code == mfe.MFE_EUNSUPPORTED
    # back to the other law: T4 is rebuilt for it
    op.set_model("nh")
    with pytest.raises(mfe.MfeError) as e:
        op.apply(_to(torch_dev, w), strategy="t4")
    assert e.value.code == mfe.MFE_ESTATE


def test_split_full_size_sampled(torch_dev):
    cfg = synthetic.get_config("box48_q2")
    verts, u, w = cfg.vertices(), cfg.displacement(), cfg.test_vector(0)
    P = Problem(BoxMesh(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts), cfg.mu, cfg.lam, chunk=256, model="split")
    dofs = np.sort(np.random.default_rng(11).choice(P.mesh.n_dofs, 200, replace=False))
    ref = P.apply_at(u, w, dofs)
    op = _op(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts, cfg.mu, cfg.lam)
    op.set_state(_to(torch_dev, u))
    full = {}
    for s in SPLIT:
        op.build_cache(s)
        full[s] = op.apply(_to(torch_dev, w), strategy=s).cpu().numpy()
        assert _rel(full[s][dofs], ref) <= TOL, s
    assert _rel(full["t4"], full["otf_ad"]) <= TOL
