"""GPU tests of the Q2 box applies' summation modes and full-size parity.

* Coloured mode (eight launches, one per parity class of the brick position,
  plain read-add-writes): agrees with the atomic mode to 1e-13 and repeats
  bitwise; matches the oracle on ragged and constrained boxes.
* Every dof of the benchmark workloads (48^3 Q2, 24^3 Q4, 12^3 Q6) against
  the oracle's naive cell loop, FP64 to 1e-12 and FP32 sweeps to 1e-5.
"""

import numpy as np
import pytest

import synthetic
from oracle.fem import Problem
from oracle.mesh import BoxMesh

pytestmark = pytest.mark.gpu

TOL = 1e-12
TOL32 = 1e-5
ALL = ["otf", "otf_geom", "t2", "t4", "otf_ad"]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda", 0)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _to(torch_dev, x, dtype=None):
    torch, dev = torch_dev
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(dev)
    return t if dtype is None else t.to(dtype)


def _op(nx, ny, nz, p, verts, mu, lam):
    import paper_2505_15535_amd as mfe
    return mfe.Operator(nx, ny, nz, p, verts, mu, lam, device=0)


def test_coloured_agrees_with_atomic_and_repeats_bitwise(torch_dev):
    torch, _ = torch_dev
    cfg = synthetic.get_config("box48_q2")
    print("case box48_q2 coloured vs atomic", flush=True)
    op = _op(cfg.nx, cfg.ny, cfg.nz, cfg.degree, cfg.vertices(), cfg.mu, cfg.lam)
    op.set_state(_to(torch_dev, cfg.displacement()))
    w = _to(torch_dev, cfg.test_vector(0))
    for prec, tol in (("fp64", 1e-13), ("fp32", 1e-6)):
        wp = w if prec == "fp64" else w.float()
        for s in ("otf", "t2", "t4", "otf_ad"):
            op.build_cache(s, precision=prec)
            op.set_deterministic(False)
            va = op.apply(wp, strategy=s, precision=prec).double()
            op.set_deterministic(True)
            v1 = op.apply(wp, strategy=s, precision=prec).clone()
            for _ in range(3):
                v2 = op.apply(wp, strategy=s, precision=prec)
                assert torch.equal(v1, v2), (prec, s)
            err = float(torch.linalg.norm(v1.double() - va) / torch.linalg.norm(va))
            assert err <= tol, (prec, s, err)
    op.set_deterministic(False)
    op.close()


@pytest.mark.parametrize("shape", [(5, 3, 1), (3, 5, 3), (9, 2, 2), (1, 1, 1)])
def test_coloured_ragged_constrained_parity(torch_dev, shape):
    """Ragged brick grids, with and without constraints, in both modes."""
    nx, ny, nz = shape
    p = 2
    rng = np.random.default_rng(sum(shape))
    verts = synthetic.box_vertices(nx, ny, nz, (1.0, 0.8, 0.9), 0.1, rng)
    u = synthetic.sine_displacement(nx, ny, nz, p, 0.02, np.random.default_rng(5 + nx))
    mesh = BoxMesh(nx, ny, nz, p, verts)
    X = mesh.node_positions()
    left = np.where(X[:, 0] < 1e-12)[0]
    cdofs = np.concatenate([(3 * left[:, None] + np.arange(3)).ravel(), [7, 7, mesh.n_dofs - 2]])
    W = np.random.default_rng(9).standard_normal((2, mesh.n_dofs))
    print(f"case coloured shape {shape}", flush=True)
    for constrained in (False, True):
        P = Problem(mesh, 1.0, 10.0, constrained_dofs=cdofs if constrained else None)
        refs = [P.apply_naive(u, wk) for wk in W]
        op = _op(nx, ny, nz, p, verts, 1.0, 10.0)
        if constrained:
            op.set_constraints(cdofs)
        op.set_state(_to(torch_dev, u))
        for det in (False, True):
            op.set_deterministic(det)
            for s in ALL:
                op.build_cache(s)
                for k in range(2):
                    v = op.apply(_to(torch_dev, W[k]), strategy=s).cpu().numpy()
                    assert _rel(v, refs[k]) <= TOL, (constrained, det, s, k, _rel(v, refs[k]))
                    if constrained:
                        assert np.array_equal(v[cdofs], W[k][cdofs])
        op.close()


def test_coloured_mode_limits(torch_dev):
    """The coloured mode covers Q2 boxes with vector-ALU sweeps only."""
    import paper_2505_15535_amd as mfe
    cfg = synthetic.get_config("cube4_q2")
    op = _op(cfg.nx, cfg.ny, cfg.nz, 3, synthetic.box_vertices(cfg.nx, cfg.ny, cfg.nz), 1.0, 1.0)
    op.set_state(_to(torch_dev, np.zeros(op.n_dofs)))
    op.set_deterministic(True)
    with pytest.raises(mfe.MfeError) as e:
        op.apply(_to(torch_dev, np.ones(op.n_dofs)), strategy="otf")
    assert e.value.code == mfe.MFE_EUNSUPPORTED
    op.close()


_FULL = {}


def _oracle_full(name):
    """The oracle's naive cell loop over every cell of a benchmark workload."""
    if name not in _FULL:
        cfg = synthetic.get_config(name)
        verts, u, w = cfg.vertices(), cfg.displacement(), cfg.test_vector(0)
        print(f"oracle {name}: naive apply over {cfg.n_elems} cells", flush=True)
        P = Problem(BoxMesh(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts), cfg.mu, cfg.lam, chunk=512)
        _FULL[name] = (cfg, verts, u, w, P.apply_naive(u, w))
        print(f"oracle {name}: done", flush=True)
    return _FULL[name]


@pytest.mark.parametrize("name", ["box48_q2", "box24_q4", "box12_q6"])
def test_full_size_every_dof(torch_dev, name):
    """Whole-vector parity at the benchmark sizes, every strategy, FP64 and
    FP32 sweeps (w rounded to FP32 for the latter, compared with the FP64
    oracle on the same rounded w)."""
    torch, _ = torch_dev
    cfg, verts, u, w, ref = _oracle_full(name)
    print(f"case {name} every dof", flush=True)
    op = _op(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts, cfg.mu, cfg.lam)
    op.set_state(_to(torch_dev, u))
    wd = _to(torch_dev, w)
    for s in ALL:
        op.build_cache(s)
        v = op.apply(wd, strategy=s).cpu().numpy()
        assert _rel(v, ref) <= TOL, (name, s, _rel(v, ref))
    # FP32: the oracle is linear in w, so compare with ref + K (w32 - w) is
    # not needed: the rounding of w (2^-24 relative) is below the 1e-5 bound
    w32 = wd.float()
    for s in ("otf", "t2", "t4"):
        op.build_cache(s, precision="fp32")
        v = op.apply(w32, strategy=s, precision="fp32").double().cpu().numpy()
        assert _rel(v, ref) <= TOL32, (name, s, "fp32", _rel(v, ref))
    op.close()
