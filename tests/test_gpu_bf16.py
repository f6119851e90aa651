"""Tangent apply with the sum-factorization sweeps of w on the matrix cores
(16x16x16 bf16 products, FP32 accumulation) against the FP64 CPU oracle.

bf16x3 splits every FP32 operand into three bf16 pieces (8 significant bits
each, so the split is exact) and keeps the six piece products of order <= 2;
the dropped products are below 2^-24 relative, the products are exact in the
FP32 accumulator and the sums round as in the FP32 sweeps, so the FP32 bound
applies: ||v - v_ref|| / ||v_ref|| <= 1e-5 (the same derivation as for the
FP32 sweeps; measured errors are of the same size as theirs).

bf16 (one product) rounds both operands of every sweep to bf16, unit roundoff
u = 2^-9 ~ 2e-3.  The w field passes through three forward stages, the
point-wise product and three backward stages, and every stage rounds its
inputs and its 1D matrix once each, so to first order the relative error of a
product is at most 2 * 6 u ~ 2.3e-2 times the conditioning of the short sums
(the derivative rows of D sum to zero, which amplifies it on smooth fields; a
random w is rough, so the amplification stays small).  The tests assert
<= 3e-2, and > 1e-4 to show that the products really ran in bf16.
"""

import numpy as np
import pytest

import synthetic
from oracle.fem import Problem
from oracle.mesh import BoxMesh

pytestmark = pytest.mark.gpu

TOL_X3 = 1e-5
TOL_BF16 = 3e-2
FLOOR_BF16 = 1e-4
ALL = ["otf", "otf_geom", "t2", "t4", "otf_ad"]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda", 0)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _to32(torch_dev, x):
    torch, dev = torch_dev
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)


def _to64(torch_dev, x):
    torch, dev = torch_dev
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(dev)


def _apply(torch_dev, op, u, W, prec, strategies=ALL):
    torch, _ = torch_dev
    op.set_state(_to64(torch_dev, u))
    out = {}
    for s in strategies:
        op.build_cache(s, precision=prec)
        out[s] = np.stack([op.apply(_to32(torch_dev, w), strategy=s, precision=prec).cpu().numpy()
                           for w in W]).astype(np.float64)
    torch.cuda.synchronize()
    return out


def _check(errs, prec, what):
    if prec == "bf16x3":
        assert max(errs) <= TOL_X3, (what, errs)
    else:
        assert FLOOR_BF16 < min(errs) and max(errs) <= TOL_BF16, (what, errs)


@pytest.mark.parametrize("prec", ["bf16x3", "bf16"])
@pytest.mark.parametrize("name", ["cube4_q2", "cube4_q2_jit"])
def test_mfma_parity_cube(torch_dev, name, prec):
    import paper_2505_15535_amd as mfe
    cfg = synthetic.get_config(name)
    verts, u, W = cfg.vertices(), cfg.displacement(), cfg.test_vectors()
    W32 = W.astype(np.float32).astype(np.float64)
    P = Problem(BoxMesh(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts), cfg.mu, cfg.lam)
    K = P.assemble_tangent(u)
    ref = np.stack([K @ w for w in W32])
    print(f"case {name} {prec}", flush=True)
    op = mfe.Operator(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts, cfg.mu, cfg.lam, device=0)
    got = _apply(torch_dev, op, u, W, prec)
    for s, V in got.items():
        errs = [_rel(V[k], ref[k]) for k in range(len(W))]
        print(f"{name} {prec} {s}: max rel err {max(errs):.2e}")
        _check(errs, prec, s)


@pytest.mark.parametrize("prec", ["bf16x3", "bf16"])
@pytest.mark.parametrize("p,shape", [(1, (5, 3, 2)), (2, (5, 3, 1)), (3, (3, 2, 2)), (4, (2, 2, 2)),
                                     (5, (2, 1, 2)), (6, (1, 2, 1))])
def test_mfma_degrees_ragged(torch_dev, p, shape, prec):
    import paper_2505_15535_amd as mfe
    nx, ny, nz = shape
    verts = synthetic.box_vertices(nx, ny, nz, (1.0, 0.7, 0.9), 0.1, np.random.default_rng(100 + p))
    u = synthetic.sine_displacement(nx, ny, nz, p, 0.02, np.random.default_rng(200 + p))
    P = Problem(BoxMesh(nx, ny, nz, p, verts), 1.0, 10.0)
    W = np.random.default_rng(300 + p).standard_normal((2, P.mesh.n_dofs)).astype(np.float32)
    ref = np.stack([P.apply_naive(u, w.astype(np.float64)) for w in W])
    print(f"case degree {p} shape {shape} {prec}", flush=True)
    op = mfe.Operator(nx, ny, nz, p, verts, 1.0, 10.0, device=0)
    got = _apply(torch_dev, op, u, W, prec)
    for s, V in got.items():
        errs = [_rel(V[k], ref[k]) for k in range(2)]
        print(f"degree {p} {prec} {s}: max rel err {max(errs):.2e}")
        _check(errs, prec, (s, p))


def test_mfma_constraints_and_agreement(torch_dev):
    """Constrained rows pass w through; bf16x3 and the FP32 vector-ALU sweeps
    agree to FP32 rounding on the same FP32 cache."""
    import paper_2505_15535_amd as mfe
    cfg = synthetic.get_config("cube4_q2_jit")
    verts, u, w = cfg.vertices(), cfg.displacement(), cfg.test_vector(0).astype(np.float32)
    mesh = BoxMesh(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts)
    left = np.where(mesh.node_positions()[:, 0] < 1e-12)[0]
    cdofs = (3 * left[:, None] + np.arange(3)).ravel()
    P = Problem(mesh, cfg.mu, cfg.lam, constrained_dofs=cdofs)
    ref = P.apply_naive(u, w.astype(np.float64))
    op = mfe.Operator(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts, cfg.mu, cfg.lam, device=0)
    op.set_constraints(cdofs)
    op.set_state(_to64(torch_dev, u))
    wd = _to32(torch_dev, w)
    for s in ALL:
        op.build_cache(s, precision="fp32")
        v32 = op.apply(wd, strategy=s, precision="fp32").cpu().numpy().astype(np.float64)
        for prec in ("bf16x3", "bf16"):
            v = op.apply(wd, strategy=s, precision=prec).cpu().numpy()
            assert np.array_equal(v[cdofs], w[cdofs]), (s, prec)
            _check([_rel(v.astype(np.float64), ref)], prec, (s, "constrained"))
            if prec == "bf16x3":
                assert _rel(v.astype(np.float64), v32) <= TOL_X3, s
    with pytest.raises(ValueError):
        op.apply(_to64(torch_dev, w), strategy="otf", precision="bf16")   # dtype checked


@pytest.mark.parametrize("name,n_samples", [("box48_q2", 300), ("box24_q4", 120), ("box12_q6", 60)])
def test_mfma_full_size_sampled(torch_dev, name, n_samples):
    """Full-size boxes (Q2 on 48^3, Q4 on 24^3, Q6 on 12^3 cells): sampled
    dofs against the oracle, the whole vector against the FP64 GPU apply."""
    import paper_2505_15535_amd as mfe
    cfg = synthetic.get_config(name)
    verts, u = cfg.vertices(), cfg.displacement()
    w = cfg.test_vector(0).astype(np.float32).astype(np.float64)
    P = Problem(BoxMesh(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts), cfg.mu, cfg.lam, chunk=256)
    dofs = np.sort(np.random.default_rng(7).choice(P.mesh.n_dofs, n_samples, replace=False))
    ref = P.apply_at(u, w, dofs)
    print(f"case {name} full size matrix-core sweeps", flush=True)
    op = mfe.Operator(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts, cfg.mu, cfg.lam, device=0)
    op.set_state(_to64(torch_dev, u))
    w64, w32 = _to64(torch_dev, w), _to32(torch_dev, w)
    v64 = op.apply(w64, strategy="otf").cpu().numpy()
    for s in ("t2", "t4", "otf"):
        op.build_cache(s, precision="fp32")
        for prec in ("bf16x3", "bf16"):
            v = op.apply(w32, strategy=s, precision=prec).cpu().numpy().astype(np.float64)
            e_samp, e_full = _rel(v[dofs], ref), _rel(v, v64)
            print(f"{name} {s} {prec}: sampled rel err {e_samp:.2e}, full-vector rel err vs FP64 {e_full:.2e}")
            _check([e_samp, e_full], prec, (s, name))
