"""Mixed-precision tangent apply (FP32 sum-factorization sweeps) against the
FP64 CPU oracle.

Metric: ||v_fp32 - v_ref||_2 / ||v_ref||_2 <= 1e-5 with v_ref the oracle's
FP64 product.  The bound follows from the arithmetic: every output entry is a
sum over at most 8 cells of short FP32 dot products (6 one-dimensional sweeps
of length p+1 <= 7 and a 3x3 point-wise product per point), each with a
relative rounding error of a few units of 2^-24 ~ 6e-8 times the conditioning
of the sums; measured errors are about 1e-7..1e-6, so 1e-5 leaves an order of
magnitude of margin while still catching any FP64-vs-FP32 indexing mistake
(those give errors of order 1).
"""

import numpy as np
import pytest

import synthetic
from oracle.fem import Problem
from oracle.mesh import BoxMesh

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
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


def _apply32(torch_dev, op, u, W, strategies=ALL):
    torch, _ = torch_dev
    op.set_state(_to64(torch_dev, u))
    out = {}
    for s in strategies:
        op.build_cache(s, precision="fp32")
        out[s] = np.stack([op.apply(_to32(torch_dev, w), strategy=s, precision="fp32").cpu().numpy()
                           for w in W]).astype(np.float64)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("name", ["cube4_q2", "cube4_q2_jit"])
def test_fp32_parity_cube(torch_dev, name):
    import paper_2505_15535_amd as mfe
    cfg = synthetic.get_config(name)
    verts, u, W = cfg.vertices(), cfg.displacement(), cfg.test_vectors()
    # the FP32 path sees w rounded to FP32: compare with the oracle on that input
    W32 = W.astype(np.float32).astype(np.float64)
    P = Problem(BoxMesh(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts), cfg.mu, cfg.lam)
    K = P.assemble_tangent(u)
    ref = np.stack([K @ w for w in W32])
    op = mfe.Operator(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts, cfg.mu, cfg.lam, device=0)
    got = _apply32(torch_dev, op, u, W)
    for s, V in got.items():
        errs = [_rel(V[k], ref[k]) for k in range(len(W))]
        print(f"{name} {s}: max rel err {max(errs):.2e}")
        assert max(errs) <= TOL32, (s, errs)
        assert max(errs) > 0.0  # really computed in FP32


@pytest.mark.parametrize("p,shape", [(1, (5, 3, 2)), (2, (5, 3, 1)), (3, (3, 2, 2)), (4, (2, 2, 2)),
                                     (5, (2, 1, 2)), (6, (1, 2, 1))])
def test_fp32_degrees_ragged(torch_dev, p, shape):
    import paper_2505_15535_amd as mfe
    nx, ny, nz = shape
    verts = synthetic.box_vertices(nx, ny, nz, (1.0, 0.7, 0.9), 0.1, np.random.default_rng(100 + p))
    u = synthetic.sine_displacement(nx, ny, nz, p, 0.02, np.random.default_rng(200 + p))
    P = Problem(BoxMesh(nx, ny, nz, p, verts), 1.0, 10.0)
    W = np.random.default_rng(300 + p).standard_normal((2, P.mesh.n_dofs)).astype(np.float32)
    ref = np.stack([P.apply_naive(u, w.astype(np.float64)) for w in W])
    print(f"case degree {p} shape {shape}", flush=True)
    op = mfe.Operator(nx, ny, nz, p, verts, 1.0, 10.0, device=0)
    got = _apply32(torch_dev, op, u, W)
    for s, V in got.items():
        for k in range(2):
            assert _rel(V[k], ref[k]) <= TOL32, (s, p, k, _rel(V[k], ref[k]))


def test_fp32_constraints_and_cache_state(torch_dev):
    import paper_2505_15535_amd as mfe
    torch, dev = torch_dev
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
    with pytest.raises(mfe.MfeError) as e:
        op.apply(wd, strategy="t2", precision="fp32")     # FP32 cache not built
    assert e.value.code == mfe.MFE_ESTATE
    op.build_cache("t2")                                  # the FP64 cache is not the FP32 one
    with pytest.raises(mfe.MfeError) as e:
        op.apply(wd, strategy="t2", precision="fp32")
    assert e.value.code == mfe.MFE_ESTATE
    for s in ALL:
        op.build_cache(s, precision="fp32")
        v = op.apply(wd, strategy=s, precision="fp32").cpu().numpy()
        assert _rel(v.astype(np.float64), ref) <= TOL32, s
        assert np.array_equal(v[cdofs], w[cdofs])
    op.set_state(_to64(torch_dev, 0.5 * u))
    with pytest.raises(mfe.MfeError) as e:
        op.apply(wd, strategy="t4", precision="fp32")     # stale after a new state
    assert e.value.code == mfe.MFE_ESTATE
    with pytest.raises(ValueError):
        op.apply(_to64(torch_dev, w), strategy="otf", precision="fp32")   # dtype checked


@pytest.mark.parametrize("name,n_samples", [("box48_q2", 300), ("box24_q4", 120), ("box12_q6", 60)])
def test_fp32_full_size_sampled(torch_dev, name, n_samples):
    """The mixed-precision configurations at full size (Q4 on 24^3 and Q6 on
    12^3 cells, and Q2 on 48^3): sampled dofs against the oracle, and the
    whole vector against the FP64 GPU apply."""
    import paper_2505_15535_amd as mfe
    torch, dev = torch_dev
    cfg = synthetic.get_config(name)
    verts, u = cfg.vertices(), cfg.displacement()
    w = cfg.test_vector(0).astype(np.float32).astype(np.float64)
    P = Problem(BoxMesh(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts), cfg.mu, cfg.lam, chunk=256)
    dofs = np.sort(np.random.default_rng(7).choice(P.mesh.n_dofs, n_samples, replace=False))
    ref = P.apply_at(u, w, dofs)
    print(f"case {name} full size fp32", flush=True)
    op = mfe.Operator(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts, cfg.mu, cfg.lam, device=0)
    op.set_state(_to64(torch_dev, u))
    w64, w32 = _to64(torch_dev, w), _to32(torch_dev, w)
    op.build_cache("otf_geom")
    v64 = op.apply(w64, strategy="otf").cpu().numpy()
    for s in ALL:
        op.build_cache(s, precision="fp32")
        v = op.apply(w32, strategy=s, precision="fp32").cpu().numpy().astype(np.float64)
        e_samp, e_full = _rel(v[dofs], ref), _rel(v, v64)
        print(f"{name} {s}: sampled rel err {e_samp:.2e}, full-vector rel err vs FP64 {e_full:.2e}")
        assert e_samp <= TOL32 and e_full <= TOL32, (s, e_samp, e_full)
