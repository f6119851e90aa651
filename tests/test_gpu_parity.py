"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Metric (FP64 path): ||v_gpu - v_ref||_2 / ||v_ref||_2 <= 1e-12, element by
element on every dof for meshes the oracle finishes in seconds, and on
sampled dofs (computed one by one by the oracle) at the full benchmark sizes.
"""

import numpy as np
import pytest

import synthetic
from oracle.fem import Problem
from oracle.mesh import BoxMesh

pytestmark = pytest.mark.gpu

TOL = 1e-12
ALL = ["otf", "otf_geom", "t2", "t4", "otf_ad"]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda", 0)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _op(torch_dev, nx, ny, nz, p, verts, mu, lam, per_cell=None):
    import paper_2505_15535_amd as mfe
    return mfe.Operator(nx, ny, nz, p, verts, mu, lam, per_cell=per_cell, device=0)


def _to(torch_dev, x):
    torch, dev = torch_dev
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(dev)


def _apply_all(torch_dev, op, u, W, strategies=ALL):
    torch, _ = torch_dev
    op.set_state(_to(torch_dev, u))
    out = {}
    for s in strategies:
        op.build_cache(s)
        out[s] = np.stack([op.apply(_to(torch_dev, w), strategy=s).cpu().numpy() for w in W])
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("name", ["cube4_q2", "cube4_q2_jit"])
def test_parity_cube_all_vectors(torch_dev, name):
    cfg = synthetic.get_config(name)
    verts, u, W = cfg.vertices(), cfg.displacement(), cfg.test_vectors()
    print(f"case {name}", flush=True)
    P = Problem(BoxMesh(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts), cfg.mu, cfg.lam)
    K = P.assemble_tangent(u)
    ref = np.stack([K @ w for w in W])
    op = _op(torch_dev, cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts, cfg.mu, cfg.lam)
    got = _apply_all(torch_dev, op, u, W)
    for s, V in got.items():
        for k in range(len(W)):
            err = _rel(V[k], ref[k])
            assert err <= TOL, (s, k, err)


@pytest.mark.parametrize("p,shape", [(1, (5, 3, 2)), (2, (5, 3, 1)), (3, (3, 2, 2)), (4, (2, 2, 2)),
                                     (5, (2, 1, 2)), (6, (1, 2, 1))])
def test_parity_degrees_ragged(torch_dev, p, shape):
    """Every degree, cell counts that leave a partial last workgroup."""
    nx, ny, nz = shape
    rng = np.random.default_rng(100 + p)
    verts = synthetic.box_vertices(nx, ny, nz, (1.0, 0.7, 0.9), 0.1, rng)
    u = synthetic.sine_displacement(nx, ny, nz, p, 0.02, np.random.default_rng(200 + p))
    P = Problem(BoxMesh(nx, ny, nz, p, verts), 1.0, 10.0)
    assert P.min_jacobian(u) > 0.1
    W = np.random.default_rng(300 + p).standard_normal((2, P.mesh.n_dofs))
    ref = np.stack([P.apply_naive(u, w) for w in W])
    print(f"case degree {p} shape {shape}", flush=True)
    op = _op(torch_dev, nx, ny, nz, p, verts, 1.0, 10.0)
    got = _apply_all(torch_dev, op, u, W)
    for s, V in got.items():
        for k in range(2):
            assert _rel(V[k], ref[k]) <= TOL, (s, p, k, _rel(V[k], ref[k]))


@pytest.mark.parametrize("p", [1, 2, 3, 6])
def test_single_cell(torch_dev, p):
    verts = synthetic.box_vertices(1, 1, 1, (1.0, 2.0, 0.5))
    verts[7] += [0.1, -0.1, 0.05]
    u = synthetic.sine_displacement(1, 1, 1, p, 0.02, np.random.default_rng(p))
    P = Problem(BoxMesh(1, 1, 1, p, verts), 0.7, 3.0)
    w = np.random.default_rng(p + 9).standard_normal(P.mesh.n_dofs)
    ref = P.apply_naive(u, w)
    op = _op(torch_dev, 1, 1, 1, p, verts, 0.7, 3.0)
    got = _apply_all(torch_dev, op, u, [w])
    for s, V in got.items():
        assert _rel(V[0], ref) <= TOL, s


def test_residual_parity(torch_dev):
    cfg = synthetic.get_config("cube4_q2_jit")
    verts, u = cfg.vertices(), cfg.displacement()
    P = Problem(BoxMesh(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts), cfg.mu, cfg.lam)
    ref = P.residual(u)
    op = _op(torch_dev, cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts, cfg.mu, cfg.lam)
    r = op.residual(_to(torch_dev, u)).cpu().numpy()
    assert _rel(r, ref) <= TOL


def test_energy_parity(torch_dev):
    """Stored energy against the oracle (uniform and per-cell material), its
    directional derivative against the residual, and a non-finite value for
    an inverted state."""
    torch, _ = torch_dev
    cfg = synthetic.get_config("cube4_q2_jit")
    verts, u, w = cfg.vertices(), cfg.displacement(), cfg.test_vector(1)
    mesh = BoxMesh(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts)
    P = Problem(mesh, cfg.mu, cfg.lam)
    op = _op(torch_dev, cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts, cfg.mu, cfg.lam)
    ud = _to(torch_dev, u)
    e = op.energy(ud)
    assert abs(e - P.energy(u)) <= 1e-12 * abs(P.energy(u))
    eps = 1e-6
    de = (op.energy(ud + eps * _to(torch_dev, w)) - op.energy(ud - eps * _to(torch_dev, w))) / (2 * eps)
    rw = float(np.dot(op.residual(ud).cpu().numpy(), w))
    assert abs(de - rw) <= 1e-6 * abs(rw)
    ml = np.tile([cfg.mu, cfg.lam], (cfg.n_elems, 1))
    ml[::3] *= 50.0
    Pc = Problem(mesh, 0.0, 0.0, elem_mu_lam=ml)
    opc = _op(torch_dev, cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts, 1.0, 1.0, per_cell=ml)
    assert abs(opc.energy(ud) - Pc.energy(u)) <= 1e-12 * abs(Pc.energy(u))
    X = mesh.node_positions()
    assert not np.isfinite(op.energy(_to(torch_dev, (-2.0 * X).reshape(-1))))


def test_constraints_parity(torch_dev):
    cfg = synthetic.get_config("cube4_q2_jit")
    verts, u, W = cfg.vertices(), cfg.displacement(), cfg.test_vectors()[:2]
    mesh = BoxMesh(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts)
    left = np.where(mesh.node_positions()[:, 0] < 1e-12)[0]
    cdofs = np.concatenate([(3 * left[:, None] + np.arange(3)).ravel(), [5, 5, 700]])
    P = Problem(mesh, cfg.mu, cfg.lam, constrained_dofs=cdofs)
    op = _op(torch_dev, cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts, cfg.mu, cfg.lam)
    op.set_constraints(cdofs)
    got = _apply_all(torch_dev, op, u, W)
    for s, V in got.items():
        for k in range(2):
            ref = P.apply_naive(u, W[k])
            assert _rel(V[k], ref) <= TOL, s
            assert np.array_equal(V[k][cdofs], W[k][cdofs])
    r = op.residual(_to(torch_dev, u)).cpu().numpy()
    assert _rel(r, P.residual(u)) <= TOL
    assert np.all(r[cdofs] == 0.0)


def test_per_cell_material_parity(torch_dev):
    cfg = synthetic.get_config("cube4_q2_jit")
    verts, u, w = cfg.vertices(), cfg.displacement(), cfg.test_vector(3)
    ml = np.tile([cfg.mu, cfg.lam], (cfg.n_elems, 1))
    ml[::5] *= 100.0   # stiff inclusions
    P = Problem(BoxMesh(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts), 0.0, 0.0, elem_mu_lam=ml)
    ref = P.apply_naive(u, w)
    op = _op(torch_dev, cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts, 5.0, 5.0, per_cell=ml)
    got = _apply_all(torch_dev, op, u, [w])
    for s, V in got.items():
        assert _rel(V[0], ref) <= TOL, s


def _sampled(name, n_samples, seed):
    cfg = synthetic.get_config(name)
    verts, u, w = cfg.vertices(), cfg.displacement(), cfg.test_vector(0)
    P = Problem(BoxMesh(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts), cfg.mu, cfg.lam, chunk=256)
    dofs = np.sort(np.random.default_rng(seed).choice(P.mesh.n_dofs, n_samples, replace=False))
    return cfg, verts, u, w, dofs, P.apply_at(u, w, dofs)


@pytest.mark.parametrize("name,n_samples", [("box48_q2", 300), ("box24_q4", 120), ("box12_q6", 60)])
def test_full_size_sampled_and_properties(torch_dev, name, n_samples):
    torch, dev = torch_dev
    cfg, verts, u, w, dofs, ref = _sampled(name, n_samples, 7)
    print(f"case {name} full size", flush=True)
    op = _op(torch_dev, cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts, cfg.mu, cfg.lam)
    ud, wd = _to(torch_dev, u), _to(torch_dev, w)
    op.set_state(ud)
    full = {}
    for s in ALL:
        op.build_cache(s)
        v = op.apply(wd, strategy=s)
        full[s] = v.cpu().numpy()
        err = _rel(full[s][dofs], ref)
        assert err <= TOL, (s, err)
    # strategies agree everywhere
    for s in ALL[1:]:
        assert _rel(full[s], full["otf"]) <= TOL, s
    # symmetry and rigid translations at full size (GPU only)
    z = _to(torch_dev, cfg.test_vector(1))
    Kz = op.apply(z, strategy="otf")
    a = float(torch.dot(wd, Kz))
    b = float(torch.dot(z, torch.from_numpy(full["otf"]).to(dev)))
    assert abs(a - b) <= 1e-12 * float(torch.linalg.norm(wd) * torch.linalg.norm(Kz))
    t = torch.zeros_like(wd)
    t[0::3] = 1.0
    assert float(torch.linalg.norm(op.apply(t, strategy="t2"))) <= 1e-11 * np.linalg.norm(full["otf"])
    # central difference of the GPU residual
    eps = 1e-6 * float(ud.abs().max() / wd.abs().max())
    fd = (op.residual(ud + eps * wd) - op.residual(ud - eps * wd)) / (2 * eps)
    assert _rel(fd.cpu().numpy(), full["otf"]) < 1e-6


def test_repeated_applies_agree(torch_dev):
    torch, _ = torch_dev
    cfg = synthetic.get_config("box48_q2")
    op = _op(torch_dev, cfg.nx, cfg.ny, cfg.nz, cfg.degree, cfg.vertices(), cfg.mu, cfg.lam)
    op.set_state(_to(torch_dev, cfg.displacement()))
    wd = _to(torch_dev, cfg.test_vector(0))
    v1 = op.apply(wd, strategy="otf").clone()
    for _ in range(3):
        v2 = op.apply(wd, strategy="otf")
        # atomics may reorder the final sums: equal to rounding only
        assert float((v2 - v1).abs().max()) <= 1e-14 * float(v1.abs().max())


def test_error_paths(torch_dev):
    import paper_2505_15535_amd as mfe
    torch, dev = torch_dev
    cfg = synthetic.get_config("cube4_q2")
    verts = cfg.vertices()
    op = _op(torch_dev, cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts, cfg.mu, cfg.lam)
    w = _to(torch_dev, cfg.test_vector(0))
    with pytest.raises(mfe.MfeError) as e:
        op.apply(w, strategy="otf")
    assert e.value.code == mfe.MFE_ESTATE
    u = cfg.displacement()
    op.set_state(_to(torch_dev, u))
    with pytest.raises(mfe.MfeError) as e:
        op.apply(w, strategy="t4")           # cache not built
    assert e.value.code == mfe.MFE_ESTATE
    op.build_cache("t4")
    op.apply(w, strategy="t4")
    op.set_state(_to(torch_dev, 0.5 * u))
    with pytest.raises(mfe.MfeError) as e:
        op.apply(w, strategy="t4")           # stale after a new state
    assert e.value.code == mfe.MFE_ESTATE
    with pytest.raises(mfe.MfeError) as e:
        op.apply(w, out=w, strategy="otf")   # aliasing
    assert e.value.code == mfe.MFE_EINVAL
    with pytest.raises(mfe.MfeError) as e:
        op.apply(w, strategy="otf", precision=7)   # no such precision
    assert e.value.code == mfe.MFE_EINVAL
    # an inverting state: u = -2 X flips every cell
    X = BoxMesh(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts).node_positions()
    with pytest.raises(mfe.MfeError) as e:
        op.set_state(_to(torch_dev, (-2.0 * X).reshape(-1)))
    assert e.value.code == mfe.MFE_EJACOBIAN
    with pytest.raises(mfe.MfeError) as e:
        op.apply(w, strategy="otf")          # the failed state is not set
    assert e.value.code == mfe.MFE_ESTATE
    # an inverted mesh is refused at creation
    bad = verts.copy()
    bad[:, 0] *= -1.0
    with pytest.raises(mfe.MfeError) as e:
        _op(torch_dev, cfg.nx, cfg.ny, cfg.nz, cfg.degree, bad, 1.0, 1.0)
    assert e.value.code == mfe.MFE_EJACOBIAN


def test_zero_state_is_textbook_linear_elasticity(torch_dev):
    """The degenerate state u = 0: every strategy gives the textbook
    small-strain stiffness B^T D B with Lame constants (2 lambda, mu) (the
    energy's lambda log^2 J term) times w, on a jittered box."""
    from oracle import linelast
    nx, ny, nz, p = 3, 2, 2, 2
    verts = synthetic.box_vertices(nx, ny, nz, (1.0, 0.7, 0.9), 0.12, np.random.default_rng(61))
    mesh = BoxMesh(nx, ny, nz, p, verts)
    K0 = linelast.assemble(mesh, 2.0 * 10.0, 1.0)
    W = np.random.default_rng(62).standard_normal((2, mesh.n_dofs))
    op = _op(torch_dev, nx, ny, nz, p, verts, 1.0, 10.0)
    got = _apply_all(torch_dev, op, np.zeros(mesh.n_dofs), W)
    for s, V in got.items():
        for k in range(2):
            assert _rel(V[k], K0 @ W[k]) <= TOL, s


def test_mesh_limits_are_refused(torch_dev):
    """Sizes past 32-bit dof indices, degrees outside 1..6, empty meshes and
    null arrays are refused before anything is read or allocated."""
    import paper_2505_15535_amd as mfe
    ctx = mfe.mfe_create(0)
    try:
        one = np.zeros(3 * 8)
        for args in [(1000, 1000, 1000, 2), (1, 1, 1, 0), (1, 1, 1, 7), (0, 1, 1, 1)]:
            with pytest.raises(mfe.MfeError) as e:
                mfe.mfe_mesh_box(ctx, *args, one.ctypes.data)
            assert e.value.code == mfe.MFE_EINVAL, args
        with pytest.raises(mfe.MfeError) as e:
            mfe.mfe_mesh_box(ctx, 1, 1, 1, 2, None)
        assert e.value.code == mfe.MFE_EINVAL
        cells = np.arange(8, dtype=np.int32)
        with pytest.raises(mfe.MfeError) as e:
            mfe.mfe_mesh_hex(ctx, 8, one.ctypes.data, 0, cells.ctypes.data, 2)
        assert e.value.code == mfe.MFE_EINVAL
        with pytest.raises(mfe.MfeError) as e:
            mfe.mfe_mesh_hex(ctx, 8, one.ctypes.data, 1, cells.ctypes.data, 7)
        assert e.value.code == mfe.MFE_EINVAL
        assert mfe.mfe_n_dofs(ctx) == 0        # no mesh was set by any of them
        # a degenerate (flat) cell is refused by the geometry check
        flat = synthetic.box_vertices(1, 1, 1)
        flat[:, 2] = 0.0
        with pytest.raises(mfe.MfeError) as e:
            mfe.mfe_mesh_box(ctx, 1, 1, 1, 1, np.ascontiguousarray(flat).ctypes.data)
        assert e.value.code == mfe.MFE_EJACOBIAN
    finally:
        mfe.mfe_destroy(ctx)


def test_timed_applies(torch_dev):
    """Timed applies (start and stop events recorded by the dispatch) give the
    same product and one positive duration per timed launch."""
    torch, dev = torch_dev
    cfg = synthetic.get_config("cube4_q2_jit")
    verts = cfg.vertices()
    op = _op(torch_dev, cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts, cfg.mu, cfg.lam)
    op.set_state(_to(torch_dev, cfg.displacement()))
    w = _to(torch_dev, cfg.test_vector(0))
    for s in ("t2", "otf"):
        op.build_cache(s)
        ref = op.apply(w, strategy=s).cpu().numpy()
        op.set_timing(True)
        outs = [op.apply(w, strategy=s).cpu().numpy() for _ in range(3)]
        ms, n = op.apply_kernel_ms()
        op.set_timing(False)
        assert n == 3 and ms > 0.0, (s, ms, n)
        for v in outs:
            assert _rel(v, ref) <= 1e-14, s
        op.apply(w, strategy=s)                 # untimed: nothing recorded
        op.set_timing(True)
        assert op.apply_kernel_ms()[1] == 0
        op.set_timing(2)                        # every second apply, starting with the first
        for _ in range(5):
            op.apply(w, strategy=s)
        assert op.apply_kernel_ms()[1] == 3
        op.set_timing(False)
    import paper_2505_15535_amd as mfe
    with pytest.raises(mfe.MfeError) as e:
        op.set_timing(-1)
    assert e.value.code == mfe.MFE_EINVAL
