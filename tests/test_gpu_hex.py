"""General hexahedral meshes on the GPU (mfe_mesh_hex) against the FP64 CPU
oracle: every strategy and degree on an unstructured cube-in-cube mesh with
random vertex numbering, cell rotations and cell order; FP32 sweeps; residual,
energy, diagonal, constraints, per-cell material, the split law; a Newton
solve; and, at full size, sampled dofs against the oracle and the
general-mesh kernels against the structured-box kernels on the same box.

Metric: ||v_gpu - v_ref||_2 / ||v_ref||_2 <= 1e-12 (FP64), <= 1e-5 (FP32
sweeps; the bound is derived with the box tests)."""

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle.solver
import synthetic
from oracle.fem import Problem
from oracle.mesh import HexMesh

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


def _to(torch_dev, x, dtype=np.float64):
    torch, dev = torch_dev
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dtype)).to(dev)


def _mesh(m, seed, relabel=True):
    v, c = synthetic.cube_in_cube(m, jitter=0.1, rng=np.random.default_rng(seed))
    if relabel:
        v, c, _, _ = synthetic.relabel(v, c, np.random.default_rng(seed + 1), shuffle_cells=True)
    return v, c


def _op(v, c, p, mu=1.0, lam=10.0, per_cell=None):
    import paper_2505_15535_amd as mfe
    return mfe.Operator.from_hex(v, c, p, mu, lam, per_cell=per_cell, device=0)


def _state(H, amp, seed):
    u = synthetic.sine_field(H.node_positions(), amp, np.random.default_rng(seed))
    return u


# Q1 groups 32 cells per workgroup, Q2 9, Q3 4, Q4 2, Q5/Q6 1: m = 3 gives 189
# cells (ragged for Q1, Q3 and Q4), m = 2 gives 56 (ragged for Q2)
@pytest.mark.parametrize("p,m", [(1, 3), (2, 2), (3, 3), (4, 3), (5, 1), (6, 1)])
def test_hex_parity_every_strategy(torch_dev, p, m):
    torch, _ = torch_dev
    v, c = _mesh(m, 10 + p)
    H = HexMesh(v, c, p)
    P = Problem(H, 1.0, 10.0)
    u = _state(H, 0.02, 20 + p)
    assert P.min_jacobian(u) > 0.1
    W = np.random.default_rng(30 + p).standard_normal((2, H.n_dofs))
    ref = [P.apply_naive(u, w) for w in W]
    print(f"case hex degree {p} m {m} cells {H.n_elems}", flush=True)
    op = _op(v, c, p)
    assert op.n_dofs == H.n_dofs and op.n_cells == H.n_elems
    assert np.abs(op.node_coordinates() - H.node_positions()).max() < 1e-14
    op.set_state(_to(torch_dev, u))
    for s in ALL:
        op.build_cache(s)
        for k in range(2):
            got = op.apply(_to(torch_dev, W[k]), strategy=s).cpu().numpy()
            assert _rel(got, ref[k]) <= TOL, (s, k, _rel(got, ref[k]))
        op.build_cache(s, precision="fp32")
        got = op.apply(_to(torch_dev, W[0], np.float32), strategy=s, precision="fp32").cpu().numpy()
        assert _rel(got.astype(np.float64), ref[0]) <= TOL32, (s, "fp32")
    torch.cuda.synchronize()


def test_hex_residual_energy_diagonal_constraints_material(torch_dev):
    torch, _ = torch_dev
    v, c = _mesh(2, 40)
    H = HexMesh(v, c, 2)
    u = _state(H, 0.03, 41)
    ud = _to(torch_dev, u)
    X = H.node_positions()
    bottom = np.where(X[:, 2] < 1e-12)[0]
    cdofs = (3 * bottom[:, None] + np.arange(3)).ravel()
    ml = np.tile([1.0, 10.0], (H.n_elems, 1))
    ml[::4] *= 30.0
    P = Problem(H, 0.0, 0.0, constrained_dofs=cdofs, elem_mu_lam=ml)
    op = _op(v, c, 2, 5.0, 5.0, per_cell=ml)
    op.set_constraints(cdofs)
    r = op.residual(ud).cpu().numpy()
    assert _rel(r, P.residual(u)) <= TOL
    assert np.all(r[cdofs] == 0.0)
    assert abs(op.energy(ud) - P.energy(u)) <= 1e-12 * abs(P.energy(u))
    op.set_state(ud)
    w = np.random.default_rng(42).standard_normal(H.n_dofs)
    ref = P.apply_naive(u, w)
    for s in ALL:
        op.build_cache(s)
        got = op.apply(_to(torch_dev, w), strategy=s).cpu().numpy()
        assert _rel(got, ref) <= TOL, s
        assert np.array_equal(got[cdofs], w[cdofs])
    d = op.diagonal().cpu().numpy()
    assert _rel(d, P.assemble_tangent(u).diagonal()) <= TOL


def test_hex_split_law(torch_dev):
    v, c = _mesh(2, 50)
    H = HexMesh(v, c, 2)
    u = _state(H, 0.03, 51)
    P = Problem(H, 1.0, 30.0, model="split")
    op = _op(v, c, 2, 1.0, 30.0)
    op.set_model("split")
    ud = _to(torch_dev, u)
    assert _rel(op.residual(ud).cpu().numpy(), P.residual(u)) <= TOL
    op.set_state(ud)
    w = np.random.default_rng(52).standard_normal(H.n_dofs)
    ref = P.apply_naive(u, w)
    for s in ("otf_ad", "t4"):
        op.build_cache(s)
        assert _rel(op.apply(_to(torch_dev, w), strategy=s).cpu().numpy(), ref) <= TOL, s


def test_hex_newton_matches_oracle(torch_dev):
    """Compress and shear the unstructured cube (bottom clamped, top moved in
    two load steps): GPU Newton-CG with Jacobi against the oracle's Newton
    with direct solves."""
    torch, dev = torch_dev
    v, c = _mesh(1, 60)
    H = HexMesh(v, c, 2)
    X = H.node_positions()
    bottom = np.where(X[:, 2] < 1e-12)[0]
    top = np.where(X[:, 2] > 1.0 - 1e-12)[0]
    cdofs = np.sort(np.concatenate([(3 * bottom[:, None] + np.arange(3)).ravel(),
                                    (3 * top[:, None] + np.arange(3)).ravel()]))

    def bc(t):
        g = np.zeros((H.n_nodes, 3))
        g[top] = t * np.array([0.04, -0.02, -0.06])
        return cdofs, g.reshape(-1)[cdofs]

    P = Problem(H, 1.0, 20.0, constrained_dofs=cdofs)
    u_ref = np.zeros(H.n_dofs)
    for t in (0.5, 1.0):
        d, g = bc(t)
        u_ref, _ = oracle.solver.newton(P, u_ref, d, g, atol=1e-11)
    op = _op(v, c, 2, 1.0, 20.0)
    op.set_constraints(cdofs)
    u = torch.zeros(H.n_dofs, dtype=torch.float64, device=dev)
    reps = op.solve_load_path(u, bc, 2, strategy="t2", preconditioner="jacobi", max_newton=30, max_cg=20000,
                              newton_atol=1e-11, cg_rtol=1e-9)
    assert all(r["converged"] for r in reps if not r.get("failed"))
    ug = u.cpu().numpy()
    assert np.linalg.norm(ug - u_ref) / np.linalg.norm(u_ref) <= 1e-8
    assert np.linalg.norm(P.residual(ug)) <= 1e-10


def test_hex_unsupported_paths(torch_dev):
    import paper_2505_15535_amd as mfe
    v, c = _mesh(1, 70)
    op = _op(v, c, 2)
    op.set_state(_to(torch_dev, np.zeros(op.n_dofs)))
    assert mfe.mfe_patch_count(op.ctx) == 0
    with pytest.raises(mfe.MfeError) as e:
        op.gmg_setup()
    assert e.value.code == mfe.MFE_EUNSUPPORTED
    torch, dev = torch_dev
    for prec in ("bf16", "bf16x3"):          # matrix-core sweeps: structured boxes only
        op.build_cache("t2", precision=prec)
        with pytest.raises(mfe.MfeError) as e:
            op.apply(torch.zeros(op.n_dofs, dtype=torch.float32, device=dev), strategy="t2", precision=prec)
        assert e.value.code == mfe.MFE_EUNSUPPORTED
    bad = c.copy()
    bad[0, [0, 1]] = bad[0, [1, 0]]          # an inverted cell
    with pytest.raises(mfe.MfeError) as e:
        _op(v, bad, 2)
    assert e.value.code in (mfe.MFE_EJACOBIAN, mfe.MFE_EINVAL)


def test_hex_full_size_sampled(torch_dev):
    """109,375-cell unstructured mesh (2,648,253 dofs), Q2, in the launch
    configuration the benchmark times: sampled dofs against the oracle,
    strategies against each other, symmetry."""
    torch, dev = torch_dev
    v, c = synthetic.cube_in_cube(25, jitter=0.1, rng=np.random.default_rng(3))
    H = HexMesh(v, c, 2)
    u = _state(H, 0.03, 5)
    w = np.random.default_rng(6).standard_normal(H.n_dofs)
    P = Problem(H, 1.0, 10.0, chunk=256)
    dofs = np.sort(np.random.default_rng(7).choice(H.n_dofs, 300, replace=False))
    ref = P.apply_at(u, w, dofs)
    print("case hex full size", flush=True)
    op = _op(v, c, 2)
    ud, wd = _to(torch_dev, u), _to(torch_dev, w)
    op.set_state(ud)
    full = {}
    for s in ALL:
        op.build_cache(s)
        full[s] = op.apply(wd, strategy=s).cpu().numpy()
        assert _rel(full[s][dofs], ref) <= TOL, s
    for s in ALL[1:]:
        assert _rel(full[s], full["otf"]) <= TOL, s
    z = _to(torch_dev, np.random.default_rng(8).standard_normal(H.n_dofs))
    Kz = op.apply(z, strategy="t2")
    a = float(torch.dot(wd, Kz))
    b = float(torch.dot(z, torch.from_numpy(full["t2"]).to(dev)))
    assert abs(a - b) <= 1e-12 * float(torch.linalg.norm(wd) * torch.linalg.norm(Kz))


def test_box_as_hex_matches_box_kernels_full_size(torch_dev):
    """The 48^3 jittered box given as a general mesh: the general-mesh kernels
    give the structured-box kernels' result (through the node permutation
    that matches positions)."""
    import paper_2505_15535_amd as mfe
    torch, dev = torch_dev
    cfg = synthetic.get_config("box48_q2")
    verts = cfg.vertices()
    box = mfe.Operator(cfg.nx, cfg.ny, cfg.nz, 2, verts, cfg.mu, cfg.lam, device=0)
    hexop = _op(verts, synthetic.box_cells(cfg.nx, cfg.ny, cfg.nz), 2, cfg.mu, cfg.lam)
    assert hexop.n_dofs == box.n_dofs
    d, perm = cKDTree(box.node_coordinates()).query(hexop.node_coordinates())
    assert d.max() < 1e-12 and np.unique(perm).size == perm.size
    dm = torch.from_numpy((3 * perm[:, None] + np.arange(3)).reshape(-1)).to(dev)
    u, w = _to(torch_dev, cfg.displacement()), _to(torch_dev, cfg.test_vector(0))
    box.set_state(u)
    hexop.set_state(u[dm].contiguous())
    print("case box as hex full size", flush=True)
    for s in ALL:
        box.build_cache(s)
        hexop.build_cache(s)
        vb = box.apply(w, strategy=s)[dm]
        vh = hexop.apply(w[dm].contiguous(), strategy=s)
        assert float(torch.linalg.norm(vh - vb) / torch.linalg.norm(vb)) <= TOL, s
