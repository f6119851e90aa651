"""GPU Newton-CG solver pieces against the oracle: matrix-free diagonal,
(preconditioned) CG solves, and Newton on a small twisted beam."""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synthetic
import oracle
from oracle.fem import Problem
from oracle.mesh import BoxMesh

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda", 0)


def _to(torch_dev, x):
    torch, dev = torch_dev
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(dev)


def _clamped_cube(torch_dev, scale=1.0):
    import paper_2505_15535_amd as mfe
    cfg = synthetic.get_config("cube4_q2_jit")
    verts, u = cfg.vertices(), scale * cfg.displacement()
    mesh = BoxMesh(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts)
    left = np.where(mesh.node_positions()[:, 0] < 1e-12)[0]
    cdofs = (3 * left[:, None] + np.arange(3)).ravel()
    P = Problem(mesh, cfg.mu, cfg.lam, constrained_dofs=cdofs)
    op = mfe.Operator(cfg.nx, cfg.ny, cfg.nz, cfg.degree, verts, cfg.mu, cfg.lam, device=0)
    op.set_constraints(cdofs)
    op.set_state(_to(torch_dev, u))
    return cfg, P, op, u, cdofs


def test_diagonal_parity(torch_dev):
    cfg, P, op, u, cdofs = _clamped_cube(torch_dev)
    ref = P.assemble_tangent(u).diagonal()
    d = op.diagonal().cpu().numpy()
    assert np.linalg.norm(d - ref) / np.linalg.norm(ref) <= 1e-12
    assert np.all(d[cdofs] == 1.0)


@pytest.mark.parametrize("pc,strategy", [("jacobi", "t2"), ("none", "otf"), ("jacobi", "t4"), ("gmg", "t2"),
                                         ("gmg", "otf")])
def test_cg_solve_parity(torch_dev, pc, strategy):
    # a state close enough to the reference configuration for K(u) to be
    # positive definite (at the full sine amplitude the neo-Hookean tangent of
    # this non-equilibrium state is indefinite and CG does not apply)
    cfg, P, op, u, cdofs = _clamped_cube(torch_dev, scale=0.1)
    K = P.assemble_tangent(u)
    ev = np.linalg.eigvalsh(K.toarray())
    assert ev[0] > 0.0
    b = cfg.test_vector(2)
    b[cdofs] = 0.0
    ref = spla.spsolve(K.tocsc(), b)
    x, it, rel, status = op.cg_solve(_to(torch_dev, b), strategy=strategy, preconditioner=pc, max_cg=30000,
                                     cg_rtol=1e-12)
    assert status == "MFE_OK" and rel <= 1e-12 and it > 1
    x = x.cpu().numpy()
    # error bound: cond(K) * tolerance
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= 1e-12 * ev[-1] / ev[0] * 10
    assert np.all(x[cdofs] == 0.0)


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_gmg_cg_beats_jacobi(torch_dev, levels):
    """GMG-preconditioned CG (all levels, a single level = plain Chebyshev-
    Jacobi, two levels) reaches the same solution as Jacobi-CG on a clamped
    16x4x4 Q2 beam with far fewer iterations; the coarse levels keep the
    clamped faces constrained."""
    import paper_2505_15535_amd as mfe
    torch, dev = torch_dev
    nx, ny, nz, L = 16, 4, 4, (4.0, 1.0, 1.0)
    verts = synthetic.box_vertices(nx, ny, nz, L, jitter=0.15, rng=synthetic.rng_for(90, 0))
    cdofs, vals = synthetic.clamp_and_twist(nx, ny, nz, 2, L, np.deg2rad(5.0))
    op = mfe.Operator(nx, ny, nz, 2, verts, 1.0, 10.0, device=0)
    op.set_constraints(cdofs)
    u = torch.zeros(op.n_dofs, dtype=torch.float64, device=dev)
    u[torch.from_numpy(cdofs).to(dev)] = _to(torch_dev, vals)
    op.set_state(u)
    b = synthetic.random_vectors(op.n_dofs, 1, synthetic.rng_for(90, 2))[0]
    b[cdofs] = 0.0
    bt = _to(torch_dev, b)
    xj, itj, relj, sj = op.cg_solve(bt, strategy="t2", preconditioner="jacobi", max_cg=50000, cg_rtol=1e-10)
    xg, itg, relg, sg = op.cg_solve(bt, strategy="t2", preconditioner="gmg", mg_levels=levels, max_cg=50000,
                                    cg_rtol=1e-10)
    print(f"levels {levels}: jacobi {itj} its, gmg {itg} its")
    assert sj == "MFE_OK" and sg == "MFE_OK"
    assert itg * (3 if levels != 1 else 1.5) < itj
    xj, xg = xj.cpu().numpy(), xg.cpu().numpy()
    assert np.linalg.norm(xg - xj) / np.linalg.norm(xj) <= 1e-7
    assert np.all(xg[cdofs] == 0.0)
    # a second solve reuses the hierarchy (the apply sums shared nodes with
    # atomics, so iterates agree to rounding, not bit for bit)
    xg2, itg2, _, _ = op.cg_solve(bt, strategy="t2", preconditioner="gmg", mg_levels=levels, max_cg=50000,
                                  cg_rtol=1e-10)
    assert abs(itg2 - itg) <= 1
    assert np.linalg.norm(xg2.cpu().numpy() - xg) / np.linalg.norm(xg) <= 1e-9


def test_gmg_fp32_vcycle_defect_correction(torch_dev):
    """FP32 V-cycle inside the FP64 CG: the outer iteration still reaches a
    relative residual of 1e-10 (the FP32 preconditioner only changes the
    search directions), with about as many iterations as the FP64 V-cycle."""
    import paper_2505_15535_amd as mfe
    torch, dev = torch_dev
    nx, ny, nz, L = 16, 4, 4, (4.0, 1.0, 1.0)
    verts = synthetic.box_vertices(nx, ny, nz, L, jitter=0.15, rng=synthetic.rng_for(90, 0))
    cdofs, vals = synthetic.clamp_and_twist(nx, ny, nz, 2, L, np.deg2rad(5.0))
    op = mfe.Operator(nx, ny, nz, 2, verts, 1.0, 10.0, device=0)
    op.set_constraints(cdofs)
    u = torch.zeros(op.n_dofs, dtype=torch.float64, device=dev)
    u[torch.from_numpy(cdofs).to(dev)] = _to(torch_dev, vals)
    op.set_state(u)
    b = synthetic.random_vectors(op.n_dofs, 1, synthetic.rng_for(90, 2))[0]
    b[cdofs] = 0.0
    bt = _to(torch_dev, b)
    res = {}
    for prec in ("fp64", "fp32"):
        for strategy in ("t2", "otf"):
            x, it, rel, st = op.cg_solve(bt, strategy=strategy, preconditioner="gmg", mg_precision=prec,
                                         max_cg=5000, cg_rtol=1e-10)
            assert st == "MFE_OK" and rel <= 1e-10, (prec, strategy, st, op.last_error())
            res[prec, strategy] = (x.cpu().numpy(), it)
    print({k: v[1] for k, v in res.items()})
    x64 = res["fp64", "t2"][0]
    for k, (x, it) in res.items():
        assert np.linalg.norm(x - x64) / np.linalg.norm(x64) <= 1e-8, k
        assert it <= 1.25 * res["fp64", "t2"][1] + 2, k


@pytest.mark.parametrize("prec,tol,direct", [("fp64", 1e-12, 1), ("fp32", 1e-5, 1), ("fp64", 1e-12, 0),
                                             ("fp32", 1e-5, 0)])
def test_gmg_preconditioner_graph_and_symmetry(torch_dev, prec, tol, direct):
    """One V-cycle replayed from the HIP graph equals the eagerly launched one
    on every replay (with other GPU work in between), B is symmetric and
    positive, and it is the identity on the constrained dofs; with the
    coarsest level (4x1x1, 243 dofs) solved directly or smoothed."""
    import paper_2505_15535_amd as mfe
    torch, dev = torch_dev
    nx, ny, nz, L = 16, 4, 4, (4.0, 1.0, 1.0)
    verts = synthetic.box_vertices(nx, ny, nz, L, jitter=0.15, rng=synthetic.rng_for(92, 0))
    cdofs, vals = synthetic.clamp_and_twist(nx, ny, nz, 2, L, np.deg2rad(5.0))
    op = mfe.Operator(nx, ny, nz, 2, verts, 1.0, 10.0, device=0)
    op.set_constraints(cdofs)
    u = torch.zeros(op.n_dofs, dtype=torch.float64, device=dev)
    u[torch.from_numpy(cdofs).to(dev)] = _to(torch_dev, vals)
    op.set_state(u)
    op.build_cache("t2")
    R = [_to(torch_dev, r) for r in synthetic.random_vectors(op.n_dofs, 2, synthetic.rng_for(92, 2))]
    opts = dict(strategy="t2", mg_precision=prec, coarse_direct=direct)
    with pytest.raises(mfe.MfeError) as e:
        op.gmg_apply(R[0], **opts)          # level data not set up yet
    assert e.value.code == mfe.MFE_ESTATE
    op.gmg_setup(**opts)
    eager = [op.gmg_apply(r, mg_graph=0, **opts).clone() for r in R]
    for rep in range(3):
        for k, r in enumerate(R):
            zg = op.gmg_apply(r, mg_graph=1, **opts)
            rel = float(torch.linalg.norm(zg - eager[k]) / torch.linalg.norm(eager[k]))
            assert rel <= tol, (rep, k, rel)
        op.apply(R[0], strategy="t2")       # unrelated eager work between replays
        torch.cuda.synchronize()
    z0, z1 = eager
    a, b = float(torch.dot(R[1], z0)), float(torch.dot(R[0], z1))
    assert abs(a - b) <= 10 * tol * max(abs(a), abs(b)) + 1e-14
    assert float(torch.dot(R[0], z0)) > 0.0 and float(torch.dot(R[1], z1)) > 0.0
    ci = torch.from_numpy(cdofs).to(dev)
    assert torch.equal(z0[ci], R[0][ci])
    # the FP32 V-cycle really runs in FP32: it differs from the FP64 one at the
    # level of FP32 rounding, not more
    other = "fp64" if prec == "fp32" else "fp32"
    op.gmg_setup(strategy="t2", mg_precision=other, coarse_direct=direct)
    with pytest.raises(mfe.MfeError) as e:
        op.gmg_apply(R[0], strategy="t2", mg_precision=other, coarse_direct=1 - direct)   # other options
    assert e.value.code == mfe.MFE_ESTATE
    zo = op.gmg_apply(R[0], strategy="t2", mg_precision=other, coarse_direct=direct)
    d = float(torch.linalg.norm(zo - z0) / torch.linalg.norm(z0))
    assert 1e-10 < d < 1e-4, d
    op.set_state(0.5 * u)
    with pytest.raises(mfe.MfeError) as e:
        op.gmg_apply(R[0], **opts)          # stale after a new state
    assert e.value.code == mfe.MFE_ESTATE


def test_gmg_per_cell_material_and_options(torch_dev):
    """Per-cell (mu, lambda) averaged onto the coarse levels; option checks."""
    import paper_2505_15535_amd as mfe
    torch, dev = torch_dev
    nx, ny, nz, L = 8, 4, 4, (2.0, 1.0, 1.0)
    verts = synthetic.box_vertices(nx, ny, nz, L, jitter=0.1, rng=synthetic.rng_for(91, 0))
    rng = synthetic.rng_for(91, 5)
    mat = np.stack([rng.uniform(0.5, 2.0, nx * ny * nz), rng.uniform(1.0, 20.0, nx * ny * nz)], 1).ravel()
    mesh = BoxMesh(nx, ny, nz, 2, verts)
    cdofs, _ = synthetic.clamp_and_twist(nx, ny, nz, 2, L, 0.0)
    op = mfe.Operator(nx, ny, nz, 2, verts, 1.0, 1.0, device=0)
    op.set_material(1.0, 1.0, per_cell=mat)
    op.set_constraints(cdofs)
    # small enough for K(u) of this non-equilibrium state to stay positive definite
    u = synthetic.sine_displacement(nx, ny, nz, 2, 0.004, synthetic.rng_for(91, 1))
    u[cdofs] = 0.0
    op.set_state(_to(torch_dev, u))
    P = Problem(mesh, 1.0, 1.0, constrained_dofs=cdofs, elem_mu_lam=mat.reshape(-1, 2))
    K = P.assemble_tangent(u)
    np.linalg.cholesky(K.toarray())  # raises unless K is positive definite
    b = synthetic.random_vectors(op.n_dofs, 1, synthetic.rng_for(91, 2))[0]
    b[cdofs] = 0.0
    ref = spla.spsolve(K.tocsc(), b)
    x, it, rel, status = op.cg_solve(_to(torch_dev, b), preconditioner="gmg", max_cg=2000, cg_rtol=1e-11)
    print(f"per-cell material: gmg {it} its, {status} {op.last_error()}")
    assert status == "MFE_OK" and it < 60
    assert np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref) <= 1e-8
    for bad in ({"cheb_degree": 0}, {"cheb_range": 1.0}, {"coarse_degree": 0}, {"coarse_range": float("nan")},
                {"mg_levels": -1}, {"mg_precision": 2}, {"mg_graph": 2}, {"mg_lag": -1}):
        with pytest.raises(mfe.MfeError, match="MFE_EINVAL"):
            op.cg_solve(_to(torch_dev, b), preconditioner="gmg", **bad)


def test_newton_twisted_beam_parity(torch_dev):
    """Load path of the twisted beam (27 degrees in 3 steps) on an 8x2x2 Q2
    beam, lambda/mu = 100: GPU Newton-CG against the oracle's Newton with
    direct solves; both converge to ||R|| <= 1e-10."""
    import paper_2505_15535_amd as mfe
    torch, dev = torch_dev
    nx, ny, nz, L, lam = 8, 2, 2, (4.0, 1.0, 1.0), 100.0
    verts = synthetic.box_vertices(nx, ny, nz, L)
    mesh = BoxMesh(nx, ny, nz, 2, verts)
    cdofs, _ = synthetic.clamp_and_twist(nx, ny, nz, 2, L, 0.0)
    P = Problem(mesh, 1.0, lam, constrained_dofs=cdofs)
    theta = np.deg2rad(27.0)
    u_ref = np.zeros(mesh.n_dofs)
    for k in (1, 2, 3):
        d, v = synthetic.clamp_and_twist(nx, ny, nz, 2, L, theta * k / 3)
        u_ref, _ = oracle.solver.newton(P, u_ref, d, v, atol=1e-10)
    op = mfe.Operator(nx, ny, nz, 2, verts, 1.0, lam, device=0)
    op.set_constraints(cdofs)
    u = torch.zeros(mesh.n_dofs, dtype=torch.float64, device=dev)
    reps = op.solve_load_path(u, lambda t: synthetic.clamp_and_twist(nx, ny, nz, 2, L, theta * t), 3,
                              strategy="t2", preconditioner="jacobi", max_newton=30, max_cg=20000,
                              newton_atol=1e-10, cg_rtol=1e-8)
    print(reps)
    assert all(r["converged"] for r in reps if not r.get("failed"))
    ug = u.cpu().numpy()
    d, v = synthetic.clamp_and_twist(nx, ny, nz, 2, L, theta)
    assert np.array_equal(ug[d], v)
    assert np.linalg.norm(ug - u_ref) / np.linalg.norm(u_ref) <= 1e-7
    # the oracle's residual at the GPU solution
    assert np.linalg.norm(P.residual(ug)) <= 1e-9


@pytest.mark.parametrize("strategy,mg_precision,mg_lag", [("t4", "fp64", 0), ("t2", "fp32", 0), ("t2", "fp64", 3),
                                                           ("t2", "fp32", 2)])
def test_newton_twisted_beam_gmg(torch_dev, strategy, mg_precision, mg_lag):
    """The same load path with the GMG preconditioner (8x2x2 -> 4x1x1), FP64
    or FP32 V-cycle, with a full multigrid set-up for every CG solve or a
    lagged one: converges to the oracle's solution."""
    import paper_2505_15535_amd as mfe
    torch, dev = torch_dev
    nx, ny, nz, L, lam = 8, 2, 2, (4.0, 1.0, 1.0), 100.0
    verts = synthetic.box_vertices(nx, ny, nz, L)
    mesh = BoxMesh(nx, ny, nz, 2, verts)
    cdofs, _ = synthetic.clamp_and_twist(nx, ny, nz, 2, L, 0.0)
    P = Problem(mesh, 1.0, lam, constrained_dofs=cdofs)
    theta = np.deg2rad(27.0)
    u_ref = np.zeros(mesh.n_dofs)
    for k in (1, 2, 3):
        d, v = synthetic.clamp_and_twist(nx, ny, nz, 2, L, theta * k / 3)
        u_ref, _ = oracle.solver.newton(P, u_ref, d, v, atol=1e-10)
    op = mfe.Operator(nx, ny, nz, 2, verts, 1.0, lam, device=0)
    op.set_constraints(cdofs)
    u = torch.zeros(mesh.n_dofs, dtype=torch.float64, device=dev)
    reps = op.solve_load_path(u, lambda t: synthetic.clamp_and_twist(nx, ny, nz, 2, L, theta * t), 3,
                              strategy=strategy, preconditioner="gmg", mg_precision=mg_precision,
                              mg_lag=mg_lag, max_newton=30, max_cg=5000, newton_atol=1e-10, cg_rtol=1e-8)
    print(reps)
    assert all(r["converged"] for r in reps if not r.get("failed"))
    ug = u.cpu().numpy()
    assert np.linalg.norm(ug - u_ref) / np.linalg.norm(u_ref) <= 1e-7
    assert np.linalg.norm(P.residual(ug)) <= 1e-9


def test_cg_reports_breakdown_on_indefinite_tangent(torch_dev):
    cfg, P, op, u, cdofs = _clamped_cube(torch_dev, scale=1.0)
    b = cfg.test_vector(2)
    b[cdofs] = 0.0
    x, it, rel, status = op.cg_solve(_to(torch_dev, b), strategy="t2", preconditioner="none", max_cg=30000,
                                     cg_rtol=1e-12)
    assert status == "MFE_ENOTCONV"


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_gmg_single_level_is_a_direct_solve(torch_dev, prec, tol):
    """With one level (135 dofs, 108 free) and coarse_direct the preconditioner is the
    exact inverse of the tangent on the free dofs (identity on the
    constrained ones): against the oracle's sparse direct solve.  The FP32
    V-cycle applies the FP64 inverse rounded to FP32 (bound 1e-4: the
    rounding of the entries times the conditioning of the product).  CG
    with it converges in one iteration; without coarse_direct the level is
    only smoothed."""
    import paper_2505_15535_amd as mfe
    torch, dev = torch_dev
    nx, ny, nz = 2, 1, 1
    verts = synthetic.box_vertices(nx, ny, nz, (1.0, 0.8, 0.7), 0.1, synthetic.rng_for(95, 0))
    mesh = BoxMesh(nx, ny, nz, 2, verts)
    u = synthetic.sine_displacement(nx, ny, nz, 2, 0.002, synthetic.rng_for(95, 1))   # K SPD, cond 8e3
    left = np.where(mesh.node_positions()[:, 0] < 1e-12)[0]
    cdofs = (3 * left[:, None] + np.arange(3)).ravel()
    P = Problem(mesh, 1.0, 10.0, constrained_dofs=cdofs)
    K = P.assemble_tangent(u).tocsc()
    r = synthetic.random_vectors(mesh.n_dofs, 1, synthetic.rng_for(95, 2))[0]
    ref = spla.spsolve(K, r)
    op = mfe.Operator(nx, ny, nz, 2, verts, 1.0, 10.0, device=0)
    op.set_constraints(cdofs)
    op.set_state(_to(torch_dev, u))
    opts = dict(strategy="t2", mg_levels=1, mg_precision=prec, coarse_direct=1)
    op.gmg_setup(**opts)
    z = op.gmg_apply(_to(torch_dev, r), **opts).cpu().numpy()
    assert np.linalg.norm(z - ref) / np.linalg.norm(ref) <= tol
    x, it, rel, status = op.cg_solve(_to(torch_dev, r), preconditioner="gmg", cg_rtol=1e-4, max_cg=50, **opts)
    assert status == "MFE_OK" and it <= 2, (it, rel)
    smooth = dict(opts, coarse_direct=0)
    op.gmg_setup(**smooth)
    z2 = op.gmg_apply(_to(torch_dev, r), **smooth).cpu().numpy()
    assert np.linalg.norm(z2 - ref) / np.linalg.norm(ref) > 1e-3


def test_gmg_direct_coarse_falls_back_on_indefinite_level(torch_dev):
    """At a state whose tangent is indefinite (smallest eigenvalue -0.03 on
    the 2x1x1 box), the sweep inversion of the one-level hierarchy meets a
    pivot <= 0 and the level is smoothed instead: set-up either reports the
    indefinite level or succeeds with a preconditioner that is not the exact
    inverse; nothing else is left changed (a later SPD state is solved
    exactly again)."""
    import paper_2505_15535_amd as mfe
    torch, dev = torch_dev
    nx, ny, nz = 2, 1, 1
    verts = synthetic.box_vertices(nx, ny, nz, (1.0, 0.8, 0.7))
    mesh = BoxMesh(nx, ny, nz, 2, verts)
    left = np.where(mesh.node_positions()[:, 0] < 1e-12)[0]
    cdofs = (3 * left[:, None] + np.arange(3)).ravel()
    P = Problem(mesh, 1.0, 10.0, constrained_dofs=cdofs)
    u_bad = synthetic.sine_displacement(nx, ny, nz, 2, 0.01, synthetic.rng_for(95, 1))
    K_bad = P.assemble_tangent(u_bad)
    assert np.linalg.eigvalsh(K_bad.toarray()).min() < 0.0
    r = synthetic.random_vectors(mesh.n_dofs, 1, synthetic.rng_for(95, 2))[0]
    op = mfe.Operator(nx, ny, nz, 2, verts, 1.0, 10.0, device=0)
    op.set_constraints(cdofs)
    opts = dict(strategy="t2", mg_levels=1, coarse_direct=1)
    op.set_state(_to(torch_dev, u_bad))
    try:
        op.gmg_setup(**opts)
        z = op.gmg_apply(_to(torch_dev, r), **opts).cpu().numpy()
        exact = spla.spsolve(K_bad.tocsc(), r)
        assert np.linalg.norm(z - exact) / np.linalg.norm(exact) > 1e-3
    except mfe.MfeError as e:
        assert e.code in (mfe.MFE_ENOTCONV, mfe.MFE_EJACOBIAN)
    u_ok = synthetic.sine_displacement(nx, ny, nz, 2, 0.002, synthetic.rng_for(95, 1))
    op.set_state(_to(torch_dev, u_ok))
    op.gmg_setup(**opts)
    z = op.gmg_apply(_to(torch_dev, r), **opts).cpu().numpy()
    ref = spla.spsolve(P.assemble_tangent(u_ok).tocsc(), r)
    assert np.linalg.norm(z - ref) / np.linalg.norm(ref) <= 1e-10


def test_load_path_resumes_from_checkpoint(torch_dev, tmp_path):
    """A load path stopped after its second step and resumed from the
    checkpoint file takes the same remaining steps as the uninterrupted path
    and ends at the same state (to the Newton tolerance)."""
    import shutil
    import paper_2505_15535_amd as mfe
    torch, dev = torch_dev
    nx, ny, nz, L, lam = 8, 2, 2, (4.0, 1.0, 1.0), 100.0
    verts = synthetic.box_vertices(nx, ny, nz, L)
    cdofs, _ = synthetic.clamp_and_twist(nx, ny, nz, 2, L, 0.0)
    # 4 degrees a step keeps every Newton solve in its quadratic phase; in a
    # damped phase (larger steps) the line search amplifies the rounding of
    # the atomic sums and two runs drift apart after a few iterations
    theta = np.deg2rad(16.0)
    bv = lambda t: synthetic.clamp_and_twist(nx, ny, nz, 2, L, theta * t)
    opts = dict(strategy="t2", preconditioner="jacobi", max_newton=30, max_cg=20000, newton_atol=1e-10,
                cg_rtol=1e-8)
    ck, ck2 = tmp_path / "path.npz", tmp_path / "after2.npz"

    def keep_second(t, uu):
        if abs(t - 0.5) < 1e-12:
            shutil.copy(ck, ck2)

    op = mfe.Operator(nx, ny, nz, 2, verts, 1.0, lam, device=0)
    op.set_constraints(cdofs)
    u = torch.zeros(op.n_dofs, dtype=torch.float64, device=dev)
    full = op.solve_load_path(u, bv, 4, on_step=keep_second, checkpoint=ck, **opts)
    op.close()
    assert ck2.exists()
    assert float(mfe.load_checkpoint(ck)["t"]) == pytest.approx(1.0)

    op = mfe.Operator(nx, ny, nz, 2, verts, 1.0, lam, device=0)
    op.set_constraints(cdofs)
    u2 = torch.full((op.n_dofs,), np.nan, dtype=torch.float64, device=dev)   # overwritten by the checkpoint
    rest = op.solve_load_path(u2, bv, 4, checkpoint=ck2, resume=True, **opts)
    op.close()
    later = [r for r in full if r["t"] > 0.5 + 1e-12]
    assert [(r["t"], r["h"], bool(r.get("failed"))) for r in rest] == \
        [(r["t"], r["h"], bool(r.get("failed"))) for r in later]
    # the residual histories agree while they are above the rounding floor
    # (the scatter's atomic sums make the last iterations, near 1e-10, vary
    # from run to run); the next step starts from the same extrapolated state
    for a, b in zip(rest, later):
        ha = [x for x in a["residual_history"] if x > 1e-7]
        hb = [x for x in b["residual_history"] if x > 1e-7]
        assert len(ha) == len(hb), (a, b)
        assert ha == pytest.approx(hb, rel=1e-3), (a, b)
        assert abs(a["newton_iterations"] - b["newton_iterations"]) <= 1, (a, b)
    assert rest[0]["residual_history"][0] == pytest.approx(later[0]["residual_history"][0], rel=1e-10)
    a, b = u.cpu().numpy(), u2.cpu().numpy()
    assert np.linalg.norm(a - b) / np.linalg.norm(a) <= 1e-8
    with pytest.raises(ValueError):
        op = mfe.Operator(nx, ny, nz, 2, verts, 1.0, lam, device=0)
        try:
            op.solve_load_path(u2, bv, 3, checkpoint=ck2, resume=True, **opts)
        finally:
            op.close()


def test_load_path_driver_through_the_c_abi(torch_dev):
    """mfe_solve_load_path called directly: the load callback sees the
    targets t of the steps, the step callback can stop the path (the state
    then says where), a second call goes on from that state to t = 1 and ends
    where an uninterrupted path ends; bad arguments are refused."""
    import ctypes
    import paper_2505_15535_amd as mfe
    torch, dev = torch_dev
    nx, ny, nz, L, lam = 8, 2, 2, (4.0, 1.0, 1.0), 100.0
    verts = synthetic.box_vertices(nx, ny, nz, L)
    cdofs, _ = synthetic.clamp_and_twist(nx, ny, nz, 2, L, 0.0)
    theta = np.deg2rad(16.0)
    order = np.unique(cdofs)

    def values(t):
        d, v = synthetic.clamp_and_twist(nx, ny, nz, 2, L, theta * t)
        g = np.zeros(3 * (2 * nx + 1) * (2 * ny + 1) * (2 * nz + 1))
        g[d] = v
        return g[order]

    op = mfe.Operator(nx, ny, nz, 2, verts, 1.0, lam, device=0)
    op.set_constraints(cdofs)
    opts = op.solve_opts(strategy="t2", preconditioner="jacobi", max_newton=30, max_cg=20000, newton_atol=1e-10,
                         cg_rtol=1e-8)
    n = op.n_dofs
    u = torch.zeros(n, dtype=torch.float64, device=dev)
    prev = torch.zeros_like(u)
    seen, steps = [], []
    st = mfe.PathState(0.0, 0.0, 0.0, 0.0)
    rc, reps = mfe.mfe_solve_load_path(op.ctx, opts, u.data_ptr(), prev.data_ptr(), 4, 1.0 / 64, True, st,
                                       lambda t: seen.append(t) or values(t),
                                       lambda s, up, pp: steps.append(s.t) or s.t >= 0.5 - 1e-12,
                                       stream=mfe._stream_handle(None))
    assert rc == mfe.MFE_OK and st.t == pytest.approx(0.5) and steps == pytest.approx([0.25, 0.5])
    assert seen == pytest.approx([0.25, 0.5]) and st.prev_h == pytest.approx(0.25) and st.h == pytest.approx(0.25)
    assert [r.failed for r in reps] == [0, 0] and all(r.solve.converged for r in reps)
    rc, reps2 = mfe.mfe_solve_load_path(op.ctx, opts, u.data_ptr(), prev.data_ptr(), 4, 1.0 / 64, True, st, values,
                                        stream=mfe._stream_handle(None))
    assert rc == mfe.MFE_OK and st.t == pytest.approx(1.0) and [r.t for r in reps2] == pytest.approx([0.75, 1.0])
    # the same path in one call
    u1 = torch.zeros_like(u)
    op.solve_load_path(u1, lambda t: synthetic.clamp_and_twist(nx, ny, nz, 2, L, theta * t), 4, extrapolate=True,
                       strategy="t2", preconditioner="jacobi", max_newton=30, max_cg=20000, newton_atol=1e-10,
                       cg_rtol=1e-8)
    assert torch.linalg.norm(u - u1) / torch.linalg.norm(u1) <= 1e-8
    # bad arguments
    for args in ((0, 1.0 / 64, False), (4, 0.0, False), (4, 2.0, False)):
        with pytest.raises(mfe.MfeError, match="MFE_EINVAL"):
            mfe.mfe_solve_load_path(op.ctx, opts, u.data_ptr(), prev.data_ptr(), args[0], args[1], args[2],
                                    mfe.PathState(), values, stream=mfe._stream_handle(None))
    # extrapolation without the previous state; no load callback with constrained dofs
    load_cb = mfe.LOAD_FN(lambda *a: 0)
    for prev_ptr, cb, extra in ((None, load_cb, 1), (prev.data_ptr(), mfe.LOAD_FN(), 0)):
        rc = mfe._lib.mfe_solve_load_path(op.ctx, ctypes.byref(opts), u.data_ptr(), prev_ptr, 4, 0.1, extra, None, cb,
                                          None, mfe.STEP_FN(), None, None, 0, None, mfe._stream_handle(None))
        assert rc == mfe.MFE_EINVAL, op.last_error()
    with pytest.raises(ValueError, match="constrained dofs"):   # a load callback with the wrong count
        mfe.mfe_solve_load_path(op.ctx, opts, u.data_ptr(), prev.data_ptr(), 4, 1.0 / 64, False, mfe.PathState(),
                                lambda t: np.zeros(3), stream=mfe._stream_handle(None))
    op.close()


def test_load_path_driver_gives_up_below_min_fraction(torch_dev):
    """Forced from the host: with one Newton iteration allowed no step can
    converge, so every attempt fails, the increment halves from 1/2 down to
    min_fraction = 1/16 (attempts at 1/2, 1/4, 1/8, 1/16) and the driver
    returns MFE_ENOTCONV with the state still at t = 0 and h_cap lowered."""
    import paper_2505_15535_amd as mfe
    torch, dev = torch_dev
    nx, ny, nz, L, lam = 8, 2, 2, (4.0, 1.0, 1.0), 100.0
    verts = synthetic.box_vertices(nx, ny, nz, L)
    cdofs, _ = synthetic.clamp_and_twist(nx, ny, nz, 2, L, 0.0)
    order = np.unique(cdofs)
    theta = np.deg2rad(60.0)

    def values(t):
        d, v = synthetic.clamp_and_twist(nx, ny, nz, 2, L, theta * t)
        g = np.zeros(3 * (2 * nx + 1) * (2 * ny + 1) * (2 * nz + 1))
        g[d] = v
        return g[order]

    op = mfe.Operator(nx, ny, nz, 2, verts, 1.0, lam, device=0)
    op.set_constraints(cdofs)
    opts = op.solve_opts(strategy="t2", preconditioner="jacobi", max_newton=1, max_cg=20000, newton_atol=1e-10,
                         cg_rtol=1e-8)
    u = torch.zeros(op.n_dofs, dtype=torch.float64, device=dev)
    prev = torch.zeros_like(u)
    st = mfe.PathState(0.0, 0.0, 0.0, 0.0)
    rc, reps = mfe.mfe_solve_load_path(op.ctx, opts, u.data_ptr(), prev.data_ptr(), 2, 1.0 / 16, True, st, values,
                                       stream=mfe._stream_handle(None))
    assert rc == mfe.MFE_ENOTCONV and "min_fraction" in op.last_error()
    assert [r.h for r in reps] == pytest.approx([0.5, 0.25, 0.125, 0.0625])
    assert all(r.failed and r.status in (mfe.MFE_ENOTCONV, mfe.MFE_EJACOBIAN) for r in reps)
    assert st.t == 0.0 and st.h_cap == pytest.approx(0.9 * 0.0625)
    assert torch.count_nonzero(u) == 0     # the state is the last converged one
    with pytest.raises(mfe.MfeError, match="MFE_ENOTCONV"):
        op.solve_load_path(u, lambda t: synthetic.clamp_and_twist(nx, ny, nz, 2, L, theta * t), 2,
                           min_fraction=1.0 / 16, strategy="t2", preconditioner="jacobi", max_newton=1,
                           max_cg=20000, newton_atol=1e-10, cg_rtol=1e-8)
    op.close()
