"""The learned smoother correction: the network's forward and backward
kernels against the FP64 oracle (oracle/net.py), the Adam kernel, the patch
gather/scatter, and the learned step of the multigrid smoother trained on
pairs the solver generates.

Tolerances: forward 1e-5 and gradients 1e-4 (relative 2-norm): FP32 sums of
up to 32*27 = 864 terms per output and of 729*P products per weight
gradient, against FP64."""

import numpy as np
import pytest

import synthetic
from oracle import net as onet

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda", 0)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("variant", ["relu", "linear"])
def test_forward_backward_loss_parity(torch_dev, variant):
    import paper_2505_15535_amd as mfe
    torch, dev = torch_dev
    lin = variant == "linear"
    var = mfe.NET_VARIANTS[variant]
    rng = np.random.default_rng(0)
    P = 3
    prm = rng.normal(0.0, 0.1, onet.N_PARAMS).astype(np.float32)
    x = rng.normal(size=(P, 6, 729)).astype(np.float32)
    t = rng.normal(size=(P, 3, 729)).astype(np.float32)
    y_ref, acts = onet.forward(prm.astype(np.float64), x.astype(np.float64), linear=lin)
    loss_ref, dy_ref = onet.mse(y_ref, t)
    g_ref = onet.backward(prm.astype(np.float64), x, acts, dy_ref, linear=lin)
    f = dict(dtype=torch.float32, device=dev)
    W, X, Tt = (torch.from_numpy(a).to(dev) for a in (prm, x, t))
    act = torch.empty((2, P, 32, 729), **f)
    y = torch.empty((P, 3, 729), **f)
    dy = torch.empty_like(y)
    work = torch.empty_like(act)
    grad = torch.empty(onet.N_PARAMS, **f)
    scratch = torch.zeros(1025, dtype=torch.float64, device=dev)
    mfe.mfe_net_forward(W.data_ptr(), X.data_ptr(), P, act.data_ptr(), y.data_ptr(), var)
    loss = mfe.mfe_net_loss(y.data_ptr(), Tt.data_ptr(), y.numel(), dy.data_ptr(), scratch.data_ptr())
    mfe.mfe_net_backward(W.data_ptr(), X.data_ptr(), act.data_ptr(), dy.data_ptr(), P, work.data_ptr(),
                         grad.data_ptr(), var)
    assert _rel(y.cpu().numpy(), y_ref) <= 1e-5
    assert _rel(act[0].cpu().numpy(), acts[0]) <= 1e-5 and _rel(act[1].cpu().numpy(), acts[1]) <= 1e-5
    assert abs(loss - loss_ref) <= 1e-5 * loss_ref
    g = grad.cpu().numpy()
    for a, b in ((0, 5184), (5184, 5216), (5216, 32864), (32864, 32896), (32896, 35488), (35488, 35491)):
        if lin and b - a <= 32:
            assert np.all(g[a:b] == 0.0)
            continue
        assert _rel(g[a:b], g_ref[a:b]) <= 1e-4, (a, b, _rel(g[a:b], g_ref[a:b]))
    # the weight gradients are reduced in a fixed order: bitwise reproducible
    grad2 = torch.empty_like(grad)
    mfe.mfe_net_backward(W.data_ptr(), X.data_ptr(), act.data_ptr(), dy.data_ptr(), P, work.data_ptr(),
                         grad2.data_ptr(), var)
    assert torch.equal(grad, grad2)


def test_adam_parity(torch_dev):
    import paper_2505_15535_amd as mfe
    torch, dev = torch_dev
    rng = np.random.default_rng(1)
    w = rng.normal(size=onet.N_PARAMS).astype(np.float32)
    m, v = np.zeros_like(w), np.zeros_like(w)
    W, M, V = (torch.from_numpy(a.copy()).to(dev) for a in (w, m, v))
    wr, mr, vr = w.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in (1, 2, 3):
        g = rng.normal(size=onet.N_PARAMS).astype(np.float32)
        G = torch.from_numpy(g).to(dev)
        mfe.mfe_net_adam(W.data_ptr(), G.data_ptr(), M.data_ptr(), V.data_ptr(), step, 1e-3)
        wr, mr, vr = onet.adam_step(wr, g.astype(np.float64), mr, vr, step, 1e-3)
    assert _rel(W.cpu().numpy() - w, wr - w) <= 1e-4



def test_training_resumes_from_checkpoint(torch_dev, tmp_path):
    """Adam training stopped after two steps, saved, loaded into a new network
    and continued gives bitwise the parameters and moments of the
    uninterrupted run (the forward, loss, backward and Adam kernels reduce in
    a fixed order)."""
    from paper_2505_15535_amd import learned
    torch, dev = torch_dev
    rng = np.random.default_rng(3)
    P = 4
    batches = [(torch.from_numpy(rng.normal(size=(P, 6, 729)).astype(np.float32)).to(dev),
                torch.from_numpy(rng.normal(size=(P, 3, 729)).astype(np.float32)).to(dev)) for _ in range(4)]
    a = learned.Net(learned.init_params(5), dev, "relu")
    path = tmp_path / "net.npz"
    losses = []
    for k, (x, t) in enumerate(batches):
        losses.append(a.train_step(x, t, 1e-3))
        if k == 1:
            a.save(path)
    b = learned.Net.load(path, dev)
    assert b.step == 2
    resumed = [b.train_step(x, t, 1e-3) for x, t in batches[2:]]
    assert resumed == losses[2:]
    assert torch.equal(a.w, b.w) and torch.equal(a.m, b.m) and torch.equal(a.v, b.v) and a.step == b.step


def test_training_loop_resumes_from_its_checkpoint(torch_dev, tmp_path):
    """learned.train stopped after one epoch and resumed from its checkpoint
    (network, Adam moments, epoch, shuffling generator, loss history) goes on
    as the uninterrupted run does: the same epoch losses and parameters, to
    the rounding of the applies' atomic sums."""
    from paper_2505_15535_amd import learned
    torch, dev = torch_dev
    data = learned.generate([(60.0, 100.0)], nx=16, ny=8, nz=8, steps=2, states_per_path=1, n_loads=1, seed=2,
                            cg_stages=(0, 2))
    full, hist = learned.train(data, nx=16, ny=8, nz=8, epochs=3, lr=1e-3, seed=4)
    ck = tmp_path / "train.npz"
    _, h1 = learned.train(data, nx=16, ny=8, nz=8, epochs=1, lr=1e-3, seed=4, checkpoint=ck)
    back, h3 = learned.train(data, nx=16, ny=8, nz=8, epochs=3, lr=1e-3, seed=4, checkpoint=ck, resume=True)
    assert len(h1) == 1 and len(h3) == 3 and h3[0] == h1[0] and back.step == full.step
    assert h3 == pytest.approx(hist, rel=1e-6)
    assert _rel(back.params(), full.params()) <= 1e-5

def test_patch_gather_scatter_and_invariants(torch_dev):
    import paper_2505_15535_amd as mfe
    torch, dev = torch_dev
    nx, ny, nz = 8, 4, 4
    verts = synthetic.box_vertices(nx, ny, nz, (2.0, 1.0, 1.0), 0.1, np.random.default_rng(3))
    op = mfe.Operator(nx, ny, nz, 2, verts, 1.0, 10.0, device=0)
    assert op.n_patches == 2
    Nx, Ny, Nz = 17, 9, 9
    # affine state: F = F0 at every cell centre
    F0 = np.array([[1.1, 0.05, -0.02], [0.03, 0.95, 0.04], [0.0, -0.06, 1.02]])
    from oracle.mesh import BoxMesh
    X = BoxMesh(nx, ny, nz, 2, verts).node_positions()
    u = ((X @ (F0 - np.eye(3)).T)).reshape(-1)
    op.set_state(torch.from_numpy(u).to(dev))
    rng = np.random.default_rng(4)
    r = rng.normal(size=op.n_dofs)
    feat, scale = op.patch_features(torch.from_numpy(r).to(dev))
    feat, scale = feat.cpu().numpy(), scale.cpu().numpy()
    nodes = onet.patch_nodes(2, 1, 1, Nx, Ny)
    R = r.reshape(-1, 3)
    for p in range(2):
        rp = R[nodes[p]]
        s = np.sqrt(np.mean(rp ** 2))
        assert abs(scale[p] - s) <= 1e-6 * s
        np.testing.assert_allclose(feat[p, :3].T, rp / s, rtol=2e-6, atol=1e-6)
    C = F0.T @ F0
    I1, I2, J = np.trace(C), 0.5 * (np.trace(C) ** 2 - np.trace(C @ C)), np.linalg.det(F0)
    np.testing.assert_allclose(feat[:, 3], I1 - 3.0, atol=2e-6)
    np.testing.assert_allclose(feat[:, 4], I2 - 3.0, atol=2e-6)
    np.testing.assert_allclose(feat[:, 5], J - 1.0, atol=2e-6)
    e = rng.normal(size=op.n_dofs)
    t = op.patch_targets(torch.from_numpy(e).to(dev), torch.from_numpy(scale).to(dev)).cpu().numpy()
    for p in range(2):
        np.testing.assert_allclose(t[p].T, e.reshape(-1, 3)[nodes[p]] / scale[p], rtol=2e-6, atol=1e-6)
    # scatter: average of the patches holding a node, times s_p
    y = rng.normal(size=(2, 3, 729)).astype(np.float32)
    z0 = rng.normal(size=op.n_dofs)
    z = op.patch_scatter(torch.from_numpy(y).to(dev), torch.from_numpy(scale).to(dev),
                         torch.from_numpy(z0.copy()).to(dev), alpha=0.5).cpu().numpy()
    acc = np.zeros((op.n_dofs // 3, 3))
    cnt = np.zeros(op.n_dofs // 3)
    for p in range(2):
        acc[nodes[p]] += scale[p] * y[p].T.astype(np.float64)
        cnt[nodes[p]] += 1
    ref = z0.reshape(-1, 3) + 0.5 * acc / cnt[:, None]
    np.testing.assert_allclose(z.reshape(-1, 3), ref, rtol=1e-6, atol=1e-9)
    assert cnt.max() == 2 and cnt.min() == 1


def test_learned_step_in_the_smoother(torch_dev):
    """Train on residuals from seeded random load paths of a 16x8x8 beam
    (twist 30-120 degrees, lambda/mu log-uniform in 10-1000) and evaluate at
    a held-out state (lambda = 100, 60 degrees).  The learned step in the
    finest post-smoother is the energy-optimal step along N, so the cycle
    with it never leaves a larger error energy than the cycle stopped before
    it (the same cycle with a zero network); on held-out residuals it also
    leaves less than the plain cycle with all its Chebyshev steps.  The
    step's graph replay matches the launch-by-launch cycle; CG with it
    reaches the tolerance with a true residual to match; the CG iteration
    counts with and without it are printed."""
    import paper_2505_15535_amd as mfe
    from paper_2505_15535_amd import learned
    torch, dev = torch_dev
    paths = learned.random_paths(3, 5)
    assert all(30.0 <= t <= 120.0 and 10.0 <= l <= 1000.0 for t, l in paths)
    data = learned.generate(paths, nx=16, ny=8, nz=8, steps=3, states_per_path=2, n_loads=2, seed=1)
    netw, hist = learned.train(data, nx=16, ny=8, nz=8, epochs=25, lr=1e-3, seed=0)
    print("mean J per epoch", [f"{h:.3e}" for h in hist])
    assert hist[-1] < 0.0 and min(hist) < hist[0]
    op, bv, cd = learned.beam(16, 8, 8, 100.0)
    cdt = torch.from_numpy(cd).to(dev)
    u = torch.zeros(op.n_dofs, dtype=torch.float64, device=dev)
    op.solve_load_path(u, bv(60.0), 3, strategy="t2", preconditioner="gmg", max_newton=20, cg_rtol=1e-3)
    op.set_state(u)
    o = dict(strategy="t2", mg_precision="fp64")
    rs = learned.residuals_at_state(op, cd, np.random.default_rng(7), n_loads=1)   # leaves a zero network set

    def energy(e, z, r):   # ||e - z||_K^2 / ||e||_K^2
        d = e - z
        return float(torch.dot(d, op.apply(d, strategy="t2"))) / float(torch.dot(e, r))

    rows = []
    for r in rs:
        e, _, _, _ = op.cg_solve(r, strategy="t2", preconditioner="gmg", max_cg=500, cg_rtol=1e-11)
        op.set_network(np.zeros(mfe.MFE_NET_PARAMS, dtype=np.float32))
        z_stop = op.gmg_apply(r, net=True, **o)            # the cycle stopped before the learned step
        op.set_network(netw.params())
        z_net = op.gmg_apply(r, net=True, **o)
        z_net0 = op.gmg_apply(r, net=True, mg_graph=0, **o)
        assert float(torch.linalg.norm(z_net - z_net0) / torch.linalg.norm(z_net)) < 1e-10
        z_plain = op.gmg_apply(r, **o)
        rows.append((energy(e, z_stop, r), energy(e, z_net, r), energy(e, z_plain, r)))
    rows = np.array(rows)
    # a new network (cleared, then set again with the other variant) is what the next cycle uses
    op.set_network(None)
    op.set_network(netw.params(), "linear")
    z_lin = op.gmg_apply(rs[0], net=True, **o)
    z_lin0 = op.gmg_apply(rs[0], net=True, mg_graph=0, **o)
    assert float(torch.linalg.norm(z_lin - z_lin0) / torch.linalg.norm(z_lin0)) < 1e-10
    assert float(torch.linalg.norm(z_lin - z_net) / torch.linalg.norm(z_net)) > 1e-8
    op.set_network(netw.params())
    print("error energy after the cycle: stopped before the step / with the learned step / plain\n", rows.round(4))
    assert np.all(rows[:, 1] <= rows[:, 0] * (1.0 + 1e-9))
    assert rows[:, 1].mean() < rows[:, 2].mean()
    b = torch.from_numpy(np.random.default_rng(9).standard_normal(op.n_dofs)).to(dev)
    b[cdt] = 0.0
    res = {}
    for pc in ("gmg", "gmg_net"):
        op.set_network(netw.params())
        x, it, rel, st = op.cg_solve(b, strategy="t2", preconditioner=pc, max_cg=500, cg_rtol=1e-8)
        true = float(torch.linalg.norm(b - op.apply(x, strategy="t2")) / torch.linalg.norm(b))
        res[pc] = (it, true, st)
    print("CG iterations, true relative residual:", res)
    for pc in res:
        assert res[pc][2] == "MFE_OK" and res[pc][1] <= 2e-8
    with pytest.raises(mfe.MfeError):   # the learned step runs in the FP64 V-cycle only
        op.cg_solve(b, strategy="t2", preconditioner="gmg_net", mg_precision="fp32", max_cg=50, cg_rtol=1e-3)


def test_bad_network_falls_back(torch_dev):
    """A network with huge random weights makes r.Br <= 0 or stalls CG: the
    solve drops the correction and still converges."""
    import paper_2505_15535_amd as mfe
    from paper_2505_15535_amd import learned
    torch, dev = torch_dev
    op, bv, cd = learned.beam(16, 8, 8, 100.0)
    u = torch.zeros(op.n_dofs, dtype=torch.float64, device=dev)
    op.set_network(np.random.default_rng(0).normal(0.0, 3.0, mfe.MFE_NET_PARAMS).astype(np.float32))
    reps = op.solve_load_path(u, bv(20.0), 2, strategy="t2", preconditioner="gmg_net", max_newton=8, cg_rtol=1e-3)
    assert all(r["converged"] for r in reps if not r.get("failed"))
    assert sum(r["net_fallbacks"] for r in reps) > 0
    with pytest.raises(mfe.MfeError):
        op.set_network(np.full(mfe.MFE_NET_PARAMS, np.nan, dtype=np.float32))
