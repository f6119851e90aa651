"""Training data, training loop and evaluation of the learned smoother
correction (preconditioner "gmg_net").

The correction is a step of the finest level's post-smoother (it replaces
the last Chebyshev step): with x the V-cycle's iterate before that step, the
residual left is r1 = r - K x, and the network maps the patch features of r1
(residual scaled by its patch RMS, strain invariants of the state) to a
correction N(r1), assembled from the patch outputs by averaging over shared
nodes; the cycle adds alpha N with the energy-optimal alpha.  Its quality
is the energy norm of the error it leaves, ||e1 - N||_K^2 with e1 = K^-1 r1,
which equals 2 J(N) + e1.r1 with J(N) = N.K N / 2 - N.r1: the loss is J, the
potential energy of the correction, whose gradient K N - r1 is the residual
after the correction -- no solved target is needed, and the norm weights the
local (high-frequency) part of the error that a patch network can represent,
not the smooth part that the coarse grid already handles.  Residuals r1 come
from the Newton-CG solver itself: states along twisted-beam load paths with
seeded random twist angles and lambda/mu (random_paths), CG residuals of
random loads after 0-8 GMG-CG iterations, one V-cycle applied up to the
learned step (the cycle with a zero network, whose step is then empty).
Every arithmetic step runs in the library's kernels (V-cycle, applies,
features, scatter and its adjoint, the network's forward and backward passes,
Adam); torch only holds the buffers.
"""

from __future__ import annotations

import numpy as np

from . import (MFE_NET_PARAMS, NET_VARIANTS, Operator, mfe_net_adam, mfe_net_backward, mfe_net_forward,
               mfe_net_loss)

LAYERS = ((6, 32), (32, 32), (32, 3))


def init_params(seed: int = 0, last_scale: float = 0.1) -> np.ndarray:
    """He-normal weights (fan-in 27 ci), zero biases; the last layer scaled down."""
    rng = np.random.default_rng(seed)
    out = []
    for li, (ci, co) in enumerate(LAYERS):
        std = np.sqrt(2.0 / (27 * ci))
        if li == len(LAYERS) - 1:
            std *= last_scale
        out.append(rng.normal(0.0, std, co * ci * 27))
        out.append(np.zeros(co))
    p = np.concatenate(out).astype(np.float32)
    assert p.size == MFE_NET_PARAMS
    return p


class Net:
    """Parameters, Adam moments and scratch of one network on the GPU."""

    def __init__(self, params: np.ndarray, device, variant="relu"):
        import torch
        self.device = device
        self.variant = variant
        self.var = NET_VARIANTS[variant]
        self.w = torch.from_numpy(np.ascontiguousarray(params, dtype=np.float32)).to(device)
        self.g = torch.zeros_like(self.w)
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.step = 0
        self.scratch = torch.zeros(1025, dtype=torch.float64, device=device)
        self._bufs = {}

    def _buf(self, P):
        import torch
        if P not in self._bufs:
            f = dict(dtype=torch.float32, device=self.device)
            self._bufs[P] = (torch.empty((2, P, 32, 729), **f), torch.empty((P, 3, 729), **f),
                             torch.empty((P, 3, 729), **f), torch.empty((2, P, 32, 729), **f))
        return self._bufs[P]

    def forward(self, x):
        P = x.shape[0]
        act, y, _, _ = self._buf(P)
        mfe_net_forward(self.w.data_ptr(), x.data_ptr(), P, act.data_ptr(), y.data_ptr(), self.var)
        return y

    def loss(self, x, t) -> float:
        y = self.forward(x)
        return mfe_net_loss(y.data_ptr(), t.data_ptr(), y.numel(), None, self.scratch.data_ptr())

    def train_step(self, x, t, lr) -> float:
        P = x.shape[0]
        act, y, dy, work = self._buf(P)
        mfe_net_forward(self.w.data_ptr(), x.data_ptr(), P, act.data_ptr(), y.data_ptr(), self.var)
        loss = mfe_net_loss(y.data_ptr(), t.data_ptr(), y.numel(), dy.data_ptr(), self.scratch.data_ptr())
        mfe_net_backward(self.w.data_ptr(), x.data_ptr(), act.data_ptr(), dy.data_ptr(), P, work.data_ptr(),
                         self.g.data_ptr(), self.var)
        self.step += 1
        mfe_net_adam(self.w.data_ptr(), self.g.data_ptr(), self.m.data_ptr(), self.v.data_ptr(), self.step, lr)
        return loss

    def params(self) -> np.ndarray:
        return self.w.cpu().numpy().copy()

    def save(self, path, **extra):
        """Parameters, Adam moments and step count (and any `extra` arrays) as
        an .npz file, written whole or not at all, so that training resumed
        from it takes the same steps as uninterrupted."""
        import os
        tmp = str(path) + ".tmp.npz"
        np.savez(tmp, w=self.params(), m=self.m.cpu().numpy(), v=self.v.cpu().numpy(), step=self.step,
                 variant=self.variant, **extra)
        os.replace(tmp, path)

    @classmethod
    def load(cls, path, device):
        with np.load(path, allow_pickle=False) as f:
            net = cls(f["w"], device, str(f["variant"]))
            net.m.copy_(torch_from(f["m"], device))
            net.v.copy_(torch_from(f["v"], device))
            net.step = int(f["step"])
        return net


def torch_from(a, device):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


def beam(nx, ny, nz, lam, device=0):
    """Operator of the twisted beam (clamped at x = 0) and its boundary data function."""
    import synthetic
    L = (nx / ny, 1.0, 1.0)
    op = Operator(nx, ny, nz, 2, synthetic.box_vertices(nx, ny, nz, L), 1.0, lam, device=device)
    cd, _ = synthetic.clamp_and_twist(nx, ny, nz, 2, L, 0.0)
    op.set_constraints(cd)

    def bv(theta_deg):
        return lambda t: synthetic.clamp_and_twist(nx, ny, nz, 2, L, np.deg2rad(theta_deg) * t)

    return op, bv, cd


def random_paths(n, seed, theta=(30.0, 120.0), lam=(10.0, 1000.0)):
    """n load paths (theta_deg, lambda/mu): theta uniform, lambda/mu log-uniform in the given ranges."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(theta[0], theta[1], n)
    lm = np.exp(rng.uniform(np.log(lam[0]), np.log(lam[1]), n))
    return [(float(a), float(b)) for a, b in zip(th, lm)]


def residuals_at_state(op, cdofs, rng, n_loads=2, cg_stages=(0, 1, 2, 4, 8), opts=None):
    """Unit-norm residuals r1 = r - K V' r, V' the V-cycle up to the learned
    step (the cycle run with a zero network), for r = CG residuals of random
    loads after 0, 1, 2, 4, 8 GMG-CG iterations, at the operator's current
    state (T2 cache and level data are built here; the operator's network is
    replaced by zeros)."""
    import torch
    from . import MFE_NET_PARAMS
    o = dict(strategy="t2", mg_precision="fp64")
    o.update(opts or {})
    dev = op.device
    op.set_network(np.zeros(MFE_NET_PARAMS, dtype=np.float32))
    op.build_cache("t2")
    op.gmg_setup(**o)
    out = []
    for _ in range(n_loads):
        b0 = torch.from_numpy(rng.standard_normal(op.n_dofs)).to(dev)
        op.zero_constrained(b0)
        for j in cg_stages:
            r = b0.clone()
            if j > 0:   # r = b0 - K x after j GMG-CG iterations
                x, _, _, _ = op.cg_solve(b0, preconditioner="gmg", max_cg=j, cg_rtol=1e-30, **o)
                op.axpby(-1.0, op.apply(x, strategy="t2"), 1.0, r)
            z = op.gmg_apply(r, net=True, **o)
            r1 = op.axpby(-1.0, op.apply(z, strategy="t2"), 1.0, r)   # r1 = r - K V' r
            op.zero_constrained(r1)
            op.axpby(0.0, r1, 1.0 / op.dot(r1, r1) ** 0.5, r1)
            out.append(r1)
    return out


class Sample:
    """One state of a load path and the residuals collected there."""

    def __init__(self, u, residuals):
        self.u = u
        self.residuals = residuals


def generate(paths, nx=64, ny=16, nz=16, steps=None, states_per_path=8, n_loads=2, seed=0, device=0, log=None,
             cg_stages=(0, 1, 2, 4, 8)):
    """Samples along load paths [(theta_deg, lam), ...] of the twisted beam
    (in `steps` load steps, default one per 9 degrees);
    returns [(lam, [Sample, ...]), ...] (each sample: one state and
    n_loads * len(cg_stages) residuals, each giving one pair per patch)."""
    import torch
    rng = np.random.default_rng(seed)
    out = []
    for theta, lam in paths:
        op, bv, cd = beam(nx, ny, nz, lam, device)
        u = torch.zeros(op.n_dofs, dtype=torch.float64, device=op.device)
        states = []
        n_steps = steps if steps else max(1, int(np.ceil(theta / 9.0)))
        op.solve_load_path(u, bv(theta), n_steps, on_step=lambda t, uu: states.append(uu.clone()),
                           extrapolate=False, strategy="t2", preconditioner="gmg", max_newton=30, cg_rtol=1e-3,
                           forcing=0.5)
        pick = np.linspace(0, len(states) - 1, min(states_per_path, len(states))).round().astype(int)
        samples = []
        for k in pick:
            op.set_state(states[k])
            samples.append(Sample(states[k], residuals_at_state(op, cd, rng, n_loads=n_loads, cg_stages=cg_stages)))
        out.append((lam, samples))
        if log:
            log(f"path theta={theta:.1f} lam={lam:.1f}: {len(states)} states, {len(samples)} sampled")
        op.close()
    return out


def energy_step(op, net, r1, lr=None):
    """J(N) = N.K N / 2 - N.r1 for the correction N of residual r1 at the
    operator's state (T2 cache built); with lr, also one Adam step on J."""
    import torch
    feat, scale = op.patch_features(r1, variant=net.variant)
    P = feat.shape[0]
    act, y, dy, work = net._buf(P)
    mfe_net_forward(net.w.data_ptr(), feat.data_ptr(), P, act.data_ptr(), y.data_ptr(), net.var)
    z = torch.zeros_like(r1)
    op.patch_scatter(y, scale, z)
    op.zero_constrained(z)
    Kz = op.apply(z, strategy="t2")
    J = 0.5 * op.dot(z, Kz) - op.dot(z, r1)
    if lr is not None:
        g = op.axpby(-1.0, r1, 1.0, Kz)   # K z - r1, in place of Kz
        op.patch_adjoint(g, scale, dy)
        mfe_net_backward(net.w.data_ptr(), feat.data_ptr(), act.data_ptr(), dy.data_ptr(), P, work.data_ptr(),
                         net.g.data_ptr(), net.var)
        net.step += 1
        mfe_net_adam(net.w.data_ptr(), net.g.data_ptr(), net.m.data_ptr(), net.v.data_ptr(), net.step, lr)
    return J


def train(data, nx=64, ny=16, nz=16, epochs=10, lr=1e-3, seed=0, device=0, log=None, variant="relu",
          checkpoint=None, resume=False):
    """Adam on the energy of the correction over every (state, residual) of
    `data` (from generate); returns (Net, per-epoch mean J).
    checkpoint: path of an .npz file rewritten after every epoch with the
    network, its Adam moments, the epoch count, the shuffling generator's
    state and the loss history; resume=True goes on from that file."""
    import json
    import torch
    dev = torch.device("cuda", device)
    rng = np.random.default_rng(seed)
    hist = []
    first = 0
    if not resume:
        net = Net(init_params(seed), dev, variant)
    else:
        net = Net.load(checkpoint, dev)
        with np.load(checkpoint, allow_pickle=False) as f:
            first = int(f["epoch"])
            rng.bit_generator.state = json.loads(str(f["rng"]))
            hist = [float(x) for x in f["hist"]]
    ops = {}
    for lam, _ in data:
        if lam not in ops:
            ops[lam] = beam(nx, ny, nz, lam, device)
    for ep in range(first, epochs):
        tot, cnt = 0.0, 0
        order = [(li, si) for li, (_, ss) in enumerate(data) for si in range(len(ss))]
        rng.shuffle(order)
        for li, si in order:
            lam, samples = data[li]
            op, _, cd = ops[lam]
            smp = samples[si]
            op.set_state(smp.u)
            op.build_cache("t2")
            for k in rng.permutation(len(smp.residuals)):
                tot += energy_step(op, net, smp.residuals[k], lr)
                cnt += 1
        hist.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep}: mean J {hist[-1]:.4e}")
        if checkpoint is not None:
            net.save(checkpoint, epoch=ep + 1, rng=json.dumps(rng.bit_generator.state), hist=np.asarray(hist))
    for op, _, _ in ops.values():
        op.close()
    return net, hist
