"""Plain FP64 reference of the learned smoother correction's network: three
3x3x3 convolutions with zero padding on the 9x9x9 nodal grid of a patch
(6 -> 32 -> 32 -> 3 channels, ReLU after the first two), the mean squared
error, the gradient of that loss with respect to every parameter, and one
Adam step (Kingma & Ba, 2015, Algorithm 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Layouts follow the library's public ones: parameters are, per layer, the
weights W[co][ci][tap] with tap = a + 3 b + 9 c for the neighbour offset
(a-1, b-1, c-1) along (x, y, z), then the biases; an activation is
[patch][channel][v] with node v = i + 9 j + 81 k, i.e. a C-ordered
[patch][channel][k][j][i] array.  The convolutions are written from their
definition (sum over input channels and the 27 neighbours, zero outside the
grid) with numpy slicing over the padded grid; nothing is shared with the
HIP kernels.
"""

from __future__ import annotations

import numpy as np

LAYERS = ((6, 32, True), (32, 32, True), (32, 3, False))
N_PARAMS = sum(co * ci * 27 + co for ci, co, _ in LAYERS)
G = 9


def unpack(params):
    """[(W [co, ci, 3(z), 3(y), 3(x)], b [co]), ...] views of a flat parameter vector."""
    params = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for ci, co, _ in LAYERS:
        W = params[o:o + co * ci * 27].reshape(co, ci, 3, 3, 3)
        o += co * ci * 27
        b = params[o:o + co]
        o += co
        out.append((W, b))
    assert o == params.size
    return out


def conv3d(x, W, b=None):
    """out[p, o, k, j, i] = b[o] + sum_c sum_{dz,dy,dx in {0,1,2}}
    W[o, c, dz, dy, dx] * x[p, c, k+dz-1, j+dy-1, i+dx-1], zero outside."""
    P, C = x.shape[:2]
    xp = np.zeros((P, C, G + 2, G + 2, G + 2))
    xp[:, :, 1:-1, 1:-1, 1:-1] = x
    out = np.zeros((P, W.shape[0], G, G, G))
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                out += np.einsum("oc,pckji->pokji", W[:, :, dz, dy, dx],
                                 xp[:, :, dz:dz + G, dy:dy + G, dx:dx + G])
    if b is not None:
        out += b[None, :, None, None, None]
    return out


def conv3d_grad(x, dout):
    """d loss / d W[o, c, dz, dy, dx] = sum_p sum_kji dout[p,o,k,j,i] x[p,c,k+dz-1,j+dy-1,i+dx-1]
    and d loss / d b[o] = sum of dout[:, o]."""
    P, C = x.shape[:2]
    xp = np.zeros((P, C, G + 2, G + 2, G + 2))
    xp[:, :, 1:-1, 1:-1, 1:-1] = x
    dW = np.zeros((dout.shape[1], C, 3, 3, 3))
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                dW[:, :, dz, dy, dx] = np.einsum("pokji,pckji->oc", dout, xp[:, :, dz:dz + G, dy:dy + G, dx:dx + G])
    return dW, dout.sum(axis=(0, 2, 3, 4))


def conv3d_input_grad(dout, W):
    """d loss / d x for out = conv3d(x, W): each input node collects the
    output gradients of the nodes it fed, through the same weights."""
    P = dout.shape[0]
    dp = np.zeros((P, W.shape[1], G + 2, G + 2, G + 2))
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                dp[:, :, dz:dz + G, dy:dy + G, dx:dx + G] += np.einsum("oc,pokji->pckji", W[:, :, dz, dy, dx], dout)
    return dp[:, :, 1:-1, 1:-1, 1:-1]


def forward(params, x, linear=False):
    """x [P, 6, 729] -> (y [P, 3, 729], activations [a1, a2] each [P, 32, 729]).
    linear: the variant without ReLUs and biases (a linear map of x)."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 6, G, G, G)
    h, acts = x, []
    for (W, b), (_, _, relu) in zip(unpack(params), LAYERS):
        h = conv3d(h, W, None if linear else b)
        if relu:
            if not linear:
                h = np.maximum(h, 0.0)
            acts.append(h)
    P = x.shape[0]
    return h.reshape(P, 3, -1), [a.reshape(P, 32, -1) for a in acts]


def mse(y, t):
    """(mean of (y - t)^2, its gradient 2 (y - t) / n)."""
    d = np.asarray(y, dtype=np.float64) - np.asarray(t, dtype=np.float64)
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(params, x, acts, dy, linear=False):
    """Gradient of a loss with d loss / d y = dy, flat like params (the
    linear variant has no ReLU masks and zero bias gradients)."""
    P = dy.shape[0]
    x = np.asarray(x, dtype=np.float64).reshape(P, 6, G, G, G)
    a1, a2 = (np.asarray(a, dtype=np.float64).reshape(P, 32, G, G, G) for a in acts)
    (W1, _), (W2, _), (W3, _) = unpack(params)
    d3 = np.asarray(dy, dtype=np.float64).reshape(P, 3, G, G, G)
    gW3, gb3 = conv3d_grad(a2, d3)
    d2 = conv3d_input_grad(d3, W3) * (1.0 if linear else (a2 > 0.0))
    gW2, gb2 = conv3d_grad(a1, d2)
    d1 = conv3d_input_grad(d2, W2) * (1.0 if linear else (a1 > 0.0))
    gW1, gb1 = conv3d_grad(x, d1)
    if linear:
        gb1, gb2, gb3 = np.zeros_like(gb1), np.zeros_like(gb2), np.zeros_like(gb3)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def adam_step(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam update; returns new (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def patch_nodes(npx, npy, npz, Nx, Ny):
    """[P, 729] box node index of every patch node (patch (px,py,pz) holds
    nodes (8px+i, 8py+j, 8pz+k))."""
    i = np.arange(G)
    k3, j3, i3 = np.meshgrid(i, i, i, indexing="ij")
    out = []
    for pz in range(npz):
        for py in range(npy):
            for px in range(npx):
                out.append(((8 * px + i3) + Nx * ((8 * py + j3) + Ny * (8 * pz + k3))).ravel())
    return np.array(out)
