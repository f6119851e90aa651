"""Pins of the network oracle (oracle/net.py) against facts that do not come
from retyping it: central finite differences of the loss, the response to a
unit impulse, constant inputs, translation equivariance, and Adam's first
step (whose size is lr times the sign of the gradient)."""

import numpy as np
import pytest

from oracle import net


def _params(seed, scale=0.2):
    return np.random.default_rng(seed).normal(0.0, scale, net.N_PARAMS)


def test_parameter_count():
    assert net.N_PARAMS == 35491


def test_impulse_response_is_the_kernel():
    rng = np.random.default_rng(1)
    W = rng.normal(size=(4, 2, 3, 3, 3))
    x = np.zeros((1, 2, 9, 9, 9))
    x[0, 1, 4, 4, 4] = 1.0
    out = net.conv3d(x, W)
    # output node (4+dz', ...) sees the input node at offset -(dz'-... ): out[4-dz+1] = W[.., dz]
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                np.testing.assert_allclose(out[0, :, 5 - dz, 5 - dy, 5 - dx], W[:, 1, dz, dy, dx], rtol=0, atol=1e-15)
    assert np.count_nonzero(out) == 4 * 27


def test_constant_input_interior_and_corner():
    rng = np.random.default_rng(2)
    W, b = rng.normal(size=(3, 2, 3, 3, 3)), rng.normal(size=3)
    x = np.full((1, 2, 9, 9, 9), 0.5)
    out = net.conv3d(x, W, b)
    np.testing.assert_allclose(out[0, :, 4, 4, 4], b + 0.5 * W.sum(axis=(1, 2, 3, 4)), rtol=1e-13)
    # at the corner only the 8 taps pointing into the grid contribute
    np.testing.assert_allclose(out[0, :, 0, 0, 0], b + 0.5 * W[:, :, 1:, 1:, 1:].sum(axis=(1, 2, 3, 4)), rtol=1e-13)


def test_translation_equivariance_away_from_the_border():
    rng = np.random.default_rng(3)
    W = rng.normal(size=(2, 2, 3, 3, 3))
    x = np.zeros((1, 2, 9, 9, 9))
    x[0, :, 2:5, 2:5, 2:5] = rng.normal(size=(2, 3, 3, 3))
    xs = np.roll(x, (1, 2, 1), axis=(2, 3, 4))
    a, b = net.conv3d(x, W), net.conv3d(xs, W)
    np.testing.assert_allclose(np.roll(a, (1, 2, 1), axis=(2, 3, 4)), b, atol=1e-13)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_against_central_differences(seed):
    rng = np.random.default_rng(10 + seed)
    P = 2
    prm = _params(seed)
    x = rng.normal(size=(P, 6, 729))
    t = rng.normal(size=(P, 3, 729))
    y, acts = net.forward(prm, x)
    loss, dy = net.mse(y, t)
    g = net.backward(prm, x, acts, dy)
    idx = rng.choice(net.N_PARAMS, 40, replace=False)
    idx = np.concatenate([idx, [net.N_PARAMS - 1, 5184, 32864, 35488]])  # biases of every layer
    h = 1e-6
    for k in idx:
        e = np.zeros(net.N_PARAMS)
        e[k] = h
        lp = net.mse(net.forward(prm + e, x)[0], t)[0]
        lm = net.mse(net.forward(prm - e, x)[0], t)[0]
        fd = (lp - lm) / (2 * h)
        # 1e-5: a ReLU pre-activation within h of its kink bends the difference
        # quotient at that level; a wrong index, sign or transpose is O(1)
        assert abs(fd - g[k]) <= 1e-5 * max(1e-3, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_relu_layers_zero_gradient_of_dead_units():
    # all first-layer pre-activations negative: every gradient but the last layer's bias... vanishes
    prm = np.zeros(net.N_PARAMS)
    prm[5184:5216] = -1.0           # b1 < 0 and W1 = 0: a1 = 0
    x = np.random.default_rng(4).normal(size=(1, 6, 729))
    y, acts = net.forward(prm, x)
    assert np.all(acts[0] == 0.0)
    g = net.backward(prm, x, acts, np.ones((1, 3, 729)))
    assert np.all(g[:35488] == 0.0)
    np.testing.assert_allclose(g[35488:], 729.0)


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(5)
    w, g = rng.normal(size=100), rng.normal(size=100)
    w1, m, v = net.adam_step(w, g, np.zeros(100), np.zeros(100), 1, 1e-3)
    np.testing.assert_allclose(w - w1, 1e-3 * np.sign(g), rtol=1e-6)


def test_patch_node_map():
    nodes = net.patch_nodes(2, 1, 1, 17, 9)
    assert nodes.shape == (2, 729)
    assert nodes[0, 0] == 0 and nodes[1, 0] == 8 and nodes[0, 728] == 8 + 17 * (8 + 9 * 8)
    # the shared face x = 8 appears in both patches
    assert len(np.intersect1d(nodes[0], nodes[1])) == 81


def test_linear_variant_is_linear_and_its_gradient_matches_differences():
    rng = np.random.default_rng(20)
    prm = _params(3)
    x1, x2 = rng.normal(size=(2, 1, 6, 729))
    y1 = net.forward(prm, x1, linear=True)[0]
    y2 = net.forward(prm, x2, linear=True)[0]
    y12 = net.forward(prm, 2.0 * x1 - 3.0 * x2, linear=True)[0]
    np.testing.assert_allclose(y12, 2.0 * y1 - 3.0 * y2, atol=1e-12)
    t = rng.normal(size=(1, 3, 729))
    y, acts = net.forward(prm, x1, linear=True)
    g = net.backward(prm, x1, acts, net.mse(y, t)[1], linear=True)
    assert np.all(g[[5184, 32864, 35488]] == 0.0)
    h = 1e-6
    for k in rng.choice(net.N_PARAMS, 10, replace=False):
        e = np.zeros(net.N_PARAMS)
        e[k] = h
        fd = (net.mse(net.forward(prm + e, x1, linear=True)[0], t)[0] -
              net.mse(net.forward(prm - e, x1, linear=True)[0], t)[0]) / (2 * h)
        if 5184 <= k < 5216 or 32864 <= k < 32896 or k >= 35488:
            continue  # biases are not parameters of this variant
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g[k])) + 1e-9
