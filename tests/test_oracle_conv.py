"""Pins of the convolution / training oracle (oracle/conv_oracle.py)
against facts that do not depend on it: brute-force loops on tiny inputs,
the identity filter, a constant input, the adjoint identity of the backward
maps, central finite differences, and the closed form of Adam's first
steps."""
import itertools

import numpy as np
import pytest

from oracle import conv_oracle as co

GEOMS = [  # (in spatial, k, stride, pad, dil)
    ((5, 6, 7), 3, 1, 1, 1),
    ((7, 6, 5), 3, 1, 2, 2),
    ((9, 9, 9), 4, 4, 2, 1),
    ((13, 10, 9), 8, 4, 4, 1),
    ((6, 5, 7), 2, 2, 0, 1),
]


def brute_conv(x, w, b, s, p, d):
    N, Ci, D, H, W = x.shape
    Co, _, k0, k1, k2 = w.shape
    o = [co.out_size(x.shape[2 + i], w.shape[2 + i], s, p, d) for i in range(3)]
    y = np.zeros((N, Co, *o))
    for n, c, i, j, l in itertools.product(range(N), range(Co), range(o[0]), range(o[1]), range(o[2])):
        acc = b[c]
        for ci, a, bb, cc in itertools.product(range(Ci), range(k0), range(k1), range(k2)):
            z, yy, xx = i * s - p + a * d, j * s - p + bb * d, l * s - p + cc * d
            if 0 <= z < D and 0 <= yy < H and 0 <= xx < W:
                acc += w[c, ci, a, bb, cc] * x[n, ci, z, yy, xx]
        y[n, c, i, j, l] = acc
    return y


@pytest.mark.parametrize("shape,k,s,p,d", GEOMS[:3] + GEOMS[4:])
def test_conv_matches_brute_force(shape, k, s, p, d):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 2, *shape))
    w = rng.standard_normal((3, 2, k, k, k))
    b = rng.standard_normal(3)
    y = co.conv3d(x, w, b, s, p, d)
    assert np.allclose(y, brute_conv(x, w, b, s, p, d), rtol=1e-13, atol=1e-12)


def test_identity_filter():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 3, 6, 7, 5))
    for d in (1, 2, 3):
        w = np.zeros((3, 3, 3, 3, 3))
        for c in range(3):
            w[c, c, 1, 1, 1] = 1.0
        assert np.array_equal(co.conv3d(x, w, None, 1, d, d), x)


def test_constant_input_gives_weight_sums():
    rng = np.random.default_rng(3)
    w = rng.standard_normal((4, 2, 3, 3, 3))
    b = rng.standard_normal(4)
    x = np.full((1, 2, 9, 9, 9), 2.5)
    y = co.conv3d(x, w, b, 1, 2, 2)
    inner = y[0, :, 2:-2, 2:-2, 2:-2]  # outputs whose taps all lie inside the input
    expect = b + 2.5 * w.sum(axis=(1, 2, 3, 4))
    assert np.allclose(inner, expect[:, None, None, None], rtol=1e-14, atol=1e-13)


@pytest.mark.parametrize("shape,k,s,p,d", GEOMS)
def test_backward_data_is_the_adjoint(shape, k, s, p, d):
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 3, *shape))
    w = rng.standard_normal((2, 3, k, k, k))
    y = co.conv3d(x, w, None, s, p, d)
    g = rng.standard_normal(y.shape)
    dx = co.conv3d_bwd_data(g, w, shape, s, p, d)
    assert dx.shape == x.shape
    lhs, rhs = np.sum(y * g), np.sum(x * dx)
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(y * g)) + 1e-12


@pytest.mark.parametrize("shape,k,s,p,d", GEOMS)
def test_backward_weight_against_finite_differences(shape, k, s, p, d):
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, 2, *shape))
    w = rng.standard_normal((3, 2, k, k, k))
    b = rng.standard_normal(3)
    y0 = co.conv3d(x, w, b, s, p, d)
    t = rng.standard_normal(y0.shape)

    def loss(w_, b_):
        return 0.5 * np.sum((co.conv3d(x, w_, b_, s, p, d) - t) ** 2)

    g = y0 - t
    dw, db = co.conv3d_bwd_weight(x, g, k, s, p, d)
    h = 1e-5
    for idx in [(0, 0, 0, 0, 0), (2, 1, k - 1, k // 2, 0), (1, 0, k // 2, k - 1, k - 1)]:
        e = np.zeros_like(w)
        e[idx] = h
        fd = (loss(w + e, b) - loss(w - e, b)) / (2 * h)
        assert abs(fd - dw[idx]) <= 1e-6 * max(1.0, abs(fd))
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        fd = (loss(w, b + e) - loss(w, b - e)) / (2 * h)
        assert abs(fd - db[c]) <= 1e-6 * max(1.0, abs(fd))


def test_transposed_layer_shape():
    """37^3 coarse -> 145^3 nodes: kernel 8, stride 4, padding 4."""
    assert co.out_size(145, 8, 4, 4, 1) == 37
    assert co.out_size(145, 4, 4, 2, 1) == 37


def test_leaky_relu_backward_through_output():
    rng = np.random.default_rng(6)
    z = rng.standard_normal(1000)
    y = co.leaky_relu(z)
    h = 1e-6
    fd = (co.leaky_relu(z + h) - co.leaky_relu(z - h)) / (2 * h)
    keep = np.abs(z) > 1e-3
    assert np.allclose(co.leaky_relu_bwd(np.ones_like(z), y)[keep], fd[keep], rtol=1e-8)


def test_mse_gradient():
    rng = np.random.default_rng(7)
    pr, tg = rng.standard_normal(50), rng.standard_normal(50)
    L, g = co.mse(pr, tg)
    assert np.isclose(L, np.sum((pr - tg) ** 2) / 50, rtol=1e-14)
    h = 1e-6
    for i in (0, 17, 49):
        e = np.zeros(50)
        e[i] = h
        fd = (co.mse(pr + e, tg)[0] - co.mse(pr - e, tg)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-8


def test_adam_first_steps_move_by_lr_sign():
    """With a constant gradient, bias correction makes m_hat = g and
    v_hat = g^2 at every step, so each step is lr * g / (|g| + eps)."""
    rng = np.random.default_rng(8)
    th = rng.standard_normal(20)
    g = rng.standard_normal(20)
    m = np.zeros(20)
    v = np.zeros(20)
    t0 = th.copy()
    for t in (1, 2, 3):
        th, m, v = co.adam_step(th, g, m, v, t, lr=0.01)
        assert np.allclose(th, t0 - t * 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)
