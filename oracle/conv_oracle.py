"""Plain FP64 reference of the learned warm start's building blocks.

TEST INFRASTRUCTURE ONLY: imported by tests/ (and nothing in the product
package).  The paper has no learned component; these are the textbook
definitions of the operations the surrogate network uses, written out
directly in numpy (one tensordot per filter tap, no blocking):

  * 3D convolution, NCDHW, cross-correlation form with zero padding p,
    stride s and dilation d per direction:
        y[n,co,o] = bias[co] + sum_{ci,t} w[co,ci,t] * xpad[n,ci,o*s + t*d]
  * its adjoint in x ("backward data", also the forward map of a transposed
    convolution): dx = A_w^T g,
  * its derivative in w ("backward weight"): dw[co,ci,t] =
    sum_{n,o} g[n,co,o] * xpad[n,ci,o*s + t*d], db[co] = sum_{n,o} g[n,co,o],
  * the leaky ReLU a(z) = z (z > 0), slope*z (z <= 0) and its derivative
    expressed through the output (the sign is preserved),
  * the mean-squared-error loss and its gradient,
  * one step of Adam (Kingma and Ba, 2015): bias-corrected first and second
    moment estimates.
"""
import numpy as np


def out_size(n_in, k, s, p, d):
    return (n_in + 2 * p - d * (k - 1) - 1) // s + 1


def _triple(v):
    return tuple(v) if np.ndim(v) else (int(v),) * 3


def _pad(x, p):
    return np.pad(x, ((0, 0), (0, 0), (p[0], p[0]), (p[1], p[1]), (p[2], p[2])))


def _tap_slice(o_shape, t, s, d):
    """Index slices of xpad read by tap t for all outputs o."""
    return tuple(slice(t[i] * d[i], t[i] * d[i] + s[i] * (o_shape[i] - 1) + 1, s[i]) for i in range(3))


def conv3d(x, w, bias=None, stride=1, pad=0, dil=1):
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    s, p, d = _triple(stride), _triple(pad), _triple(dil)
    N, Ci = x.shape[:2]
    Co, Ci2, kd, kh, kw = w.shape
    assert Ci == Ci2
    o = tuple(out_size(x.shape[2 + i], w.shape[2 + i], s[i], p[i], d[i]) for i in range(3))
    xp = _pad(x, p)
    y = np.zeros((N, Co) + o)
    for t in np.ndindex(kd, kh, kw):
        sl = _tap_slice(o, t, s, d)
        xs = xp[(slice(None), slice(None)) + sl]               # N, Ci, o
        y += np.einsum("ncdhw,kc->nkdhw", xs, w[(slice(None), slice(None)) + t])
    if bias is not None:
        y += np.asarray(bias, dtype=np.float64)[None, :, None, None, None]
    return y


def conv3d_bwd_data(g, w, in_shape, stride=1, pad=0, dil=1, bias=None):
    """dx = A_w^T g for a convolution with input spatial shape in_shape.
    With bias (one per input channel) this is the forward map of the
    transposed convolution."""
    g = np.asarray(g, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    s, p, d = _triple(stride), _triple(pad), _triple(dil)
    N, Co = g.shape[:2]
    _, Ci, kd, kh, kw = w.shape
    o = g.shape[2:]
    xp = np.zeros((N, Ci) + tuple(in_shape[i] + 2 * p[i] for i in range(3)))
    for t in np.ndindex(kd, kh, kw):
        sl = _tap_slice(o, t, s, d)
        xp[(slice(None), slice(None)) + sl] += np.einsum("nkdhw,kc->ncdhw", g, w[(slice(None), slice(None)) + t])
    dx = xp[:, :, p[0]:p[0] + in_shape[0], p[1]:p[1] + in_shape[1], p[2]:p[2] + in_shape[2]]
    if bias is not None:
        dx = dx + np.asarray(bias, dtype=np.float64)[None, :, None, None, None]
    return dx


def conv3d_bwd_weight(x, g, ksize, stride=1, pad=0, dil=1):
    """(dw, db) of sum(g * conv3d(x, w, b)) with respect to w and b."""
    x = np.asarray(x, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    s, p, d = _triple(stride), _triple(pad), _triple(dil)
    k = _triple(ksize)
    Ci, Co = x.shape[1], g.shape[1]
    o = g.shape[2:]
    xp = _pad(x, p)
    dw = np.zeros((Co, Ci) + k)
    for t in np.ndindex(*k):
        sl = _tap_slice(o, t, s, d)
        xs = xp[(slice(None), slice(None)) + sl]
        dw[(slice(None), slice(None)) + t] = np.einsum("nkdhw,ncdhw->kc", g, xs)
    return dw, g.sum(axis=(0, 2, 3, 4))


def leaky_relu(z, slope=0.1):
    z = np.asarray(z, dtype=np.float64)
    return np.where(z > 0, z, slope * z)


def leaky_relu_bwd(dy, y, slope=0.1):
    """dL/dz from dL/dy and the activation's output y = a(z)."""
    return np.where(np.asarray(y) > 0, dy, slope * np.asarray(dy, dtype=np.float64))


def mse(pred, target):
    """(L, dL/dpred) with L = mean((pred - target)^2)."""
    r = np.asarray(pred, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return float(np.mean(r * r)), 2.0 * r / r.size


def adam_step(theta, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Returns (theta', m', v') after step number t (t >= 1)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
