"""ctypes binding of the warm-start network kernels (include/mfnn.h).

Argument marshalling only: every operation runs in the library's HIP
kernels.  Tensors are torch device tensors (bfloat16, float32 or float64),
contiguous, NCDHW.
"""
import ctypes

from . import mfcg

OK, EINVAL, EHIP = 0, -1, -3
BF16, F32, F64 = 0, 1, 2
ACT_NONE, ACT_LEAKY = 0, 1
LEAKY_SLOPE = 0.1
NOALLOC_WORK_FLOATS = 1 << 20   # workspace of mfnn_conv3d_bwd_weight_noalloc (floats per GPU)

EXPORTED = [
    "mfnn_conv3d_fwd", "mfnn_conv3d_bwd_data", "mfnn_conv3d_bwd_weight", "mfnn_conv3d_bwd_weight_work",
    "mfnn_conv3d_bwd_weight_noalloc", "mfnn_mse_loss", "mfnn_adam_step",
    "mfnn_act_bwd", "mfnn_mse", "mfnn_adam", "mfnn_convert", "mfnn_features", "mfnn_channel_sum",
    "mfnn_channel_sum_work",
    "mfnn_normalize", "mfnn_last_error",
]


class NnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mfnn error {code}: {msg}")
        self.code = code


class ConvDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("c_in", ctypes.c_int32), ("c_out", ctypes.c_int32),
                ("inp", ctypes.c_int32 * 3), ("out", ctypes.c_int32 * 3), ("k", ctypes.c_int32 * 3),
                ("stride", ctypes.c_int32 * 3), ("pad", ctypes.c_int32 * 3), ("dil", ctypes.c_int32 * 3)]


def out_size(n_in, k, s, p, d):
    return (n_in + 2 * p - d * (k - 1) - 1) // s + 1


def desc(n, c_in, c_out, inp, k, stride=1, pad=0, dil=1):
    """Descriptor with the output size derived from the input size."""
    t = lambda v: tuple(v) if hasattr(v, "__len__") else (int(v),) * 3
    inp, k, stride, pad, dil = t(inp), t(k), t(stride), t(pad), t(dil)
    d = ConvDesc()
    d.n, d.c_in, d.c_out = int(n), int(c_in), int(c_out)
    for i in range(3):
        d.inp[i], d.k[i], d.stride[i], d.pad[i], d.dil[i] = inp[i], k[i], stride[i], pad[i], dil[i]
        d.out[i] = out_size(inp[i], k[i], stride[i], pad[i], dil[i])
    return d


def with_batch(d, n):
    e = ConvDesc.from_buffer_copy(d)
    e.n = int(n)
    return e


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = mfcg.lib()
        P, I32, I64, F, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double
        DP = ctypes.POINTER(ConvDesc)
        L.mfnn_conv3d_fwd.argtypes = [DP, P, I32, P, P, I32, P, I32, P]
        L.mfnn_conv3d_bwd_data.argtypes = [DP, P, I32, P, P, P, I32, P]
        L.mfnn_conv3d_bwd_weight.argtypes = [DP, P, I32, P, I32, P, P, P, I64, P]
        L.mfnn_conv3d_bwd_weight_work.argtypes = [DP]
        L.mfnn_conv3d_bwd_weight_work.restype = I64
        L.mfnn_conv3d_bwd_weight_noalloc.argtypes = [DP, P, I32, P, I32, P, P, P]
        L.mfnn_act_bwd.argtypes = [I64, P, P, I32, I32, P, P]
        L.mfnn_mse.argtypes = [I64, P, P, P, P, P, P]
        L.mfnn_adam.argtypes = [I64, P, P, P, P, P, I32, F, F, F, F, P]
        L.mfnn_adam_step.argtypes = L.mfnn_adam.argtypes
        L.mfnn_mse_loss.argtypes = L.mfnn_mse.argtypes
        L.mfnn_convert.argtypes = [I64, P, I32, P, I32, P]
        L.mfnn_features.argtypes = [ctypes.POINTER(I32), I32, P, P, P, P, P, P]
        L.mfnn_channel_sum.argtypes = [I32, I32, ctypes.POINTER(I32), P, I32, P, P]
        L.mfnn_channel_sum_work.argtypes = [I32, I32, ctypes.POINTER(I32), P, I32, P, P, I64, P]
        L.mfnn_normalize.argtypes = [I64, P, P, P, P]
        L.mfnn_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(code):
    if code != OK:
        raise NnError(code, lib().mfnn_last_error().decode())


def _dt(t):
    import torch
    m = {torch.bfloat16: BF16, torch.float32: F32, torch.float64: F64}
    if t.dtype not in m or not t.is_cuda or not t.is_contiguous():
        raise ValueError("tensors must be contiguous bfloat16/float32/float64 device tensors")
    return m[t.dtype]


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _s(stream=None):
    return mfcg._stream(stream)


def _need(t, numel, name):
    if t.numel() != numel:
        raise ValueError(f"{name}: {t.numel()} elements, expected {numel}")


def _sizes(d):
    iv = d.inp[0] * d.inp[1] * d.inp[2]
    ov = d.out[0] * d.out[1] * d.out[2]
    kk = d.k[0] * d.k[1] * d.k[2]
    return iv, ov, kk


def conv_fwd(d, x, w, bias, act, y, stream=None):
    iv, ov, kk = _sizes(d)
    _need(x, d.n * d.c_in * iv, "x")
    _need(w, d.c_out * d.c_in * kk, "w")
    _need(y, d.n * d.c_out * ov, "y")
    if bias is not None:
        _need(bias, d.c_out, "bias")
    _check(lib().mfnn_conv3d_fwd(ctypes.byref(d), _p(x), _dt(x), _p(w), _p(bias), int(act), _p(y), _dt(y), _s(stream)))
    return y


def conv_bwd_data(d, g, w, bias_in, dx, stream=None):
    iv, ov, kk = _sizes(d)
    _need(g, d.n * d.c_out * ov, "g")
    _need(w, d.c_out * d.c_in * kk, "w")
    _need(dx, d.n * d.c_in * iv, "dx")
    if bias_in is not None:
        _need(bias_in, d.c_in, "bias_in")
    _check(lib().mfnn_conv3d_bwd_data(ctypes.byref(d), _p(g), _dt(g), _p(w), _p(bias_in), _p(dx), _dt(dx), _s(stream)))
    return dx


def wgrad_work(d):
    return int(lib().mfnn_conv3d_bwd_weight_work(ctypes.byref(d)))


def conv_bwd_weight(d, x, g, dw, db, work, stream=None):
    iv, ov, kk = _sizes(d)
    _need(x, d.n * d.c_in * iv, "x")
    _need(g, d.n * d.c_out * ov, "g")
    _need(dw, d.c_out * d.c_in * kk, "dw")
    if db is not None:
        _need(db, d.c_out, "db")
    _check(lib().mfnn_conv3d_bwd_weight(ctypes.byref(d), _p(x), _dt(x), _p(g), _dt(g), _p(dw), _p(db), _p(work),
                                        int(work.numel()), _s(stream)))
    return dw


def conv_bwd_weight_noalloc(d, x, g, dw, db, stream=None):
    """conv_bwd_weight with the library's own per-GPU workspace (no caller buffer)."""
    iv, ov, kk = _sizes(d)
    _need(x, d.n * d.c_in * iv, "x")
    _need(g, d.n * d.c_out * ov, "g")
    _need(dw, d.c_out * d.c_in * kk, "dw")
    if db is not None:
        _need(db, d.c_out, "db")
    _check(lib().mfnn_conv3d_bwd_weight_noalloc(ctypes.byref(d), _p(x), _dt(x), _p(g), _dt(g), _p(dw), _p(db),
                                                _s(stream)))
    return dw


def act_bwd(dy, y, dz, stream=None):
    _need(y, dy.numel(), "y")
    _need(dz, dy.numel(), "dz")
    _check(lib().mfnn_act_bwd(int(dy.numel()), _p(dy), _p(y), _dt(y), ACT_LEAKY, _p(dz), _s(stream)))
    return dz


def mse(pred, target, grad, loss, work, stream=None):
    _need(target, pred.numel(), "target")
    _need(grad, pred.numel(), "grad")
    _check(lib().mfnn_mse(int(pred.numel()), _p(pred), _p(target), _p(grad), _p(loss), _p(work), _s(stream)))


def adam(theta, theta_bf16, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    n = theta.numel()
    for t, name in ((g, "g"), (m, "m"), (v, "v")):
        _need(t, n, name)
    if theta_bf16 is not None:
        _need(theta_bf16, n, "theta_bf16")
    _check(lib().mfnn_adam(int(n), _p(theta), _p(theta_bf16), _p(g), _p(m), _p(v), int(step), float(lr),
                           float(beta1), float(beta2), float(eps), _s(stream)))


def convert(src, dst, stream=None):
    _need(dst, src.numel(), "dst")
    _check(lib().mfnn_convert(int(src.numel()), _p(src), _dt(src), _p(dst), _dt(dst), _s(stream)))
    return dst


def features(cells, k, log_coeff, b, diag, work, out, stream=None):
    c = (ctypes.c_int32 * 3)(*[int(v) for v in cells])
    n = 1
    for v in cells:
        n *= int(v) * int(k) + 1
    _need(b, n, "b")
    _need(diag, n, "diag")
    _need(out, 3 * n, "out")
    _need(log_coeff, int(cells[0]) * int(cells[1]) * int(cells[2]), "log_coeff")
    _check(lib().mfnn_features(c, int(k), _p(log_coeff), _p(b), _p(diag), _p(work), _p(out), _s(stream)))
    return out


def channel_sum(n, c, spatial, g, out, work=None, stream=None):
    """Per-channel sum over samples and points; with work (a float32 device
    tensor) spread over many blocks per channel."""
    sp = (ctypes.c_int32 * 3)(*[int(v) for v in spatial])
    _need(g, n * c * int(spatial[0]) * int(spatial[1]) * int(spatial[2]), "g")
    _need(out, c, "out")
    if work is None:
        _check(lib().mfnn_channel_sum(int(n), int(c), sp, _p(g), _dt(g), _p(out), _s(stream)))
    else:
        _check(lib().mfnn_channel_sum_work(int(n), int(c), sp, _p(g), _dt(g), _p(out), _p(work), int(work.numel()),
                                           _s(stream)))
    return out


def normalize(src, work, out, stream=None):
    _need(out, src.numel(), "out")
    _check(lib().mfnn_normalize(int(src.numel()), _p(src), _p(work), _p(out), _s(stream)))
    return out
