"""GPU parity of the warm-start network kernels (include/mfnn.h) against the
FP64 oracle (oracle/conv_oracle.py) on BF16-representable inputs.

Tolerance: the kernels accumulate in FP32, so each output may differ from
the exact value by a few FP32 roundings of the sum of absolute terms:
|y - y_ref| <= 1e-5 * (|w| * |x|) componentwise (the oracle applied to the
absolute values), plus BF16 rounding (2^-8 relative) where the output is
stored in BF16.
"""
import numpy as np
import pytest

from oracle import conv_oracle as co

pytestmark = pytest.mark.gpu

GEOMS = [  # (n, c_in, c_out, in spatial, k, stride, pad, dil)
    (2, 3, 32, (13, 12, 11), 4, 4, 2, 1),   # layer 1 shape, ragged
    (1, 32, 32, (7, 6, 5), 3, 1, 1, 1),     # layer 2
    (2, 32, 32, (9, 8, 7), 3, 1, 3, 3),     # layer 3 (dilated)
    (1, 1, 32, (17, 13, 9), 8, 4, 4, 1),    # layer 4 geometry (fine -> coarse conv)
    (2, 3, 5, (6, 7, 5), 3, 2, 1, 1),       # channel counts not multiple of 8
    # 32 -> 32 channels at stride 1 run on the matrix cores (BF16 inputs):
    # several 128-point blocks per plane with a ragged last one, rows that
    # a block spans partly, a dilated kernel
    (2, 32, 32, (5, 19, 37), 3, 1, 3, 3),
    (1, 32, 32, (3, 2, 130), 3, 1, 1, 1),
]


def bf16_round(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _rand(rng, shape, scale=1.0):
    return bf16_round(rng.standard_normal(shape) * scale)


def _dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dtype).cuda().reshape(-1)


def _host(t, shape):
    return t.to(dtype=__import__("torch").float64).cpu().numpy().reshape(shape)


def _desc(n, ci, cout, sp, k, s, p, d):
    from paper_2205_08909_amd import nn
    return nn.desc(n, ci, cout, sp, k, s, p, d)


@pytest.mark.parametrize("geom", GEOMS)
@pytest.mark.parametrize("xdt,ydt,act", [("bf16", "f32", 0), ("bf16", "bf16", 1), ("f32", "f32", 1)])
def test_conv_forward(geom, xdt, ydt, act):
    import torch
    from paper_2205_08909_amd import nn
    n, ci, cout, sp, k, s, p, d = geom
    rng = np.random.default_rng(11)
    x = _rand(rng, (n, ci) + sp)
    w = _rand(rng, (cout, ci, k, k, k), 0.2)
    b = rng.standard_normal(cout).astype(np.float32).astype(np.float64)
    D = _desc(*geom)
    tt = {"bf16": torch.bfloat16, "f32": torch.float32}
    y = torch.empty(n * cout * int(np.prod(tuple(D.out))), dtype=tt[ydt], device="cuda")
    nn.conv_fwd(D, _dev(x, tt[xdt]), _dev(w, torch.bfloat16), _dev(b, torch.float32), act, y)
    ref = co.conv3d(x, w, b, s, p, d)
    scale = co.conv3d(np.abs(x), np.abs(w), np.abs(b), s, p, d)
    if act:
        ref = co.leaky_relu(ref)
    got = _host(y, ref.shape)
    tol = 1e-5 * scale + 1e-30
    if ydt == "bf16":
        tol = tol + 2.0 ** -8 * np.abs(ref)
    assert np.all(np.abs(got - ref) <= tol), np.max(np.abs(got - ref) / tol)


@pytest.mark.parametrize("geom", GEOMS)
@pytest.mark.parametrize("gdt,bias", [("f32", False), ("bf16", True), ("bf16", False)])
def test_conv_backward_data(geom, gdt, bias):
    import torch
    from paper_2205_08909_amd import nn
    n, ci, cout, sp, k, s, p, d = geom
    D = _desc(*geom)
    out = tuple(D.out)
    rng = np.random.default_rng(12)
    g = _rand(rng, (n, cout) + out)
    w = _rand(rng, (cout, ci, k, k, k), 0.2)
    bi = rng.standard_normal(ci).astype(np.float32).astype(np.float64) if bias else None
    tt = {"bf16": torch.bfloat16, "f32": torch.float32}
    dx = torch.empty(n * ci * int(np.prod(sp)), dtype=torch.float32, device="cuda")
    nn.conv_bwd_data(D, _dev(g, tt[gdt]), _dev(w, torch.bfloat16), _dev(bi, torch.float32) if bias else None, dx)
    ref = co.conv3d_bwd_data(g, w, sp, s, p, d, bias=bi)
    scale = co.conv3d_bwd_data(np.abs(g), np.abs(w), sp, s, p, d, bias=np.abs(bi) if bias else None)
    got = _host(dx, ref.shape)
    assert np.all(np.abs(got - ref) <= 1e-5 * scale + 1e-30)


@pytest.mark.parametrize("geom", GEOMS)
@pytest.mark.parametrize("xdt,gdt", [("bf16", "f32"), ("f32", "bf16"), ("bf16", "bf16")])
def test_conv_backward_weight(geom, xdt, gdt):
    import torch
    from paper_2205_08909_amd import nn
    n, ci, cout, sp, k, s, p, d = geom
    D = _desc(*geom)
    out = tuple(D.out)
    rng = np.random.default_rng(13)
    x = _rand(rng, (n, ci) + sp)
    g = _rand(rng, (n, cout) + out)
    tt = {"bf16": torch.bfloat16, "f32": torch.float32}
    dw = torch.empty(cout * ci * k ** 3, dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    work = torch.empty(nn.wgrad_work(D), dtype=torch.float32, device="cuda")
    nn.conv_bwd_weight(D, _dev(x, tt[xdt]), _dev(g, tt[gdt]), dw, db, work)
    rw, rb = co.conv3d_bwd_weight(x, g, k, s, p, d)
    sw, sb = co.conv3d_bwd_weight(np.abs(x), np.abs(g), k, s, p, d)
    assert np.all(np.abs(_host(dw, rw.shape) - rw) <= 1e-5 * sw + 1e-30)
    assert np.all(np.abs(_host(db, rb.shape) - rb) <= 1e-5 * sb + 1e-30)
    # channel sum = the bias gradient
    cs = torch.empty(cout, dtype=torch.float32, device="cuda")
    nn.channel_sum(n, cout, out, _dev(g, tt[gdt]), cs)
    assert np.all(np.abs(_host(cs, rb.shape) - rb) <= 1e-5 * sb + 1e-30)
    # and spread over many blocks per channel with a workspace
    cw = torch.empty(cout, dtype=torch.float32, device="cuda")
    nn.channel_sum(n, cout, out, _dev(g, tt[gdt]), cw, work=torch.empty(4096, dtype=torch.float32, device="cuda"))
    assert np.all(np.abs(_host(cw, rb.shape) - rb) <= 1e-5 * sb + 1e-30)


def test_special_cases_on_gpu():
    """Identity filter reproduces the input exactly; a constant input gives
    the weight sums (bias included) away from the padding."""
    import torch
    from paper_2205_08909_amd import nn
    rng = np.random.default_rng(14)
    x = _rand(rng, (1, 8, 6, 7, 5))
    w = np.zeros((8, 8, 3, 3, 3))
    for c in range(8):
        w[c, c, 1, 1, 1] = 1.0
    D = _desc(1, 8, 8, (6, 7, 5), 3, 1, 2, 2)
    y = torch.empty(8 * 6 * 7 * 5, dtype=torch.float32, device="cuda")
    nn.conv_fwd(D, _dev(x, torch.bfloat16), _dev(w, torch.bfloat16), None, 0, y)
    assert np.array_equal(_host(y, x.shape), x)
    w = _rand(rng, (8, 2, 3, 3, 3), 0.3)
    b = bf16_round(rng.standard_normal(8))
    xc = np.full((1, 2, 9, 9, 9), 1.5)
    D = _desc(1, 2, 8, (9, 9, 9), 3, 1, 2, 2)
    y = torch.empty(8 * 9 ** 3, dtype=torch.float32, device="cuda")
    nn.conv_fwd(D, _dev(xc, torch.bfloat16), _dev(w, torch.bfloat16), _dev(b, torch.float32), 0, y)
    inner = _host(y, (1, 8, 9, 9, 9))[0, :, 2:-2, 2:-2, 2:-2]
    expect = b + 1.5 * w.sum(axis=(1, 2, 3, 4))
    assert np.allclose(inner, expect[:, None, None, None], rtol=1e-5, atol=1e-5)


def test_elementwise_kernels():
    import torch
    from paper_2205_08909_amd import nn
    rng = np.random.default_rng(15)
    n = 100_003
    dy = rng.standard_normal(n).astype(np.float32)
    y = bf16_round(rng.standard_normal(n))
    dz = torch.empty(n, dtype=torch.float32, device="cuda")
    nn.act_bwd(_dev(dy, torch.float32), _dev(y, torch.bfloat16), dz)
    # the kernel multiplies by the FP32 slope 0.1f: one FP32 rounding from the FP64 value
    assert np.allclose(dz.cpu().numpy(), co.leaky_relu_bwd(dy, y), rtol=2e-7, atol=0)
    # MSE
    pr, tg = rng.standard_normal(n).astype(np.float32), rng.standard_normal(n).astype(np.float32)
    grad = torch.empty(n, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    work = torch.empty(1024, dtype=torch.float64, device="cuda")
    nn.mse(_dev(pr, torch.float32), _dev(tg, torch.float32), grad, loss, work)
    L, g = co.mse(pr, tg)
    assert abs(loss.item() - L) <= 1e-6 * L
    assert np.allclose(grad.cpu().numpy(), g, rtol=1e-6, atol=1e-12)
    # Adam, three steps against the FP64 definition
    th = rng.standard_normal(n).astype(np.float32)
    gr = rng.standard_normal(n).astype(np.float32)
    tht, thb = _dev(th, torch.float32), torch.empty(n, dtype=torch.bfloat16, device="cuda")
    m, v = torch.zeros(n, dtype=torch.float32, device="cuda"), torch.zeros(n, dtype=torch.float32, device="cuda")
    rth, rm, rv = th.astype(np.float64), np.zeros(n), np.zeros(n)
    for t in (1, 2, 3):
        nn.adam(tht, thb, _dev(gr * t, torch.float32), m, v, t, 1e-2)
        rth, rm, rv = co.adam_step(rth, (gr * t).astype(np.float64), rm, rv, t, lr=1e-2)
    assert np.allclose(tht.cpu().numpy(), rth, rtol=0, atol=1e-5)
    assert torch.equal(thb.cpu(), tht.cpu().to(torch.bfloat16))
    # conversions: FP32 -> BF16 rounds to nearest even like torch's cast
    a = rng.standard_normal(n).astype(np.float32) * 1e3
    ab = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    nn.convert(_dev(a, torch.float32), ab)
    assert torch.equal(ab.cpu(), torch.from_numpy(a).to(torch.bfloat16))
    a64 = torch.empty(n, dtype=torch.float64, device="cuda")
    nn.convert(ab, a64)
    assert torch.equal(a64.cpu(), torch.from_numpy(a).to(torch.bfloat16).to(torch.float64))
    # normalisation of a solver vector
    u = rng.standard_normal(n) * 3.0
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    nn.normalize(torch.from_numpy(u).cuda(), work, out)
    assert np.allclose(out.cpu().numpy(), u / np.sqrt(np.mean(u * u)), rtol=1e-6)


def test_features():
    import torch
    from paper_2205_08909_amd import nn
    cells, k = (5, 4, 3), 3
    rng = np.random.default_rng(16)
    L = [c * k + 1 for c in cells]
    n = L[0] * L[1] * L[2]
    logc = rng.standard_normal(cells[0] * cells[1] * cells[2])
    b = rng.standard_normal(n)
    diag = rng.uniform(0.5, 2.0, n)
    out = torch.empty(3 * n, dtype=torch.bfloat16, device="cuda")
    work = torch.empty(2048, dtype=torch.float64, device="cuda")
    nn.features(cells, k, torch.from_numpy(logc).cuda(), torch.from_numpy(b).cuda(), torch.from_numpy(diag).cuda(),
                work, out)
    got = out.float().cpu().numpy().reshape(3, n)
    # channel 0 by brute force: average over all cells whose closure contains the node
    lc = logc.reshape(cells[2], cells[1], cells[0])
    ref0 = np.zeros((L[2], L[1], L[0]))
    for z in range(L[2]):
        for y in range(L[1]):
            for x in range(L[0]):
                vals = [lc[cz, cy, cx] for cz in range(cells[2]) for cy in range(cells[1]) for cx in range(cells[0])
                        if cx * k <= x <= (cx + 1) * k and cy * k <= y <= (cy + 1) * k and cz * k <= z <= (cz + 1) * k]
                ref0[z, y, x] = np.mean(vals)
    ref = [ref0.ravel(), b / np.sqrt(np.mean(b * b)), (b / diag) / np.sqrt(np.mean((b / diag) ** 2))]
    for c in range(3):
        assert np.allclose(got[c], ref[c], rtol=2 ** -8, atol=1e-6), c


def test_conv_matrix_core_5x5x5():
    """The matrix-core path with a 5^3 kernel (BF16 operands only: its
    direct-convolution weights would not fit the LDS budget)."""
    import torch
    from paper_2205_08909_amd import nn
    geom = (1, 32, 32, (5, 6, 8), 5, 1, 2, 1)
    n, ci, cout, sp, k, s, p, d = geom
    rng = np.random.default_rng(14)
    D = _desc(*geom)
    x = _rand(rng, (n, ci) + sp)
    w = _rand(rng, (cout, ci, k, k, k), 0.2)
    y = torch.empty(n * cout * int(np.prod(tuple(D.out))), dtype=torch.float32, device="cuda")
    nn.conv_fwd(D, _dev(x, torch.bfloat16), _dev(w, torch.bfloat16), None, 0, y)
    ref = co.conv3d(x, w, None, s, p, d)
    scale = co.conv3d(np.abs(x), np.abs(w), None, s, p, d)
    assert np.all(np.abs(_host(y, ref.shape) - ref) <= 1e-5 * scale + 1e-30)
    g = _rand(rng, (n, cout) + tuple(D.out))
    dx = torch.empty(n * ci * int(np.prod(sp)), dtype=torch.float32, device="cuda")
    nn.conv_bwd_data(D, _dev(g, torch.bfloat16), _dev(w, torch.bfloat16), None, dx)
    ref = co.conv3d_bwd_data(g, w, sp, s, p, d)
    scale = co.conv3d_bwd_data(np.abs(g), np.abs(w), sp, s, p, d)
    assert np.all(np.abs(_host(dx, ref.shape) - ref) <= 1e-5 * scale + 1e-30)
