"""The allocation-free weight-gradient entry point
(mfnn_conv3d_bwd_weight_noalloc) against mfnn_conv3d_bwd_weight on the same
inputs, through the C ABI: two calls in a row on the library's per-GPU
workspace, the second on a smaller layer, each bitwise equal to the entry
point with a caller workspace (same kernels, same fixed summation order)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case(rng, n, ci, co, inp, k, s, p, dil):
    import torch
    from paper_2205_08909_amd import nn
    d = nn.desc(n, ci, co, inp, k, s, p, dil)
    iv, ov, kk = nn._sizes(d)
    x = torch.from_numpy(rng.standard_normal(n * ci * iv).astype(np.float32)).to(torch.bfloat16).cuda()
    g = torch.from_numpy(rng.standard_normal(n * co * ov).astype(np.float32)).cuda()
    return d, x, g, kk


def test_noalloc_matches_workspace_entry_point_twice():
    import torch
    from paper_2205_08909_amd import nn
    rng = np.random.default_rng(20261203)
    L = nn.lib()
    cases = [(2, 32, 32, (19, 17, 15), 3, 1, 1, 1),   # the larger layer first
             (1, 3, 8, (9, 7, 6), 3, 2, 1, 1)]        # then a smaller one on the same workspace
    for args in cases:
        print("noalloc case", args, flush=True)
        d, x, g, kk = _case(rng, *args)
        need = L.mfnn_conv3d_bwd_weight_work(ctypes.byref(d))
        assert 0 < need <= nn.NOALLOC_WORK_FLOATS
        work = torch.empty(need, dtype=torch.float32, device="cuda")
        dw_ref = torch.empty(d.c_out * d.c_in * kk, dtype=torch.float32, device="cuda")
        db_ref = torch.empty(d.c_out, dtype=torch.float32, device="cuda")
        nn.conv_bwd_weight(d, x, g, dw_ref, db_ref, work)
        dw = torch.full_like(dw_ref, float("nan"))
        db = torch.full_like(db_ref, float("nan"))
        nn.conv_bwd_weight_noalloc(d, x, g, dw, db)
        torch.cuda.synchronize()
        assert torch.equal(dw, dw_ref), args
        assert torch.equal(db, db_ref), args
        assert torch.isfinite(dw).all()
