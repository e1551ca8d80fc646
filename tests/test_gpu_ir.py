"""Mixed precision: FP64 iterative refinement around the FP32 fused solver,
with fresh inner solves and with the search direction kept across
corrections (residual replacement).

Pinned: the final residual in FP64 (the library's and the oracle's own
matrix) is below 1e-10 ||b||, and every correction with fresh inner solves to
1e-4 reduces the outer residual by at least 10^3 except the last one, which
only goes as far as the target needs (an FP32 inner solve to 1e-4 can only
do that if the FP32 operator equals A to single precision; residual
replacement, which keeps the direction, corrects every 10x).  The FP32
operator itself is compared with the oracle's FP64 matrix directly.  The total FP32 iteration count
stays below 1.6x the FP64 oracle's count plus the polling granularity (16
iterations per correction).  The forward error against the FP64
oracle solution is reported and only bounded (parity unpinned for its value:
refinement follows a different iterate sequence than Algorithm 1).
"""
import numpy as np
import pytest

from paper_2205_08909_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("keep", [False, True])  # fresh inner solves to 1e-4 / residual replacement every 10x
@pytest.mark.parametrize("cells,k,seed", [((16, 16, 16), 4, 0), ((7, 6, 8), 3, 1), ((4, 4, 4), 6, 2)])
def test_ir_converges_to_fp64_tolerance(cells, k, seed, keep, oracle_mod, torch_cuda):
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    coeff = inputs.grf_coefficient(cells, 0.1, 1.0, seed=seed)
    m = oracle_mod.Mesh(cells, k, map_kind=1, amp=0.05, coeff=coeff)
    A = oracle_mod.assemble(m)
    b = oracle_mod.rhs(m)
    xo, its_o, _, rc = oracle_mod.pcg(A, A.diagonal(), b, tol=1e-12, maxit=20000)
    _, its10, _, _ = oracle_mod.pcg(A, A.diagonal(), b, tol=1e-10, maxit=20000)
    P = mfcg.Problem(cells, k, coeff=coeff, map_kind=1, amplitude=0.05)
    bt = torch.from_numpy(b).cuda()
    xt = torch.zeros_like(bt)
    itol = 1e-1 if keep else 1e-4
    code, outer, inner, hist, tr = P.solve_ir(bt, xt, tol=1e-10, inner_tol=itol, keep_direction=keep)
    assert code == 0 and tr < 1e-10 and hist[-1] < 1e-10
    # every correction but the last (which stops at what the target needs) reduces the residual
    assert np.all(hist[1:-1] <= (1e-1 if keep else 1e-3) * hist[:-2]), hist
    x = xt.cpu().numpy()
    nb = np.linalg.norm(b)
    assert np.linalg.norm(b - A.matvec(x)) <= 2e-10 * nb
    ferr = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    print(f"IR (keep direction {keep}): outer {outer}, inner {inner} (FP64 oracle {its10}), true rel res {tr:.2e}, "
          f"forward error vs oracle {ferr:.2e}")
    assert ferr < 1e-6
    assert inner <= 1.6 * its10 + 16 * outer
    P.close()


def test_ir_edge_cases(torch_cuda):
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    P = mfcg.Problem((3, 3, 3), 2, map_kind=1, amplitude=0.05)
    z = torch.zeros(P.n, dtype=torch.float64, device="cuda")
    x = torch.ones_like(z)
    code, outer, inner, hist, tr = P.solve_ir(z, x)
    assert code == 0 and outer == 0 and torch.count_nonzero(x).item() == 0
    b = torch.from_numpy(inputs.random_rhs((3, 3, 3), 2, seed=1)).cuda()
    for bad in (dict(inner_tol=1.5), dict(tol=0.0), dict(max_outer=0)):
        code, *_ = P.solve_ir(b, x, raise_on=False, **bad)
        assert code == mfcg.EINVAL
    code, outer, inner, hist, tr = P.solve_ir(b, x, tol=1e-10, max_outer=1, raise_on=False)
    assert code == mfcg.ENOTCONV and outer == 1
    P.close()


# componentwise FP32 bound: c * 2^-24 * (|A| |u|)_i.  The sum-factorised
# product S^T D^T G D S (contractions of k+1 terms and the 3-term tensor
# apply, each rounded in FP32, plus G_q rounded to FP32) errs by a few tens of
# roundings of the terms' absolute sums, which exceed |A| |u| only by the
# cancellation inside the element matrices; measured on MI355X: at most 7.5
# (k = 2..6, curved map, random-field coefficient), so c = 2^5 leaves a
# factor 4; normwise 2.2e-7 relative, bound 2^-20
@pytest.mark.parametrize("cells,k,seed", [((5, 4, 6), 4, 3), ((8, 8, 8), 2, 4), ((3, 4, 3), 6, 5), ((9, 7, 8), 3, 6)])
def test_fp32_operator_matches_oracle(cells, k, seed, oracle_mod, torch_cuda):
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    coeff = inputs.grf_coefficient(cells, 0.1, 1.0, seed=seed)
    m = oracle_mod.Mesh(cells, k, map_kind=1, amp=0.05, coeff=coeff)
    A = oracle_mod.assemble(m)
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(A.n)
    u32 = u.astype(np.float32).astype(np.float64)  # the FP32 operator sees src rounded to FP32
    ref = A.matvec(u32)
    scale = A.abs_matvec(u32)
    P = mfcg.Problem(cells, k, coeff=coeff, map_kind=1, amplitude=0.05)
    out = torch.empty(P.n, dtype=torch.float64, device="cuda")
    P.vmult_fp32(out, torch.from_numpy(u).cuda())
    got = out.cpu().numpy()
    ratio = np.abs(got - ref) / (2.0 ** -24 * scale)
    print(f"FP32 operator: max |A32 u - A u| / (2^-24 |A||u|) = {ratio.max():.1f}, "
          f"normwise {np.linalg.norm(got - ref) / np.linalg.norm(ref):.2e}")
    assert np.all(np.isfinite(got))
    assert ratio.max() <= 2.0 ** 5
    assert np.linalg.norm(got - ref) <= 2.0 ** -20 * np.linalg.norm(ref)
    # it is not the FP64 operator: the difference is of FP32 size somewhere
    out64 = torch.empty_like(out)
    P.vmult(out64, torch.from_numpy(u32).cuda())
    assert np.abs(got - out64.cpu().numpy()).max() > 2.0 ** -40 * scale.max()
    P.close()
