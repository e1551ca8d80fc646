"""Many right-hand sides on one operator (mfcg_solve_multi) against single
solves and against the oracle.

Every right-hand side runs Algorithm 5 with its own scalars: its tiles,
shared-node blocks and finish block compute exactly what the scalar solve
computes, in the same order, so each x_c, its iteration count and status
must equal the scalar solve's bitwise, also when the right-hand sides stop
at different iterations (warm starts close to the solution, a zero
right-hand side, the iteration limit).  One case is also checked against the
oracle's Algorithm 1 (iterations within its summation-order range +-2,
x within 1e-10 relative).
"""
import numpy as np
import pytest

from paper_2205_08909_amd import inputs
from tests.test_gpu_solve import _problem, oracle_noise, torch_cuda  # noqa: F401

pytestmark = pytest.mark.gpu


def _singles(torch, P, bs, x0s, tol, maxit):
    out = []
    for b, x0 in zip(bs, x0s):
        x = x0.clone()
        code, its, _, _ = P.solve(b, x, tol=tol, maxit=maxit, want_hist=False, raise_on=False)
        out.append((code, its, x))
    return out


@pytest.mark.parametrize("cells,k,coeff_seed,tile,m", [
    ((6, 7, 5), 3, 4, (2, 3, 2), 3),     # ragged tiles
    ((8, 8, 8), 2, None, None, 5),
    ((4, 4, 4), 5, 2, (2, 2, 2), 2),
    ((3, 2, 3), 7, 1, (2, 1, 2), 1),
])
def test_multi_equals_single_solves(cells, k, coeff_seed, tile, m, oracle_mod, torch_cuda):
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    _, A, P = _problem(oracle_mod, cells, k, 1, 0.05, coeff_seed, tile)
    print("case", cells, k, tile, "m", m, flush=True)
    bs = [torch.from_numpy(inputs.random_rhs(cells, k, seed=40 + c)).cuda() for c in range(m)]
    x0s = [torch.zeros_like(bs[0]) for _ in range(m)]
    if m > 1:
        # a warm start near the solution: this right-hand side stops early
        xs1 = x0s[1].clone()
        P.solve(bs[1], xs1, tol=1e-6, maxit=5000, want_hist=False)
        x0s[1] = xs1
    ref = _singles(torch, P, bs, x0s, 1e-10, 5000)
    xs = [x.clone() for x in x0s]
    code, its, status, tr = P.solve_multi(bs, xs, tol=1e-10, maxit=5000, want_true_res=True)
    print("multi its", its, "single", [r[1] for r in ref], "true res", tr)
    assert code == mfcg.OK and all(s == mfcg.OK for s in status)
    for c in range(m):
        assert its[c] == ref[c][1]
        assert torch.equal(xs[c], ref[c][2]), f"rhs {c}"
        assert tr[c] <= 2e-10
    if m > 1:
        assert its[1] < its[0]


def test_multi_matches_oracle(oracle_mod, torch_cuda):
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    cells, k = (6, 5, 7), 4
    _, A, P = _problem(oracle_mod, cells, k, 1, 0.05, 3, (3, 2, 3))
    bn = [inputs.random_rhs(cells, k, seed=60 + c) for c in range(3)]
    bs = [torch.from_numpy(b).cuda() for b in bn]
    xs = [torch.zeros_like(bs[0]) for _ in range(3)]
    code, its, status, _ = P.solve_multi(bs, xs, tol=1e-10, maxit=5000)
    assert code == mfcg.OK
    d = A.diagonal()
    for c in range(3):
        xo, its_o, _, rc_o = oracle_mod.pcg(A, d, bn[c], tol=1e-10, maxit=5000)
        lo, hi, _ = oracle_noise(oracle_mod, A, bn[c], nperm=2)
        x = xs[c].cpu().numpy()
        print("rhs", c, "its", its[c], "oracle", its_o, (lo, hi))
        assert rc_o == 0 and lo - 2 <= its[c] <= hi + 2
        assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo)


@pytest.mark.parametrize("maxit", [1, 2, 5])
def test_multi_zero_rhs_and_iteration_limit(maxit, oracle_mod, torch_cuda):
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    cells, k = (5, 4, 6), 3
    _, A, P = _problem(oracle_mod, cells, k, 1, 0.05, 2, (3, 2, 3))
    bs = [torch.from_numpy(inputs.random_rhs(cells, k, seed=70 + c)).cuda() for c in range(3)]
    bs[1].zero_()
    x0s = [torch.zeros_like(bs[0]) for _ in range(3)]
    x0s[2] = torch.from_numpy(inputs.random_rhs(cells, k, seed=79)).cuda() * 1e-3
    x0s[1].fill_(7.0)        # ignored for a zero right-hand side: x = 0
    ref = _singles(torch, P, bs, x0s, 1e-12, maxit)
    xs = [x.clone() for x in x0s]
    code, its, status, _ = P.solve_multi(bs, xs, tol=1e-12, maxit=maxit)
    print("maxit", maxit, "its", its, "status", status, "single", [(r[0], r[1]) for r in ref])
    assert code == mfcg.ENOTCONV
    assert status == [mfcg.ENOTCONV, mfcg.OK, mfcg.ENOTCONV]
    assert its == [maxit, 0, maxit]
    assert float(xs[1].abs().max()) == 0.0
    for c in (0, 2):
        assert ref[c][0] == mfcg.ENOTCONV and ref[c][1] == maxit
        assert torch.equal(xs[c], ref[c][2]), f"rhs {c}"


def test_multi_reuses_buffers_and_rejects_bad_m(oracle_mod, torch_cuda):
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    cells, k = (4, 4, 4), 2
    _, A, P = _problem(oracle_mod, cells, k, 1, 0.05, None, None)
    bs = [torch.from_numpy(inputs.random_rhs(cells, k, seed=80 + c)).cuda() for c in range(4)]
    first = [torch.zeros_like(bs[0]) for _ in range(4)]
    P.solve_multi(bs, first, tol=1e-10, maxit=500)
    # a smaller m on the same handle, then the scalar solve, give the same x
    again = [torch.zeros_like(bs[0]) for _ in range(2)]
    P.solve_multi(bs[2:], again, tol=1e-10, maxit=500)
    assert torch.equal(again[0], first[2]) and torch.equal(again[1], first[3])
    x = torch.zeros_like(bs[0])
    P.solve(bs[0], x, tol=1e-10, maxit=500)
    assert torch.equal(x, first[0])
    with pytest.raises(ValueError):
        P.solve_multi([], [], tol=1e-10)
    many = [bs[0]] * (mfcg.MULTI_MAX + 1)
    with pytest.raises(ValueError):
        P.solve_multi(many, [torch.zeros_like(bs[0]) for _ in many], tol=1e-10)


def test_multi_fullsize_equals_single_solves(torch_cuda):
    """At the benchmark's size (Q4, 64^3 curved cells, default tiles), m = 3
    right-hand sides for a few iterations in the launch configuration the
    benchmark times: each equals its single solve bitwise (the operator and
    the solve at this size are pinned against the oracle by the full-size
    tests)."""
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    P = mfcg.Problem(64, 4, map_kind=mfcg.MAP_SINE_SHEAR, amplitude=0.05)
    bs = [torch.from_numpy(inputs.random_rhs(64, 4, seed=90 + c)).cuda() for c in range(3)]
    for maxit in (3, 4):
        ref = _singles(torch, P, bs, [torch.zeros_like(bs[0]) for _ in bs], 1e-12, maxit)
        xs = [torch.zeros_like(bs[0]) for _ in bs]
        code, its, status, _ = P.solve_multi(bs, xs, tol=1e-12, maxit=maxit)
        assert code == mfcg.ENOTCONV and its == [maxit] * 3
        for c in range(3):
            assert torch.equal(xs[c], ref[c][2]), f"rhs {c} maxit {maxit}"
    P.close()


def test_multi_failed_history_allocation_leaves_handle_usable(oracle_mod, torch_cuda):
    """A residual history that cannot be allocated (64 right-hand sides x
    2^31 entries, 1 TiB) is refused with MFCG_ENOMEM before any launch, and
    the handle still solves afterwards: the iteration limit's 32-bit
    maximum is sized in 64 bits, and a failed allocation leaves no stale
    capacity behind."""
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    cells, k = (4, 4, 4), 2
    _, A, P = _problem(oracle_mod, cells, k, 1, 0.05, None, None)
    b = torch.from_numpy(inputs.random_rhs(cells, k, seed=85)).cuda()
    m = mfcg.MULTI_MAX
    xs = [torch.zeros_like(b) for _ in range(m)]
    print("m", m, "maxit 2^31 - 1", flush=True)
    code, _, _, _ = P.solve_multi([b] * m, xs, tol=1e-10, maxit=2**31 - 1, raise_on=False)
    assert code == mfcg.ENOMEM
    x1 = [torch.zeros_like(b)]
    code, its, status, _ = P.solve_multi([b], x1, tol=1e-10, maxit=500)
    ref = torch.zeros_like(b)
    P.solve(b, ref, tol=1e-10, maxit=500)
    assert code == mfcg.OK and status == [mfcg.OK]
    assert torch.equal(x1[0], ref)
