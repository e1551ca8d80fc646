"""GPU solve parity: the fused Algorithm 5 against the oracle's Algorithm 1.

In exact arithmetic both produce the same iterates (Sec. 4.2: Eq. 6-8 only
regroup the inner products).  In FP64 the iteration count and the residual
history are compared against the oracle's own sensitivity to summation
order (the same system solved in permuted node orders): the GPU's count
must lie within that range +-2 and its history within 10x that deviation;
the first iterations must agree to rounding; the converged solutions must
agree to 1e-10 relative (the required solution tolerance) and the GPU
solution's residual in the oracle's matrix must be below 2e-10 ||b||.  Also checked: the exit
reconstruction of x for both parities of the last iteration (maxit exits),
warm starts, a zero right-hand side, reproducibility.
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


def _problem(oracle_mod, cells, k, kind, amp, coeff_seed=None, tile=None, bc=0):
    from paper_2205_08909_amd import mfcg
    coeff = inputs.grf_coefficient(cells, 0.1, 1.0, seed=coeff_seed) if coeff_seed is not None else None
    m = oracle_mod.Mesh(cells, k, map_kind=kind, amp=amp, bc=bc, coeff=coeff)
    A = oracle_mod.assemble(m)
    P = mfcg.Problem(cells, k, coeff=coeff, map_kind=kind, amplitude=amp, bc=bc, tile=tile)
    return m, A, P


def oracle_noise(oracle_mod, A, b, x0=None, tol=1e-10, maxit=5000, nperm=3, diag=None):
    """The oracle's own sensitivity to summation order: the same system
    solved in other node orders (P A P^T, P b).  Returns the range of
    iteration counts and the largest relative deviation of the residual
    history from the unpermuted solve.  diag: the preconditioner's
    diagonal (default diag(A); ones for plain CG)."""
    from oracle.oracle import CSR
    d = A.diagonal() if diag is None else diag
    _, its1, h1, _ = oracle_mod.pcg(A, d, b, x0=x0, tol=tol, maxit=maxit)
    lo = hi = its1
    dev = 0.0
    for seed in range(nperm):
        perm = np.random.default_rng(seed).permutation(A.n)
        S = A.to_scipy()[perm][:, perm].tocsr()
        S.sort_indices()
        Ap = CSR(S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data.copy())
        xp = None if x0 is None else x0[perm]
        _, its2, h2, _ = oracle_mod.pcg(Ap, d[perm], b[perm], x0=xp, tol=tol, maxit=maxit)
        lo, hi = min(lo, its2), max(hi, its2)
        j = min(its1, its2)
        dev = max(dev, np.max(np.abs(h1[:j + 1] - h2[:j + 1]) / h1[:j + 1]))
    return lo, hi, dev


def _compare(torch, oracle_mod, A, P, b, x0=None, tol=1e-10, maxit=5000):
    d = A.diagonal()
    xo, its_o, hist_o, rc_o = oracle_mod.pcg(A, d, b, x0=x0, tol=tol, maxit=maxit)
    bt = torch.from_numpy(b).cuda()
    xt = torch.from_numpy(x0 if x0 is not None else np.zeros_like(b)).cuda()
    code, its, hist, tr = P.solve(bt, xt, tol=tol, maxit=maxit, want_true_res=True)
    return xo, its_o, hist_o, rc_o, xt.cpu().numpy(), its, hist, tr, code


@pytest.mark.parametrize("cells,k,kind,coeff_seed,tile", [
    ((8, 8, 8), 2, 0, None, None),           # the plain Q2 workload, f from the manufactured solution
    ((16, 16, 16), 4, 1, 3, None),           # curved Q4, random coefficient
    ((6, 7, 5), 3, 1, 4, (2, 3, 2)),         # ragged tiles
    ((4, 4, 4), 8, 1, 5, (2, 1, 3)),
])
def test_solve_matches_oracle(cells, k, kind, coeff_seed, tile, oracle_mod, torch_cuda):
    torch = torch_cuda
    m, A, P = _problem(oracle_mod, cells, k, kind, 0.05, coeff_seed, tile)
    b = oracle_mod.rhs(m, oracle_mod.F_SINE)
    xo, its_o, hist_o, rc_o, x, its, hist, tr, code = _compare(torch, oracle_mod, A, P, b)
    assert rc_o == 0 and code == 0
    lo, hi, floor = oracle_noise(oracle_mod, A, b)
    assert lo - 2 <= its <= hi + 2, (its, lo, hi)
    assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo)
    nb = np.linalg.norm(b)
    j = min(its, its_o)
    # early iterations agree to rounding; later ones within 10x the
    # oracle's own order-of-summation noise floor
    e = min(j, 5)
    assert np.abs(hist[:e + 1] - hist_o[:e + 1]).max() <= 1e-12 * max(nb, hist_o[:e + 1].max())
    dev = np.max(np.abs(hist[:j + 1] - hist_o[:j + 1]) / hist_o[:j + 1])
    assert dev <= 10 * floor + 1e-12, (dev, floor)
    assert hist[its] < 1e-10 * nb
    assert tr <= 2e-10
    # the oracle's own residual of the GPU solution
    assert np.linalg.norm(b - A.matvec(x)) <= 2e-10 * nb
    P.close()


def test_random_rhs_warm_start_and_reproducible(oracle_mod, torch_cuda):
    torch = torch_cuda
    cells, k = (6, 6, 6), 4
    m, A, P = _problem(oracle_mod, cells, k, 1, 0.05, coeff_seed=8)
    b = inputs.random_rhs(cells, k, seed=9)
    x0 = 0.1 * inputs.random_vector(A.n, seed=10)
    x0[m.constrained_mask()] = 0.0
    xo, its_o, _, _, x, its, _, tr, code = _compare(torch, oracle_mod, A, P, b, x0=x0)
    lo, hi, _ = oracle_noise(oracle_mod, A, b, x0=x0)
    assert code == 0 and lo - 2 <= its <= hi + 2, (its, lo, hi)
    assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo)
    # bitwise reproducible
    xt = torch.from_numpy(x0).cuda()
    bt = torch.from_numpy(b).cuda()
    P.solve(bt, xt, tol=1e-10, maxit=5000)
    assert np.array_equal(xt.cpu().numpy(), x)
    P.close()


@pytest.mark.parametrize("maxit", [1, 2, 3, 4, 7])
def test_maxit_exit_both_parities(maxit, oracle_mod, torch_cuda):
    """x after exactly maxit iterations (not converged) equals Algorithm 1's
    x_maxit: the delayed x update is reconstructed for odd and even exits."""
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    cells, k = (5, 4, 6), 3
    m, A, P = _problem(oracle_mod, cells, k, 1, 0.05, coeff_seed=2, tile=(2, 2, 3))
    b = inputs.random_rhs(cells, k, seed=1)
    xo, its_o, hist_o, rc_o = oracle_mod.pcg(A, A.diagonal(), b, tol=1e-14, maxit=maxit)
    assert rc_o == -4 and its_o == maxit
    bt = torch.from_numpy(b).cuda()
    xt = torch.zeros_like(bt)
    code, its, hist, _ = P.solve(bt, xt, tol=1e-14, maxit=maxit)
    assert code == mfcg.ENOTCONV and its == maxit
    x = xt.cpu().numpy()
    assert np.linalg.norm(x - xo) <= 1e-12 * np.linalg.norm(xo)
    assert np.abs(hist - hist_o).max() <= 1e-12 * np.linalg.norm(b)
    P.close()


def test_zero_rhs_and_exact_warm_start(oracle_mod, torch_cuda):
    torch = torch_cuda
    cells, k = (4, 4, 4), 2
    m, A, P = _problem(oracle_mod, cells, k, 1, 0.05)
    z = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    x = torch.ones_like(z)
    code, its, hist, tr = P.solve(z, x, tol=1e-10, maxit=10, want_true_res=True)
    assert code == 0 and its == 0 and torch.count_nonzero(x).item() == 0 and tr == 0.0
    # warm start at the (oracle) solution: converged before the first iteration
    import scipy.sparse.linalg as spla
    b = oracle_mod.rhs(m)
    xs = spla.spsolve(A.to_scipy().tocsc(), b)
    xt = torch.from_numpy(xs).cuda()
    code, its, hist, _ = P.solve(torch.from_numpy(b).cuda(), xt, tol=1e-8, maxit=10)
    assert code == 0 and its == 0
    P.close()


def test_breakdown_on_nan(oracle_mod, torch_cuda):
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    cells, k = (3, 3, 3), 2
    P = mfcg.Problem(cells, k)
    b = torch.from_numpy(inputs.random_rhs(cells, k, seed=3)).cuda()
    b[P.n // 2] = float("nan")
    x = torch.zeros_like(b)
    code, its, hist, _ = P.solve(b, x, tol=1e-10, maxit=20, raise_on=False)
    assert code in (mfcg.EBREAKDOWN,)
    P.close()
