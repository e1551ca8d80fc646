"""GPU parity of the comparison solvers of Sec. 4.1 against the oracle:
pipelined CG (Algorithm 2) and s-step CG (Algorithm 3, monomial basis), both
without preconditioner as the paper compares them.

The oracle runs the same recurrences in FP64 on the assembled matrix.  As
for the fused solver, the GPU's iteration count must lie within the
oracle's own range under permuted node orders (widened by 2, or by the
range's own width where that is larger), its residual history
within 10x the oracle's deviation under those permutations (and to 1e-9 in
the first iterations, for s < 6), its solution within 10x that deviation's effect on
x (at least 1e-9 relative), its true residual within 3x the oracle's
(pipelined CG's recursive residual drifts from the true one); after a fixed number of s-step phases (not
converged) the GPU iterate matches the oracle's to the same bar.  Edge
cases: zero right-hand side, an iteration limit that is not a multiple of
s, a warm start at the solution, switching solvers on one handle.
"""
import numpy as np
import pytest

from paper_2205_08909_amd import inputs
from tests.test_gpu_solve import _problem, torch_cuda  # noqa: F401

pytestmark = pytest.mark.gpu


def _oracle_run(KO, name, s, A, b, tol, maxit, x0=None):
    if name == "pipe":
        return KO.pipelined_cg(A.matvec, b, x0=x0, tol=tol, maxit=maxit)
    return KO.s_step_cg(A.matvec, b, s, x0=x0, tol=tol, maxit=maxit)


def _noise(KO, name, s, A, b, tol, maxit, nperm=2):
    """The oracle's spread under permuted node orders: iteration range, the
    largest relative deviation of the (defined) history and of x, and the
    largest true relative residual ||b - A x|| / ||b|| of its solutions."""
    from oracle.oracle import CSR
    x1, its1, h1, _ = _oracle_run(KO, name, s, A, b, tol, maxit)
    lo = hi = its1
    dh = dx = 0.0
    nb = np.linalg.norm(b)
    trmax = np.linalg.norm(b - A.matvec(x1)) / nb
    for seed in range(nperm):
        perm = np.random.default_rng(100 + seed).permutation(A.n)
        S = A.to_scipy()[perm][:, perm].tocsr()
        S.sort_indices()
        Ap = CSR(S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data.copy())
        x2, its2, h2, _ = _oracle_run(KO, name, s, Ap, b[perm], tol, maxit)
        xb = np.empty_like(x2)
        xb[perm] = x2
        lo, hi = min(lo, its2), max(hi, its2)
        j = min(its1, its2)
        ok = ~np.isnan(h1[:j + 1])
        dh = max(dh, np.max(np.abs(h1[:j + 1][ok] - h2[:j + 1][ok]) / h1[:j + 1][ok]))
        dx = max(dx, np.linalg.norm(xb - x1) / np.linalg.norm(x1))
        trmax = max(trmax, np.linalg.norm(b - A.matvec(xb)) / nb)
    return x1, its1, h1, lo, hi, dh, dx, trmax


def _gpu_solve(torch, P, solver, s, b, tol, maxit, x0=None):
    from paper_2205_08909_amd import mfcg
    P.set_solver(solver)
    if s:
        P.set_sstep(s)
    bt = torch.from_numpy(b).cuda()
    xt = torch.from_numpy(np.zeros_like(b) if x0 is None else x0.copy()).cuda()
    code, its, hist, tr = P.solve(bt, xt, tol=tol, maxit=maxit, want_true_res=True, raise_on=False)
    assert code in (mfcg.OK, mfcg.ENOTCONV), code
    return code, its, hist, tr, xt.cpu().numpy()


def _check(name, s, its, hist, x, ref):
    xo, its_o, hist_o, lo, hi, dh, dx, _ = ref
    # margin: 2, or the oracle's own spread where it is wider (the s-step
    # tail on a rough coefficient moves by phases under reordering)
    margin = max(2, hi - lo)
    assert lo - margin <= its <= hi + margin, (name, s, its, lo, hi)
    j = min(its, its_o)
    ok = ~np.isnan(hist_o[:j + 1])
    assert np.array_equal(np.isnan(hist[:j + 1]), ~ok)
    e = min(j, 10)
    early = np.abs(hist[:e + 1][ok[:e + 1]] - hist_o[:e + 1][ok[:e + 1]]) / hist_o[:e + 1][ok[:e + 1]]
    # the monomial basis of s >= 6 amplifies rounding from the first phase on
    assert early.max() <= (1e-9 if s < 6 else max(1e-9, 10 * dh)), early
    dev = np.max(np.abs(hist[:j + 1][ok] - hist_o[:j + 1][ok]) / hist_o[:j + 1][ok])
    assert dev <= 10 * dh + 1e-9, (dev, dh)
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    assert err <= max(1e-9, 10 * dx), (err, dx)


@pytest.mark.parametrize("cells,k,coeff_seed,tile", [
    ((5, 4, 3), 4, 3, None),
    ((6, 7, 5), 3, 4, (2, 3, 2)),   # several tiles, ragged tails
    ((3, 3, 3), 6, None, (2, 2, 2)),
    ((8, 8, 8), 1, 5, (4, 4, 4)),
])
def test_pipelined_matches_oracle(cells, k, coeff_seed, tile, oracle_mod, torch_cuda):
    from oracle import krylov_oracle as KO
    from paper_2205_08909_amd import mfcg
    m, A, P = _problem(oracle_mod, cells, k, 1, 0.05, coeff_seed, tile)
    b = inputs.random_rhs(cells, k, seed=11)
    ref = _noise(KO, "pipe", 0, A, b, 1e-10, 5000)
    code, its, hist, tr, x = _gpu_solve(torch_cuda, P, mfcg.SOLVER_PIPELINED, 0, b, 1e-10, 5000)
    print(cells, k, "pipelined its", its, "oracle", ref[1], (ref[3], ref[4]), "true res", tr)
    assert code == mfcg.OK
    _check("pipe", 0, its, hist, x, ref)
    # pipelined CG stops on its recursively updated residual, which drifts
    # from the true one (the oracle's own solutions show the same gap): the
    # true residual is bounded by the oracle's, not by tol
    bound = max(2e-10, 3 * ref[7])
    assert tr <= bound, (tr, ref[7])
    assert np.linalg.norm(b - A.matvec(x)) <= bound * np.linalg.norm(b)
    P.close()


@pytest.mark.parametrize("s", [1, 2, 3, 6, 8])
def test_s_step_phases_match_oracle(s, oracle_mod, torch_cuda):
    """A fixed number of phases (no convergence test hit): every phase-end
    residual and the iterate against the oracle."""
    from oracle import krylov_oracle as KO
    from paper_2205_08909_amd import mfcg
    cells, k = (5, 4, 6), 3
    m, A, P = _problem(oracle_mod, cells, k, 1, 0.05, 2, (2, 2, 3))
    b = inputs.random_rhs(cells, k, seed=12)
    maxit = 4 * s
    ref = _noise(KO, "sstep", s, A, b, 0.0, maxit)
    code, its, hist, tr, x = _gpu_solve(torch_cuda, P, mfcg.SOLVER_SSTEP, s, b, 0.0, maxit)
    print("s", s, "its", its, "phase residuals", hist[::s], ref[2][::s])
    assert code == mfcg.ENOTCONV and its == maxit
    _check("sstep", s, its, hist, x, ref)
    P.close()


# Solves to convergence with a rough coefficient only for s = 2: for s >= 4
# the monomial basis makes the oracle itself break down in some node orders
# on such problems (the instability the paper notes), so those cases use a
# constant coefficient.
@pytest.mark.parametrize("s,cells,k,tile,coeff_seed", [
    (2, (6, 7, 5), 3, (2, 3, 2), 6),
    (6, (5, 4, 3), 4, None, None),
    (4, (3, 3, 3), 6, (2, 2, 2), None),
])
def test_s_step_converges_like_oracle(s, cells, k, tile, coeff_seed, oracle_mod, torch_cuda):
    from oracle import krylov_oracle as KO
    from paper_2205_08909_amd import mfcg
    m, A, P = _problem(oracle_mod, cells, k, 1, 0.05, coeff_seed, tile)
    b = inputs.random_rhs(cells, k, seed=13)
    ref = _noise(KO, "sstep", s, A, b, 1e-10, 5000, nperm=3)
    code, its, hist, tr, x = _gpu_solve(torch_cuda, P, mfcg.SOLVER_SSTEP, s, b, 1e-10, 5000)
    print("s", s, cells, k, "its", its, "oracle", ref[1], (ref[3], ref[4]), "true res", tr)
    assert code == mfcg.OK and its % s == 0
    _check("sstep", s, its, hist, x, ref)
    assert tr < 1e-10
    P.close()


def test_edge_cases_and_solver_switching(oracle_mod, torch_cuda):
    torch = torch_cuda
    from oracle import krylov_oracle as KO
    from paper_2205_08909_amd import mfcg
    cells, k = (4, 5, 3), 3
    m, A, P = _problem(oracle_mod, cells, k, 1, 0.05, None, (2, 2, 2))
    b = inputs.random_rhs(cells, k, seed=14)
    zero = np.zeros_like(b)
    for bad in (lambda: P.set_sstep(0), lambda: P.set_sstep(9), lambda: P.set_solver(5), lambda: P.set_solver(-1)):
        with pytest.raises(mfcg.MfcgError):
            bad()
    for solver, s in ((mfcg.SOLVER_PIPELINED, 0), (mfcg.SOLVER_SSTEP, 3)):
        code, its, hist, tr, x = _gpu_solve(torch, P, solver, s, zero, 1e-10, 100)
        assert code == mfcg.OK and its == 0 and not x.any()
    # an iteration limit that is not a multiple of s: whole phases only
    code, its, hist, tr, x = _gpu_solve(torch, P, mfcg.SOLVER_SSTEP, 3, b, 1e-10, 8)
    assert code == mfcg.ENOTCONV and its == 6
    xo, its_o, _, rc_o = KO.s_step_cg(A.matvec, b, 3, tol=1e-10, maxit=8)
    assert its_o == 6 and np.linalg.norm(x - xo) <= 1e-9 * np.linalg.norm(xo)
    # pipelined iteration limit
    code, its, hist, tr, x = _gpu_solve(torch, P, mfcg.SOLVER_PIPELINED, 0, b, 1e-10, 5)
    xo, its_o, hist_o, rc_o = KO.pipelined_cg(A.matvec, b, tol=1e-10, maxit=5)
    assert code == mfcg.ENOTCONV and its == 5 and rc_o == KO.NOT_CONVERGED
    assert np.linalg.norm(x - xo) <= 1e-12 * np.linalg.norm(xo)
    assert np.abs(hist - hist_o).max() <= 1e-12 * np.linalg.norm(b)
    # a warm start at the solution needs no iteration
    xs = np.linalg.solve(A.to_scipy().toarray(), b)
    for solver, s in ((mfcg.SOLVER_PIPELINED, 0), (mfcg.SOLVER_SSTEP, 6)):
        code, its, hist, tr, x = _gpu_solve(torch, P, solver, s, b, 1e-8, 100, x0=xs)
        assert code == mfcg.OK and its == 0
    # switching back and forth on one handle: each solver still matches
    # its own first run bitwise
    runs = {}
    for solver, s in ((mfcg.SOLVER_FUSED, 0), (mfcg.SOLVER_PIPELINED, 0), (mfcg.SOLVER_SSTEP, 4),
                      (mfcg.SOLVER_PCG_BASIC, 0), (mfcg.SOLVER_SSTEP, 2), (mfcg.SOLVER_FUSED, 0),
                      (mfcg.SOLVER_PIPELINED, 0), (mfcg.SOLVER_SSTEP, 4), (mfcg.SOLVER_SSTEP, 2)):
        code, its, hist, tr, x = _gpu_solve(torch, P, solver, s, b, 1e-10, 5000)
        assert code == mfcg.OK and tr < 2e-10
        key = (solver, s)
        if key in runs:
            assert runs[key][0] == its and np.array_equal(runs[key][1], x)
        runs[key] = (its, x)
    P.close()
