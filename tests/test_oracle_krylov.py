"""Pins for the oracle's comparison solvers (Sec. 4.1): pipelined CG
(Algorithm 2) and s-step CG (Algorithm 3).

In exact arithmetic both produce the iterates of plain CG (pipelined CG at
every iteration, s-step CG at every multiple of s), so they are pinned to
scipy's CG (a library routine, iterates taken from its callback) on a small
well-conditioned problem; to the closed form that CG on an operator with m
distinct eigenvalues reaches the solution in m steps; to the invariant that
pipelined CG's recursively updated gamma_k is ||b - A x_k||^2; and to the
edge cases (zero right-hand side, iteration limit, indefinite operator).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import krylov_oracle as KO


def _problem(O, ncells=(3, 3, 2), k=2, seed=0):
    rng = np.random.default_rng(seed)
    m = O.Mesh(ncells, k, map_kind=1, amp=0.05)
    A = O.assemble(m)
    b = rng.normal(size=A.n)
    b[m.constrained_mask()] = 0.0
    return m, A, b


def _scipy_iterates(A, b, maxiter):
    xs = []
    spla.cg(A.to_scipy(), b, rtol=1e-30, atol=0.0, maxiter=maxiter, callback=lambda xk: xs.append(xk.copy()))
    return xs


def _few_eigenvalues(n=40, values=(1.0, 2.0, 5.0, 10.0), seed=1):
    rng = np.random.default_rng(seed)
    Qm, _ = np.linalg.qr(rng.normal(size=(n, n)))
    lam = np.array([values[i % len(values)] for i in range(n)])
    M = (Qm * lam) @ Qm.T
    M = 0.5 * (M + M.T)
    return M, rng.normal(size=n)


def test_pipelined_iterates_match_cg(oracle_mod):
    m, A, b = _problem(oracle_mod)
    ref = _scipy_iterates(A, b, 25)
    x, its, hist, rc, xs = KO.pipelined_cg(A.matvec, b, tol=1e-10, maxit=2000, return_iterates=True)
    assert rc == KO.OK
    nb = np.linalg.norm(ref[-1])
    for j in range(1, 26):
        d = np.linalg.norm(xs[j] - ref[j - 1]) / nb
        assert d <= 1e-9, (j, d)
    # converged to the solution, with about CG's iteration count
    xd = spla.spsolve(A.to_scipy().tocsc(), b)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
    _, its_cg, _, _ = oracle_mod.pcg(A, np.ones(A.n), b, tol=1e-10)
    assert abs(its - its_cg) <= 3


def test_pipelined_gamma_is_the_residual(oracle_mod):
    m, A, b = _problem(oracle_mod, seed=3)
    x, its, hist, rc, xs = KO.pipelined_cg(A.matvec, b, tol=1e-10, maxit=2000, return_iterates=True)
    nb = np.linalg.norm(b)
    for j in range(0, min(its, 30) + 1):
        true = np.linalg.norm(b - A.matvec(xs[j]))
        assert abs(hist[j] - true) <= 1e-9 * nb, (j, hist[j], true)


@pytest.mark.parametrize("s", [1, 2, 3])
def test_s_step_iterates_match_cg(oracle_mod, s):
    m, A, b = _problem(oracle_mod, seed=5)
    ref = _scipy_iterates(A, b, 5 * s)
    x, its, hist, rc, xs = KO.s_step_cg(A.matvec, b, s, tol=1e-10, maxit=5 * s, return_iterates=True)
    assert its == 5 * s and len(xs) == 6
    nb = np.linalg.norm(ref[-1])
    for j in range(1, 6):
        d = np.linalg.norm(xs[j] - ref[j * s - 1]) / nb
        assert d <= 1e-8, (s, j, d)
    # the history holds the true residual at the phase ends, NaN between
    for j in range(1, 6):
        assert hist[j * s] == pytest.approx(np.linalg.norm(b - A.matvec(xs[j])), rel=1e-12)
        assert np.all(np.isnan(hist[(j - 1) * s + 1: j * s]))


def test_s_step_converges(oracle_mod):
    m, A, b = _problem(oracle_mod, seed=7)
    xd = spla.spsolve(A.to_scipy().tocsc(), b)
    for s in (1, 2, 4):
        x, its, hist, rc = KO.s_step_cg(A.matvec, b, s, tol=1e-10, maxit=4000)
        assert rc == KO.OK and its % s == 0
        assert np.linalg.norm(b - A.matvec(x)) < 1e-10 * np.linalg.norm(b)
        assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)


def test_few_distinct_eigenvalues():
    """CG on an operator with 4 distinct eigenvalues ends in 4 steps."""
    M, b = _few_eigenvalues()
    mv = lambda u: M @ u
    xd = np.linalg.solve(M, b)
    x, its, hist, rc = KO.pipelined_cg(mv, b, tol=1e-10, maxit=50)
    assert rc == KO.OK and its == 4
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    x, its, hist, rc = KO.s_step_cg(mv, b, 4, tol=1e-10, maxit=50)
    assert rc == KO.OK and its == 4
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    x, its, hist, rc = KO.s_step_cg(mv, b, 2, tol=1e-10, maxit=50)
    assert rc == KO.OK and its == 4
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)


def test_edge_cases(oracle_mod):
    m, A, b = _problem(oracle_mod, ncells=(2, 2, 2))
    for f in (lambda bb, **kw: KO.pipelined_cg(A.matvec, bb, **kw),
              lambda bb, **kw: KO.s_step_cg(A.matvec, bb, 3, **kw)):
        x, its, hist, rc = f(np.zeros(A.n), tol=1e-10)
        assert rc == KO.OK and its == 0 and np.all(x == 0)
    x, its, hist, rc = KO.pipelined_cg(A.matvec, b, tol=1e-10, maxit=2)
    assert rc == KO.NOT_CONVERGED and its == 2
    x, its, hist, rc = KO.s_step_cg(A.matvec, b, 3, tol=1e-10, maxit=8)
    assert rc == KO.NOT_CONVERGED and its == 6
    # an indefinite (negated) operator breaks pipelined CG down at once
    x, its, hist, rc = KO.pipelined_cg(lambda u: -A.matvec(u), b, tol=1e-10)
    assert rc == KO.BREAKDOWN and its == 1
