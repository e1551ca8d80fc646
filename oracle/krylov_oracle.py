"""Plain FP64 numpy versions of the comparison Krylov solvers of Sec. 4.1
(alternative CG methods): pipelined CG (Algorithm 2) and s-step CG with the
monomial basis (Algorithm 3), both without preconditioner as the paper
compares them.  (Algorithm 1 with M = I is the C oracle's pcg with a unit
diagonal.)

TEST INFRASTRUCTURE ONLY: imported by tests/ (and bench.py's cpu_baseline
leg).  The product package never imports it.

Every solver takes the operator as a callable `matvec(u) -> A u` (the
oracle's CSR product), stops on the residual norm it carries falling below
tol * ||b||_2, and returns (x, iterations, hist, rc) with rc 0 converged,
-4 iteration limit, -5 breakdown (a non-positive or non-finite denominator,
or a singular s x s block).

Readings of the paper's listings (they omit the initialisation):
  * pipelined CG starts from r_0 = b - A x_0, w_0 = A r_0,
    gamma_0 = r_0^T r_0, a_0 = w_0^T r_0 and p = s = z = 0; the first
    iteration takes beta = 0 and alpha = gamma_0 / a_0 (the recurrence of
    Algorithm 2 with no previous step); hist[k] = sqrt(gamma_k), the
    recursively updated residual norm.
  * s-step CG: R_k = [r_k, A r_k, .., A^{s-1} r_k] and Q_k = A R_k (the first
    and the last s columns of T_k); the block B_k makes P_k A-conjugate to
    P_{k-1}, i.e. B_k = -W_{k-1}^{-1} (P_{k-1}^T Q_k).  That s x s block is
    symmetric in exact arithmetic (r_k is orthogonal to the previous Krylov
    space, so the (i, l) entry reduces to (A^{i+l+1} r_{k-1})^T r_k, a Hankel
    matrix), so it equals the printed Q_k^T P_{k-1}.  The first phase takes P_0 = R_0.  One phase counts as s iterations; the residual is recomputed
    as b - A x at the end of every phase and hist holds its norm at the
    multiples of s (NaN in between).
"""
import numpy as np

OK, NOT_CONVERGED, BREAKDOWN = 0, -4, -5


def pipelined_cg(matvec, b, x0=None, tol=1e-10, maxit=10000, return_iterates=False):
    """Algorithm 2: one mat-vec q = A w per iteration, the scalars of the
    iteration from the previous iteration's two inner products, then the six
    vector updates and the two inner products gamma = r^T r, a = w^T r."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - matvec(x)
    w = matvec(r)
    gamma, a = r @ r, w @ r
    p, s, z = np.zeros_like(b), np.zeros_like(b), np.zeros_like(b)
    eps = tol * np.linalg.norm(b)
    hist = [np.sqrt(gamma)]
    its = [x.copy()] if return_iterates else None

    def out(k, rc):
        res = (x, k, np.array(hist), rc)
        return res + (its,) if return_iterates else res

    if gamma == 0.0 or np.sqrt(gamma) < eps:
        return out(0, OK)
    gamma_prev, alpha_prev = 0.0, 0.0
    for k in range(1, maxit + 1):
        q = matvec(w)
        if k == 1:
            beta = 0.0
            den = a
        else:
            beta = gamma / gamma_prev
            den = a - beta * gamma / alpha_prev
        if not (den > 0) or not np.isfinite(den):
            return out(k, BREAKDOWN)
        alpha = gamma / den
        p = r + beta * p
        x = x + alpha * p
        s = w + beta * s
        r = r - alpha * s
        z = q + beta * z
        w = w - alpha * z
        gamma_prev, alpha_prev = gamma, alpha
        gamma, a = r @ r, w @ r
        hist.append(np.sqrt(gamma))
        if return_iterates:
            its.append(x.copy())
        if not np.isfinite(gamma):
            return out(k, BREAKDOWN)
        if np.sqrt(gamma) < eps:
            return out(k, OK)
    return out(maxit, NOT_CONVERGED)


def s_step_cg(matvec, b, s, x0=None, tol=1e-10, maxit=10000, return_iterates=False):
    """Algorithm 3 with the monomial basis.  Per phase: s mat-vecs for the
    basis T = [r, A r, .., A^s r], the block products P_prev^T Q, Q^T P and
    P^T r, two s x s solves, x += P a, and one more mat-vec for the true
    residual r = b - A x.  Only whole phases run: the iteration count is a
    multiple of s and at most maxit."""
    assert 1 <= s <= 16
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - matvec(x)
    eps = tol * np.linalg.norm(b)
    hist = [np.linalg.norm(r)]
    its = [x.copy()] if return_iterates else None

    def out(k, rc):
        res = (x, k, np.array(hist), rc)
        return res + (its,) if return_iterates else res

    if hist[0] == 0.0 or hist[0] < eps:
        return out(0, OK)
    P_prev = W_prev = None
    k = 0
    while k + s <= maxit:
        # basis T = [r, A r, .., A^s r]; R = first s columns, Q = last s
        T = [r]
        for _ in range(s):
            T.append(matvec(T[-1]))
        R = np.stack(T[:s], axis=1)
        Q = np.stack(T[1:], axis=1)
        if P_prev is None:
            P = R
        else:
            C = P_prev.T @ Q
            try:
                B = -np.linalg.solve(W_prev, C)
            except np.linalg.LinAlgError:
                return out(k + s, BREAKDOWN)
            P = R + P_prev @ B
        W = Q.T @ P
        g = P.T @ r
        try:
            a = np.linalg.solve(W, g)
        except np.linalg.LinAlgError:
            return out(k + s, BREAKDOWN)
        if not np.all(np.isfinite(a)):
            return out(k + s, BREAKDOWN)
        x = x + P @ a
        r = b - matvec(x)
        k += s
        rho = np.linalg.norm(r)
        hist.extend([np.nan] * (s - 1) + [rho])
        if return_iterates:
            its.append(x.copy())
        if not np.isfinite(rho):
            return out(k, BREAKDOWN)
        if rho < eps:
            return out(k, OK)
        P_prev, W_prev = P, W
    return out(k, NOT_CONVERGED)
