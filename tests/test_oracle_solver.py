"""Pins for the oracle's solver (Algorithm 1), load vector and L2 error.

* Algorithm 1 with the Jacobi preconditioner against scipy's preconditioned
  CG (a library routine computing the same recurrence) and a direct solve,
* a numpy toy of Algorithm 5 (merged PCG, Sec. 4.2) reproduces Algorithm 1:
  same iteration count, same x, both exit parities,
* sum of the load vector = integral of f (partition of unity),
* O(h^{k+1}) L2 convergence to u = prod sin(pi x_j) on the Cartesian mesh
  and on the boundary-preserving sine-product map.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla


def _problem(O, ncells=(4, 3, 5), k=2, kind=1, seed=0):
    rng = np.random.default_rng(seed)
    coeff = np.exp(rng.normal(size=int(np.prod(ncells))))
    m = O.Mesh(ncells, k, map_kind=kind, amp=0.05, coeff=coeff)
    A = O.assemble(m)
    b = rng.normal(size=A.n)
    b[m.constrained_mask()] = 0.0
    return m, A, b


def test_pcg_matches_scipy_cg(oracle_mod):
    O = oracle_mod
    m, A, b = _problem(O)
    d = A.diagonal()
    tol = 1e-10
    x, its, hist, rc = O.pcg(A, d, b, tol=tol, maxit=2000)
    assert rc == 0
    S = A.to_scipy()
    M = spla.LinearOperator(S.shape, matvec=lambda r: r / d)
    count = [0]

    def cb(_):
        count[0] += 1
    xs, info = spla.cg(S, b, rtol=tol, atol=0.0, M=M, maxiter=2000, callback=cb)
    assert info == 0
    assert abs(count[0] - its) <= 1
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    xd = spla.spsolve(S.tocsc(), b)
    assert np.linalg.norm(x - xd) <= 1e-7 * np.linalg.norm(xd)
    # history: starts at ||b||, ends below tol*||b||, the one before not
    nb = np.linalg.norm(b)
    assert hist[0] == pytest.approx(nb, rel=1e-14)
    assert hist[-1] < tol * nb <= hist[-2]
    assert np.linalg.norm(b - A.matvec(x)) <= 2 * tol * nb


def test_pcg_edge_cases(oracle_mod):
    O = oracle_mod
    m, A, b = _problem(O, ncells=(2, 2, 2))
    d = A.diagonal()
    x, its, hist, rc = O.pcg(A, d, np.zeros(A.n), tol=1e-10)
    assert rc == 0 and its == 0 and np.all(x == 0)
    x, its, hist, rc = O.pcg(A, d, b, tol=1e-10, maxit=1)
    assert rc == -4 and its == 1
    # a warm start at the solution needs no iteration
    xs = spla.spsolve(A.to_scipy().tocsc(), b)
    x, its, hist, rc = O.pcg(A, d, b, x0=xs, tol=1e-8)
    assert rc == 0 and its == 0
    # non-SPD (negated operator) breaks down in the first iteration
    from oracle.oracle import CSR
    An = CSR(A.rowptr, A.col, -A.val)
    x, its, hist, rc = O.pcg(An, np.abs(d), b, tol=1e-10)
    assert rc == -5


def merged_pcg_toy(A, d, b, tol, maxit):
    """Algorithm 5 in numpy, with the reading x_1 = x_0 (x updated every
    other iteration and reconstructed at exit)."""
    x = np.zeros_like(b)
    r = b - A @ x
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    alpha, beta = 0.0, 0.0
    alpha_prev, beta_prev = 0.0, 0.0
    eps = tol * np.linalg.norm(b)
    if np.linalg.norm(r) < eps:
        return x, 0
    for k in range(1, maxit + 1):
        if k > 1 and k % 2 == 1:
            x = x + alpha * p + (alpha_prev / beta_prev) * (p - r / d)
        r = r - alpha * v
        p = r / d + beta * p
        v = A @ p
        g, a, bb, c = r @ r, p @ v, r @ v, v @ v
        dd, e, f = r @ (r / d), r @ (v / d), v @ (v / d)
        alpha_new = dd / a
        if np.sqrt(max(g - 2 * alpha_new * bb + alpha_new ** 2 * c, 0.0)) < eps:
            if k % 2 == 1:
                x = x + alpha_new * p
            else:
                x = x + alpha_new * p + (alpha / beta) * (p - r / d)
            return x, k
        beta_new = (dd - 2 * alpha_new * e + alpha_new ** 2 * f) / dd
        alpha_prev, beta_prev = alpha, beta
        alpha, beta = alpha_new, beta_new
    return x, maxit


@pytest.mark.parametrize("seed,tol", [(0, 1e-6), (1, 1e-9), (2, 1e-12), (3, 1e-4)])
def test_algorithm5_toy_reproduces_algorithm1(oracle_mod, seed, tol):
    O = oracle_mod
    m, A, b = _problem(O, ncells=(3, 3, 2), k=2, seed=seed)
    d = A.diagonal()
    x1, its1, _, rc = O.pcg(A, d, b, tol=tol)
    S = A.to_scipy()
    x5, its5 = merged_pcg_toy(S, d, b, tol, 1000)
    assert rc == 0 and abs(its5 - its1) <= 1
    assert np.linalg.norm(x5 - x1) <= 1e-10 * np.linalg.norm(x1)


def test_algorithm5_toy_both_parities(oracle_mod):
    O = oracle_mod
    m, A, b = _problem(O, ncells=(3, 3, 2), k=2, seed=7)
    d = A.diagonal()
    S = A.to_scipy()
    parities = set()
    for tol in np.logspace(-2, -10, 9):
        x1, its1, _, _ = O.pcg(A, d, b, tol=tol)
        x5, its5 = merged_pcg_toy(S, d, b, tol, 1000)
        if its1 == its5:
            parities.add(its1 % 2)
            assert np.linalg.norm(x5 - x1) <= 1e-10 * np.linalg.norm(x1)
    assert parities == {0, 1}


@pytest.mark.parametrize("kind", [0, 2])
def test_rhs_integral(oracle_mod, kind):
    O = oracle_mod
    m = O.Mesh(4, 2, map_kind=kind, amp=0.05, bc=O.BC_NONE)
    b = O.rhs(m, O.F_SINE)
    assert b.sum() == pytest.approx(24.0 / np.pi, rel=2e-5)


@pytest.mark.parametrize("kind", [0, 2])
@pytest.mark.parametrize("k,Ns", [(1, (4, 8)), (2, (4, 8)), (3, (3, 6)), (4, (4, 8))])
def test_l2_convergence_rate(oracle_mod, kind, k, Ns):
    O = oracle_mod
    errs = []
    for N in Ns:
        m = O.Mesh(N, k, map_kind=kind, amp=0.05)
        A = O.assemble(m)
        b = O.rhs(m, O.F_SINE)
        x, its, _, rc = O.pcg(A, A.diagonal(), b, tol=1e-13, maxit=5000)
        assert rc == 0
        errs.append(O.l2_error(m, x))
    rate = np.log2(errs[0] / errs[1]) / np.log2(Ns[1] / Ns[0])
    assert abs(rate - (k + 1)) < 0.35, (errs, rate)


def _bump_moments(params):
    """Closed forms of int f and int f x_d over the unit cube for
    f = sum_m A_m exp(-|x - c_m|^2 / (2 s_m^2)): per direction,
    int_0^1 exp(-(t-c)^2/(2s^2)) dt = s sqrt(pi/2) [erf((1-c)/(s sqrt2)) + erf(c/(s sqrt2))]
    and int_0^1 t exp(-(t-c)^2/(2s^2)) dt = c I0 + s^2 [exp(-c^2/(2s^2)) - exp(-(1-c)^2/(2s^2))]."""
    from math import erf, exp, pi, sqrt
    nb = int(params[0])
    m0, m1 = 0.0, np.zeros(3)
    for b in range(nb):
        A, cx, cy, cz, s = params[1 + 5 * b: 6 + 5 * b]
        i0, i1 = [], []
        for c in (cx, cy, cz):
            z = s * sqrt(2.0)
            I0 = s * sqrt(pi / 2.0) * (erf((1.0 - c) / z) + erf(c / z))
            I1 = c * I0 + s * s * (exp(-c * c / (2 * s * s)) - exp(-(1.0 - c) ** 2 / (2 * s * s)))
            i0.append(I0)
            i1.append(I1)
        m0 += A * i0[0] * i0[1] * i0[2]
        m1 += A * np.array([i1[0] * i0[1] * i0[2], i0[0] * i1[1] * i0[2], i0[0] * i0[1] * i1[2]])
    return m0, m1


@pytest.mark.parametrize("k,N", [(3, 12), (4, 10)])
def test_rhs_bumps_closed_form(oracle_mod, k, N):
    """Gaussian-bump forcing (the warm-start workload's load vector): with no
    boundary condition on the affine unit cube, sum_i b_i = int f (partition
    of unity) and sum_i x_d(node i) b_i = int f x_d (the Q_k basis reproduces
    linear functions), against the closed-form integrals, to Gauss-quadrature
    accuracy.  A wrong width factor, centre, amplitude or sign fails."""
    O = oracle_mod
    rng = np.random.default_rng(5)
    nb = 4
    params = [nb]
    for _ in range(nb):
        params += [rng.normal(), *rng.uniform(0.25, 0.75, 3), rng.uniform(0.08, 0.12)]
    params = np.array(params)
    m = O.Mesh(N, k, map_kind=O.MAP_AFFINE, amp=0.0, bc=O.BC_NONE)
    b = O.rhs(m, O.F_BUMPS, params)
    m0, m1 = _bump_moments(params)
    nn = N * k + 1
    # node coordinates of the lexicographic order (GLL nodes in each cell)
    g = np.asarray(O.gll(k))
    x1 = np.concatenate([(c + g[:-1]) / N for c in range(N)] + [np.array([1.0])])
    assert x1.size == nn
    X = x1[np.arange(b.size) % nn]
    Y = x1[(np.arange(b.size) // nn) % nn]
    Z = x1[np.arange(b.size) // (nn * nn)]
    scale = np.abs(params[1::5]).sum() * 0.01  # size of the bumps' integrals
    assert abs(b.sum() - m0) <= 1e-8 * scale, (b.sum(), m0)
    for d, C in enumerate((X, Y, Z)):
        assert abs((C * b).sum() - m1[d]) <= 1e-8 * scale, (d, (C * b).sum(), m1[d])
    # the same bumps with a width 1/sqrt(2) too small give a clearly different integral
    wrong = params.copy()
    wrong[5::5] /= np.sqrt(2.0)
    assert abs(_bump_moments(wrong)[0] - m0) > 1e-3 * scale


def _node_coords(cells, k, oracle_mod):
    """Reference coordinates of the Q_k nodes along each axis."""
    x = oracle_mod.gll(k)
    out = []
    for N in cells:
        g = np.arange(N * k + 1)
        e = np.minimum(g // k, N - 1)
        out.append((e + x[g - k * e]) / N)
    return out


@pytest.mark.parametrize("cells,kf,kt", [((3, 2, 4), 1, 3), ((2, 3, 2), 2, 4), ((2, 2, 3), 1, 1), ((3, 1, 2), 3, 5)])
def test_interpolate_reproduces_polynomials(oracle_mod, cells, kf, kt):
    """Nested spaces: a polynomial of degree kf in each variable (the Q_kf
    space contains it) sampled at the Q_kf nodes must come out at the Q_kt
    nodes exactly; a dropped basis term, a wrong cell index at the right end
    or transposed axes all fail this."""
    cx, cy, cz = _node_coords(cells, kf, oracle_mod)
    tx, ty, tz = _node_coords(cells, kt, oracle_mod)
    rng = np.random.default_rng(kf * 10 + kt)
    coef = rng.standard_normal((kf + 1, kf + 1, kf + 1))

    def f(X, Y, Z):
        out = np.zeros(np.broadcast(X, Y, Z).shape)
        for a in range(kf + 1):
            for b in range(kf + 1):
                for c in range(kf + 1):
                    out += coef[a, b, c] * X ** a * Y ** b * Z ** c
        return out

    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    src = f(X, Y, Z).ravel()
    Z2, Y2, X2 = np.meshgrid(tz, ty, tx, indexing="ij")
    want = f(X2, Y2, Z2).ravel()
    got = oracle_mod.interpolate(cells, kf, kt, src)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_interpolate_piecewise_not_global(oracle_mod):
    """A Q1 hat function (one interior node = 1) is piecewise trilinear: at
    the Q3 nodes it is the product of 1D hats, zero outside the 8 cells
    around the node."""
    cells, kf, kt = (4, 3, 3), 1, 3
    src = np.zeros((4, 4, 5))
    src[1, 2, 2] = 1.0  # z = 1, y = 2, x = 2
    got = oracle_mod.interpolate(cells, kf, kt, src.ravel()).reshape(10, 10, 13)
    tx, ty, tz = _node_coords(cells, kt, oracle_mod)
    hat = lambda t, c, N: np.maximum(0.0, 1.0 - np.abs(t * N - c))
    want = hat(tz, 1, 3)[:, None, None] * hat(ty, 2, 3)[None, :, None] * hat(tx, 2, 4)[None, None, :]
    assert np.abs(got - want).max() <= 1e-14
