"""Quadratic geometry evaluated in the operator kernel (Sec. 2.2: per cell
the map at 27 interpolation points instead of the stored tensor G_q)
against the oracle's quadratic-geometry operator, on k+1 and on k+2 Gauss
points per direction, for the Laplacian and the mass operator.

Checked: the GPU operator equals the oracle's CSR matrix (1e-12 relative,
componentwise within 1e-13 (|A| |u|)) on curved meshes with a rough
coefficient, every degree, several tiles with ragged tails, with and
without boundary condition; it differs from the exact-map operator; the
diagonal and the load vector; the fused Jacobi-CG solve, scalar and
vector (three components, BP4), against the oracle's Algorithm 1 (iteration
count within the oracle's summation-order range +-2, x within 1e-10); the
comparison solvers reach the same solution; the mass operator's BP1 and
BP2 solves; a coefficient update re-writes the per-cell values; combinations the
library does not offer are rejected.
"""
import numpy as np
import pytest

from paper_2205_08909_amd import inputs
from tests.test_gpu_solve import oracle_noise, torch_cuda  # noqa: F401

pytestmark = pytest.mark.gpu

CASES = [
    # (cells, k, map, bc, tile)
    ((8, 8, 8), 2, 1, 0, None),
    ((12, 12, 12), 4, 1, 0, None),
    ((5, 6, 7), 1, 2, 1, (3, 2, 3)),
    ((4, 5, 3), 3, 1, 0, (3, 2, 2)),
    ((3, 4, 5), 5, 2, 1, (2, 3, 2)),
    ((3, 3, 4), 6, 1, 0, (2, 2, 3)),
    ((3, 2, 3), 7, 1, 1, (2, 1, 2)),
    ((3, 3, 2), 8, 2, 0, (2, 1, 1)),
]


def _ids(c):
    return "x".join(map(str, c[0])) + f"-k{c[1]}-map{c[2]}-bc{c[3]}-t{c[4]}"


# with k+2 Gauss points per direction (the BP4 base case of the paper:
# quadratic geometry and (k+2)^3 points)
CASES_Q2 = [
    ((6, 5, 4), 2, 1, 0, (5, 3, 2)),
    ((10, 10, 10), 4, 1, 0, None),
    ((3, 4, 3), 5, 2, 1, (2, 3, 2)),
    ((3, 2, 3), 7, 1, 0, (2, 1, 2)),
]


def _setup(case, oracle_mod, coeff_seed=23, amp=0.08, kplus2=False, mass=False):
    from paper_2205_08909_amd import mfcg
    cells, k, kind, bc, tile = case
    coeff = inputs.grf_coefficient(cells, 0.3, 1.0, seed=coeff_seed)
    nq1 = k + 2 if kplus2 else None
    m = oracle_mod.Mesh(cells, k, nq1=nq1, map_kind=kind, amp=amp, bc=bc, coeff=coeff, geometry="quadratic",
                        op="mass" if mass else "laplace")
    P = mfcg.Problem(cells, k, coeff=coeff, map_kind=kind, amplitude=amp, bc=bc, tile=tile,
                     geometry=mfcg.GEOM_QUADRATIC, n_q_1d=nq1 or 0, op=mfcg.OP_MASS if mass else mfcg.OP_LAPLACE)
    return m, P


MASS_CASES = [(CASES[2], False), (CASES[4], False), (CASES_Q2[0], True), (CASES_Q2[2], True)]


@pytest.mark.parametrize("case,kplus2,mass",
                         [(c, False, False) for c in CASES] + [(c, True, False) for c in CASES_Q2] +
                         [(c, q, True) for c, q in MASS_CASES],
                         ids=[_ids(c) for c in CASES] + [_ids(c) + "-kplus2" for c in CASES_Q2] +
                         [_ids(c) + ("-kplus2" if q else "") + "-mass" for c, q in MASS_CASES])
def test_vmult_and_diagonal_match_oracle(case, kplus2, mass, oracle_mod, torch_cuda):
    torch = torch_cuda
    print("case", _ids(case), "k+2" if kplus2 else "", "mass" if mass else "", flush=True)
    m, P = _setup(case, oracle_mod, kplus2=kplus2, mass=mass)
    A = oracle_mod.assemble(m)
    assert P.n == A.n
    u = inputs.random_vector(A.n, seed=9)
    ref = A.matvec(u)
    scale = A.abs_matvec(u)
    src = torch.from_numpy(u).cuda()
    dst = torch.empty_like(src)
    P.vmult(dst, src)
    d = dst.cpu().numpy() - ref
    assert np.abs(d).max() <= 1e-12 * np.abs(ref).max()
    assert np.all(np.abs(d) <= 1e-13 * scale + 1e-300)
    np.testing.assert_allclose(P.diagonal().cpu().numpy(), A.diagonal(), rtol=1e-13, atol=0)
    P.close()


def test_differs_from_the_exact_map(oracle_mod, torch_cuda):
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    cells, k = (4, 4, 4), 3
    u = torch.from_numpy(inputs.random_vector((4 * 3 + 1) ** 3, seed=4)).cuda()
    out = []
    for geom in (mfcg.GEOM_STORED, mfcg.GEOM_QUADRATIC):
        P = mfcg.Problem(cells, k, map_kind=1, amplitude=0.1, bc=1, geometry=geom)
        out.append(P.vmult(P.empty(), u).cpu().numpy())
        P.close()
    ref = oracle_mod.assemble(oracle_mod.Mesh(cells, k, map_kind=1, amp=0.1, bc=1, geometry="quadratic")).matvec(
        u.cpu().numpy())
    assert np.abs(out[1] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(out[0] - ref).max() > 1e-6 * np.abs(ref).max()


def test_rhs_matches_oracle(oracle_mod, torch_cuda):
    from paper_2205_08909_amd import mfcg
    m, P = _setup(CASES[3], oracle_mod)
    b = P.rhs(mfcg.RHS_SINE).cpu().numpy()
    ref = oracle_mod.rhs(m, oracle_mod.F_SINE)
    assert np.abs(b - ref).max() <= 1e-13 * np.abs(ref).max()
    P.close()


@pytest.mark.parametrize("case", [CASES[1], CASES[3], CASES[5]], ids=_ids)
def test_solve_matches_oracle(case, oracle_mod, torch_cuda):
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    print("case", _ids(case), flush=True)
    m, P = _setup(case, oracle_mod)
    A = oracle_mod.assemble(m)
    cells, k = case[0], case[1]
    b = inputs.random_rhs(cells, k, seed=91, dirichlet=case[3] == 0)
    if case[3] == 1:  # no boundary condition: the singular Laplacian is solved on a consistent right-hand side
        b = b - b.mean()
    xo, its_o, _, rc_o = oracle_mod.pcg(A, A.diagonal(), b, tol=1e-10, maxit=5000)
    lo, hi, _ = oracle_noise(oracle_mod, A, b, nperm=2)
    bt = torch.from_numpy(b).cuda()
    xs = {}
    for solver in (mfcg.SOLVER_FUSED, mfcg.SOLVER_ALG5_SPLIT, mfcg.SOLVER_PCG_BASIC):
        P.set_solver(solver)
        xt = torch.zeros_like(bt)
        code, its, hist, tr = P.solve(bt, xt, tol=1e-10, maxit=5000, want_true_res=True)
        x = xt.cpu().numpy()
        print(_ids(case), "solver", solver, "its", its, "oracle", its_o, (lo, hi), "true res", tr)
        assert rc_o == 0 and code == mfcg.OK and lo - 2 <= its <= hi + 2
        assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo) and tr <= 2e-10
        xs[solver] = x
    P.close()


def test_coefficient_update(oracle_mod, torch_cuda):
    """mfcg_set_coefficient re-writes a_e in the per-cell array: the operator
    follows the new coefficient."""
    torch = torch_cuda
    case = CASES[3]
    m, P = _setup(case, oracle_mod)
    cells, k = case[0], case[1]
    c2 = inputs.grf_coefficient(cells, 0.3, 1.0, seed=77)
    P.set_coefficient(c2)
    m2 = oracle_mod.Mesh(cells, k, map_kind=case[2], amp=0.08, bc=case[3], coeff=c2, geometry="quadratic")
    A2 = oracle_mod.assemble(m2)
    u = inputs.random_vector(A2.n, seed=3)
    ref = A2.matvec(u)
    v = P.vmult(P.empty(), torch.from_numpy(u).cuda()).cpu().numpy()
    assert np.abs(v - ref).max() <= 1e-12 * np.abs(ref).max()
    np.testing.assert_allclose(P.diagonal().cpu().numpy(), A2.diagonal(), rtol=1e-13, atol=0)
    P.close()


@pytest.mark.parametrize("kplus2", [False, True], ids=["k+1", "k+2"])
def test_vector_solve_matches_oracle(kplus2, oracle_mod, torch_cuda):
    """The vector Laplacian with quadratic geometry, on k+1 and on k+2 Gauss
    points per direction (BP4 as the paper runs it): three components, one
    CG, against the block-diagonal oracle."""
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    from tests.test_gpu_vector import _block3
    case = CASES[3]
    m, P = _setup(case, oracle_mod, kplus2=kplus2)
    A = oracle_mod.assemble(m)
    cells, k = case[0], case[1]
    A3 = _block3(A)
    d3 = np.tile(A.diagonal(), 3)
    b3 = np.concatenate([inputs.random_rhs(cells, k, seed=95 + c) for c in range(3)])
    xo3, its_o3, _, rc_o3 = oracle_mod.pcg(A3, d3, b3, tol=1e-10, maxit=5000)
    lo3, hi3, _ = oracle_noise(oracle_mod, A3, b3, nperm=2, diag=d3)
    bt3 = torch.from_numpy(b3).cuda()
    xt3 = torch.zeros_like(bt3)
    code3, its3, _, tr3 = P.solve_vector(bt3, xt3, tol=1e-10, maxit=5000, want_true_res=True)
    x3 = xt3.cpu().numpy()
    print("vector its", its3, "oracle", its_o3, (lo3, hi3), "true res", tr3)
    assert rc_o3 == 0 and code3 == mfcg.OK and lo3 - 2 <= its3 <= hi3 + 2
    assert np.linalg.norm(x3 - xo3) <= 1e-10 * np.linalg.norm(xo3) and tr3 <= 2e-10
    P.close()


@pytest.mark.parametrize("kplus2", [False, True], ids=["k+1", "k+2"])
def test_mass_solves_match_oracle(kplus2, oracle_mod, torch_cuda):
    """BP1 (scalar) and BP2 (three components) with quadratic geometry."""
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    from tests.test_gpu_vector import _block3
    case = CASES_Q2[0]
    m, P = _setup(case, oracle_mod, kplus2=kplus2, mass=True)
    A = oracle_mod.assemble(m)
    cells, k = case[0], case[1]
    b = inputs.random_rhs(cells, k, seed=97)
    xo, its_o, _, rc_o = oracle_mod.pcg(A, A.diagonal(), b, tol=1e-10, maxit=2000)
    lo, hi, _ = oracle_noise(oracle_mod, A, b, nperm=2)
    bt = torch.from_numpy(b).cuda()
    xt = torch.zeros_like(bt)
    code, its, _, tr = P.solve(bt, xt, tol=1e-10, maxit=2000, want_true_res=True)
    print("BP1 its", its, "oracle", its_o, (lo, hi), "true res", tr)
    assert rc_o == 0 and code == mfcg.OK and lo - 2 <= its <= hi + 2
    assert np.linalg.norm(xt.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo) and tr <= 2e-10
    A3 = _block3(A)
    d3 = np.tile(A.diagonal(), 3)
    b3 = np.concatenate([inputs.random_rhs(cells, k, seed=98 + c) for c in range(3)])
    xo3, its_o3, _, rc_o3 = oracle_mod.pcg(A3, d3, b3, tol=1e-10, maxit=2000)
    lo3, hi3, _ = oracle_noise(oracle_mod, A3, b3, nperm=2, diag=d3)
    bt3 = torch.from_numpy(b3).cuda()
    xt3 = torch.zeros_like(bt3)
    code3, its3, _, tr3 = P.solve_vector(bt3, xt3, tol=1e-10, maxit=2000, want_true_res=True)
    print("BP2 its", its3, "oracle", its_o3, (lo3, hi3), "true res", tr3)
    assert rc_o3 == 0 and code3 == mfcg.OK and lo3 - 2 <= its3 <= hi3 + 2
    assert np.linalg.norm(xt3.cpu().numpy() - xo3) <= 1e-10 * np.linalg.norm(xo3) and tr3 <= 2e-10
    P.close()


def test_unsupported_combinations_rejected(torch_cuda):
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    G = mfcg.GEOM_QUADRATIC
    for kw in (dict(quad=mfcg.QUAD_GLL), dict(n_q_1d=6)):
        with pytest.raises(mfcg.MfcgError):
            mfcg.Problem((4, 4, 4), 3, geometry=G, **kw)
    with pytest.raises(mfcg.MfcgError):
        mfcg.Problem((4, 4, 4), 3, geometry=2)
    P = mfcg.Problem((4, 4, 4), 3, map_kind=1, amplitude=0.05, geometry=G)
    b = P.rhs()
    x = torch.zeros_like(b)
    code, *_ = P.solve_ir(b, x, raise_on=False)
    assert code == mfcg.EINVAL
    P.close()
