"""k+2 Gauss points per direction (the n_q = (k+2)^3 rule of the BP1-BP4
benchmarks of Sec. 6) against the oracle assembled with the same rule.

Checked: the GPU operator equals the oracle's CSR matrix (1e-12 relative,
componentwise within 1e-13 (|A| |u|)) for the Laplacian and the mass
operator, curved meshes with a rough coefficient, every degree 1..7,
several tiles with ragged tails, with and without boundary condition; the
diagonal and the load vector; the fused Jacobi-CG solve (scalar: BP3 / BP1)
and the vector solve (three components: BP4 / BP2) against the oracle's
Algorithm 1 (iteration count within the oracle's summation-order range
+-2, x within 1e-10); the comparison solvers reach the same solution;
combinations the library does not offer are rejected.
"""
import numpy as np
import pytest

from paper_2205_08909_amd import inputs
from tests.test_gpu_solve import oracle_noise, torch_cuda  # noqa: F401
from tests.test_gpu_vector import _block3

pytestmark = pytest.mark.gpu

CASES = [
    # (cells, k, map, bc, tile, op)
    ((8, 8, 8), 2, 1, 0, None, "laplace"),
    ((10, 10, 10), 4, 1, 0, None, "laplace"),
    ((5, 6, 7), 1, 2, 1, (3, 2, 3), "laplace"),
    ((4, 5, 3), 3, 1, 0, (3, 2, 2), "laplace"),
    ((3, 4, 5), 5, 1, 1, (2, 3, 2), "laplace"),
    ((3, 3, 4), 6, 2, 0, (2, 2, 3), "laplace"),
    ((3, 2, 3), 7, 1, 1, (2, 1, 2), "laplace"),
    ((4, 5, 3), 4, 1, 1, (3, 2, 2), "mass"),
    ((6, 5, 4), 2, 2, 0, (5, 3, 2), "mass"),
    ((3, 3, 2), 7, 1, 0, (2, 2, 1), "mass"),
]


def _ids(c):
    return "x".join(map(str, c[0])) + f"-k{c[1]}-map{c[2]}-bc{c[3]}-t{c[4]}-{c[5]}"


def _setup(case, oracle_mod, coeff_seed=17):
    from paper_2205_08909_amd import mfcg
    cells, k, kind, bc, tile, op = case
    coeff = inputs.grf_coefficient(cells, 0.3, 1.0, seed=coeff_seed)
    m = oracle_mod.Mesh(cells, k, nq1=k + 2, map_kind=kind, amp=0.05, bc=bc, coeff=coeff, op=op)
    P = mfcg.Problem(cells, k, coeff=coeff, map_kind=kind, amplitude=0.05, bc=bc, tile=tile, n_q_1d=k + 2,
                     op=mfcg.OP_MASS if op == "mass" else mfcg.OP_LAPLACE)
    return m, P


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_vmult_and_diagonal_match_oracle(case, oracle_mod, torch_cuda):
    torch = torch_cuda
    print("case", _ids(case), flush=True)
    m, P = _setup(case, oracle_mod)
    A = oracle_mod.assemble(m)
    assert P.n == A.n
    u = inputs.random_vector(A.n, seed=5)
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


def test_differs_from_kplus1_rule(oracle_mod, torch_cuda):
    """On a curved mesh the two rules give different operators: the k+2
    handle must not silently run the k+1 kernel."""
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    cells, k = (4, 4, 4), 3
    u = torch.from_numpy(inputs.random_vector((4 * 3 + 1) ** 3, seed=2)).cuda()
    out = []
    for nq in (k + 1, k + 2):
        P = mfcg.Problem(cells, k, map_kind=1, amplitude=0.1, bc=1, n_q_1d=nq)
        out.append(P.vmult(P.empty(), u).cpu().numpy())
        P.close()
    m2 = oracle_mod.Mesh(cells, k, nq1=k + 2, map_kind=1, amp=0.1, bc=1)
    ref = oracle_mod.assemble(m2).matvec(u.cpu().numpy())
    assert np.abs(out[1] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(out[0] - ref).max() > 1e-9 * np.abs(ref).max()


def test_rhs_matches_oracle(oracle_mod, torch_cuda):
    from paper_2205_08909_amd import mfcg
    m, P = _setup(CASES[3], oracle_mod)
    b = P.rhs(mfcg.RHS_SINE).cpu().numpy()
    ref = oracle_mod.rhs(m, oracle_mod.F_SINE)
    assert np.abs(b - ref).max() <= 1e-13 * np.abs(ref).max()
    P.close()


@pytest.mark.parametrize("case", [CASES[1], CASES[3], CASES[5], CASES[7]], ids=_ids)
def test_scalar_solve_matches_oracle(case, oracle_mod, torch_cuda):
    """BP3 (Laplacian) / BP1 (mass) with the Jacobi preconditioner."""
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    print("case", _ids(case), flush=True)
    m, P = _setup(case, oracle_mod)
    A = oracle_mod.assemble(m)
    cells, k = case[0], case[1]
    b = inputs.random_rhs(cells, k, seed=71, dirichlet=case[3] == 0)
    xo, its_o, _, rc_o = oracle_mod.pcg(A, A.diagonal(), b, tol=1e-10, maxit=5000)
    lo, hi, _ = oracle_noise(oracle_mod, A, b, nperm=2)
    bt = torch.from_numpy(b).cuda()
    xt = torch.zeros_like(bt)
    code, its, hist, tr = P.solve(bt, xt, tol=1e-10, maxit=5000, want_true_res=True)
    x = xt.cpu().numpy()
    print(_ids(case), "its", its, "oracle", its_o, (lo, hi), "true res", tr)
    assert rc_o == 0 and code == mfcg.OK and lo - 2 <= its <= hi + 2
    assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo) and tr <= 2e-10
    P.close()


@pytest.mark.parametrize("case", [CASES[3], CASES[8]], ids=_ids)
def test_vector_solve_matches_oracle(case, oracle_mod, torch_cuda):
    """BP4 (vector Laplacian) / BP2 (vector mass): three components sharing
    the geometry tensor, against the block-diagonal oracle."""
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    print("case", _ids(case), flush=True)
    m, P = _setup(case, oracle_mod)
    A = oracle_mod.assemble(m)
    cells, k = case[0], case[1]
    A3 = _block3(A)
    d3 = np.tile(A.diagonal(), 3)
    b3 = np.concatenate([inputs.random_rhs(cells, k, seed=80 + c, dirichlet=case[3] == 0) for c in range(3)])
    xo3, its_o3, _, rc_o3 = oracle_mod.pcg(A3, d3, b3, tol=1e-10, maxit=5000)
    lo3, hi3, _ = oracle_noise(oracle_mod, A3, b3, nperm=2, diag=d3)
    bt3 = torch.from_numpy(b3).cuda()
    xt3 = torch.zeros_like(bt3)
    code3, its3, _, tr3 = P.solve_vector(bt3, xt3, tol=1e-10, maxit=5000, want_true_res=True)
    x3 = xt3.cpu().numpy()
    print(_ids(case), "vector its", its3, "oracle", its_o3, (lo3, hi3), "true res", tr3)
    assert rc_o3 == 0 and code3 == mfcg.OK and lo3 - 2 <= its3 <= hi3 + 2
    assert np.linalg.norm(x3 - xo3) <= 1e-10 * np.linalg.norm(xo3) and tr3 <= 2e-10
    P.close()


def test_comparison_solvers_reach_the_oracle_solution(oracle_mod, torch_cuda):
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    case = CASES[3]
    m, P = _setup(case, oracle_mod)
    A = oracle_mod.assemble(m)
    b = inputs.random_rhs(case[0], case[1], seed=72)
    xo, its_o, _, rc_o = oracle_mod.pcg(A, A.diagonal(), b, tol=1e-10, maxit=5000)
    bt = torch.from_numpy(b).cuda()
    for solver in (mfcg.SOLVER_ALG5_SPLIT, mfcg.SOLVER_PCG_BASIC, mfcg.SOLVER_PIPELINED):
        P.set_solver(solver)
        xt = torch.zeros_like(bt)
        code, its, _, tr = P.solve(bt, xt, tol=1e-10, maxit=5000, want_true_res=True)
        print("solver", solver, "its", its, "oracle", its_o, "true res", tr)
        assert code == mfcg.OK
        assert np.linalg.norm(xt.cpu().numpy() - xo) <= 1e-9 * np.linalg.norm(xo)
    P.set_solver(mfcg.SOLVER_FUSED)
    P.set_preconditioner(mfcg.PRECOND_NONE)
    xo1, _, _, _ = oracle_mod.pcg(A, np.ones(A.n), b, tol=1e-10, maxit=5000)
    xt = torch.zeros_like(bt)
    code, its, _, _ = P.solve(bt, xt, tol=1e-10, maxit=5000)
    assert code == mfcg.OK
    assert np.linalg.norm(xt.cpu().numpy() - xo1) <= 1e-9 * np.linalg.norm(xo1)
    P.close()


def test_unsupported_combinations_rejected(torch_cuda):
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    for kw in (dict(degree=8, n_q_1d=10), dict(degree=3, n_q_1d=5, quad=mfcg.QUAD_GLL), dict(degree=3, n_q_1d=6),
               dict(degree=3, n_q_1d=3)):
        d = kw.pop("degree")
        with pytest.raises(mfcg.MfcgError):
            mfcg.Problem((4, 4, 4), d, **kw)
    P = mfcg.Problem((4, 4, 4), 3, map_kind=1, amplitude=0.05, n_q_1d=5)
    b = P.rhs()
    x = torch.zeros_like(b)
    code, *_ = P.solve_ir(b, x, raise_on=False)
    assert code == mfcg.EINVAL
    P.close()
