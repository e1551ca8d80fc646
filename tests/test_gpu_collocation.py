"""GLL collocation (quadrature on the k+1 nodes per direction, the BP5
variation of Sec. 6) against the oracle's Gauss-Lobatto operator.

Checked: the GPU operator equals the oracle's CSR matrix assembled with the
GLL rule (1e-12 relative, componentwise within 1e-13 (|A| |u|)), on curved
meshes, several tiles with ragged tails, every degree; the diagonal and the
load vector; the fused solve against the oracle's Algorithm 1 (iteration
count within the oracle's summation-order range +-2, x within 1e-10); the
comparison solvers reach the same solution; mixed precision and batches,
which only exist for Gauss quadrature, reject such a handle.
"""
import numpy as np
import pytest

from paper_2205_08909_amd import inputs
from tests.test_gpu_solve import oracle_noise, torch_cuda  # noqa: F401

pytestmark = pytest.mark.gpu

CASES = [
    # (cells, k, map, tile, coeff)
    ((8, 8, 8), 2, 0, None, False),
    ((12, 12, 12), 4, 1, None, True),
    ((5, 6, 7), 1, 1, (3, 2, 3), True),
    ((4, 5, 3), 3, 1, (3, 2, 2), True),
    ((3, 4, 5), 5, 2, (2, 3, 2), True),
    ((3, 3, 4), 6, 1, (2, 2, 3), True),
    ((3, 2, 3), 7, 1, (2, 1, 2), True),
    ((3, 3, 2), 8, 1, (2, 1, 1), True),
]


def _ids(c):
    return "x".join(map(str, c[0])) + f"-k{c[1]}-map{c[2]}-t{c[3]}"


def _setup(case, oracle_mod):
    from paper_2205_08909_amd import mfcg
    cells, k, kind, tile, use_coeff = case
    coeff = inputs.grf_coefficient(cells, 0.3, 1.0, seed=12) if use_coeff else None
    m = oracle_mod.Mesh(cells, k, map_kind=kind, amp=0.05, coeff=coeff, quad="gll")
    P = mfcg.Problem(cells, k, coeff=coeff, map_kind=kind, amplitude=0.05, tile=tile, quad=mfcg.QUAD_GLL)
    return m, P


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_vmult_matches_oracle(case, oracle_mod, torch_cuda):
    torch = torch_cuda
    m, P = _setup(case, oracle_mod)
    A = oracle_mod.assemble(m)
    u = inputs.random_vector(A.n, seed=6)
    ref = A.matvec(u)
    scale = A.abs_matvec(u)
    src = torch.from_numpy(u).cuda()
    dst = torch.empty_like(src)
    P.vmult(dst, src)
    d = dst.cpu().numpy() - ref
    assert np.abs(d).max() <= 1e-12 * np.abs(ref).max()
    assert np.all(np.abs(d) <= 1e-13 * scale + 1e-300)
    P.close()


@pytest.mark.parametrize("case", [CASES[1], CASES[4]], ids=_ids)
def test_diagonal_and_rhs_match_oracle(case, oracle_mod, torch_cuda):
    from paper_2205_08909_amd import mfcg
    m, P = _setup(case, oracle_mod)
    A = oracle_mod.assemble(m)
    np.testing.assert_allclose(P.diagonal().cpu().numpy(), A.diagonal(), rtol=1e-13, atol=0)
    b = P.rhs(mfcg.RHS_SINE).cpu().numpy()
    ref = oracle_mod.rhs(m, oracle_mod.F_SINE)
    assert np.abs(b - ref).max() <= 1e-13 * np.abs(ref).max()
    P.close()


@pytest.mark.parametrize("case", [CASES[1], CASES[3], CASES[5]], ids=_ids)
def test_solve_matches_oracle(case, oracle_mod, torch_cuda):
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    m, P = _setup(case, oracle_mod)
    A = oracle_mod.assemble(m)
    b = oracle_mod.rhs(m, oracle_mod.F_SINE)
    xo, its_o, hist_o, rc_o = oracle_mod.pcg(A, A.diagonal(), b, tol=1e-10, maxit=5000)
    lo, hi, _ = oracle_noise(oracle_mod, A, b, nperm=2)
    bt = torch.from_numpy(b).cuda()
    xs = {}
    for solver in (mfcg.SOLVER_FUSED, mfcg.SOLVER_ALG5_SPLIT, mfcg.SOLVER_PCG_BASIC):
        P.set_solver(solver)
        xt = torch.zeros_like(bt)
        code, its, hist, tr = P.solve(bt, xt, tol=1e-10, maxit=5000, want_true_res=True)
        x = xt.cpu().numpy()
        print(case[0], case[1], "solver", solver, "its", its, "oracle", its_o, (lo, hi), "true res", tr)
        assert rc_o == 0 and code == mfcg.OK
        assert lo - 2 <= its <= hi + 2
        assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo)
        assert tr <= 2e-10
        xs[solver] = x
    P.close()


def test_gauss_only_paths_reject_collocation(torch_cuda):
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    P = mfcg.Problem((4, 4, 4), 3, map_kind=1, amplitude=0.05, quad=mfcg.QUAD_GLL)
    b = P.rhs()
    x = torch.zeros_like(b)
    code, *_ = P.solve_ir(b, x, raise_on=False)
    assert code == mfcg.EINVAL
    P.close()
    with pytest.raises(mfcg.MfcgError):
        mfcg.Problem((4, 4, 4), 3, quad=7)
