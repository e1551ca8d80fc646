"""The mass operator (the BP1/BP2 variations of Sec. 6) against the
oracle's brute-force mass matrix (a_e w_q det J_q phi_i phi_j on the Gauss
points).

Checked: the GPU operator equals the oracle's CSR matrix (1e-12 relative,
componentwise within 1e-13 (|M| |u|)) on curved meshes with a rough
coefficient, several tiles with ragged tails, every degree, with and
without boundary condition; the diagonal; the fused Jacobi-CG solve of the
scalar problem (BP1) and of the three-component problem (BP2, through the
vector solve) against the oracle's Algorithm 1 (iteration count within the
oracle's summation-order range +-2, x within 1e-10); combinations the
library does not offer are rejected.
"""
import numpy as np
import pytest

from paper_2205_08909_amd import inputs
from tests.test_gpu_solve import oracle_noise, torch_cuda  # noqa: F401
from tests.test_gpu_vector import _block3

pytestmark = pytest.mark.gpu

CASES = [
    # (cells, k, map, bc, tile)
    ((8, 8, 8), 2, 1, 1, None),
    ((12, 12, 12), 4, 1, 0, None),
    ((5, 6, 7), 1, 2, 1, (3, 2, 3)),
    ((4, 5, 3), 3, 1, 0, (3, 2, 2)),
    ((3, 4, 5), 5, 1, 1, (2, 3, 2)),
    ((3, 3, 4), 6, 2, 0, (2, 2, 3)),
    ((3, 2, 3), 7, 1, 1, (2, 1, 2)),
    ((3, 3, 2), 8, 1, 0, (2, 1, 1)),
]


def _ids(c):
    return "x".join(map(str, c[0])) + f"-k{c[1]}-map{c[2]}-bc{c[3]}-t{c[4]}"


def _setup(case, oracle_mod):
    from paper_2205_08909_amd import mfcg
    cells, k, kind, bc, tile = case
    coeff = inputs.grf_coefficient(cells, 0.3, 1.0, seed=13)
    m = oracle_mod.Mesh(cells, k, map_kind=kind, amp=0.05, bc=bc, coeff=coeff, op="mass")
    P = mfcg.Problem(cells, k, coeff=coeff, map_kind=kind, amplitude=0.05, bc=bc, tile=tile, op=mfcg.OP_MASS)
    return m, P


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_mass_vmult_and_diagonal(case, oracle_mod, torch_cuda):
    torch = torch_cuda
    m, P = _setup(case, oracle_mod)
    A = oracle_mod.assemble(m)
    u = inputs.random_vector(A.n, seed=7)
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


@pytest.mark.parametrize("case", [CASES[0], CASES[1], CASES[4]], ids=_ids)
def test_mass_solves_match_oracle(case, oracle_mod, torch_cuda):
    """BP1 (scalar) and BP2 (three components) with the Jacobi preconditioner."""
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    m, P = _setup(case, oracle_mod)
    A = oracle_mod.assemble(m)
    cells, k = case[0], case[1]
    b = inputs.random_rhs(cells, k, seed=51, dirichlet=case[3] == 0)
    xo, its_o, _, rc_o = oracle_mod.pcg(A, A.diagonal(), b, tol=1e-10, maxit=2000)
    lo, hi, _ = oracle_noise(oracle_mod, A, b, nperm=2)
    bt = torch.from_numpy(b).cuda()
    xt = torch.zeros_like(bt)
    code, its, hist, tr = P.solve(bt, xt, tol=1e-10, maxit=2000, want_true_res=True)
    x = xt.cpu().numpy()
    print(case, "BP1 its", its, "oracle", its_o, (lo, hi), "true res", tr)
    assert rc_o == 0 and code == mfcg.OK and lo - 2 <= its <= hi + 2
    assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo) and tr <= 2e-10
    # BP2: the vector mass problem
    A3 = _block3(A)
    d3 = np.tile(A.diagonal(), 3)
    b3 = np.concatenate([inputs.random_rhs(cells, k, seed=60 + c, dirichlet=case[3] == 0) for c in range(3)])
    xo3, its_o3, _, rc_o3 = oracle_mod.pcg(A3, d3, b3, tol=1e-10, maxit=2000)
    lo3, hi3, _ = oracle_noise(oracle_mod, A3, b3, nperm=2, diag=d3)
    bt3 = torch.from_numpy(b3).cuda()
    xt3 = torch.zeros_like(bt3)
    code3, its3, _, tr3 = P.solve_vector(bt3, xt3, tol=1e-10, maxit=2000, want_true_res=True)
    x3 = xt3.cpu().numpy()
    print(case, "BP2 its", its3, "oracle", its_o3, (lo3, hi3), "true res", tr3)
    assert rc_o3 == 0 and code3 == mfcg.OK and lo3 - 2 <= its3 <= hi3 + 2
    assert np.linalg.norm(x3 - xo3) <= 1e-10 * np.linalg.norm(xo3) and tr3 <= 2e-10
    P.close()


def test_mass_rejects_unsupported_combinations(torch_cuda):
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    with pytest.raises(mfcg.MfcgError):
        mfcg.Problem((4, 4, 4), 3, op=mfcg.OP_MASS, quad=mfcg.QUAD_GLL)
    with pytest.raises(mfcg.MfcgError):
        mfcg.Problem((4, 4, 4), 3, op=5)
    P = mfcg.Problem((4, 4, 4), 3, map_kind=1, amplitude=0.05, op=mfcg.OP_MASS)
    b = P.rhs()
    x = torch.zeros_like(b)
    code, *_ = P.solve_ir(b, x, raise_on=False)
    assert code == mfcg.EINVAL
    P.close()
