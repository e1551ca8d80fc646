"""The vector Laplacian (three uncoupled components, the paper's BP4 family)
against the oracle: Algorithm 1 with the Jacobi preconditioner on the
block-diagonal matrix I_3 (x) A assembled from the oracle's scalar matrix.

Checked: iteration count within the oracle's own summation-order range
(+-2), converged x within 1e-10 relative, true residual below 2e-10 ||b||,
the first residual norms to rounding; with one non-zero component the
vector solve reproduces the scalar solve of that component bitwise (the
other components contribute exact zeros to every inner product); a zero
right-hand side; iteration limits of both exit parities.  (For a non-zero
component 1 or 2 its records sit at other offsets of the fixed-order finish,
so there the agreement is to rounding.)
"""
import numpy as np
import pytest

from paper_2205_08909_amd import inputs
from tests.test_gpu_solve import _problem, oracle_noise, torch_cuda  # noqa: F401

pytestmark = pytest.mark.gpu


def _block3(A):
    import scipy.sparse as sp
    from oracle.oracle import CSR
    S = sp.block_diag([A.to_scipy()] * 3, format="csr")
    S.sort_indices()
    return CSR(S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data.copy())


def _rhs3(cells, k, seed):
    return np.concatenate([inputs.random_rhs(cells, k, seed=seed + c) for c in range(3)])


@pytest.mark.parametrize("cells,k,coeff_seed,tile", [
    ((6, 7, 5), 3, 4, (2, 3, 2)),
    ((8, 8, 8), 2, None, None),
    ((4, 4, 4), 5, 2, (2, 2, 2)),
])
def test_vector_solve_matches_oracle(cells, k, coeff_seed, tile, oracle_mod, torch_cuda):
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    m, A, P = _problem(oracle_mod, cells, k, 1, 0.05, coeff_seed, tile)
    A3 = _block3(A)
    d3 = np.tile(A.diagonal(), 3)
    b = _rhs3(cells, k, 20)
    xo, its_o, hist_o, rc_o = oracle_mod.pcg(A3, d3, b, tol=1e-10, maxit=5000)
    lo, hi, floor = oracle_noise(oracle_mod, A3, b, nperm=2, diag=d3)
    bt = torch.from_numpy(b).cuda()
    xt = torch.zeros_like(bt)
    code, its, hist, tr = P.solve_vector(bt, xt, tol=1e-10, maxit=5000, want_true_res=True)
    x = xt.cpu().numpy()
    print(cells, k, "vector its", its, "oracle", its_o, (lo, hi), "true res", tr)
    assert rc_o == 0 and code == mfcg.OK
    assert lo - 2 <= its <= hi + 2
    assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo)
    nb = np.linalg.norm(b)
    e = min(its, its_o, 5)
    assert np.abs(hist[:e + 1] - hist_o[:e + 1]).max() <= 1e-12 * max(nb, hist_o[:e + 1].max())
    assert tr <= 2e-10
    assert np.linalg.norm(b - A3.matvec(x)) <= 2e-10 * nb
    P.close()


def test_single_component_is_the_scalar_solve(oracle_mod, torch_cuda):
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    cells, k = (5, 6, 4), 4
    m, A, P = _problem(oracle_mod, cells, k, 1, 0.05, 3, (2, 2, 2))
    n = P.n
    b1 = inputs.random_rhs(cells, k, seed=31)
    for c in range(3):
        b = np.zeros(3 * n)
        b[c * n:(c + 1) * n] = b1
        bt = torch.from_numpy(b).cuda()
        xt = torch.zeros_like(bt)
        code, its, hist, _ = P.solve_vector(bt, xt, tol=1e-10, maxit=5000)
        x1 = torch.zeros(n, dtype=torch.float64, device="cuda")
        code1, its1, hist1, _ = P.solve(torch.from_numpy(b1).cuda(), x1, tol=1e-10, maxit=5000)
        x = xt.cpu().numpy()
        xs = x1.cpu().numpy()
        assert code == code1 == mfcg.OK
        assert not np.delete(x, np.s_[c * n:(c + 1) * n]).any()
        if c == 0:
            # the zero records of components 1 and 2 come after component 0's
            # in the fixed-order finish: every sum is the scalar one plus zeros
            assert its == its1 and np.array_equal(hist, hist1)
            assert np.array_equal(x[:n], xs)
        else:
            # the records sit at other offsets, so the finish groups the sums
            # differently: agreement to rounding
            assert abs(its - its1) <= 2
            assert np.linalg.norm(x[c * n:(c + 1) * n] - xs) <= 1e-10 * np.linalg.norm(xs)
    P.close()


def test_vector_edge_cases(oracle_mod, torch_cuda):
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    cells, k = (4, 5, 3), 3
    m, A, P = _problem(oracle_mod, cells, k, 1, 0.05, 5, (2, 2, 2))
    A3 = _block3(A)
    d3 = np.tile(A.diagonal(), 3)
    n = P.n
    bt = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
    xt = torch.ones_like(bt)
    code, its, hist, tr = P.solve_vector(bt, xt, tol=1e-10, maxit=10, want_true_res=True)
    assert code == mfcg.OK and its == 0 and not xt.any().item() and tr == 0.0
    b = _rhs3(cells, k, 40)
    bt = torch.from_numpy(b).cuda()
    for maxit in (3, 4):
        xo, its_o, hist_o, rc_o = oracle_mod.pcg(A3, d3, b, tol=1e-14, maxit=maxit)
        xt = torch.zeros_like(bt)
        code, its, hist, _ = P.solve_vector(bt, xt, tol=1e-14, maxit=maxit)
        assert code == mfcg.ENOTCONV and its == maxit and rc_o == -4
        assert np.linalg.norm(xt.cpu().numpy() - xo) <= 1e-12 * np.linalg.norm(xo)
        assert np.abs(hist - hist_o).max() <= 1e-12 * np.linalg.norm(b)
    with pytest.raises(ValueError):
        P.solve_vector(torch.zeros(n, dtype=torch.float64, device="cuda"), torch.zeros(n, dtype=torch.float64,
                                                                                         device="cuda"))
    P.close()


def test_vector_solve_with_collocation(oracle_mod, torch_cuda):
    """The vector problem on a GLL-collocation handle (the one-launch kernel's
    collocation variant) against the block-diagonal oracle."""
    torch = torch_cuda
    from paper_2205_08909_amd import mfcg
    cells, k = (5, 4, 6), 3
    coeff = inputs.grf_coefficient(cells, 0.1, 1.0, seed=8)
    m = oracle_mod.Mesh(cells, k, map_kind=1, amp=0.05, coeff=coeff, quad="gll")
    A = oracle_mod.assemble(m)
    P = mfcg.Problem(cells, k, coeff=coeff, map_kind=1, amplitude=0.05, tile=(2, 3, 2), quad=mfcg.QUAD_GLL)
    A3 = _block3(A)
    d3 = np.tile(A.diagonal(), 3)
    b = _rhs3(cells, k, 70)
    xo, its_o, _, rc_o = oracle_mod.pcg(A3, d3, b, tol=1e-10, maxit=5000)
    lo, hi, _ = oracle_noise(oracle_mod, A3, b, nperm=2, diag=d3)
    bt = torch.from_numpy(b).cuda()
    xt = torch.zeros_like(bt)
    code, its, hist, tr = P.solve_vector(bt, xt, tol=1e-10, maxit=5000, want_true_res=True)
    x = xt.cpu().numpy()
    print("GLL vector its", its, "oracle", its_o, (lo, hi), "true res", tr)
    assert rc_o == 0 and code == mfcg.OK and lo - 2 <= its <= hi + 2
    assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo) and tr <= 2e-10
    P.close()

