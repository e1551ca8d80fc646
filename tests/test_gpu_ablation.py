"""The comparison solvers (Algorithm 5 in three passes, basic Algorithm 1)
against the oracle and against the fused solver, with the Jacobi
preconditioner and without one (M = I: the fused and split solvers then run
Algorithm 4, the basic one textbook CG; the oracle runs Algorithm 1 with a
unit diagonal).

All three produce the same iterates in exact arithmetic.  Checked: each
solver's iteration count lies within the oracle's own summation-order range
(+-2), its converged x agrees with the oracle's to 1e-10 relative and its
residual in the oracle's matrix is below 2e-10 ||b||; the two Algorithm 5
variants differ only in the order of the inner-product sums, so their
solutions agree to within 1e-10 relative as well; the basic solver's first
residual norms agree with the oracle's Algorithm 1 history to rounding.
"""
import numpy as np
import pytest

from paper_2205_08909_amd import inputs

from tests.test_gpu_solve import oracle_noise

pytestmark = pytest.mark.gpu

CASES = [
    ((8, 8, 8), 2, 0, None, None),
    ((12, 12, 12), 4, 1, 3, None),
    ((6, 7, 5), 3, 1, 4, (2, 3, 2)),
]


@pytest.mark.parametrize("precond", [0, 1])
@pytest.mark.parametrize("cells,k,kind,coeff_seed,tile", CASES)
def test_comparison_solvers(cells, k, kind, coeff_seed, tile, precond, oracle_mod):
    import torch
    from paper_2205_08909_amd import mfcg
    coeff = inputs.grf_coefficient(cells, 0.1, 1.0, seed=coeff_seed) if coeff_seed is not None else None
    m = oracle_mod.Mesh(cells, k, map_kind=kind, amp=0.05, coeff=coeff)
    A = oracle_mod.assemble(m)
    b = oracle_mod.rhs(m, oracle_mod.F_SINE)
    d = A.diagonal() if precond == mfcg.PRECOND_JACOBI else np.ones(A.n)
    xo, its_o, hist_o, _ = oracle_mod.pcg(A, d, b, tol=1e-10, maxit=5000)
    lo, hi, _ = oracle_noise(oracle_mod, A, b, diag=d)
    P = mfcg.Problem(cells, k, coeff=coeff, map_kind=kind, amplitude=0.05, tile=tile)
    P.set_preconditioner(precond)
    bt = torch.from_numpy(b).cuda()
    xs = {}
    for solver in (mfcg.SOLVER_FUSED, mfcg.SOLVER_ALG5_SPLIT, mfcg.SOLVER_PCG_BASIC):
        P.set_solver(solver)
        xt = torch.zeros_like(bt)
        code, its, hist, tr = P.solve(bt, xt, tol=1e-10, maxit=5000, want_true_res=True)
        x = xt.cpu().numpy()
        xs[solver] = x
        err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
        res = np.linalg.norm(b - A.matvec(x)) / np.linalg.norm(b)
        print(f"precond {precond} solver {solver}: its {its} (oracle {its_o}, range {lo}..{hi}), x err {err:.2e}, oracle res {res:.2e}")
        assert code == mfcg.OK
        assert lo - 2 <= its <= hi + 2
        assert err <= 1e-10
        assert res <= 2e-10
        assert tr <= 2e-10
        if solver == mfcg.SOLVER_PCG_BASIC:
            j = min(5, its, its_o)
            scale = np.maximum(hist_o[:j + 1], 1e-300)
            assert np.all(np.abs(hist[:j + 1] - hist_o[:j + 1]) <= 1e-12 * np.maximum(scale, hist_o[0]))
    split = np.linalg.norm(xs[mfcg.SOLVER_ALG5_SPLIT] - xs[mfcg.SOLVER_FUSED]) / np.linalg.norm(xs[mfcg.SOLVER_FUSED])
    print(f"fused vs split: {split:.2e}")
    assert split <= 1e-10
    P.close()


@pytest.mark.parametrize("precond", [0, 1])
def test_comparison_solvers_fixed_iterations(precond, oracle_mod):
    """tol = 0: exactly maxit iterations, both exit parities, ENOTCONV
    (without preconditioner also for the fused solver: its exit
    reconstruction of x then takes a unit diagonal)."""
    import torch
    from paper_2205_08909_amd import mfcg
    cells, k = (6, 6, 6), 3
    m = oracle_mod.Mesh(cells, k, map_kind=1, amp=0.05)
    A = oracle_mod.assemble(m)
    b = oracle_mod.rhs(m, oracle_mod.F_SINE)
    P = mfcg.Problem(cells, k, map_kind=1, amplitude=0.05)
    P.set_preconditioner(precond)
    d = A.diagonal() if precond == mfcg.PRECOND_JACOBI else np.ones(A.n)
    bt = torch.from_numpy(b).cuda()
    solvers = (mfcg.SOLVER_ALG5_SPLIT, mfcg.SOLVER_PCG_BASIC)
    if precond == mfcg.PRECOND_NONE:
        solvers = (mfcg.SOLVER_FUSED,) + solvers
    for maxit in (1, 2, 5, 8):
        xo, its_o, _, _ = oracle_mod.pcg(A, d, b, tol=0.0, maxit=maxit)
        for solver in solvers:
            P.set_solver(solver)
            xt = torch.zeros_like(bt)
            code, its, _, _ = P.solve(bt, xt, tol=0.0, maxit=maxit, raise_on=False)
            assert code == mfcg.ENOTCONV and its == maxit
            x = xt.cpu().numpy()
            assert np.linalg.norm(x - xo) <= 1e-12 * np.linalg.norm(xo), (solver, maxit)
    with pytest.raises(mfcg.MfcgError):
        P.set_solver(7)
    with pytest.raises(mfcg.MfcgError):
        P.set_preconditioner(2)
    P.close()
