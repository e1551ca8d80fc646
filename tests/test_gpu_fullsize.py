"""Parity at the benchmark's full size, in the configuration bench.py times
(Q4, 64^3 cells of the sine-shear mesh, 16,974,593 DoFs, default tiles),
and the GLL-collocation, k+2-point and quadratic-geometry operators at the
same size.

The oracle cannot assemble this matrix in a test (3.7e9 nonzeros), so it
evaluates sampled rows of A u cell by cell (oracle_apply_rows): random rows
plus the rows where the enumeration changes class (tile boundary planes,
edges and corners, the Dirichlet boundary).  Checked: the GPU operator on a
random-normal vector, and on the converged solution of the benchmark's
solve; the solve's residual in the GPU operator (pinned by the first check)
is below 1e-10 ||b||, and the sampled residual rows in the oracle's operator
agree with it.
"""
import numpy as np
import pytest

from paper_2205_08909_amd import inputs

pytestmark = pytest.mark.gpu

N, K = 64, 4


def _rows(problem, nsample=3000, seed=0):
    L = N * K + 1
    rng = np.random.default_rng(seed)
    rows = set(rng.integers(0, L ** 3, nsample).tolist())
    tile = problem.layout_info()["tile"]
    # nodes on tile boundary planes in each direction, their crossings, and the domain boundary
    planes = [np.arange(0, L, t * K) for t in tile]
    for _ in range(nsample // 3):
        ijk = [int(rng.integers(0, L)) for _ in range(3)]
        d = int(rng.integers(0, 3))
        ijk[d] = int(rng.choice(planes[d]))
        if rng.random() < 0.5:
            e = (d + 1) % 3
            ijk[e] = int(rng.choice(planes[e]))
        rows.add(ijk[0] + L * (ijk[1] + L * ijk[2]))
    for corner in ((0, 0, 0), (L - 1, 0, 0), (1, 1, 1), (L - 2, L - 2, L - 2), (K * tile[0], K * tile[1], K * tile[2])):
        rows.add(corner[0] + L * (corner[1] + L * corner[2]))
    return np.array(sorted(rows), dtype=np.int64)


def test_fullsize_operator_and_solve(oracle_mod):
    import torch
    from paper_2205_08909_amd import mfcg
    P = mfcg.Problem(N, K, map_kind=mfcg.MAP_SINE_SHEAR, amplitude=0.05)
    assert P.n == 257 ** 3
    m = oracle_mod.Mesh(N, K, map_kind=oracle_mod.MAP_SINE_SHEAR, amp=0.05)
    rows = _rows(P)
    # operator on a random-normal vector
    u = inputs.random_vector(P.n, seed=21)
    v = P.vmult(P.empty(), torch.from_numpy(u).cuda()).cpu().numpy()
    ref = oracle_mod.apply_rows(m, u, rows)
    err = np.max(np.abs(v[rows] - ref)) / np.max(np.abs(ref))
    print("sampled rows", rows.size, "operator max rel err", err)
    assert err <= 1e-12
    # the benchmark's solve
    b = P.rhs(mfcg.RHS_SINE)
    x = torch.zeros_like(b)
    code, its, _, tr = P.solve(b, x, tol=1e-10, maxit=5000, want_hist=False, want_true_res=True)
    print("iterations", its, "true rel res", tr)
    assert code == mfcg.OK and tr <= 1e-10 * 1.5
    xh = x.cpu().numpy()
    ax = P.vmult(P.empty(), x).cpu().numpy()
    ref = oracle_mod.apply_rows(m, xh, rows)
    # A x of the smooth solution cancels down to the size of b (h^3 f), far
    # below its terms: compare on the scale of the terms, ||A||_inf ||x||_inf
    # with ||A||_inf >= 8 max diag(A) over free nodes (the diagonal is pinned separately)
    free = ~inputs.boundary_mask(N, K)
    scale = 8.0 * P.diagonal().cpu().numpy()[free].max() * np.max(np.abs(xh))
    d = np.max(np.abs(ax[rows] - ref))
    print("solution rows: max |A x - oracle| =", d, "scale", scale)
    assert d <= 1e-12 * scale
    bh = b.cpu().numpy()
    res_rows = bh[rows] - ref
    # the sampled residual entries are small on the scale of the whole residual norm
    assert np.max(np.abs(res_rows)) <= 1.5e-10 * np.linalg.norm(bh)
    P.close()


def test_fullsize_collocation_operator(oracle_mod):
    """GLL collocation (BP5) at the same full size: sampled operator rows
    against the oracle's Gauss-Lobatto rows."""
    import torch
    from paper_2205_08909_amd import mfcg
    P = mfcg.Problem(N, K, map_kind=mfcg.MAP_SINE_SHEAR, amplitude=0.05, quad=mfcg.QUAD_GLL)
    m = oracle_mod.Mesh(N, K, map_kind=oracle_mod.MAP_SINE_SHEAR, amp=0.05, quad="gll")
    rows = _rows(P, nsample=1500, seed=1)
    u = inputs.random_vector(P.n, seed=22)
    v = P.vmult(P.empty(), torch.from_numpy(u).cuda()).cpu().numpy()
    ref = oracle_mod.apply_rows(m, u, rows)
    err = np.max(np.abs(v[rows] - ref)) / np.max(np.abs(ref))
    print("sampled rows", rows.size, "operator max rel err", err)
    assert err <= 1e-12
    P.close()



@pytest.mark.parametrize("variant", ["kplus2", "quadratic", "quadratic_kplus2"])
def test_fullsize_operator_variants(variant, oracle_mod):
    """k+2 Gauss points per direction, the quadratic geometry evaluated in the
    kernel, and both together (BP4's scalar operator as the paper runs it) at
    the same full size: sampled operator rows against the oracle's rows of
    the same rule."""
    import torch
    from paper_2205_08909_amd import mfcg
    nq = K + 2 if "kplus2" in variant else 0
    quad = variant.startswith("quadratic")
    P = mfcg.Problem(N, K, map_kind=mfcg.MAP_SINE_SHEAR, amplitude=0.05, n_q_1d=nq,
                     geometry=mfcg.GEOM_QUADRATIC if quad else mfcg.GEOM_STORED)
    m = oracle_mod.Mesh(N, K, nq1=nq or None, map_kind=oracle_mod.MAP_SINE_SHEAR, amp=0.05,
                        geometry="quadratic" if quad else "exact")
    rows = _rows(P, nsample=1500, seed=2)
    u = inputs.random_vector(P.n, seed=23)
    v = P.vmult(P.empty(), torch.from_numpy(u).cuda()).cpu().numpy()
    ref = oracle_mod.apply_rows(m, u, rows)
    err = np.max(np.abs(v[rows] - ref)) / np.max(np.abs(ref))
    print(variant, "sampled rows", rows.size, "operator max rel err", err)
    assert err <= 1e-12
    P.close()
