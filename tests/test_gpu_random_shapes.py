"""Operator parity over a seeded random sample of shapes: cells per
direction, degree, tile (ragged in any direction, one-cell tiles), map,
boundary condition, coefficient and operator variant (Laplacian on Gauss
points, GLL collocation, mass; a second sample: k+2 Gauss points and the
quadratic geometry, each for the Laplacian and the mass operator), each
against the
oracle's brute-force CSR
matrix (1e-12 relative; componentwise within 1e-13 (|A| |u|)), and, where
the operator is definite, five fused iterations against the oracle's fifth
Algorithm 1 iterate.
"""
import numpy as np
import pytest

from paper_2205_08909_amd import inputs

pytestmark = pytest.mark.gpu


def _draw(i):
    rng = np.random.default_rng(1000 + i)
    k = int(rng.integers(1, 9))
    cmax = max(2, 9 - k)
    cells = tuple(int(c) for c in rng.integers(1, cmax + 1, 3))
    tile = tuple(int(rng.integers(1, c + 1)) for c in cells) if rng.random() < 0.7 else None
    if tile is not None:
        # the compiled x/y tile limits shrink with the degree
        limx = {1: 8, 2: 8, 3: 8, 4: 4, 5: 4, 6: 2, 7: 2, 8: 2}[k]
        limy = {1: 8, 2: 8, 3: 4, 4: 4, 5: 3, 6: 2, 7: 2, 8: 1}[k]
        tile = (min(tile[0], limx), min(tile[1], limy), tile[2])
    kind = int(rng.integers(0, 3))
    bc = int(rng.random() < 0.3)
    variant = ["laplace", "gll", "mass"][int(rng.integers(0, 3))]
    coeff_seed = int(rng.integers(0, 100)) if rng.random() < 0.6 else None
    return cells, k, tile, kind, bc, variant, coeff_seed


@pytest.mark.parametrize("i", range(24))
def test_random_shape_parity(i, oracle_mod):
    import torch
    from paper_2205_08909_amd import mfcg
    cells, k, tile, kind, bc, variant, coeff_seed = _draw(i)
    print("case", i, cells, k, tile, kind, bc, variant, coeff_seed, flush=True)
    coeff = inputs.grf_coefficient(cells, 0.3, 1.0, seed=coeff_seed) if coeff_seed is not None else None
    quad = "gll" if variant == "gll" else "gauss"
    op = "mass" if variant == "mass" else "laplace"
    m = oracle_mod.Mesh(cells, k, map_kind=kind, amp=0.05, bc=bc, coeff=coeff, quad=quad, op=op)
    P = mfcg.Problem(cells, k, coeff=coeff, map_kind=kind, amplitude=0.05, bc=bc, tile=tile,
                     quad=mfcg.QUAD_GLL if variant == "gll" else mfcg.QUAD_GAUSS,
                     op=mfcg.OP_MASS if variant == "mass" else mfcg.OP_LAPLACE)
    A = oracle_mod.assemble(m)
    assert P.n == A.n
    u = inputs.random_vector(A.n, seed=i)
    ref = A.matvec(u)
    v = P.vmult(P.empty(), torch.from_numpy(u).cuda()).cpu().numpy()
    d = v - ref
    assert np.abs(d).max() <= 1e-12 * np.abs(ref).max()
    assert np.all(np.abs(d) <= 1e-13 * A.abs_matvec(u) + 1e-300)
    # five fused iterations against Algorithm 1's fifth iterate
    if bc == 1 and variant != "mass":  # singular Laplacian without boundary condition: operator only
        P.close()
        return
    b = inputs.random_rhs(cells, k, seed=i, dirichlet=bc == 0)
    if not b.any():
        P.close()
        return
    xo, its_o, _, rc_o = oracle_mod.pcg(A, A.diagonal(), b, tol=0.0, maxit=5)
    xt = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    code, its, _, _ = P.solve(torch.from_numpy(b).cuda(), xt, tol=0.0, maxit=5, raise_on=False)
    assert its == 5 == its_o
    assert np.linalg.norm(xt.cpu().numpy() - xo) <= 1e-11 * np.linalg.norm(xo)
    P.close()


def _draw_variant(i):
    rng = np.random.default_rng(2000 + i)
    variant = ["kplus2", "kplus2_mass", "qgeom", "qgeom_mass"][i % 4]
    kmax = 7 if variant.startswith("kplus2") else 8
    k = int(rng.integers(1, kmax + 1))
    cmax = max(2, 9 - k)
    cells = tuple(int(c) for c in rng.integers(1, cmax + 1, 3))
    limx = {1: 8, 2: 8, 3: 8, 4: 4, 5: 4, 6: 2, 7: 2, 8: 2}[k]
    limy = {1: 8, 2: 8, 3: 4, 4: 4, 5: 3, 6: 2, 7: 2, 8: 1}[k]
    tile = tuple(int(rng.integers(1, c + 1)) for c in cells) if rng.random() < 0.7 else None
    if tile is not None:
        tile = (min(tile[0], limx), min(tile[1], limy), tile[2])
    kind = int(rng.integers(0, 3))
    bc = int(rng.random() < 0.3)
    coeff_seed = int(rng.integers(0, 100)) if rng.random() < 0.6 else None
    return cells, k, tile, kind, bc, variant, coeff_seed


@pytest.mark.parametrize("i", range(24))
def test_random_shape_parity_kplus2_and_quadratic_geometry(i, oracle_mod):
    """The same check for k+2 Gauss points per direction (Laplacian and
    mass) and for the quadratic geometry evaluated in the kernel."""
    import torch
    from paper_2205_08909_amd import mfcg
    cells, k, tile, kind, bc, variant, coeff_seed = _draw_variant(i)
    print("case", i, cells, k, tile, kind, bc, variant, coeff_seed, flush=True)
    coeff = inputs.grf_coefficient(cells, 0.3, 1.0, seed=coeff_seed) if coeff_seed is not None else None
    op = "mass" if variant.endswith("mass") else "laplace"
    nq1 = k + 2 if variant.startswith("kplus2") else None
    geometry = "quadratic" if variant.startswith("qgeom") else "exact"
    m = oracle_mod.Mesh(cells, k, nq1=nq1, map_kind=kind, amp=0.05, bc=bc, coeff=coeff, op=op, geometry=geometry)
    P = mfcg.Problem(cells, k, coeff=coeff, map_kind=kind, amplitude=0.05, bc=bc, tile=tile,
                     op=mfcg.OP_MASS if op == "mass" else mfcg.OP_LAPLACE, n_q_1d=nq1 or 0,
                     geometry=mfcg.GEOM_QUADRATIC if variant.startswith("qgeom") else mfcg.GEOM_STORED)
    A = oracle_mod.assemble(m)
    assert P.n == A.n
    u = inputs.random_vector(A.n, seed=i)
    ref = A.matvec(u)
    v = P.vmult(P.empty(), torch.from_numpy(u).cuda()).cpu().numpy()
    d = v - ref
    assert np.abs(d).max() <= 1e-12 * np.abs(ref).max()
    assert np.all(np.abs(d) <= 1e-13 * A.abs_matvec(u) + 1e-300)
    if bc == 1 and op != "mass":
        P.close()
        return
    b = inputs.random_rhs(cells, k, seed=i, dirichlet=bc == 0)
    if not b.any():
        P.close()
        return
    xo, its_o, _, rc_o = oracle_mod.pcg(A, A.diagonal(), b, tol=0.0, maxit=5)
    xt = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    code, its, _, _ = P.solve(torch.from_numpy(b).cuda(), xt, tol=0.0, maxit=5, raise_on=False)
    assert its == 5 == its_o
    assert np.linalg.norm(xt.cpu().numpy() - xo) <= 1e-11 * np.linalg.norm(xo)
    P.close()
