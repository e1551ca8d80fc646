"""Pins for the oracle's operator (Sec. 2, Eq. 3-5) and diagonal (Sec. 3).

* affine mesh: the assembled matrix equals the Kronecker sum of exactly
  integrated 1D stiffness and mass matrices,
* Q1 on a uniform mesh: the textbook 27-point stencil,
* curved maps: element matrices agree with an FD-Jacobian numpy build,
  the assembled matrix is symmetric, positive definite on the free nodes
  and annihilates constants without boundary conditions,
* the diagonal equals the Kronecker closed form on affine meshes,
* the mass operator (BP1): the affine Kronecker product of 1D masses (lumped
  under GLL), total mass 1, curved element matrices against the FD build,
* with GLL collocation (quadrature at the k+1 nodes, BP5): the affine matrix
  is the Kronecker sum with the diagonal (lumped) 1D mass of the basis
  integrals, and curved element matrices match the FD-Jacobian build,
* quadratic geometry (the map replaced per cell by its quadratic
  interpolant through 27 points, Sec. 2.2): element matrices against a numpy
  build from the closed-form quadratic basis with exact central
  differences, identical to the exact geometry for an affine map, and
  converging to the exact-geometry matrices at second order in h,
* with k+2 Gauss points per direction (the BP1-BP4 rule): affine matrices
  equal the same exact Kronecker forms (both rules integrate them exactly),
  curved element matrices (Laplacian and mass) match the FD build on k+2
  points and differ from the (k+1)-point ones.
"""
import os

import numpy as np
import pytest

from tests import fe_numpy

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("k,ncells", [(1, (2, 3, 2)), (2, (2, 2, 3)), (3, (2, 1, 2)), (4, (1, 2, 1))])
def test_kronecker_closed_form(oracle_mod, k, ncells):
    O = oracle_mod
    m = O.Mesh(ncells, k, bc=O.BC_NONE)
    A = O.assemble(m).to_scipy().toarray()
    ref = fe_numpy.kronecker_laplacian(k, ncells)
    assert np.abs(A - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("k,ncells", [(1, (2, 3, 2)), (2, (2, 2, 3)), (4, (1, 2, 1)), (6, (1, 1, 2))])
def test_kronecker_gll_collocation(oracle_mod, k, ncells):
    O = oracle_mod
    m = O.Mesh(ncells, k, bc=O.BC_NONE, quad="gll")
    A = O.assemble(m).to_scipy().toarray()
    ref = fe_numpy.kronecker_laplacian(k, ncells, lumped=True)
    assert np.abs(A - ref).max() <= 1e-13 * np.abs(ref).max()
    # and it differs from the Gauss-integrated operator (the mass is lumped)
    if k > 1:
        assert np.abs(A - fe_numpy.kronecker_laplacian(k, ncells)).max() > 1e-6 * np.abs(ref).max()


@pytest.mark.parametrize("kind,amp,k", [(1, 0.05, 2), (2, 0.05, 4)])
def test_element_matrix_fd_jacobian_gll(oracle_mod, kind, amp, k):
    O = oracle_mod
    ncells = (2, 3, 2)
    m = O.Mesh(ncells, k, map_kind=kind, amp=amp, quad="gll")
    for cell in [(0, 0, 0), (1, 2, 1)]:
        A = O.element_matrix(m, cell)
        ref = fe_numpy.element_matrix_fd(k, 0, ncells, cell, kind, amp, quad="gll")
        assert np.abs(A - ref).max() <= 1e-8 * np.abs(ref).max()


@pytest.mark.parametrize("k,ncells,quad", [(1, (2, 3, 2), "gauss"), (3, (2, 1, 2), "gauss"), (4, (1, 2, 1), "gauss"),
                                           (2, (2, 2, 3), "gll"), (5, (1, 1, 2), "gll")])
def test_mass_kronecker_closed_form(oracle_mod, k, ncells, quad):
    """The mass operator (BP1): (k+1)-point Gauss integrates the affine mass
    exactly (degree 2k per direction); GLL collocation gives the lumped mass."""
    O = oracle_mod
    m = O.Mesh(ncells, k, bc=O.BC_NONE, quad=quad, op="mass")
    A = O.assemble(m).to_scipy().toarray()
    ref = fe_numpy.kronecker_mass(k, ncells, lumped=(quad == "gll"))
    assert np.abs(A - ref).max() <= 1e-14 * np.abs(ref).max() + 1e-17
    # total mass = volume of the unit cube
    assert A.sum() == pytest.approx(1.0, rel=1e-13)


@pytest.mark.parametrize("kind,amp,k", [(1, 0.05, 2), (2, 0.05, 3)])
def test_mass_element_fd_jacobian(oracle_mod, kind, amp, k):
    O = oracle_mod
    ncells = (2, 3, 2)
    coeff = np.linspace(0.5, 2.0, 12)
    m = O.Mesh(ncells, k, map_kind=kind, amp=amp, coeff=coeff, op="mass")
    for cell in [(0, 0, 0), (1, 2, 1)]:
        A = O.element_matrix(m, cell)
        ae = coeff[cell[0] + 2 * (cell[1] + 3 * cell[2])]
        ref = fe_numpy.element_mass_fd(k, ncells, cell, kind, amp, a_e=ae)
        assert np.abs(A - ref).max() <= 1e-8 * np.abs(ref).max()


@pytest.mark.parametrize("k", [1, 3])
def test_kronecker_with_dirichlet(oracle_mod, k):
    O = oracle_mod
    ncells = (3, 2, 2)
    m = O.Mesh(ncells, k, bc=O.BC_DIRICHLET)
    A = O.assemble(m).to_scipy().toarray()
    ref = fe_numpy.kronecker_laplacian(k, ncells)
    c = m.constrained_mask()
    ref[c, :] = 0
    ref[:, c] = 0
    ref[c, c] = 1.0
    assert np.abs(A - ref).max() <= 1e-13 * np.abs(ref).max()


def test_q1_stencil(oracle_mod):
    O = oracle_mod
    st = dict(tuple(map(float, l.split())) for l in open(os.path.join(GOLDEN, "q1_stencil.txt"))
              if l.strip() and not l.startswith("#"))
    N = 4
    h = 1.0 / N
    m = O.Mesh(N, 1)
    A = O.assemble(m).to_scipy()
    L = N + 1
    centre = 2 + L * (2 + L * 2)
    row = A.getrow(centre).toarray().ravel()
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                cls = abs(dx) + abs(dy) + abs(dz)
                j = centre + dx + L * (dy + L * dz)
                assert row[j] == pytest.approx(st[cls] * h, abs=1e-15)
    assert abs(row.sum()) < 1e-15


@pytest.mark.parametrize("kind,amp,k", [(1, 0.05, 2), (2, 0.05, 3), (1, 0.1, 1)])
def test_element_matrix_fd_jacobian(oracle_mod, kind, amp, k):
    O = oracle_mod
    ncells = (2, 3, 2)
    m = O.Mesh(ncells, k, map_kind=kind, amp=amp)
    for cell in [(0, 0, 0), (1, 2, 1), (0, 1, 1)]:
        A = O.element_matrix(m, cell)
        ref = fe_numpy.element_matrix_fd(k, k + 1, ncells, cell, kind, amp)
        assert np.abs(A - ref).max() <= 1e-8 * np.abs(ref).max()


def test_element_matrix_coefficient_scaling(oracle_mod):
    O = oracle_mod
    ncells = (2, 2, 2)
    coeff = np.arange(1, 9, dtype=np.float64) * 0.37
    m1 = O.Mesh(ncells, 2, map_kind=1, amp=0.05)
    m2 = O.Mesh(ncells, 2, map_kind=1, amp=0.05, coeff=coeff)
    for c in range(8):
        cell = (c % 2, (c // 2) % 2, c // 4)
        np.testing.assert_allclose(O.element_matrix(m2, cell), coeff[c] * O.element_matrix(m1, cell), rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("kind,k", [(1, 2), (2, 3), (1, 4)])
def test_symmetry_nullspace_spd(oracle_mod, kind, k):
    O = oracle_mod
    rng = np.random.default_rng(3)
    ncells = (3, 2, 2)
    coeff = np.exp(rng.normal(size=12))
    m = O.Mesh(ncells, k, map_kind=kind, amp=0.05, bc=O.BC_NONE, coeff=coeff)
    A = O.assemble(m)
    S = A.to_scipy()
    x = rng.normal(size=A.n)
    y = rng.normal(size=A.n)
    scale = np.linalg.norm(x) * np.linalg.norm(y) * abs(S).sum(axis=1).max()
    assert abs(y @ A.matvec(x) - x @ A.matvec(y)) <= 1e-13 * scale
    assert abs(S - S.T).max() <= 1e-15 * abs(S).max()
    rowabs = np.asarray(abs(S).sum(axis=1)).ravel()
    assert np.abs(A.matvec(np.ones(A.n))).max() <= 1e-13 * rowabs.max()
    # Dirichlet version: symmetric positive definite
    md = O.Mesh(ncells, k, map_kind=kind, amp=0.05, bc=O.BC_DIRICHLET, coeff=coeff)
    D = O.assemble(md).to_scipy().toarray()
    assert np.linalg.eigvalsh(D).min() > 0


@pytest.mark.parametrize("k,ncells", [(2, (3, 2, 2)), (4, (2, 2, 1))])
def test_diagonal_closed_form(oracle_mod, k, ncells):
    O = oracle_mod
    m = O.Mesh(ncells, k, bc=O.BC_NONE)
    d = O.assemble(m).diagonal()
    ref = np.diag(fe_numpy.kronecker_laplacian(k, ncells))
    np.testing.assert_allclose(d, ref, rtol=1e-13)


def test_apply_rows_matches_csr(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(5)
    for bc in (O.BC_DIRICHLET, O.BC_NONE):
        m = O.Mesh((3, 2, 4), 3, map_kind=1, amp=0.05, bc=bc, coeff=np.exp(rng.normal(size=24)))
        A = O.assemble(m)
        u = rng.normal(size=A.n)
        rows = rng.choice(A.n, size=200, replace=False)
        out = O.apply_rows(m, u, rows)
        ref = A.matvec(u)[rows]
        scale = A.abs_matvec(u)[rows]
        assert np.all(np.abs(out - ref) <= 1e-13 * scale + 1e-300)


def test_maps_invertible(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(0)
    X = rng.random((2000, 3))
    for kind, lo, hi in [(1, 0.85, 1.15), (2, 0.6, 1.4)]:
        dets = np.array([O.map_det(kind, 0.05, x) for x in X])
        assert dets.min() > lo and dets.max() < hi


@pytest.mark.parametrize("k,ncells", [(1, (2, 3, 2)), (3, (2, 1, 2)), (5, (1, 1, 2))])
def test_kplus2_kronecker_closed_form(oracle_mod, k, ncells):
    """k+2 Gauss points integrate the affine Laplacian and mass exactly, like k+1."""
    O = oracle_mod
    A = O.assemble(O.Mesh(ncells, k, nq1=k + 2, bc=O.BC_NONE)).to_scipy().toarray()
    ref = fe_numpy.kronecker_laplacian(k, ncells)
    assert np.abs(A - ref).max() <= 1e-13 * np.abs(ref).max()
    M = O.assemble(O.Mesh(ncells, k, nq1=k + 2, bc=O.BC_NONE, op="mass")).to_scipy().toarray()
    refm = fe_numpy.kronecker_mass(k, ncells)
    assert np.abs(M - refm).max() <= 1e-14 * np.abs(refm).max() + 1e-17


@pytest.mark.parametrize("kind,amp,k", [(1, 0.05, 2), (2, 0.05, 3), (1, 0.1, 1)])
def test_kplus2_element_fd_jacobian(oracle_mod, kind, amp, k):
    O = oracle_mod
    ncells = (2, 3, 2)
    coeff = np.linspace(0.5, 2.0, 12)
    m2 = O.Mesh(ncells, k, nq1=k + 2, map_kind=kind, amp=amp)
    m1 = O.Mesh(ncells, k, map_kind=kind, amp=amp)
    mm = O.Mesh(ncells, k, nq1=k + 2, map_kind=kind, amp=amp, coeff=coeff, op="mass")
    for cell in [(0, 0, 0), (1, 2, 1)]:
        A = O.element_matrix(m2, cell)
        ref = fe_numpy.element_matrix_fd(k, k + 2, ncells, cell, kind, amp)
        assert np.abs(A - ref).max() <= 1e-8 * np.abs(ref).max()
        # under the curved map the two rules give different matrices
        assert np.abs(A - O.element_matrix(m1, cell)).max() > 1e-7 * np.abs(ref).max()
        M = O.element_matrix(mm, cell)
        ae = coeff[cell[0] + 2 * (cell[1] + 3 * cell[2])]
        refm = fe_numpy.element_mass_fd(k, ncells, cell, kind, amp, a_e=ae, nq1=k + 2)
        assert np.abs(M - refm).max() <= 1e-8 * np.abs(refm).max()


@pytest.mark.parametrize("kind,amp,k", [(1, 0.05, 2), (2, 0.05, 4), (1, 0.1, 1)])
def test_quadratic_geometry_element_fd(oracle_mod, kind, amp, k):
    O = oracle_mod
    ncells = (2, 3, 2)
    m = O.Mesh(ncells, k, map_kind=kind, amp=amp, geometry="quadratic")
    me = O.Mesh(ncells, k, map_kind=kind, amp=amp)
    for cell in [(0, 0, 0), (1, 2, 1)]:
        A = O.element_matrix(m, cell)
        ref = fe_numpy.element_matrix_fd(k, k + 1, ncells, cell, kind, amp, geometry="quadratic")
        assert np.abs(A - ref).max() <= 1e-11 * np.abs(ref).max()
        assert np.abs(A - O.element_matrix(me, cell)).max() > 1e-6 * np.abs(ref).max()


def test_quadratic_geometry_affine_and_convergence(oracle_mod):
    O = oracle_mod
    # an affine map is reproduced exactly
    A = O.assemble(O.Mesh((2, 2, 3), 3, bc=O.BC_NONE, geometry="quadratic")).to_scipy().toarray()
    ref = fe_numpy.kronecker_laplacian(3, (2, 2, 3))
    assert np.abs(A - ref).max() <= 1e-13 * np.abs(ref).max()
    # curved: the element matrix error against the exact map falls like h^2
    # (the same physical cell, refined; ratios 3.6, 3.9, 4.0 -> 4)
    errs = []
    for n in (16, 32, 64, 128):
        c = (n // 4, n // 2, n // 4)
        me = O.Mesh((n, n, n), 2, map_kind=1, amp=0.1)
        mq = O.Mesh((n, n, n), 2, map_kind=1, amp=0.1, geometry="quadratic")
        Ae = O.element_matrix(me, c)
        errs.append(np.abs(O.element_matrix(mq, c) - Ae).max() / np.abs(Ae).max())
    rates = [errs[i] / errs[i + 1] for i in range(3)]
    assert rates[0] > 3.3 and rates[1] > 3.7 and 3.8 < rates[2] < 4.2, errs
