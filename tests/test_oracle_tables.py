"""Pins for the oracle's 1D tables (GLL nodes, Gauss rule, Lagrange basis).

The paper's basis is the tensor product of 1D Lagrange polynomials of degree
k (Sec. 2, Eq. 2) integrated by tensor Gauss quadrature (Sec. 2, after Eq. 5);
node placement (GLL) is a reading.
"""
import os

import numpy as np
import pytest

from tests import fe_numpy

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_gll_closed_forms(oracle_mod):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "gll_nodes.txt")) if l.strip() and not l.startswith("#")]
    for r in rows:
        k = int(r[0])
        ref = np.array([float(v) for v in r[1:]])
        np.testing.assert_allclose(oracle_mod.gll(k), ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("k", range(1, 11))
def test_gll_matches_numpy_roots(oracle_mod, k):
    np.testing.assert_allclose(oracle_mod.gll(k), fe_numpy.gll_nodes(k), rtol=0, atol=2e-15)


@pytest.mark.parametrize("n", range(1, 12))
def test_gauss_exactness(oracle_mod, n):
    x, w = oracle_mod.gauss(n)
    assert np.all(np.diff(x) > 0) and np.all(w > 0)
    for m in range(2 * n):
        assert abs(np.sum(w * x ** m) - 1.0 / (m + 1)) < 1e-15 * 4
    # degree 2n is not integrated exactly: this is the n-point Gauss rule
    if n <= 6:
        assert abs(np.sum(w * x ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-12


def test_gauss_three_point_closed_form(oracle_mod):
    x, w = oracle_mod.gauss(3)
    r = np.sqrt(3.0 / 5.0)
    np.testing.assert_allclose(x, [(1 - r) / 2, 0.5, (1 + r) / 2], atol=1e-16)
    np.testing.assert_allclose(w, [5 / 18, 8 / 18, 5 / 18], atol=1e-16)


@pytest.mark.parametrize("n", [1, 4, 9, 20])
def test_gauss_matches_numpy(oracle_mod, n):
    x, w = oracle_mod.gauss(n)
    xr, wr = fe_numpy.gauss_rule(n)
    np.testing.assert_allclose(x, xr, atol=1e-15)
    np.testing.assert_allclose(w, wr, atol=1e-15)


@pytest.mark.parametrize("k", [1, 2, 4, 8])
def test_lagrange_properties(oracle_mod, k):
    nodes = oracle_mod.gll(k)
    for i in range(k + 1):
        for j in range(k + 1):
            assert oracle_mod.lagrange(nodes, i, nodes[j]) == pytest.approx(float(i == j), abs=1e-14)
    xs = np.linspace(0, 1, 17)
    val, der = fe_numpy.basis_1d(nodes, xs)
    for xi, x in enumerate(xs):
        v = [oracle_mod.lagrange(nodes, i, x) for i in range(k + 1)]
        d = [oracle_mod.lagrange_deriv(nodes, i, x) for i in range(k + 1)]
        assert abs(sum(v) - 1.0) < 1e-13          # partition of unity
        assert abs(sum(d)) < 1e-11 * k * k        # derivative of 1
        np.testing.assert_allclose(v, val[xi], atol=1e-12)
        np.testing.assert_allclose(d, der[xi], atol=1e-10 * k * k)


@pytest.mark.parametrize("k", range(1, 10))
def test_gll_weights(oracle_mod, k):
    """The (k+1)-point GLL rule: weights are the integrals of the nodal
    basis, positive, symmetric; exact to degree 2k-1 and not for 2k."""
    w = oracle_mod.gll_weights(k)
    x = oracle_mod.gll(k)
    np.testing.assert_allclose(w, fe_numpy.gll_weights_exact(k), rtol=0, atol=2e-15)
    assert np.all(w > 0) and np.allclose(w, w[::-1], atol=1e-15)
    for m in range(2 * k):
        assert abs(np.sum(w * x ** m) - 1.0 / (m + 1)) < 1e-14
    assert abs(np.sum(w * x ** (2 * k)) - 1.0 / (2 * k + 1)) > 1e-12
    if k == 2:  # Simpson's rule
        np.testing.assert_allclose(w, [1 / 6, 4 / 6, 1 / 6], atol=1e-16)

