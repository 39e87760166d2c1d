"""Pins of the oracle's 1-D building blocks: quadrature points and weights (xi^Q, w^Q of
section 2), Gauss-Lobatto-Legendre nodes and the Lagrange basis (phi of section 2).

Pinned against closed forms, a library routine (numpy's Gauss-Legendre rule and Legendre
derivative roots) and properties that any correct implementation satisfies."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from polyexact import gll_nodes_numpy, lagrange_polys


def test_gauss_legendre_closed_forms(oracle_lib):
    x, w = oracle_lib.gauss_legendre(1)
    assert x[0] == pytest.approx(0.0, abs=1e-16) and w[0] == pytest.approx(2.0, rel=1e-15)
    x, w = oracle_lib.gauss_legendre(2)
    np.testing.assert_allclose(x, [-1 / np.sqrt(3), 1 / np.sqrt(3)], rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, [1.0, 1.0], rtol=1e-15)
    x, w = oracle_lib.gauss_legendre(3)
    np.testing.assert_allclose(x, [-np.sqrt(0.6), 0.0, np.sqrt(0.6)], rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, [5 / 9, 8 / 9, 5 / 9], rtol=1e-14)


@pytest.mark.parametrize("n", range(1, 13))
def test_gauss_legendre_vs_numpy(oracle_lib, n):
    x, w = oracle_lib.gauss_legendre(n)
    xr, wr = npleg.leggauss(n)
    np.testing.assert_allclose(x, xr, rtol=0, atol=2e-15)
    np.testing.assert_allclose(w, wr, rtol=2e-14, atol=0)
    assert np.all(np.diff(x) > 0)
    assert w.sum() == pytest.approx(2.0, rel=1e-14)


@pytest.mark.parametrize("n", range(1, 9))
def test_gauss_legendre_exactness(oracle_lib, n):
    x, w = oracle_lib.gauss_legendre(n)
    for m in range(2 * n):
        exact = 2.0 / (m + 1) if m % 2 == 0 else 0.0
        assert np.dot(w, x ** m) == pytest.approx(exact, abs=1e-14)
    # and not exact one degree higher (degree 2n)
    assert abs(np.dot(w, x ** (2 * n)) - 2.0 / (2 * n + 1)) > 1e-6


def test_gll_closed_forms(oracle_lib):
    np.testing.assert_allclose(oracle_lib.gll_nodes(1), [-1, 1], atol=0)
    np.testing.assert_allclose(oracle_lib.gll_nodes(2), [-1, 0, 1], atol=1e-16)
    np.testing.assert_allclose(oracle_lib.gll_nodes(3), [-1, -1 / np.sqrt(5), 1 / np.sqrt(5), 1],
                               atol=1e-15)
    np.testing.assert_allclose(oracle_lib.gll_nodes(4),
                               [-1, -np.sqrt(3 / 7), 0, np.sqrt(3 / 7), 1], atol=1e-15)


@pytest.mark.parametrize("p", range(1, 8))
def test_gll_vs_legendre_derivative_roots(oracle_lib, p):
    np.testing.assert_allclose(oracle_lib.gll_nodes(p), gll_nodes_numpy(p), atol=5e-15)


@pytest.mark.parametrize("p", range(1, 8))
def test_lagrange_properties(oracle_lib, p):
    nodes = oracle_lib.gll_nodes(p)
    n = p + 1
    for b in range(n):
        val, _ = oracle_lib.lagrange(nodes, nodes[b])
        np.testing.assert_allclose(val, np.eye(n)[b], atol=1e-14)
    rng = np.random.default_rng(11)
    polys = lagrange_polys(gll_nodes_numpy(p))
    for x in rng.uniform(-1, 1, 7):
        val, der = oracle_lib.lagrange(nodes, x)
        assert val.sum() == pytest.approx(1.0, abs=1e-13)          # partition of unity
        assert der.sum() == pytest.approx(0.0, abs=1e-11)
        assert np.dot(nodes, der) == pytest.approx(1.0, abs=1e-11)  # reproduces x
        np.testing.assert_allclose(val, [pl(x) for pl in polys], atol=1e-12)
        np.testing.assert_allclose(der, [pl.deriv()(x) for pl in polys], atol=1e-10)


def test_field_eval_special_values(oracle_lib):
    d = np.zeros((7, 5, 5))
    # field 0: one mode sin(2 pi x1); field 1: cos via theta = pi/2 on k=(0,1,0);
    # field 2: constant 0.25 (k = 0, theta = pi/2); field 3: two modes that cancel
    d[0, 0] = [1.0, 1, 0, 0, 0.0]
    d[1, 0] = [0.5, 0, 1, 0, np.pi / 2]
    d[2, 0] = [0.25, 0, 0, 0, np.pi / 2]
    d[3, 0] = [0.5, 1, 1, 1, 0.0]
    d[3, 1] = [0.5, -1, -1, -1, 0.0]
    d[4, 0] = [1.0, 2, -1, 0, 0.3]
    g = oracle_lib.field_eval(d, [0.25, 0.0, 0.7])
    assert g[0] == pytest.approx(1.0, abs=1e-15)
    assert g[1] == pytest.approx(0.5, abs=1e-15)
    assert g[2] == pytest.approx(0.25, abs=1e-15)
    assert g[3] == pytest.approx(0.0, abs=1e-15)
    assert g[4] == pytest.approx(np.sin(2 * np.pi * (0.5 - 0.0) + 0.3), abs=1e-14)
    assert g[5] == 0.0 and g[6] == 0.0
    # integer periodicity
    g2 = oracle_lib.field_eval(d, [1.25, -2.0, 3.7])
    np.testing.assert_allclose(g2, g, atol=1e-12)
