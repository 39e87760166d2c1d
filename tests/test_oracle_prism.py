"""Pins of the prism oracle (the paper's reference element, section 2, Tables 1-2) against what
the paper and the mathematics fix: the sizes the paper prints, exact polynomial integration (a
different construction of the basis and no quadrature), closed-form properties of the basis and
invariants of the element matrices on distorted prisms."""
import math
import os

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle
from oracle import prism_rule
from prismexact import (affine_prism, exact_affine_cdr, exact_affine_elastic,
                        exact_load_distorted, exact_volume, lattice, reference_vertices)
from polyexact import gll_nodes_numpy

HERE = os.path.dirname(os.path.abspath(__file__))
DEGREES = range(1, 8)


def golden_sizes():
    rows = {}
    for line in open(os.path.join(HERE, "golden", "prism_table1_table2.txt")):
        if line.strip() and not line.startswith("#"):
            v = [int(x) for x in line.split()]
            rows[v[0]] = dict(nsh=v[1], nq=v[2], xiw=v[3], phi_pt=v[4], phi_all=v[5], blocks=v[6])
    return rows


# ---------------------------------------------------------------------------------------------
# sizes printed in the paper
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("p", DEGREES)
def test_sizes_match_tables_1_and_2(p):
    g = golden_sizes()[p]
    pts, w = prism_rule.triangle_rule(p)
    nq = pts.shape[0] * (p + 1)
    nsh = oracle.prism_ns(p)
    assert nsh == g["nsh"]
    assert nq == g["nq"]
    assert 4 * nq == g["xiw"]               # 3 coordinates and a weight per point
    assert 4 * nsh == g["phi_pt"]           # value and 3 derivatives per shape function
    assert 4 * nsh * nq == g["phi_all"]
    assert nsh * nsh == g["blocks"]
    assert oracle.prism_shape(p, 0.2, 0.3, 0.1).shape == (nsh, 4)


# ---------------------------------------------------------------------------------------------
# triangle rule: degree 2p, against a collapsed Gauss-Legendre rule from numpy (a library
# routine; the map (u, v) -> (u, (1-u) v) with Jacobian 1-u is exact for polynomials)
# ---------------------------------------------------------------------------------------------
def _collapsed_integral(f, n):
    x, w = npleg.leggauss(n)
    u, wu = (x + 1) / 2, w / 2
    tot = 0.0
    for a in range(n):
        for b in range(n):
            tot += wu[a] * wu[b] * (1 - u[a]) * f(u[a], (1 - u[a]) * u[b])
    return tot


@pytest.mark.parametrize("p", DEGREES)
def test_triangle_rule_is_exact_to_degree_2p(p):
    pts, w = prism_rule.triangle_rule(p)
    assert (w > 0).all()
    assert ((pts > 0).all(axis=1) & (pts.sum(axis=1) < 1)).all()
    rng = np.random.default_rng(p)
    d = 2 * p
    for _ in range(5):
        coef = rng.normal(size=(d + 1, d + 1))
        coef[np.add.outer(np.arange(d + 1), np.arange(d + 1)) > d] = 0.0
        f = lambda x, y: np.polynomial.polynomial.polyval2d(x, y, coef)
        ref = _collapsed_integral(f, d + 2)
        got = float((w * f(pts[:, 0], pts[:, 1])).sum())
        assert abs(got - ref) <= 1e-14 * max(1.0, np.abs(coef).sum())
    # and not exact for every polynomial of degree 2p + 2 (the degree is what the rule claims)
    f = lambda x, y: x ** (d + 2) + y ** (d + 2) + (1 - x - y) ** (d + 2)
    assert abs(float((w * f(pts[:, 0], pts[:, 1])).sum()) - _collapsed_integral(f, d + 3)) > 1e-12


@pytest.mark.parametrize("p", DEGREES)
def test_triangle_rule_is_fully_symmetric(p):
    pts, w = prism_rule.triangle_rule(p)
    lam = np.column_stack([1 - pts.sum(axis=1), pts])
    key = {tuple(np.round(l, 12)): round(float(x), 14) for l, x in zip(lam, w)}
    for l, x in zip(lam, w):
        for perm in [(0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]:
            k = tuple(np.round(l[list(perm)], 12))
            assert k in key and abs(key[k] - round(float(x), 14)) < 1e-13


# ---------------------------------------------------------------------------------------------
# shape functions
# ---------------------------------------------------------------------------------------------
def _nodes(p):
    gll = gll_nodes_numpy(p)
    return [(a / p, b / p, gll[c]) for c in range(p + 1) for (a, b) in lattice(p)]


@pytest.mark.parametrize("p", DEGREES)
def test_basis_is_nodal_and_reproduces_polynomials(p):
    nodes = _nodes(p)
    ns = len(nodes)
    for i, (x, y, z) in enumerate(nodes[:: max(1, ns // 40)]):
        phi = oracle.prism_shape(p, x, y, z)[:, 0]
        e = np.zeros(ns)
        e[nodes.index((x, y, z))] = 1.0
        np.testing.assert_allclose(phi, e, atol=1e-11)
    rng = np.random.default_rng(7 + p)
    for _ in range(4):
        x, y = rng.uniform(0, 0.5, 2)
        z = rng.uniform(-1, 1)
        phi = oracle.prism_shape(p, x, y, z)
        assert abs(phi[:, 0].sum() - 1.0) < 1e-12
        np.testing.assert_allclose(phi[:, 1:].sum(axis=0), 0.0, atol=1e-10)
        # a polynomial of the space (degree p in the triangle times degree p in zeta) and its
        # gradient are reproduced from its nodal values
        g = lambda X, Y, Z: (X ** p + 2 * X * Y ** (p - 1) - Y + 0.5) * (Z ** p - 0.3 * Z)
        gx = lambda X, Y, Z: (p * X ** (p - 1) + 2 * Y ** (p - 1)) * (Z ** p - 0.3 * Z)
        gz = lambda X, Y, Z: (X ** p + 2 * X * Y ** (p - 1) - Y + 0.5) * (p * Z ** (p - 1) - 0.3)
        vals = np.array([g(*nd) for nd in nodes])
        assert abs(vals @ phi[:, 0] - g(x, y, z)) < 1e-10
        assert abs(vals @ phi[:, 1] - gx(x, y, z)) < 1e-9
        assert abs(vals @ phi[:, 3] - gz(x, y, z)) < 1e-9


# ---------------------------------------------------------------------------------------------
# element matrices on affine prisms: exact (the integrands are polynomials of degree <= 2p in the
# triangle and <= 2p in zeta, which the rule integrates exactly)
# ---------------------------------------------------------------------------------------------
def _random_affine(rng):
    M = np.eye(3) * rng.uniform(0.5, 1.5, 3) + 0.2 * rng.normal(size=(3, 3))
    if np.linalg.det(M) < 0:
        M[:, 0] *= -1
    return M, rng.normal(size=3)


@pytest.mark.parametrize("p", DEGREES)
def test_affine_prism_cdr_is_exact(p):
    rng = np.random.default_rng(100 + p)
    M, x0 = _random_affine(rng)
    K = rng.normal(size=(3, 3))  # full, non-symmetric
    bv, c, f = rng.normal(size=3), 0.7, -1.3
    X = affine_prism(M, x0)
    rec = np.concatenate([K.reshape(-1), bv, [c, f]])[None]
    A, b, fl = oracle.integrate_prism(X[None], rec, p)
    Aex, bex = exact_affine_cdr(p, M, K, bv, c, f)
    scale = np.abs(Aex).max()
    np.testing.assert_allclose(A[0], Aex, atol=1e-11 * scale)
    np.testing.assert_allclose(b[0], bex, atol=1e-12 * np.abs(bex).max())
    assert fl[0] == 0


@pytest.mark.parametrize("p", [1, 2, 3, 5, 7])
def test_affine_prism_elasticity_is_exact(p):
    rng = np.random.default_rng(200 + p)
    M, x0 = _random_affine(rng)
    E, nu, fv = 3.0, 0.28, np.array([0.5, -1.0, 2.0])
    X = affine_prism(M, x0)
    A, b, fl = oracle.integrate_prism(X[None], np.array([[E, nu, *fv]]), p, mode=oracle.ELASTIC)
    Aex, bex = exact_affine_elastic(p, M, E, nu, fv)
    np.testing.assert_allclose(A[0], Aex, atol=1e-11 * np.abs(Aex).max())
    np.testing.assert_allclose(b[0], bex, atol=1e-12 * np.abs(bex).max())


# ---------------------------------------------------------------------------------------------
# distorted prisms (the map is bilinear in (triangle, zeta); the integrands are rational)
# ---------------------------------------------------------------------------------------------
def _distorted(rng, amp=0.15):
    return reference_vertices() * np.array([1.3, 0.9, 0.6]) + amp * rng.uniform(-1, 1, (6, 3))


@pytest.mark.parametrize("p", DEGREES)
def test_distorted_prism_load_and_volume_are_exact(p):
    """phi_i detJ is a polynomial of degree <= p + 1 in the triangle and <= p + 2 in zeta."""
    rng = np.random.default_rng(300 + p)
    X = _distorted(rng)
    K = np.eye(3)
    rec = np.concatenate([K.reshape(-1), [0, 0, 0], [0.0, 2.5]])[None]
    _, b, fl = oracle.integrate_prism(X[None], rec, p)
    np.testing.assert_allclose(b[0], exact_load_distorted(p, X, 2.5), atol=1e-13, rtol=1e-12)
    assert abs(b[0].sum() - 2.5 * exact_volume(X)) < 1e-12
    assert fl[0] == 0


@pytest.mark.parametrize("p", DEGREES)
def test_distorted_prism_invariants(p):
    rng = np.random.default_rng(400 + p)
    X = _distorted(rng)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    K = Q @ np.diag([0.3, 1.0, 4.0]) @ Q.T
    bv = rng.normal(size=3)
    # diffusion + convection rows sum to zero (sum_j phi_j = 1); with c the rows sum to the
    # load of f = c
    A, b, _ = oracle.integrate_prism(X[None], np.concatenate([K.ravel(), bv, [0.0, 0.8]])[None], p)
    assert np.abs(A[0].sum(axis=1)).max() < 1e-11 * np.abs(A[0]).max()
    A2, _, _ = oracle.integrate_prism(X[None], np.concatenate([K.ravel(), bv, [0.8, 0.8]])[None], p)
    np.testing.assert_allclose(A2[0].sum(axis=1), b[0], atol=1e-12 * np.abs(A2[0]).max())
    # symmetric iff b = 0; PSD with the constants as the only null vector
    As, _, _ = oracle.integrate_prism(X[None], np.concatenate([K.ravel(), [0, 0, 0], [0.0, 0.0]])[None], p)
    assert np.abs(As[0] - As[0].T).max() < 1e-13 * np.abs(As[0]).max()
    assert np.abs(A[0] - A[0].T).max() > 1e-6 * np.abs(A[0]).max()
    ev = np.linalg.eigvalsh(As[0])
    assert ev[0] > -1e-11 * ev[-1] and ev[1] > 1e-9 * ev[-1]


@pytest.mark.parametrize("p", [1, 2, 4])
def test_rigid_motion_and_scaling(p):
    rng = np.random.default_rng(500 + p)
    X = _distorted(rng)
    K = np.diag([1.0, 2.0, 3.0])
    bv = np.array([0.3, -0.2, 0.5])
    rec = np.concatenate([K.ravel(), bv, [0.4, 1.0]])[None]
    A, b, _ = oracle.integrate_prism(X[None], rec, p)
    R, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    Xr = X @ R.T + np.array([1.0, -2.0, 3.0])
    recr = np.concatenate([(R @ K @ R.T).ravel(), R @ bv, [0.4, 1.0]])[None]
    Ar, br, _ = oracle.integrate_prism(Xr[None], recr, p)
    np.testing.assert_allclose(Ar[0], A[0], atol=1e-12 * np.abs(A[0]).max())
    np.testing.assert_allclose(br[0], b[0], atol=1e-13)
    # x -> s x: diffusion * s, convection * s^2, reaction and load * s^3
    s = 1.7
    parts = []
    for r in ([*K.ravel(), 0, 0, 0, 0, 0], [*np.zeros(9), *bv, 0, 0], [*np.zeros(12), 0.4, 1.0]):
        a1, b1, _ = oracle.integrate_prism(X[None], np.array([r]), p)
        a2, b2, _ = oracle.integrate_prism((s * X)[None], np.array([r]), p)
        parts.append((a1[0], a2[0], b1[0], b2[0]))
    for (a1, a2, _, _), k in zip(parts, (1, 2, 3)):
        np.testing.assert_allclose(a2, s ** k * a1, atol=1e-12 * np.abs(a2).max())
    np.testing.assert_allclose(parts[2][3], s ** 3 * parts[2][2], atol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_distorted_prism_elasticity_has_six_rigid_modes(p):
    rng = np.random.default_rng(600 + p)
    X = _distorted(rng)
    A, _, _ = oracle.integrate_prism(X[None], np.array([[2.0, 0.3, 0, 0, 0]]), p, mode=oracle.ELASTIC)
    ns = oracle.prism_ns(p)
    big = A[0].transpose(0, 2, 1, 3).reshape(3 * ns, 3 * ns)
    assert np.abs(big - big.T).max() < 1e-12 * np.abs(big).max()
    ev = np.linalg.eigvalsh(big)
    assert np.abs(ev[:6]).max() < 1e-10 * ev[-1] and ev[6] > 1e-8 * ev[-1]
    # the rigid motions (physical positions of the nodes) are in the kernel
    phys = []
    for (x, y, z) in _nodes(p):
        lam = [1 - x - y, x, y]
        phys.append(sum(lam[t] * (1 + (2 * h - 1) * z) / 2 * X[t + 3 * h] for h in range(2) for t in range(3)))
    phys = np.array(phys)
    for mode in [np.eye(3)[0], np.eye(3)[1], np.eye(3)[2]]:
        u = np.tile(mode, (ns, 1)).T.reshape(-1)
        assert np.abs(big @ u).max() < 1e-10 * np.abs(big).max()
    u = np.concatenate([-phys[:, 1], phys[:, 0], 0 * phys[:, 0]])  # rotation about x3
    assert np.abs(big @ u).max() < 1e-10 * np.abs(big).max()


def test_field_mode_with_zero_amplitudes_equals_element_mode():
    rng = np.random.default_rng(700)
    X = _distorted(rng)
    field = np.zeros((7, 5, 5))
    field[:, :, 1:4] = rng.integers(-2, 3, size=(7, 5, 3))
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    A1, b1, _ = oracle.integrate_prism(X[None], np.concatenate([Q.ravel(), [0.9]])[None], 3,
                                       mode=oracle.FIELD, field=field)
    # g = 0: K = Q Q^T = I, b = 0, c = 1/2
    A2, b2, _ = oracle.integrate_prism(X[None], np.concatenate([np.eye(3).ravel(), [0, 0, 0], [0.5, 0.9]])[None], 3)
    np.testing.assert_allclose(A1, A2, atol=1e-13 * np.abs(A2).max())
    np.testing.assert_allclose(b1, b2, atol=1e-14)


def test_flags_and_argument_errors():
    X = reference_vertices().copy()
    X[3:, 2] = -3.0  # top below the bottom: detJ < 0
    rec = np.concatenate([np.eye(3).ravel(), [0, 0, 0], [0, 1.0]])[None]
    _, _, fl = oracle.integrate_prism(X[None], rec, 2)
    assert fl[0] & oracle.FLAG_DETJ
    tri = np.array([[0.2, 0.2, 0.5]])
    with pytest.raises(ValueError):
        oracle.integrate_prism(X[None], rec, 8, tri=tri)
    with pytest.raises(ValueError):
        oracle.integrate_prism(X[None], rec, 2, tri=np.zeros((0, 3)))
