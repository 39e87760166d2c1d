"""Pins of the oracle's element integrals against exact results.

* p = 1 Poisson on a cube of side h: the closed-form 8x8 trilinear stiffness matrix.
* Any p on an axis-aligned box with constant (K, b, c): Kronecker products of exact 1-D
  matrices (the (p+1)-point Gauss rule integrates every term exactly there).
* Any p on a parallelepiped with a full K: exact polynomial integration.
* Any p on a distorted trilinear element: the convection term and the load vector have
  polynomial integrands of degree <= 2p+1 per variable, so the quadrature sum must equal the
  exact integral; the mass term's row sums likewise.
These compare the quadrature sum of Algorithm 2 (section 2) with integrals computed without
any quadrature rule."""
import numpy as np
import pytest

import polyexact as px


def box_vertices(lo, h):
    return np.array([[lo[0] + (v & 1) * h[0], lo[1] + ((v >> 1) & 1) * h[1],
                      lo[2] + ((v >> 2) & 1) * h[2]] for v in range(8)], dtype=np.float64)


def elem_record(K, b, c, f):
    rec = np.zeros(14)
    rec[0:9] = np.asarray(K, dtype=np.float64).reshape(9)
    rec[9:12] = b
    rec[12] = c
    rec[13] = f
    return rec


def rel_err(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("h", [1.0, 0.5, 1.0 / 16])
def test_cube_p1_poisson_closed_form(oracle_lib, h):
    X = box_vertices([0.3, -0.1, 2.0], [h, h, h])
    A, b, fl = oracle_lib.integrate(X[None], elem_record(np.eye(3), [0, 0, 0], 0.0, 1.0)[None], p=1)
    ref = np.zeros((8, 8))
    for i in range(8):
        for j in range(8):
            ndiff = bin(i ^ j).count("1")
            ref[i, j] = {0: 4.0, 1: 0.0, 2: -1.0, 3: -1.0}[ndiff] * h / 12.0
    np.testing.assert_allclose(A[0], ref, rtol=0, atol=1e-15 * max(1.0, h))
    np.testing.assert_allclose(b[0], np.full(8, h ** 3 / 8), rtol=1e-14)
    assert fl[0] == 0


def one_d_matrices(p):
    polys = px.lagrange_polys(px.gll_nodes_numpy(p))
    n = p + 1

    def integ(poly):
        ant = poly.integ()
        return ant(1.0) - ant(-1.0)

    M = np.array([[integ(polys[a] * polys[b]) for b in range(n)] for a in range(n)])
    S = np.array([[integ(polys[a].deriv() * polys[b].deriv()) for b in range(n)] for a in range(n)])
    C = np.array([[integ(polys[a] * polys[b].deriv()) for b in range(n)] for a in range(n)])
    return M, S, C


def kron3(F):
    return np.kron(F[2], np.kron(F[1], F[0]))


@pytest.mark.parametrize("p", range(1, 8))
def test_box_kronecker_formula(oracle_lib, p):
    rng = np.random.default_rng(100 + p)
    h = rng.uniform(0.2, 1.5, 3)
    X = box_vertices(rng.uniform(-1, 1, 3), h)
    G = rng.standard_normal((3, 3))
    K = G @ G.T + np.eye(3)
    K[0, 1] += 0.3  # a non-symmetric K is allowed by the form
    bvec = rng.uniform(-1, 1, 3)
    c = rng.uniform(0, 1)
    f = rng.uniform(-1, 1)
    A, b, fl = oracle_lib.integrate(X[None], elem_record(K, bvec, c, f)[None], p=p)

    M, S, C = one_d_matrices(p)
    det = np.prod(h) / 8.0
    ref = c * det * kron3([M, M, M])
    for k in range(3):
        F = [M, M, M]
        F[k] = C
        ref += det * bvec[k] * (2.0 / h[k]) * kron3(F)
        for l in range(3):
            F = [M, M, M]
            if k == l:
                F[k] = S
            else:
                F[k] = C.T
                F[l] = C
            ref += det * K[k, l] * (2.0 / h[k]) * (2.0 / h[l]) * kron3(F)
    assert rel_err(A[0], ref) < 1e-12
    # load vector: b_i = f det * prod of 1-D integrals of l_a
    m1 = M.sum(axis=1)
    np.testing.assert_allclose(b[0], f * det * kron3([m1[None], m1[None], m1[None]])[0],
                               rtol=1e-12, atol=1e-15)
    assert fl[0] == 0


def parallelepiped(rng, scale=1.0):
    x0 = rng.uniform(-1, 1, 3)
    E = np.eye(3) * scale + rng.uniform(-0.3, 0.3, (3, 3)) * scale
    X = np.array([x0 + ((v & 1) * E[:, 0] + ((v >> 1) & 1) * E[:, 1] + ((v >> 2) & 1) * E[:, 2])
                  for v in range(8)])
    return X


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_parallelepiped_exact(oracle_lib, p):
    rng = np.random.default_rng(200 + p)
    X = parallelepiped(rng, 0.7)
    G = rng.standard_normal((3, 3))
    K = G @ G.T + 0.5 * np.eye(3)
    bvec = rng.uniform(-1, 1, 3)
    c = rng.uniform(0, 1)
    A, b, fl = oracle_lib.integrate(X[None], elem_record(K, bvec, c, 0.5)[None], p=p)
    ref = px.exact_affine_full(p, X, K, bvec, c)
    assert rel_err(A[0], ref) < 1e-12
    np.testing.assert_allclose(b[0], px.exact_load(p, X, 0.5), rtol=1e-11, atol=1e-14)


def jittered_element(rng, alpha=0.25):
    X = box_vertices([0, 0, 0], [1, 1, 1]) + rng.uniform(-alpha, alpha, (8, 3))
    return X


def test_polyexact_adjugate_identity():
    rng = np.random.default_rng(5)
    X = jittered_element(rng)
    _, J = px.geometry_polys(X)
    adj = px.adjugate(J)
    det = px.det3(J)
    xi = rng.uniform(-1, 1, 3)

    def ev(P):
        return np.polynomial.polynomial.polyval3d(xi[0], xi[1], xi[2], P)

    Jn = np.array([[ev(J[a][b]) for b in range(3)] for a in range(3)])
    An = np.array([[ev(adj[m][k]) for k in range(3)] for m in range(3)])
    np.testing.assert_allclose(An @ Jn, ev(det) * np.eye(3), atol=1e-13)
    assert ev(det) == pytest.approx(np.linalg.det(Jn), rel=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_trilinear_convection_exact(oracle_lib, p):
    rng = np.random.default_rng(300 + p)
    X = jittered_element(rng)
    bvec = rng.uniform(-1, 1, 3)
    A, b, fl = oracle_lib.integrate(X[None], elem_record(np.zeros((3, 3)), bvec, 0.0, 0.0)[None],
                                    p=p)
    ref = px.exact_convection(p, X, bvec)
    assert rel_err(A[0], ref) < 1e-12
    assert fl[0] == 0


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_trilinear_load_and_mass_rowsum_exact(oracle_lib, p):
    rng = np.random.default_rng(400 + p)
    X = jittered_element(rng)
    c, f = 0.7, -1.3
    A, b, fl = oracle_lib.integrate(X[None], elem_record(np.zeros((3, 3)), [0, 0, 0], c, f)[None],
                                    p=p)
    ex = px.exact_load(p, X, 1.0)
    np.testing.assert_allclose(b[0], f * ex, rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(A[0].sum(axis=1), c * ex, rtol=1e-11, atol=1e-14)
