"""Exact integration on the reference prism, independent of any quadrature rule (pins the prism
oracle).

Polynomials are dense coefficient arrays c[i, j, k] of xi1^i xi2^j zeta^k. The reference prism is
T x [-1, 1] with T = {xi1, xi2 >= 0, xi1 + xi2 <= 1}; monomials integrate exactly as
    int_T xi1^i xi2^j = i! j! / (i + j + 2)!,   int_{-1}^{1} zeta^k = 2/(k+1) (k even), 0 (odd).
The triangle's Lagrange basis on the principal lattice is built here with Silvester's product
formula phi_(a,b,c) = R_a(lambda1) R_b(lambda2) R_c(lambda0), R_m(l) = prod_{k<m} (p l - k)/(k+1)
(the oracle inverts a Vandermonde matrix instead); the vertical factors are the GLL Lagrange
polynomials of polyexact (numpy's Legendre roots).
"""
from __future__ import annotations

import functools
import math
from fractions import Fraction

import numpy as np

from polyexact import gll_nodes_numpy, lagrange_polys, pmul, padd, pderiv


def tri_moment(i: int, j: int) -> float:
    return math.factorial(i) * math.factorial(j) / math.factorial(i + j + 2)


def line_moment(k: int) -> float:
    return 2.0 / (k + 1) if k % 2 == 0 else 0.0


def integrate_prism_poly(P: np.ndarray) -> float:
    tot = 0.0
    for (i, j, k), c in np.ndenumerate(P):
        if c != 0.0:
            tot += c * tri_moment(i, j) * line_moment(k)
    return tot


def integrate_triangle_poly(P: np.ndarray) -> float:
    """P: 2-D coefficient array c[i, j] of xi1^i xi2^j."""
    return sum(c * tri_moment(i, j) for (i, j), c in np.ndenumerate(P) if c != 0.0)


def lattice(p: int):
    """Triangle nodes t -> (a, b), a + b <= p, b outer, a inner."""
    return [(a, b) for b in range(p + 1) for a in range(p + 1 - b)]


def _poly_mul(a: dict, b: dict) -> dict:
    out = {}
    for (i1, j1), c1 in a.items():
        for (i2, j2), c2 in b.items():
            k = (i1 + i2, j1 + j2)
            out[k] = out.get(k, Fraction(0)) + c1 * c2
    return {k: v for k, v in out.items() if v != 0}


def _R(m: int, p: int, lam: dict) -> dict:
    """prod_{k<m} (p lam - k) / (k + 1) with exact rational coefficients."""
    out = {(0, 0): Fraction(1)}
    for k in range(m):
        term = {key: p * c for key, c in lam.items()}
        term[(0, 0)] = term.get((0, 0), Fraction(0)) - k
        out = {key: c / (k + 1) for key, c in _poly_mul(out, term).items()}
    return out


def triangle_basis_exact(p: int):
    """Silvester Lagrange basis as exact rational polynomials {(i, j): c} of xi1^i xi2^j."""
    lam1 = {(1, 0): Fraction(1)}
    lam2 = {(0, 1): Fraction(1)}
    lam0 = {(0, 0): Fraction(1), (1, 0): Fraction(-1), (0, 1): Fraction(-1)}
    return [_poly_mul(_poly_mul(_R(a, p, lam1), _R(b, p, lam2)), _R(p - a - b, p, lam0))
            for a, b in lattice(p)]


def triangle_basis(p: int):
    """The same basis as float coefficient arrays [(p+1), (p+1)]."""
    out = []
    for poly in triangle_basis_exact(p):
        full = np.zeros((p + 1, p + 1))
        for (i, j), c in poly.items():
            full[i, j] = float(c)
        out.append(full)
    return out


@functools.lru_cache(maxsize=None)
def triangle_matrices(p: int):
    """TT[d][e][t][t'] = int_T (D_d T_t)(D_e T_t'), d, e in {0 value, 1 d/dxi1, 2 d/dxi2}, in
    exact rational arithmetic (Gram matrix of the monomials), rounded once."""
    basis = triangle_basis_exact(p)
    monos = [(i, j) for j in range(p + 1) for i in range(p + 1 - j)]
    index = {m: k for k, m in enumerate(monos)}
    nt, nm = len(basis), len(monos)

    def coef_matrix(polys):
        Cm = [[Fraction(0)] * nt for _ in range(nm)]
        for t, poly in enumerate(polys):
            for key, c in poly.items():
                Cm[index[key]][t] = c
        return Cm

    def deriv(poly, axis):
        out = {}
        for (i, j), c in poly.items():
            if axis == 0 and i:
                out[(i - 1, j)] = out.get((i - 1, j), Fraction(0)) + i * c
            if axis == 1 and j:
                out[(i, j - 1)] = out.get((i, j - 1), Fraction(0)) + j * c
        return out

    mats = [coef_matrix(basis), coef_matrix([deriv(b, 0) for b in basis]),
            coef_matrix([deriv(b, 1) for b in basis])]
    gram = [[Fraction(math.factorial(m[0] + n[0]) * math.factorial(m[1] + n[1]),
                      math.factorial(m[0] + n[0] + m[1] + n[1] + 2)) for n in monos] for m in monos]
    TT = np.zeros((3, 3, nt, nt))
    for d in range(3):
        # G_d[n][t] = sum_m gram[n][m] C_d[m][t]
        left = mats[d]
        for e in range(3):
            right = mats[e]
            GR = [[sum(gram[n][m] * right[m][u] for m in range(nm) if right[m][u] != 0)
                   for u in range(nt)] for n in range(nm)]
            for t in range(nt):
                col = [left[n][t] for n in range(nm)]
                for u in range(nt):
                    TT[d, e, t, u] = float(sum(col[n] * GR[n][u] for n in range(nm) if col[n] != 0))
    return TT


def line_matrices(p: int):
    """LL[d][e][c][c'] = int_{-1}^{1} (D_d l_c)(D_e l_c'), d, e in {0 value, 1 derivative}."""
    polys = lagrange_polys(gll_nodes_numpy(p))
    D = [polys, [pl.deriv() for pl in polys]]
    n = p + 1
    LL = np.zeros((2, 2, n, n))
    for d in range(2):
        for e in range(2):
            for c in range(n):
                for u in range(n):
                    LL[d, e, c, u] = (D[d][c] * D[e][u]).integ()(1.0) - (D[d][c] * D[e][u]).integ()(-1.0)
    return LL


# reference-gradient component m of the prism basis -> (triangle factor, line factor)
_COMP = {0: (0, 0), 1: (1, 0), 2: (2, 0), 3: (0, 1)}


def reference_pair_matrices(p: int):
    """G[m][n][i][j] = int (D_m phi_i)(D_n phi_j) over the reference prism, i = t + Nt c, for
    m, n in 0 (value), 1..3 (d/dxi1, d/dxi2, d/dzeta): Kronecker products kron(line, triangle)."""
    TT, LL = triangle_matrices(p), line_matrices(p)
    nt, n = TT.shape[2], LL.shape[2]
    G = np.zeros((4, 4, nt * n, nt * n))
    for m in range(4):
        for k in range(4):
            (dm, em), (dk, ek) = _COMP[m], _COMP[k]
            G[m, k] = np.kron(LL[em, ek], TT[dm, dk])
    return G


def reference_vertices():
    """Reference coordinates (xi1, xi2, zeta) of prism vertex v = t + 3h."""
    tri = [(0.0, 0.0), (1.0, 0.0), (0.0, 1.0)]
    return np.array([[tri[t][0], tri[t][1], -1.0 + 2.0 * h] for h in range(2) for t in range(3)])


def affine_prism(M: np.ndarray, x0: np.ndarray) -> np.ndarray:
    """Vertices [6, 3] of the affine image x = x0 + M (xi1, xi2, zeta) of the reference prism."""
    return reference_vertices() @ np.asarray(M).T + np.asarray(x0)


def exact_affine_cdr(p: int, M, K, bvec, c, f):
    """Exact A and b of the scalar form on the affine prism x = x0 + M xi."""
    G = reference_pair_matrices(p)
    M = np.asarray(M, dtype=float)
    det = np.linalg.det(M)
    Mi = np.linalg.inv(M)
    Kh = det * Mi @ np.asarray(K) @ Mi.T
    bh = det * Mi @ np.asarray(bvec)
    A = det * c * G[0, 0]
    for n in range(3):
        A = A + bh[n] * G[0, 1 + n]
        for m in range(3):
            A = A + Kh[m, n] * G[1 + m, 1 + n]
    # load: int phi_i = sum over the basis of value integrals (times det f)
    mass_row = G[0, 0].sum(axis=1)  # int phi_i * sum_j phi_j = int phi_i
    return A, det * f * mass_row


def exact_affine_elastic(p: int, M, E, nu, fvec):
    """Exact blocks A[i][k][s][r] = sum_jl c_ijkl int d_l phi_r d_j phi_s and b[i][s] on the
    affine prism x = x0 + M xi (isotropic c_ijkl of E and nu)."""
    G = reference_pair_matrices(p)
    M = np.asarray(M, dtype=float)
    det = np.linalg.det(M)
    Mi = np.linalg.inv(M)
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    ns = G.shape[2]
    # P[j][l][s][r] = int d_xj phi_s d_xl phi_r = det sum_mn Mi[m, j] Mi[n, l] G[m][n][s][r]
    P = np.einsum("mj,nl,mnsr->jlsr", Mi, Mi, G[1:, 1:]) * det
    A = np.zeros((3, 3, ns, ns))
    for i in range(3):
        for k in range(3):
            for j in range(3):
                for l in range(3):
                    cijkl = lam * (i == j) * (k == l) + mu * ((i == k) * (j == l) + (i == l) * (j == k))
                    if cijkl:
                        A[i, k] += cijkl * P[j, l]
    mass_row = G[0, 0].sum(axis=1)
    b = det * np.outer(np.asarray(fvec), mass_row)
    return A, b


def prism_map_polys(X: np.ndarray):
    """x_a(xi1, xi2, zeta) of the prism map as (2, 2, 2) arrays and J[a][b] = dx_a/dxi_b."""
    lam = [np.array([[1.0, -1.0], [-1.0, 0.0]]), np.array([[0.0], [1.0]]), np.array([[0.0, 1.0]])]
    xs = []
    for a in range(3):
        poly = np.zeros((2, 2, 2))
        for h in range(2):
            fz = np.array([0.5, 0.5 if h else -0.5])
            for t in range(3):
                lt = np.zeros((2, 2))
                lt[:lam[t].shape[0], :lam[t].shape[1]] = lam[t]
                poly += X[t + 3 * h, a] * np.einsum("ij,k->ijk", lt, fz)
        xs.append(poly)
    J = [[pderiv(xs[a], b) for b in range(3)] for a in range(3)]
    return xs, J


def prism_basis_polys(p: int):
    """phi_i as 3-D arrays (i = t + Nt c)."""
    T = triangle_basis(p)
    L = lagrange_polys(gll_nodes_numpy(p))
    out = []
    for c in range(p + 1):
        lc = L[c].coef
        for t in range(len(T)):
            out.append(np.einsum("ij,k->ijk", T[t], lc))
    return out


def exact_load_distorted(p: int, X: np.ndarray, f: float) -> np.ndarray:
    """Exact int f phi_i dx = f int phi_i detJ dxi on any prism: detJ = sum d_abk xi1^a xi2^b
    zeta^k is a polynomial, int_T T_t xi1^a xi2^b is summed in rational arithmetic and
    int l_c zeta^k from numpy's polynomial of l_c."""
    from polyexact import det3
    _, J = prism_map_polys(X)
    det = det3(J)
    basis = triangle_basis_exact(p)
    L = lagrange_polys(gll_nodes_numpy(p))
    nt = len(basis)
    out = np.zeros(nt * (p + 1))
    for (a, b, k), dv in np.ndenumerate(det):
        if dv == 0.0:
            continue
        tri = [float(sum(c * Fraction(math.factorial(i + a) * math.factorial(j + b),
                                      math.factorial(i + a + j + b + 2))
                         for (i, j), c in poly.items())) for poly in basis]
        zk = np.polynomial.Polynomial([0.0] * k + [1.0])
        for c in range(p + 1):
            F = (L[c] * zk).integ()
            line = F(1.0) - F(-1.0)
            for t in range(nt):
                out[t + nt * c] += dv * tri[t] * line
    return f * out


def exact_volume(X: np.ndarray) -> float:
    from polyexact import det3
    _, J = prism_map_polys(X)
    return integrate_prism_poly(det3(J))
