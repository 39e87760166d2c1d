"""Exact integration of polynomial integrands on [-1,1]^3, independent of any quadrature rule.

Used to pin the oracle: polynomials are dense monomial coefficient arrays c[i, j, k] (the
coefficient of xi1^i xi2^j xi3^k); products are N-D convolutions; integrals over the reference
cube use the moments int_{-1}^{1} t^m dt = 2/(m+1) for even m, 0 for odd m.

The 1-D Lagrange polynomials on the Gauss-Lobatto-Legendre nodes are built from the nodes that
numpy's Legendre class gives as roots of P_p' (a library routine, not the oracle's Newton
iteration).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import Polynomial
from numpy.polynomial import legendre as npleg
from scipy.signal import convolve


def gll_nodes_numpy(p: int) -> np.ndarray:
    if p == 1:
        return np.array([-1.0, 1.0])
    inner = npleg.Legendre.basis(p).deriv().roots()
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


def lagrange_polys(nodes) -> list[Polynomial]:
    out = []
    for a, xa in enumerate(nodes):
        others = [xb for b, xb in enumerate(nodes) if b != a]
        poly = Polynomial.fromroots(others) if others else Polynomial([1.0])
        out.append(poly / poly(xa))
    return out


def moments(m: int) -> np.ndarray:
    k = np.arange(m)
    return np.where(k % 2 == 0, 2.0 / (k + 1.0), 0.0)


def pmul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    return convolve(a, b, mode="full", method="direct")


def padd(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    shape = tuple(max(x, y) for x, y in zip(a.shape, b.shape))
    out = np.zeros(shape)
    out[tuple(slice(0, s) for s in a.shape)] += a
    out[tuple(slice(0, s) for s in b.shape)] += b
    return out


def pscale(a: np.ndarray, s: float) -> np.ndarray:
    return a * s


def pderiv(a: np.ndarray, axis: int) -> np.ndarray:
    n = a.shape[axis]
    if n == 1:
        shape = list(a.shape)
        return np.zeros(shape)
    idx = np.arange(1, n, dtype=np.float64)
    sl = [slice(None)] * 3
    sl[axis] = slice(1, n)
    out = a[tuple(sl)].copy()
    bshape = [1, 1, 1]
    bshape[axis] = n - 1
    return out * idx.reshape(bshape)


def basis_arrays(p: int):
    """phi_i and d phi_i / d xi_m as coefficient arrays of shape (Ns, n, n, n), node i = a + n b + n^2 c."""
    n = p + 1
    polys = lagrange_polys(gll_nodes_numpy(p))
    L = np.zeros((n, n))   # L[a, power]
    Ld = np.zeros((n, n))
    for a, pl in enumerate(polys):
        co = pl.coef
        L[a, :co.size] = co
        dco = pl.deriv().coef
        Ld[a, :dco.size] = dco
    ns = n ** 3
    phi = np.zeros((ns, n, n, n))
    dphi = np.zeros((3, ns, n, n, n))
    for c in range(n):
        for b in range(n):
            for a in range(n):
                i = a + n * b + n * n * c
                phi[i] = np.einsum("i,j,k->ijk", L[a], L[b], L[c])
                dphi[0, i] = np.einsum("i,j,k->ijk", Ld[a], L[b], L[c])
                dphi[1, i] = np.einsum("i,j,k->ijk", L[a], Ld[b], L[c])
                dphi[2, i] = np.einsum("i,j,k->ijk", L[a], L[b], Ld[c])
    return phi, dphi


def geometry_polys(X: np.ndarray):
    """x_a(xi) of the trilinear map of 8 vertices (vertex v = v1 + 2 v2 + 4 v3 at
    xi = 2 v - 1) as (2,2,2) arrays, and the Jacobian entries J[a][b] = dx_a/dxi_b."""
    xs = []
    for a in range(3):
        poly = np.zeros((2, 2, 2))
        for v in range(8):
            s = [1.0 if (v >> d) & 1 else -1.0 for d in range(3)]
            f = [np.array([1.0, s[d]]) / 2.0 for d in range(3)]
            poly += X[v, a] * np.einsum("i,j,k->ijk", f[0], f[1], f[2])
        xs.append(poly)
    J = [[pderiv(xs[a], b) for b in range(3)] for a in range(3)]
    return xs, J


def det3(M):
    t1 = pmul(M[0][0], padd(pmul(M[1][1], M[2][2]), -pmul(M[1][2], M[2][1])))
    t2 = pmul(M[0][1], padd(pmul(M[1][0], M[2][2]), -pmul(M[1][2], M[2][0])))
    t3 = pmul(M[0][2], padd(pmul(M[1][0], M[2][1]), -pmul(M[1][1], M[2][0])))
    return padd(padd(t1, -t2), t3)


def adjugate(M):
    """adj(M)[m][k] = (-1)^(m+k) * minor of M without row k and column m, so that
    adj(M) M = det(M) I."""
    adj = [[None] * 3 for _ in range(3)]
    for m in range(3):
        for k in range(3):
            rows = [r for r in range(3) if r != k]
            cols = [c for c in range(3) if c != m]
            minor = padd(pmul(M[rows[0]][cols[0]], M[rows[1]][cols[1]]),
                         -pmul(M[rows[0]][cols[1]], M[rows[1]][cols[0]]))
            adj[m][k] = minor * (1.0 if (m + k) % 2 == 0 else -1.0)
    return adj


def integrate_pairs(P: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """Exact I[i, j] = int_{[-1,1]^3} P_i Q_j for stacks P (ni, a, b, c) and Q (nj, d, e, f)."""
    d = max(P.shape[1] + Q.shape[1], P.shape[2] + Q.shape[2], P.shape[3] + Q.shape[3])
    mom = moments(d)
    H1 = mom[np.add.outer(np.arange(P.shape[1]), np.arange(Q.shape[1]))]
    H2 = mom[np.add.outer(np.arange(P.shape[2]), np.arange(Q.shape[2]))]
    H3 = mom[np.add.outer(np.arange(P.shape[3]), np.arange(Q.shape[3]))]
    T = np.einsum("iabc,ad->idbc", P, H1)
    T = np.einsum("idbc,be->idec", T, H2)
    T = np.einsum("idec,cf->idef", T, H3)
    return np.einsum("idef,jdef->ij", T, Q)


def integrate_single(P: np.ndarray) -> float:
    mom = [moments(s) for s in P.shape]
    return float(np.einsum("abc,a,b,c->", P, mom[0], mom[1], mom[2]))


def stack_pad(polys, shape):
    out = np.zeros((len(polys),) + tuple(shape))
    for t, pl in enumerate(polys):
        out[(t,) + tuple(slice(0, s) for s in pl.shape)] = pl
    return out


def exact_convection(p: int, X: np.ndarray, bvec) -> np.ndarray:
    """Exact int phi_i (b . grad phi_j) dx on the trilinear element X (any distortion).
    With grad_x phi detJ = adj(J)^T grad_xi phi the integrand is a polynomial of degree
    <= 2p+1 per variable."""
    phi, dphi = basis_arrays(p)
    _, J = geometry_polys(X)
    adj = adjugate(J)
    ns = phi.shape[0]
    G = []
    for j in range(ns):
        acc = np.zeros((1, 1, 1))
        for k in range(3):
            for m in range(3):
                acc = padd(acc, pmul(adj[m][k], dphi[m, j]) * bvec[k])
        G.append(acc)
    shape = tuple(max(g.shape[d] for g in G) for d in range(3))
    return integrate_pairs(phi, stack_pad(G, shape))


def exact_load(p: int, X: np.ndarray, f: float) -> np.ndarray:
    """Exact int f phi_i dx = f int phi_i detJ dxi (degree <= p+2 per variable)."""
    phi, _ = basis_arrays(p)
    _, J = geometry_polys(X)
    det = det3(J)
    return f * integrate_pairs(phi, det[None])[:, 0]


def exact_affine_full(p: int, X: np.ndarray, K, bvec, c) -> np.ndarray:
    """Exact element matrix on an affine element (parallelepiped: J constant): every term is a
    polynomial integrand, integrated by moments."""
    phi, dphi = basis_arrays(p)
    _, J = geometry_polys(X)
    Jc = np.array([[J[a][b].reshape(-1)[0] for b in range(3)] for a in range(3)])
    for a in range(3):
        for b in range(3):
            assert np.allclose(J[a][b].reshape(-1)[1:], 0.0), "element is not affine"
    det = np.linalg.det(Jc)
    Ji = np.linalg.inv(Jc)
    Khat = det * Ji @ np.asarray(K) @ Ji.T
    bhat = det * Ji @ np.asarray(bvec)
    A = c * det * integrate_pairs(phi, phi)
    for m in range(3):
        A += integrate_pairs(phi, dphi[m]) * bhat[m]
        for l in range(3):
            A += Khat[m, l] * integrate_pairs(dphi[m], dphi[l])
    return A
