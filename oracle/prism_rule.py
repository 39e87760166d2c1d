"""The oracle's triangle quadrature for prisms (test infrastructure, like the rest of ``oracle/``).

Section 2 of the paper integrates its reference prism with a Gaussian rule whose point counts
Table 1 lists: N_Q = 6, 18, 48, 80, 150, 231, 336 for p = 1..7, i.e. (p+1) Gauss-Legendre points
in the vertical direction times 3, 6, 12, 16, 25, 33, 42 points on the triangle. The paper gives
no triangle rule. The reading used here: the fully symmetric triangle rule of degree 2p (exact
for every polynomial of degree <= 2p, the degree of phi_i phi_j) with that many points, all
inside the triangle with positive weights, made of orbits of the permutations of barycentric
coordinates:
    S3    (1/3, 1/3, 1/3)                       1 point,  parameter: weight
    S21   (a, a, 1 - 2a) and its permutations   3 points, parameters: weight, a
    S111  (a, b, 1 - a - b) and permutations    6 points, parameters: weight, a, b
Such a rule integrates every polynomial of degree <= 2p exactly over the triangle
{x, y >= 0, x + y <= 1}; where several such rules exist, the one meant is the one near the orbit
parameters in SEEDS (found offline by a seeded search). This module refines those parameters to
full FP64 precision by Gauss-Newton on the moment equations of the products of shifted Legendre
polynomials P_i(2x-1) P_j(2y-1), i + j <= 2p, and returns the points (x, y) =
(lambda_1, lambda_2) and weights (summing to 1/2).
"""
from __future__ import annotations

import functools
import math
from fractions import Fraction

import numpy as np

# per p: list of orbits, ("S3", w) / ("S21", w, a) / ("S111", w, a, b); values are starting points
SEEDS = {
    1: [("S21", 0.1667, 0.1667)],
    2: [("S21", 0.11169, 0.44595), ("S21", 0.054976, 0.091576)],
    3: [("S21", 0.085667, 0.21943), ("S21", 0.040366, 0.48014),
        ("S111", 0.020317, 0.019372, 0.83901)],
    4: [("S3", 0.072158), ("S21", 0.016229, 0.050547), ("S21", 0.047546, 0.45929),
        ("S21", 0.051609, 0.17057), ("S111", 0.013615, 0.0083948, 0.72849)],
    5: [("S3", 0.040872), ("S21", 0.022979, 0.14216), ("S21", 0.0066765, 0.032055),
        ("S111", 0.017092, 0.029620, 0.60123), ("S111", 0.012649, 0.16370, 0.028368),
        ("S111", 0.031952, 0.32181, 0.14813)],
    6: [("S21", 0.021846, 0.43972), ("S21", 0.031429, 0.27121), ("S21", 0.0030831, 0.021317),
        ("S21", 0.012866, 0.48822), ("S21", 0.017398, 0.12758),
        ("S111", 0.011178, 0.022838, 0.28133), ("S111", 0.020186, 0.11534, 0.27571),
        ("S111", 0.0086581, 0.025734, 0.11625)],
    7: [("S21", 0.010942, 0.48896), ("S21", 0.0024617, 0.019391), ("S21", 0.016394, 0.41764),
        ("S21", 0.021081, 0.17721), ("S21", 0.0072168, 0.061800), ("S21", 0.025887, 0.27348),
        ("S111", 0.019286, 0.092916, 0.33686), ("S111", 0.012333, 0.057125, 0.17227),
        ("S111", 0.0025051, 0.0012683, 0.11897), ("S111", 0.0072182, 0.014647, 0.29837)],
}
POINTS = {1: 3, 2: 6, 3: 12, 4: 16, 5: 25, 6: 33, 7: 42}


def _orbit_points(kind, prm):
    """Points (lambda_1, lambda_2) of one orbit and their derivatives with respect to the
    orbit's coordinate parameters (a) or (a, b)."""
    if kind == "S3":
        return np.array([[1 / 3, 1 / 3]]), np.zeros((1, 2, 0))
    if kind == "S21":
        a = prm[0]
        lam = [(a, a, 1 - 2 * a), (a, 1 - 2 * a, a), (1 - 2 * a, a, a)]
        dlam = [(1, 1, -2), (1, -2, 1), (-2, 1, 1)]
        pts = np.array([[l[1], l[2]] for l in lam])
        der = np.array([[[d[1]], [d[2]]] for d in dlam], dtype=float)
        return pts, der
    a, b = prm
    c = 1 - a - b
    # each permutation puts (a, b, c) into the slots of lambda_0, lambda_1, lambda_2
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    vals = (a, b, c)
    dvals = ((1.0, 0.0), (0.0, 1.0), (-1.0, -1.0))   # d(a, b, c) / d(a, b)
    pts = np.array([[vals[pm[1]], vals[pm[2]]] for pm in perms])
    der = np.array([[dvals[pm[1]], dvals[pm[2]]] for pm in perms])
    return pts, der


def _expand(orbits, theta):
    """Points, weights and d(points, weights)/d(theta) for the parameter vector theta."""
    pts, wts, dp, dw = [], [], [], []
    k = 0
    ntheta = theta.size
    for kind, *_ in orbits:
        npar = {"S3": 0, "S21": 1, "S111": 2}[kind]
        w = theta[k]
        P, D = _orbit_points(kind, theta[k + 1:k + 1 + npar])
        for r in range(P.shape[0]):
            g = np.zeros((2, ntheta))
            g[:, k + 1:k + 1 + npar] = D[r]
            gw = np.zeros(ntheta)
            gw[k] = 1.0
            pts.append(P[r])
            wts.append(w)
            dp.append(g)
            dw.append(gw)
        k += 1 + npar
    return np.array(pts), np.array(wts), np.array(dp), np.array(dw)


def _shifted_legendre(n: int):
    """Integer coefficients c_k of P_n(2x - 1) = sum_k c_k x^k (the shifted Legendre polynomial):
    c_k = (-1)^(n-k) C(n, k) C(n+k, k)."""
    return [(-1) ** (n - k) * math.comb(n, k) * math.comb(n + k, k) for k in range(n + 1)]


def _moments(d):
    """The moment equations in the products P_i(2x-1) P_j(2y-1), i + j <= d (values bounded by 1,
    far better conditioned than monomials at degree 14), and their exact integrals over the
    triangle, int x^k y^l = k! l! / (k + l + 2)!, summed in rational arithmetic."""
    idx = [(i, j) for i in range(d + 1) for j in range(d + 1 - i)]
    exact = []
    for i, j in idx:
        ci, cj = _shifted_legendre(i), _shifted_legendre(j)
        tot = Fraction(0)
        for k, a in enumerate(ci):
            for l, b in enumerate(cj):
                tot += Fraction(a * b * math.factorial(k) * math.factorial(l),
                                math.factorial(k + l + 2))
        exact.append(float(tot))
    return idx, np.array(exact)


def _leg(n, t):
    """P_0..P_n and their derivatives at t (three-term recurrence)."""
    P = np.zeros((n + 1,) + t.shape)
    D = np.zeros((n + 1,) + t.shape)
    P[0] = 1.0
    if n >= 1:
        P[1] = t
        D[1] = 1.0
    for k in range(1, n):
        P[k + 1] = ((2 * k + 1) * t * P[k] - k * P[k - 1]) / (k + 1)
        D[k + 1] = D[k - 1] + (2 * k + 1) * P[k]
    return P, D


@functools.lru_cache(maxsize=None)
def _triangle_rule(p: int):
    if p not in SEEDS:
        raise NotImplementedError(f"no triangle rule seed for p = {p}")
    orbits = SEEDS[p]
    theta = np.array([v for orb in orbits for v in orb[1:]], dtype=np.float64)
    d = 2 * p
    idx, exact = _moments(d)

    def system(theta):
        P, W, dP, dW = _expand(orbits, theta)
        x, y = P[:, 0], P[:, 1]
        Lx, Dx = _leg(d, 2 * x - 1)
        Ly, Dy = _leg(d, 2 * y - 1)
        res = np.empty(len(idx))
        jac = np.empty((len(idx), theta.size))
        for r, (i, j) in enumerate(idx):
            f = Lx[i] * Ly[j]
            fx, fy = 2 * Dx[i] * Ly[j], 2 * Lx[i] * Dy[j]
            res[r] = (W * f).sum() - exact[r]
            # d/dtheta of sum_k w_k f(x_k, y_k)
            jac[r] = (dW * f[:, None]).sum(0) + (W[:, None] * (fx[:, None] * dP[:, 0, :] +
                                                            fy[:, None] * dP[:, 1, :])).sum(0)
        return res, jac

    for _ in range(60):
        res, jac = system(theta)
        step = np.linalg.lstsq(jac, -res, rcond=None)[0]
        theta = theta + step
        if np.abs(step).max() < 1e-17:
            break
    P, W, _, _ = _expand(orbits, theta)
    x, y = P[:, 0], P[:, 1]
    resid = np.abs(system(theta)[0]).max()
    if resid > 1e-14 or not (W > 0).all() or not ((x > 0) & (y > 0) & (x + y < 1)).all():
        raise RuntimeError(f"triangle rule p = {p}: refinement failed (residual {resid:.2e})")
    if P.shape[0] != POINTS[p]:
        raise RuntimeError(f"triangle rule p = {p}: {P.shape[0]} points, Table 1 needs {POINTS[p]}")
    return P, W


def triangle_rule(p: int):
    """(points [ntq, 2] = (xi1, xi2), weights [ntq]) of the degree-2p rule for prisms of degree p."""
    P, W = _triangle_rule(int(p))
    return P.copy(), W.copy()
