"""Pins of the oracle's linear-elastostatics element matrices (the vector model problem of
section 5.1, eq. (sum_int) with an isotropic tensor from Young's modulus and Poisson's ratio).

* Parallelepipeds: every block equals the exact integral of the scalar form with the 3x3
  coefficient matrix K_jl = c_ijkl, computed by polynomial moments (no quadrature).
* Distorted trilinear elements: the six rigid motions (translations and infinitesimal
  rotations, interpolated at the physical node positions) lie in the kernel of A; A is
  symmetric, positive semi-definite, and its kernel has dimension exactly six.
* The load vector: summed over the nodes it is f_i times the element volume.
"""
import numpy as np
import pytest

import polyexact as px
from test_oracle_exact import jittered_element, parallelepiped


def lame(E, nu):
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


def elastic_tensor(E, nu):
    lam, mu = lame(E, nu)
    d = np.eye(3)
    return (lam * np.einsum("ij,kl->ijkl", d, d)
            + mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))


def physical_nodes(p, X):
    """Physical positions of the GLL nodes under the trilinear map of the vertices X."""
    n = p + 1
    g = px.gll_nodes_numpy(p)
    pts = np.zeros((n ** 3, 3))
    for c in range(n):
        for b in range(n):
            for a in range(n):
                xi = (g[a], g[b], g[c])
                w = [(1 + (2 * ((v >> d) & 1) - 1) * xi[d]) / 2 for v in range(8) for d in range(3)]
                w = np.array(w).reshape(8, 3).prod(axis=1)
                pts[a + n * b + n * n * c] = w @ X
    return pts


def rigid_modes(pts):
    """Six rigid displacement fields at the given points, as vectors indexed (k, r)."""
    modes = []
    for k in range(3):
        u = np.zeros((3, len(pts)))
        u[k] = 1.0
        modes.append(u.reshape(-1))
    for axis in range(3):
        w = np.zeros(3)
        w[axis] = 1.0
        modes.append(np.cross(w, pts).T.reshape(-1))  # u = w x x
    return np.array(modes)


def full_matrix(Ablocks):
    """[3][3][Ns][Ns] blocks -> (3 Ns) x (3 Ns) matrix indexed ((i, s), (k, r))."""
    ns = Ablocks.shape[-1]
    return Ablocks.transpose(0, 2, 1, 3).reshape(3 * ns, 3 * ns)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_parallelepiped_blocks_exact(oracle_lib, p):
    rng = np.random.default_rng(300 + p)
    X = parallelepiped(rng, 0.8)
    E, nu = 2.5, 0.3
    coef = np.array([[E, nu, 0.2, -0.4, 0.7]])
    A, b, fl = oracle_lib.integrate_elastic(X[None], coef, p)
    c = elastic_tensor(E, nu)
    for i in range(3):
        for k in range(3):
            ref = px.exact_affine_full(p, X, c[i, :, k, :], np.zeros(3), 0.0)
            assert np.linalg.norm(A[0, i, k] - ref) <= 1e-12 * np.linalg.norm(ref) + 1e-14, (i, k)
    for i, f in enumerate([0.2, -0.4, 0.7]):
        np.testing.assert_allclose(b[0, i], px.exact_load(p, X, f), rtol=1e-11, atol=1e-14)
    assert fl[0] == 0


@pytest.mark.parametrize("p", range(1, 8))
def test_rigid_motions_are_in_the_kernel(oracle_lib, p):
    rng = np.random.default_rng(400 + p)
    X = jittered_element(rng, 0.2)
    coef = np.array([[1.7, 0.27, 0.0, 0.0, 0.0]])
    A, _, fl = oracle_lib.integrate_elastic(X[None], coef, p, with_b=False)
    M = full_matrix(A[0])
    U = rigid_modes(physical_nodes(p, X))
    scale = np.linalg.norm(M) * np.linalg.norm(U, axis=1)
    res = np.linalg.norm(U @ M.T, axis=1)
    assert np.all(res <= 1e-12 * scale), res / scale
    assert fl[0] == 0


@pytest.mark.parametrize("p", [1, 2, 3])
def test_symmetric_psd_with_six_zero_modes(oracle_lib, p):
    rng = np.random.default_rng(500 + p)
    X = jittered_element(rng, 0.2)
    A, _, _ = oracle_lib.integrate_elastic(X[None], np.array([[3.0, 0.35, 0, 0, 0]]), p, with_b=False)
    M = full_matrix(A[0])
    np.testing.assert_allclose(M, M.T, rtol=0, atol=1e-13 * np.abs(M).max())
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    tol = 1e-10 * ev.max()
    assert ev.min() > -tol
    assert int(np.sum(ev < tol)) == 6


def test_load_sums_to_force_times_volume(oracle_lib):
    rng = np.random.default_rng(7)
    X = jittered_element(rng, 0.2)
    f = np.array([0.5, -1.5, 2.0])
    _, b, _ = oracle_lib.integrate_elastic(X[None], np.array([[1.0, 0.25, *f]]), 3)
    vol = oracle_lib.integrate(X[None], np.array([[0] * 12 + [0.0, 1.0]], dtype=float), p=3)[1][0].sum()
    np.testing.assert_allclose(b[0].sum(axis=1), f * vol, rtol=1e-12)


def test_elastic_rejects_bad_arguments(oracle_lib):
    X = jittered_element(np.random.default_rng(1))
    with pytest.raises(ValueError):
        oracle_lib.integrate_elastic(X[None], np.array([[1.0, 0.3, 0, 0, 0]]), 8)
