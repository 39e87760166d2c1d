"""The library's prism reference data (its own triangle-rule solver and Silvester basis, no GPU)
against the oracle's (its own solver on other moment equations and a Vandermonde basis), and the
synthetic prism meshes."""
import numpy as np
import pytest

import oracle
from oracle import prism_rule
from paper_1310_1191_amd import fem, synth


def _sorted_rule(P, W):
    order = np.lexsort((P[:, 1], P[:, 0]))
    return P[order], W[order]


@pytest.mark.parametrize("p", range(1, 8))
def test_library_triangle_rule_equals_oracle_rule(p):
    tri, _ = fem.fem_prism_reference_tables(p)
    Pl, Wl = _sorted_rule(tri[:, :2], tri[:, 2])
    Po, Wo = _sorted_rule(*prism_rule.triangle_rule(p))
    assert Pl.shape == Po.shape == (fem.PRISM_TRI_POINTS[p], 2)
    np.testing.assert_allclose(Pl, Po, atol=2e-15)
    np.testing.assert_allclose(Wl, Wo, rtol=1e-13)


@pytest.mark.parametrize("p", range(1, 8))
def test_library_reference_operand_equals_oracle_basis(p):
    """B[q][r][i] at the library's points q = qt + ntq qz against the oracle's shape functions."""
    tri, B = fem.fem_prism_reference_tables(p)
    zx, _ = oracle.gauss_legendre(p + 1)
    ntq = tri.shape[0]
    for q in range(0, B.shape[0], max(1, B.shape[0] // 24)):
        qt, qz = q % ntq, q // ntq
        ref = oracle.prism_shape(p, tri[qt, 0], tri[qt, 1], zx[qz])  # [Ns, 4]
        np.testing.assert_allclose(B[q].T, ref, atol=2e-12 * max(1.0, np.abs(ref).max()))


def test_prism_meshes_are_valid():
    for kind in ("cdr", "elastic", "field"):
        w = synth.make_prism(kind, 2, grid=(4, 3, 2))
        assert w.geom.shape == (48, 6, 3)
        # every prism has positive volume everywhere: the oracle flags none
        mode = {"cdr": oracle.ELEMENT, "elastic": oracle.ELASTIC, "field": oracle.FIELD}[kind]
        _, _, fl = oracle.integrate_prism(w.geom, w.coef, 1, mode=mode, field=w.field)
        assert fl.max() == 0
    # the two prisms of a cell tile it: their volumes add up to the domain's (exactly 1)
    w = synth.make_prism("cdr", 1, grid=(3, 3, 3))
    rec = synth.poisson_coeffs(w.nel)
    _, b, _ = oracle.integrate_prism(w.geom, rec, 1)
    assert abs(b.sum() - 1.0) < 1e-13
