"""GPU parity of the p = 1 vector-ALU kernel (the default for trilinear hexahedra with ELEMENT
coefficients) through the C ABI: ragged element counts around its 8-element waves and
32-element workgroups in every precision, element lists and packed offsets (the per-degree
launches of a mixed-degree ELEMENT call, offsets not 16-byte aligned), supplied Jacobian terms,
the status counts, and agreement with the tile kernels it replaces."""
import numpy as np
import pytest

from gpu_cases import TOL_A, TOL_B, cdr_case, log, oracle_uniform, rel_fro, rel_vec, to_dev
from paper_1310_1191_amd import synth

pytestmark = pytest.mark.gpu

PRECS = ["fp64", "fp32", "split_fp16", "split_bf16", "bf16"]


@pytest.fixture(scope="module")
def fem():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_1310_1191_amd import fem as F
    F.fem_init(0)
    for prec in range(5):
        assert F.fem_get_variant(1, prec, F.ELEMENT) == F.trilinear_variant(prec)
    return F


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("nel", [1, 7, 8, 9, 31, 33, 1000])
def test_ragged_counts(fem, prec, nel):
    import torch
    geom, coef, A_ref, b_ref, _ = oracle_uniform(1)
    g, c = to_dev(geom[:nel], coef[:nel])
    status = torch.zeros(2, dtype=torch.int32, device="cuda")
    print(f"[trilinear] nel={nel} prec={prec}", flush=True)
    A, b = fem.integrate(g, c, 1, precision=prec, status=status)
    torch.cuda.synchronize()
    ea = rel_fro(A.double().cpu().numpy(), A_ref[:nel])
    eb = rel_vec(b.double().cpu().numpy(), b_ref[:nel])
    log(f"[trilinear] nel={nel} prec={prec} errA max={ea.max():.3e} errb max={eb.max():.3e}")
    assert status.cpu().tolist() == [0, 0]
    assert ea.max() <= TOL_A[prec] and eb.max() <= TOL_B[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "split_fp16"])
def test_agrees_with_tile_variants(fem, prec):
    """The same mesh through every tile variant of p = 1 and through the vector kernel."""
    import torch
    geom, coef, A_ref, _, _ = oracle_uniform(1)
    g, c = to_dev(geom, coef)
    code = fem.PRECISIONS[prec]
    tri = fem.trilinear_variant(code)
    out = {}
    try:
        for v in range(fem.fem_variant_count(1, code)):
            fem.fem_set_variant(1, code, fem.ELEMENT, v)
            print(f"[trilinear-vs-tile] prec={prec} v={v}", flush=True)
            A, _ = fem.integrate(g, c, 1, precision=prec)
            torch.cuda.synchronize()
            out[v] = A.double().cpu().numpy()
    finally:
        fem.fem_set_variant(1, code, fem.ELEMENT, tri)
    for v, A in out.items():
        d = rel_fro(A, out[tri])
        log(f"[trilinear-vs-tile] prec={prec} v={v} rel diff to the vector kernel {d.max():.3e}")
        assert d.max() <= 2 * TOL_A[prec]


@pytest.mark.parametrize("prec", ["fp64", "split_fp16"])
def test_mixed_degree_element_mode(fem, prec):
    """A mixed-degree ELEMENT call (per-degree launches): the p = 1 bucket runs the vector kernel
    on an element list, writing at packed offsets that follow larger elements."""
    import oracle
    import torch
    w = synth.make(4, grid=(9, 7, 5))
    # ELEMENT records with the CDR law for every element
    coef = synth.cdr_element_coeffs(w.nel, np.random.default_rng(5))
    deg = np.minimum(w.degree, 3).astype(np.int8)  # degrees 1..3 keep the oracle quick
    g, c, d = to_dev(w.geom, coef, deg)
    code = fem.PRECISIONS[prec]
    saved = fem.fem_get_variant(0, code, fem.ELEMENT)
    fem.fem_set_variant(0, code, fem.ELEMENT, 1)  # one launch per degree
    try:
        print(f"[trilinear-mixed] prec={prec} nel={w.nel}", flush=True)
        A, b, a_off, b_off = fem.integrate_mixed(g, c, d, precision=prec, mode=fem.ELEMENT)
        torch.cuda.synchronize()
    finally:
        fem.fem_set_variant(0, code, fem.ELEMENT, saved)
    a_np, b_np = a_off.cpu().numpy(), b_off.cpu().numpy()
    A_np, b_np_v = A.double().cpu().numpy(), b.double().cpu().numpy()
    assert (a_np[:-1][deg == 1] % 4 != 0).any()  # some p = 1 matrices start off a 16-byte boundary
    ea_all, eb_all = [], []
    for p in (1, 2, 3):
        sel = np.nonzero(deg == p)[0]
        A_ref, b_ref, _ = oracle.integrate(w.geom[sel], coef[sel], p=p)
        ns = (p + 1) ** 3
        Ag = np.stack([A_np[a_np[e]:a_np[e] + ns * ns].reshape(ns, ns) for e in sel])
        bg = np.stack([b_np_v[b_np[e]:b_np[e] + ns] for e in sel])
        ea, eb = rel_fro(Ag, A_ref), rel_vec(bg, b_ref)
        log(f"[trilinear-mixed] prec={prec} p={p} n={sel.size} errA max={ea.max():.3e} errb max={eb.max():.3e}")
        ea_all.append(ea.max())
        eb_all.append(eb.max())
    assert max(ea_all) <= TOL_A[prec] and max(eb_all) <= TOL_B[prec]


def test_status_counts(fem):
    """An inverted element (detJ < 0 at every point) and one with a NaN coefficient are counted
    once each; the other elements are unaffected."""
    import torch
    geom, coef = cdr_case(1)
    geom = geom[:40].copy()
    coef = coef[:40].copy()
    geom[5] = geom[5][[1, 0, 3, 2, 5, 4, 7, 6]]  # mirror: detJ < 0
    coef[17, 13] = np.nan                          # f = NaN
    _, _, A_ref, b_ref, _ = oracle_uniform(1)
    g, c = to_dev(geom, coef)
    status = torch.zeros(2, dtype=torch.int32, device="cuda")
    A, b = fem.integrate(g, c, 1, precision="fp64", status=status)
    torch.cuda.synchronize()
    assert status.cpu().tolist() == [1, 1]
    keep = np.array([e for e in range(40) if e not in (5, 17)])
    ea = rel_fro(A.cpu().numpy()[keep], A_ref[keep])
    assert ea.max() <= TOL_A["fp64"]
