"""GPU parity for coefficient fields (c^Q per quadrature point) and mixed-degree batches, against
the FP64 oracle; the device offset scans against their plain definition."""
import numpy as np
import pytest

from gpu_cases import TOL_A, TOL_B, log, rel_fro, rel_vec, to_dev
from paper_1310_1191_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fem():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_1310_1191_amd import fem as F
    F.fem_init(0)
    return F


@pytest.fixture(scope="module")
def field_case():
    import oracle
    w = synth.make(4, grid=(7, 5, 4))          # 140 elements, degrees 1..7, FIELD coefficients
    A, b, fl, a_off, b_off = oracle.integrate(w.geom, w.coef, degree=w.degree, mode=oracle.FIELD,
                                              field=w.field)
    return w, A, b, a_off, b_off


def split_packed(A, b, a_off, b_off, degree):
    outA, outb = [], []
    for e, p in enumerate(degree):
        ns = (int(p) + 1) ** 3
        outA.append(A[a_off[e]:a_off[e + 1]].reshape(ns, ns))
        outb.append(b[b_off[e]:b_off[e + 1]])
    return outA, outb


def test_mixed_offsets_match_definition(fem):
    import torch
    rng = np.random.default_rng(3)
    for nel in [1, 5, 1023, 1024, 1025, 5000]:
        deg = rng.integers(1, 8, size=nel).astype(np.int8)
        d = torch.from_numpy(deg).cuda()
        a_off, b_off = fem.mixed_offsets(d)
        torch.cuda.synchronize()
        ns = (deg.astype(np.int64) + 1) ** 3
        ref_a = np.concatenate([[0], np.cumsum(ns * ns)])
        ref_b = np.concatenate([[0], np.cumsum(ns)])
        np.testing.assert_array_equal(a_off.cpu().numpy(), ref_a)
        np.testing.assert_array_equal(b_off.cpu().numpy(), ref_b)


STRATEGIES = {0: "single launch", 1: "per-degree launches"}


@pytest.mark.parametrize("strategy", [0, 1])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "split_fp16", "split_bf16"])
def test_mixed_degree_field_parity(fem, field_case, prec, strategy):
    import torch
    w, A_ref, b_ref, a_ref_off, b_ref_off = field_case
    g, c, f, d = to_dev(w.geom, w.coef, w.field, w.degree)
    status = torch.zeros(2, dtype=torch.int32, device="cuda")
    code = fem.PRECISIONS[prec]
    saved = fem.fem_get_variant(0, code, fem.FIELD)
    fem.fem_set_variant(0, code, fem.FIELD, strategy)
    try:
        A, b, a_off, b_off = fem.integrate_mixed(g, c, d, precision=prec, mode=fem.FIELD, field=f,
                                                 status=status)
        torch.cuda.synchronize()
    finally:
        fem.fem_set_variant(0, code, fem.FIELD, saved)
    np.testing.assert_array_equal(a_off.cpu().numpy(), a_ref_off)
    Ag, bg = split_packed(A.double().cpu().numpy(), b.double().cpu().numpy(), a_ref_off,
                          b_ref_off, w.degree)
    Ar, br = split_packed(A_ref, b_ref, a_ref_off, b_ref_off, w.degree)
    ea = np.array([rel_fro(x[None], y[None])[0] for x, y in zip(Ag, Ar)])
    eb = np.array([rel_vec(x[None], y[None])[0] for x, y in zip(bg, br)])
    log(f"[parity] mixed FIELD prec={prec} {STRATEGIES[strategy]} nel={w.nel} "
        f"errA max={ea.max():.3e} errb max={eb.max():.3e}")
    assert status.cpu().tolist() == [0, 0]
    assert ea.max() <= TOL_A[prec]
    assert eb.max() <= TOL_B[prec]


@pytest.mark.parametrize("p", [2, 5])
def test_uniform_field_parity(fem, p):
    import oracle
    import torch
    w = synth.make(4, grid=(4, 3, 2))
    A_ref, b_ref, _ = oracle.integrate(w.geom, w.coef, p=p, mode=oracle.FIELD, field=w.field)
    g, c, f = to_dev(w.geom, w.coef, w.field)
    for prec in ["fp64", "split_fp16"]:
        A, b = fem.integrate(g, c, p, precision=prec, mode=fem.FIELD, field=f)
        torch.cuda.synchronize()
        ea = rel_fro(A.double().cpu().numpy(), A_ref)
        log(f"[parity] FIELD p={p} prec={prec} errA max={ea.max():.3e}")
        assert ea.max() <= TOL_A[prec]


def test_mixed_equals_uniform_launches_bitwise(fem, field_case):
    """A mixed-degree call computes each element with the same kernel as a uniform call of its
    degree, so the results agree bit for bit."""
    import torch
    w = field_case[0]
    g, c, f, d = to_dev(w.geom, w.coef, w.field, w.degree)
    A, b, a_off, b_off = fem.integrate_mixed(g, c, d, precision="split_fp16", mode=fem.FIELD, field=f)
    torch.cuda.synchronize()
    a_off = a_off.cpu().numpy()
    for p in range(1, 8):
        idx = np.nonzero(w.degree == p)[0]
        if idx.size == 0:
            continue
        ti = torch.from_numpy(idx).cuda()
        Au, bu = fem.integrate(g[ti].contiguous(), c[ti].contiguous(), p, precision="split_fp16",
                               mode=fem.FIELD, field=f)
        torch.cuda.synchronize()
        ns = (p + 1) ** 3
        for t, e in enumerate(idx):
            assert torch.equal(A[a_off[e]:a_off[e + 1]].view(ns, ns), Au[t]), (p, e)


@pytest.mark.parametrize("alt", [0, 1])
@pytest.mark.parametrize("prec", ["split_fp16", "fp32", "fp64"])
def test_single_launch_equals_per_degree_launches_bitwise(fem, prec, alt):
    """With the per-degree launches set to the tiles the single persistent launch uses (its
    default tiles, alt 0, or the other alternative of every degree, alt 1), both strategies give
    identical bits; a larger batch makes every workgroup handle several degrees in turn."""
    import torch
    w = synth.make(4, grid=(16, 12, 10))        # 1920 elements, degrees 1..7
    g, c, f, d = to_dev(w.geom, w.coef, w.field, w.degree)
    code = fem.PRECISIONS[prec]
    keys = list(range(8)) + [fem.mixed(p) for p in range(1, 8)]
    saved = {p: fem.fem_get_variant(p, code, fem.FIELD) for p in keys}
    # the single launch's tile of each degree, and per-degree launches with the same tiles
    tiles = {}
    for p in range(1, 8):
        fem.fem_set_variant(fem.mixed(p), code, fem.FIELD, min(alt, fem.fem_variant_count(fem.mixed(p), code) - 1))
        tiles[p] = fem.mixed_tile_variant(p, code, fem.FIELD)
        fem.fem_set_variant(p, code, fem.FIELD, tiles[p])
    print(f"[mixed-bitwise] prec={prec} alt={alt} tiles={tiles}", flush=True)
    out = []
    for strategy in (0, 1):
        fem.fem_set_variant(0, code, fem.FIELD, strategy)
        A, b, a_off, b_off = fem.integrate_mixed(g, c, d, precision=prec, mode=fem.FIELD, field=f)
        torch.cuda.synchronize()
        out.append((A, b))
    for p, v in saved.items():
        fem.fem_set_variant(p, code, fem.FIELD, v)
    log(f"[mixed] {prec} tiles {tiles}: single vs per-degree, {w.nel} elements")
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][1], out[1][1])
