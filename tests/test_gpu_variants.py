"""Every compiled kernel variant (tile configuration) of every (degree, precision) against the
FP64 oracle, and the per-degree autotuner with its tuning file. Calls go through the C ABI."""
import json

import numpy as np
import pytest

from gpu_cases import TOL_A, TOL_B, log, oracle_uniform, rel_fro, rel_vec, to_dev

pytestmark = pytest.mark.gpu

PRECS = ["fp64", "fp32", "split_bf16", "split_fp16", "bf16"]


@pytest.fixture(scope="module")
def fem():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_1310_1191_amd import fem as F
    F.fem_init(0)
    saved = {(p, c, m): F.fem_get_variant(p, c, m) for p in range(8) for c in range(5) for m in F.MODES}
    yield F
    for (p, c, m), v in saved.items():
        F.fem_set_variant(p, c, m, v)


@pytest.mark.parametrize("p", range(1, 8))
@pytest.mark.parametrize("prec", PRECS)
def test_every_variant_parity(fem, p, prec):
    import torch
    code = fem.PRECISIONS[prec]
    n = fem.fem_variant_count(p, code)
    assert 1 <= n <= fem.MAX_VARIANTS
    geom, coef, A_ref, b_ref, _ = oracle_uniform(p)
    g, c = to_dev(geom, coef)
    first = None
    v_default = fem.fem_get_variant(p, code, fem.ELEMENT)
    for v in range(n):
        fem.fem_set_variant(p, code, fem.ELEMENT, v)
        assert fem.fem_get_variant(p, code, fem.ELEMENT) == v
        status = torch.zeros(2, dtype=torch.int32, device="cuda")
        A, b = fem.integrate(g, c, p, precision=prec, status=status)
        torch.cuda.synchronize()
        An, bn = A.double().cpu().numpy(), b.double().cpu().numpy()
        ea, eb = rel_fro(An, A_ref), rel_vec(bn, b_ref)
        log(f"[variant] p={p} prec={prec} v={v} errA max={ea.max():.3e} errb max={eb.max():.3e}")
        assert status.cpu().tolist() == [0, 0]
        assert ea.max() <= TOL_A[prec] and eb.max() <= TOL_B[prec]
        if p == 1 and v == fem.trilinear_variant(code):
            continue  # the vector-ALU kernel sums b_i in its own order (checked above)
        if first is None:
            first = bn
        else:  # the load vector does not depend on the tile configuration
            np.testing.assert_array_equal(bn, first)
    fem.fem_set_variant(p, code, fem.ELEMENT, v_default)


def test_set_variant_rejects_missing_variant(fem):
    for p in range(1, 8):
        n = fem.fem_variant_count(p, fem.FP64)
        with pytest.raises(fem.FemError):
            fem.fem_set_variant(p, fem.FP64, fem.ELEMENT, n)


def test_autotune_writes_and_reloads_choice(fem, tmp_path):
    """Tuning per (degree, precision, coefficient mode): ELEMENT, FIELD and ELASTIC batches, the
    mixed-degree strategy (after the tile of every degree inside the single launch, keys
    FEM_MIXED(d), recorded in the same file), the JSON file keyed by mode, and its reload."""
    path = tmp_path / "tuning.json"
    seen = {}
    keys = list(range(8)) + [fem.mixed(d) for d in range(1, 8)]
    saved = {(p, c, m): fem.fem_get_variant(p, c, m) for p in keys for c in range(5) for m in fem.MODES}
    cases = [(2, fem.SPLIT_FP16, fem.ELEMENT), (4, fem.SPLIT_FP16, fem.ELEMENT), (3, fem.FP64, fem.ELEMENT),
             (0, fem.SPLIT_FP16, fem.ELEMENT), (3, fem.SPLIT_FP16, fem.FIELD), (0, fem.FP32, fem.FIELD),
             (2, fem.SPLIT_FP16, fem.ELASTIC), (1, fem.FP32, fem.ELEMENT), (1, fem.FP32, fem.FIELD)]
    for p, prec, mode in cases:
        other = {m: fem.fem_get_variant(p, prec, m) for m in fem.MODES if m != mode}
        v, times = fem.fem_autotune(p, prec, mode, 3000 if mode != fem.ELASTIC else 1000, str(path))
        log(f"[autotune] p={p} prec={prec} mode={mode} chosen={v} ms={times}")
        assert 0 <= v < fem.fem_variant_count(p, prec)
        assert len(times) == fem.fem_variant_count(p, prec)
        # p = 1: the vector-ALU variant takes ELEMENT coefficients only (-1 in other modes)
        tri = fem.trilinear_variant(prec) if p == 1 else -1
        timed = [t for k, t in enumerate(times) if not (k == tri and mode != fem.ELEMENT)]
        assert min(timed) > 0 and times[v] == min(timed)
        if tri >= 0 and mode != fem.ELEMENT:
            assert times[tri] == -1 and v != tri
        assert fem.fem_get_variant(p, prec, mode) == v
        assert {m: fem.fem_get_variant(p, prec, m) for m in other} == other  # other modes untouched
        seen[(p, prec, mode)] = v
        if p == 0:
            for d in range(1, 8):
                seen[(fem.mixed(d), prec, mode)] = fem.fem_get_variant(fem.mixed(d), prec, mode)
    doc = json.loads(path.read_text())
    got = {(e["p"], e["precision"], e["mode"]): e["variant"] for e in doc["entries"]}
    assert got == seen
    for (p, prec, mode) in seen:
        n = fem.fem_variant_count(p, prec) - (p == 1)  # p = 1: skip the vector-ALU variant
        fem.fem_set_variant(p, prec, mode, (seen[(p, prec, mode)] + 1) % n)
    assert fem.fem_load_tuning(str(path)) == len(seen)
    for (p, prec, mode), v in seen.items():
        assert fem.fem_get_variant(p, prec, mode) == v
    with pytest.raises(fem.FemError):  # the elasticity mode takes a uniform degree
        fem.fem_autotune(0, fem.SPLIT_FP16, fem.ELASTIC, 100)
    for (p, c, m), v in saved.items():
        fem.fem_set_variant(p, c, m, v)


@pytest.mark.parametrize("p", range(1, 8))
def test_every_variant_field_mode(fem, p):
    """Coefficient fields (FIELD mode) through every compiled variant of the split-FP16 path."""
    import oracle
    import torch
    from paper_1310_1191_amd import synth
    w = synth.make(4, grid=(5, 3, 2) if p <= 4 else (3, 2, 1))
    A_ref, b_ref, _ = oracle.integrate(w.geom, w.coef, p=p, mode=oracle.FIELD, field=w.field)
    g, c, f = (torch.from_numpy(x).cuda() for x in (w.geom, w.coef, w.field))
    code = fem.SPLIT_FP16
    v_default = fem.fem_get_variant(p, code, fem.FIELD)
    try:
        for v in range(fem.fem_variant_count(p, code)):
            if p == 1 and v == fem.trilinear_variant(code):
                continue  # ELEMENT mode only
            fem.fem_set_variant(p, code, fem.FIELD, v)
            A, b = fem.integrate(g, c, p, precision="split_fp16", mode=fem.FIELD, field=f)
            torch.cuda.synchronize()
            ea = rel_fro(A.double().cpu().numpy(), A_ref)
            eb = rel_vec(b.double().cpu().numpy(), b_ref)
            log(f"[variant FIELD] p={p} v={v} errA max={ea.max():.3e} errb max={eb.max():.3e}")
            assert ea.max() <= TOL_A["split_fp16"] and eb.max() <= TOL_B["split_fp16"]
    finally:
        fem.fem_set_variant(p, code, fem.FIELD, v_default)
