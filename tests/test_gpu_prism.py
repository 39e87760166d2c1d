"""GPU parity for prismatic elements (the paper's reference element, section 2, Tables 1-2)
through the C ABI (fem_integrate_prism): every degree, precision and compiled variant against the
FP64 prism oracle element by element, the elastostatics of section 5.1, coefficient fields,
empty input and argument errors."""
import functools

import numpy as np
import pytest

from gpu_cases import TOL_A, TOL_B, log, rel_fro, rel_vec, to_dev
from paper_1310_1191_amd import synth

pytestmark = pytest.mark.gpu

# cells per degree (two prisms each): several work items of every tile, ragged tails
GRIDS = {1: (7, 5, 3), 2: (5, 4, 3), 3: (5, 3, 2), 4: (3, 3, 2), 5: (3, 2, 2), 6: (3, 2, 1),
         7: (2, 2, 1)}
PRECS = ["fp64", "fp32", "split_fp16", "split_bf16", "bf16"]


@pytest.fixture(scope="module")
def fem():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_1310_1191_amd import fem as F
    F.fem_init(0)
    keys = [F.prism(p) for p in range(1, 8)]
    saved = {(k, c, m): F.fem_get_variant(k, c, m) for k in keys for c in range(5) for m in F.MODES}
    yield F
    for (k, c, m), v in saved.items():
        F.fem_set_variant(k, c, m, v)


@functools.lru_cache(maxsize=None)
def prism_case(kind: str, p: int):
    import oracle
    w = synth.make_prism(kind, p, grid=GRIDS[p])
    mode = {"cdr": oracle.ELEMENT, "elastic": oracle.ELASTIC, "field": oracle.FIELD}[kind]
    A, b, fl = oracle.integrate_prism(w.geom, w.coef, p, mode=mode, field=w.field)
    assert fl.max() == 0
    return w, A, b


@pytest.mark.parametrize("p", range(1, 8))
@pytest.mark.parametrize("prec", PRECS)
def test_prism_every_variant_parity(fem, p, prec):
    import torch
    w, A_ref, b_ref = prism_case("cdr", p)
    g, c = to_dev(w.geom, w.coef)
    code, key = fem.PRECISIONS[prec], fem.prism(p)
    n = fem.fem_variant_count(key, code)
    assert 1 <= n <= fem.MAX_VARIANTS
    first = None
    for v in range(n):
        fem.fem_set_variant(key, code, fem.ELEMENT, v)
        status = torch.zeros(2, dtype=torch.int32, device="cuda")
        print(f"[prism] p={p} prec={prec} variant={v} nel={w.nel}", flush=True)
        A, b = fem.integrate_prism(g, c, p, precision=prec, status=status)
        torch.cuda.synchronize()
        An, bn = A.double().cpu().numpy(), b.double().cpu().numpy()
        ea, eb = rel_fro(An, A_ref), rel_vec(bn, b_ref)
        log(f"[prism] p={p} prec={prec} v={v} errA max={ea.max():.3e} errb max={eb.max():.3e}")
        assert status.cpu().tolist() == [0, 0]
        assert ea.max() <= TOL_A[prec] and eb.max() <= TOL_B[prec]
        if first is None:
            first = bn
        else:  # the load vector does not depend on the tile configuration
            np.testing.assert_array_equal(bn, first)


@pytest.mark.parametrize("p", range(1, 8))
@pytest.mark.parametrize("prec", ["fp64", "fp32", "split_fp16"])
def test_prism_elasticity_parity(fem, p, prec):
    import torch
    w, A_ref, b_ref = prism_case("elastic", p)
    g, c = to_dev(w.geom, w.coef)
    print(f"[prism-elastic] p={p} prec={prec} nel={w.nel}", flush=True)
    A, b = fem.integrate_prism(g, c, p, precision=prec, mode=fem.ELASTIC)
    torch.cuda.synchronize()
    ns = fem.prism_ns(p)
    An = A.double().cpu().numpy().transpose(0, 1, 3, 2, 4).reshape(w.nel, 3 * ns, 3 * ns)
    Ar = A_ref.transpose(0, 1, 3, 2, 4).reshape(w.nel, 3 * ns, 3 * ns)
    ea = rel_fro(An, Ar)
    eb = rel_vec(b.double().cpu().numpy().reshape(w.nel, -1), b_ref.reshape(w.nel, -1))
    log(f"[prism-elastic] p={p} prec={prec} errA max={ea.max():.3e} errb max={eb.max():.3e}")
    assert ea.max() <= TOL_A[prec] and eb.max() <= TOL_B[prec]
    if p >= 2:  # lower blocks: transposes of the upper ones, from the epilogue or the copy kernel
        for i in range(3):
            for k in range(i + 1, 3):
                assert torch.equal(A[:, k, i], A[:, i, k].transpose(1, 2)), (i, k)


@pytest.mark.parametrize("p", [1, 3, 5, 7])
@pytest.mark.parametrize("prec", ["fp64", "split_fp16"])
def test_prism_field_mode_parity(fem, p, prec):
    import torch
    w, A_ref, b_ref = prism_case("field", p)
    g, c, f = to_dev(w.geom, w.coef, w.field)
    print(f"[prism-field] p={p} prec={prec} nel={w.nel}", flush=True)
    A, b = fem.integrate_prism(g, c, p, precision=prec, mode=fem.FIELD, field=f)
    torch.cuda.synchronize()
    ea = rel_fro(A.double().cpu().numpy(), A_ref)
    eb = rel_vec(b.double().cpu().numpy(), b_ref)
    log(f"[prism-field] p={p} prec={prec} errA max={ea.max():.3e} errb max={eb.max():.3e}")
    assert ea.max() <= TOL_A[prec] and eb.max() <= TOL_B[prec]


def test_prism_single_element_and_empty(fem):
    import torch
    import oracle
    w = synth.make_prism("cdr", 4, grid=(1, 1, 1))
    g, c = to_dev(w.geom[:1], w.coef[:1])
    A, b = fem.integrate_prism(g, c, 4, precision="fp64")
    torch.cuda.synchronize()
    A_ref, b_ref, _ = oracle.integrate_prism(w.geom[:1], w.coef[:1], 4)
    assert rel_fro(A.cpu().numpy(), A_ref).max() <= 1e-12
    empty = fem.make_coeffs("fp64", fem.ELEMENT, c)
    assert fem.fem_integrate_prism(0, 4, None, empty, None, None, None) == fem.FEM_OK


def test_prism_argument_errors(fem):
    import torch
    w = synth.make_prism("cdr", 2, grid=(1, 1, 1))
    g, c = to_dev(w.geom, w.coef)
    out = torch.empty(w.nel * 18 * 18, dtype=torch.float32, device="cuda")
    coeffs = fem.make_coeffs("split_fp16", fem.ELEMENT, c)
    assert fem.fem_integrate_prism(w.nel, 8, fem._ptr(g), coeffs, fem._ptr(out), None, None) == fem.FEM_EDEGREE
    assert fem.fem_integrate_prism(w.nel, 0, fem._ptr(g), coeffs, fem._ptr(out), None, None) == fem.FEM_EDEGREE
    assert fem.fem_integrate_prism(w.nel, 2, None, coeffs, fem._ptr(out), None, None) == fem.FEM_EINVAL
    jac = fem.make_coeffs("split_fp16", fem.ELEMENT, c, jac=c)
    assert fem.fem_integrate_prism(w.nel, 2, fem._ptr(g), jac, fem._ptr(out), None, None) == fem.FEM_EINVAL
    with pytest.raises(ValueError):  # the binding checks the geometry's shape before any launch
        fem.integrate_prism(torch.zeros((w.nel, 8, 3), dtype=torch.float64, device="cuda"), c, 2)


def test_prism_autotune(fem, tmp_path):
    path = tmp_path / "tuning.json"
    for p, prec in [(3, fem.SPLIT_FP16), (7, fem.FP32)]:
        v, times = fem.fem_autotune(fem.prism(p), prec, fem.ELEMENT, 2000 if p < 5 else 200, str(path))
        log(f"[prism-autotune] p={p} prec={prec} chosen={v} ms={times}")
        assert times[v] == min(times) and fem.fem_get_variant(fem.prism(p), prec, fem.ELEMENT) == v
    assert fem.fem_load_tuning(str(path)) == 2
