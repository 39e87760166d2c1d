"""fem_integrate_noalloc (the allocation-free entry point) against fem_integrate, through the C
ABI: the same mixed-degree batch through both, bitwise equal, on two calls in a row with the
second one smaller (the static scratch keeps the first call's contents), plus the uniform-degree
path and the size limit."""
import numpy as np
import pytest

from gpu_cases import log, to_dev
from paper_1310_1191_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fem():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_1310_1191_amd import fem as F
    F.fem_init(0)
    return F


def _mixed_pair(fem, w, prec, nel):
    """Packed outputs of fem_integrate (caller workspace) and fem_integrate_noalloc (static
    scratch) for the first nel elements of w, same stream, same offsets."""
    import torch
    g, c, f, d = to_dev(w.geom[:nel], w.coef[:nel], w.field, w.degree[:nel])
    a_off, b_off = fem.mixed_offsets(d)
    ntot_a, ntot_b = int(a_off[-1].item()), int(b_off[-1].item())
    dt = fem.out_dtype(prec)
    outs = []
    for noalloc in (False, True):
        A = torch.full((ntot_a,), float("nan"), dtype=dt, device="cuda")
        b = torch.full((ntot_b,), float("nan"), dtype=dt, device="cuda")
        status = torch.zeros(2, dtype=torch.int32, device="cuda")
        ws = None if noalloc else torch.empty(fem.fem_workspace_bytes(nel), dtype=torch.uint8,
                                              device="cuda")
        coeffs = fem.make_coeffs(prec, fem.FIELD, c, field=f, degree=d, a_off=a_off,
                                 b_off=b_off, status=status, workspace=ws)
        call = fem.fem_integrate_noalloc if noalloc else fem.fem_integrate
        rc = call(nel, 0, fem._ptr(g), coeffs, fem._ptr(A), fem._ptr(b), fem._stream(None))
        assert rc == fem.FEM_OK, fem.fem_strerror(rc)
        torch.cuda.synchronize()
        outs.append((A.cpu().numpy(), b.cpu().numpy(), status.cpu().numpy()))
    return outs


@pytest.mark.parametrize("strategy", [0, 1])
@pytest.mark.parametrize("prec", ["split_fp16", "fp32", "fp64"])
def test_noalloc_mixed_equals_workspace_call(fem, prec, strategy):
    w = synth.make(4, grid=(9, 7, 5))  # 315 elements of degrees 1..7, FIELD coefficients
    code = fem.PRECISIONS[prec]
    saved = fem.fem_get_variant(0, code, fem.FIELD)
    fem.fem_set_variant(0, code, fem.FIELD, strategy)
    try:
        # the larger call first, then a smaller one: the scratch still holds the first call's
        # buckets and counters, which the second must not see
        for nel in (w.nel, 97):
            (A0, b0, s0), (A1, b1, s1) = _mixed_pair(fem, w, prec, nel)
            assert not np.isnan(A1).any() and not np.isnan(b1).any()
            np.testing.assert_array_equal(A1, A0)
            np.testing.assert_array_equal(b1, b0)
            np.testing.assert_array_equal(s1, s0)
            log(f"[noalloc] mixed FIELD prec={prec} strategy={strategy} nel={nel}: bitwise equal")
    finally:
        fem.fem_set_variant(0, code, fem.FIELD, saved)


def test_noalloc_uniform_equals_integrate(fem):
    import torch
    w = synth.make(2, p=3, grid=(5, 4, 3))
    g, c = to_dev(w.geom, w.coef)
    A0, b0 = fem.integrate(g, c, 3, precision="split_fp16")
    A1 = torch.empty_like(A0)
    b1 = torch.empty_like(b0)
    coeffs = fem.make_coeffs("split_fp16", fem.ELEMENT, c)
    rc = fem.fem_integrate_noalloc(w.nel, 3, fem._ptr(g), coeffs, fem._ptr(A1), fem._ptr(b1),
                                   fem._stream(None))
    assert rc == fem.FEM_OK, fem.fem_strerror(rc)
    torch.cuda.synchronize()
    assert torch.equal(A0, A1) and torch.equal(b0, b1)


def test_noalloc_rejects_more_elements_than_the_scratch(fem):
    import torch
    d = torch.ones(4, dtype=torch.int8, device="cuda")
    c = torch.zeros((4, 10), dtype=torch.float64, device="cuda")
    coeffs = fem.make_coeffs("split_fp16", fem.FIELD, c, field=c, degree=d, a_off=c, b_off=c)
    # host-side check on the count only: nothing is enqueued, no buffer is touched
    rc = fem.fem_integrate_noalloc(fem.NOALLOC_MAX_NEL + 1, 0, fem._ptr(c), coeffs, fem._ptr(c),
                                   fem._ptr(c), fem._stream(None))
    assert rc == fem.FEM_ETOOBIG
    assert "static scratch" in fem.fem_strerror(rc)
