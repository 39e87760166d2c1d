"""GPU tests of the host-staged pipeline (meshes in host memory, chunks over several streams):
bitwise equal to the device-resident call for every chunking and stream count, within the
tolerance of the FP64 oracle, in every coefficient mode; pageable and pinned host memory;
status counts; stage statistics; argument errors."""
import numpy as np
import pytest

from gpu_cases import TOL_A, cdr_case, log, oracle_uniform, rel_fro, to_dev
from paper_1310_1191_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fem():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_1310_1191_amd import fem as F
    F.fem_init(0)
    return F


def host(*arrays, pin=True):
    import torch
    out = []
    for a in arrays:
        t = torch.from_numpy(np.ascontiguousarray(a))
        out.append(t.pin_memory() if pin else t)
    return out


@pytest.mark.parametrize("chunk,nstreams", [(1, 2), (37, 1), (37, 3), (100, 2), (504, 3), (5000, 4)])
def test_staged_equals_device_path(fem, chunk, nstreams):
    import torch
    geom, coef, A_ref, b_ref, _ = oracle_uniform(2)
    g, c = to_dev(geom, coef)
    A0, b0 = fem.integrate(g, c, 2, precision="split_fp16")
    torch.cuda.synchronize()
    gh, ch = host(geom, coef)
    A, b, st = fem.integrate_staged(gh, ch, 2, precision="split_fp16", chunk=chunk, nstreams=nstreams)
    log(f"[staged] chunk={chunk} streams={nstreams} chunks={st['chunks']} total {st['total_ms']:.2f} ms")
    assert torch.equal(A, A0.cpu()) and torch.equal(b, b0.cpu())
    assert rel_fro(A.double().numpy(), A_ref).max() <= TOL_A["split_fp16"]
    nel = geom.shape[0]
    assert st["chunks"] == -(-nel // min(chunk, nel))
    assert st["h2d_bytes"] == nel * (192 + 14 * 8)
    assert st["d2h_bytes"] == nel * (27 * 27 + 27) * 4
    assert st["total_ms"] > 0 and st["kernel_ms"] > 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_staged_pageable_memory(fem, prec):
    import torch
    geom, coef = cdr_case(3)
    g, c = to_dev(geom, coef)
    A0, b0 = fem.integrate(g, c, 3, precision=prec)
    torch.cuda.synchronize()
    gh, ch = host(geom, coef, pin=False)
    A, b, _ = fem.integrate_staged(gh, ch, 3, precision=prec, chunk=25, nstreams=2,
                                   out_A=torch.empty(A0.shape, dtype=A0.dtype),
                                   out_b=torch.empty(b0.shape, dtype=b0.dtype))
    assert torch.equal(A, A0.cpu()) and torch.equal(b, b0.cpu())


def test_staged_field_and_elastic(fem):
    import torch
    w = synth.make(4, grid=(4, 3, 2))
    g, c, f = to_dev(w.geom, w.coef, w.field)
    A0, b0 = fem.integrate(g, c, 3, precision="split_fp16", mode=fem.FIELD, field=f)
    torch.cuda.synchronize()
    gh, ch, fh = host(w.geom, w.coef, w.field)
    A, b, _ = fem.integrate_staged(gh, ch, 3, precision="split_fp16", mode=fem.FIELD, field=fh,
                                   chunk=7, nstreams=3)
    assert torch.equal(A, A0.cpu()) and torch.equal(b, b0.cpu())
    rng = np.random.default_rng(5)
    geom = synth.element_vertices(synth.node_grid(3, 2, 2, 0.15, rng))
    coef = synth.elastic_coeffs(geom.shape[0], rng)
    g, c = to_dev(geom, coef)
    A0, b0 = fem.integrate(g, c, 2, precision="fp32", mode=fem.ELASTIC)
    torch.cuda.synchronize()
    gh, ch = host(geom, coef)
    A, b, st = fem.integrate_staged(gh, ch, 2, precision="fp32", mode=fem.ELASTIC, chunk=5, nstreams=2)
    assert torch.equal(A, A0.cpu()) and torch.equal(b, b0.cpu())
    assert st["d2h_bytes"] == geom.shape[0] * (9 * 27 * 27 + 3 * 27) * 4


def test_staged_without_load_vector_and_status(fem):
    import torch
    geom, coef = cdr_case(2)
    geom = geom.copy()
    geom[[3, 40]] = geom[[3, 40]][:, [1, 0, 3, 2, 5, 4, 7, 6]]   # two mirrored elements
    gh, ch = host(geom, coef)
    status = torch.tensor([5, 0], dtype=torch.int32)
    A, b, _ = fem.integrate_staged(gh, ch, 2, precision="fp32", chunk=64, nstreams=2,
                                   with_b=False, status=status)
    assert b is None
    assert status.tolist() == [7, 0]     # added to what the array held


def test_staged_argument_errors(fem):
    import torch
    geom, coef = cdr_case(2)
    gh, ch = host(geom, coef)
    nel = geom.shape[0]
    out = torch.empty(nel * 27 * 27, dtype=torch.float32)
    c = fem.make_coeffs("fp32", fem.ELEMENT, ch)
    call = lambda p, chunk, ns, cc=c: fem.fem_integrate_staged(nel, p, gh.data_ptr(), cc,
                                                                out.data_ptr(), None, chunk, ns, None)
    assert call(0, 10, 1) == fem.FEM_EDEGREE
    assert call(8, 10, 1) == fem.FEM_EDEGREE
    assert call(2, 0, 1) == fem.FEM_EINVAL
    assert call(2, 10, 0) == fem.FEM_EINVAL
    assert call(2, 10, fem.STAGED_MAX_STREAMS + 1) == fem.FEM_EINVAL
    jac = torch.zeros(10, dtype=torch.float64)
    assert call(2, 10, 1, fem.make_coeffs("fp32", fem.ELEMENT, ch, jac=jac)) == fem.FEM_EINVAL
    assert fem.fem_integrate_staged(0, 2, None, c, None, None, 10, 1, None) == fem.FEM_OK
