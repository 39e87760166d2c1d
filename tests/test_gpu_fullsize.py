"""Parity at the workloads' full sizes, in the launch configuration the benchmark times (the
default tile variant of each degree and precision, the default mixed-degree strategy):

* p = 1..4 (the Poisson meshes 16^3 and 128^3, the p = 2, 3, 4 CDR meshes of 262144, 131072
  and 65536 elements): EVERY element of every checked precision against the FP64 oracle, which
  runs chunk by chunk on the host; the maximum, p99 and median of the per-element errors are
  printed;
* p = 5..7: seeded samples (48, 24, 16 elements, plus the first and the last), one oracle run
  per degree shared by the precisions;
* the mixed-degree batch of 200000 elements through both strategies (samples against the oracle;
  with the same tiles the two strategies agree bit for bit on every element), and the 50-step
  time-stepped replay of 100000 elements on its samples;
* the limits: an output indexed past 2^31 entries, and meshes scaled by 1e-4 and 1e4.
"""
import functools

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


def sample(nel, k, seed):
    idx = np.random.default_rng(seed).choice(nel, k, replace=False)
    return np.unique(np.concatenate([[0, nel - 1], idx]))


def every_element(fem, torch, w, p, precs, chunk):
    """Integrate the whole mesh in each precision, then compare every element with the oracle,
    which runs on chunks of `chunk` elements; the per-element relative errors are reduced on
    the device. Returns {prec: (errA [nel], errb [nel])}."""
    import oracle
    g, c = to_dev(w.geom, w.coef)
    outs = {}
    for prec in precs:
        print(f"[fullsize-every] p={p} prec={prec} nel={w.nel}", flush=True)
        outs[prec] = fem.integrate(g, c, p, precision=prec)
    torch.cuda.synchronize()
    errs = {prec: (np.empty(w.nel), np.empty(w.nel)) for prec in precs}
    for s in range(0, w.nel, chunk):
        e = min(w.nel, s + chunk)
        Aref, bref, fl = oracle.integrate(w.geom[s:e], w.coef[s:e], p=p)
        assert fl.max() == 0
        Ar, br = to_dev(Aref, bref)
        nA = Ar.square().sum(dim=(1, 2)).sqrt()
        nb = br.square().sum(dim=1).sqrt().clamp_min(1e-300)
        for prec in precs:
            A, b = outs[prec]
            dA = (A[s:e].double() - Ar).square().sum(dim=(1, 2)).sqrt() / nA
            db = (b[s:e].double() - br).square().sum(dim=1).sqrt() / nb
            errs[prec][0][s:e] = dA.cpu().numpy()
            errs[prec][1][s:e] = db.cpu().numpy()
        del Ar, br
    for prec in precs:
        ea, eb = errs[prec]
        log(f"[fullsize-every] p={p} prec={prec} nel={w.nel} errA max={ea.max():.3e} "
            f"p99={np.percentile(ea, 99):.3e} median={np.median(ea):.3e} errb max={eb.max():.3e}")
    del outs
    torch.cuda.empty_cache()
    return errs


@pytest.mark.parametrize("p", [2, 3, 4])
def test_every_element_full_size(fem, p):
    import torch
    w = synth.make(2, p=p)
    precs = ["split_fp16", "fp32"]
    errs = every_element(fem, torch, w, p, precs, {2: 32768, 3: 16384, 4: 4096}[p])
    for prec in precs:
        ea, eb = errs[prec]
        assert ea.max() <= TOL_A[prec] and eb.max() <= TOL_B[prec], prec


@pytest.mark.parametrize("grid", [(16, 16, 16), (128, 128, 128)])
def test_poisson_every_element(fem, grid):
    import torch
    w = synth.make(1, grid=grid)
    precs = ["fp64", "fp32", "split_fp16"]
    errs = every_element(fem, torch, w, 1, precs, 262144)
    for prec in precs:
        ea, eb = errs[prec]
        assert ea.max() <= TOL_A[prec] and eb.max() <= TOL_B[prec], prec


@functools.lru_cache(maxsize=None)
def high_order_reference(p):
    import oracle
    w = synth.make(3, p=p)
    idx = sample(w.nel, {5: 48, 6: 24, 7: 16}[p], 100 + p)
    Aref, bref, fl = oracle.integrate(w.geom[idx], w.coef[idx], p=p)
    assert fl.max() == 0
    return w, idx, Aref, bref


@pytest.mark.parametrize("p", [5, 6, 7])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "split_fp16", "bf16"])
def test_high_order_full_size(fem, p, prec):
    import torch
    w, idx, Aref, bref = high_order_reference(p)
    g, c = to_dev(w.geom, w.coef)
    print(f"[fullsize] p={p} prec={prec} nel={w.nel}", flush=True)
    A, b = fem.integrate(g, c, p, precision=prec)
    torch.cuda.synchronize()
    ti = torch.from_numpy(idx).to(A.device)
    ea = rel_fro(A[ti].double().cpu().numpy(), Aref)
    eb = rel_vec(b[ti].double().cpu().numpy(), bref)
    log(f"[fullsize] p={p} prec={prec} nel={w.nel} sample={idx.size} errA max={ea.max():.3e} "
        f"p99={np.percentile(ea, 99):.3e} errb max={eb.max():.3e}")
    assert ea.max() <= TOL_A[prec] and eb.max() <= TOL_B[prec]
    del A, b
    torch.cuda.empty_cache()


def packed_errors(A, b, a_off, b_off, w, idx, ref):
    ea, eb = [], []
    for k, e in enumerate(idx):
        ns = (int(w.degree[e]) + 1) ** 3
        Ag = A[a_off[e]:a_off[e + 1]].double().cpu().numpy().reshape(ns, ns)
        bg = b[b_off[e]:b_off[e + 1]].double().cpu().numpy()
        ea.append(rel_fro(Ag[None], ref[k][0][None])[0])
        eb.append(rel_vec(bg[None], ref[k][1][None])[0])
    return max(ea), max(eb)


def oracle_field_sample(w, field, idx):
    import oracle
    out = {}
    for p in range(1, 8):
        sel = [e for e in idx if int(w.degree[e]) == p]
        if sel:
            A, b, _ = oracle.integrate(w.geom[sel], w.coef[sel], p=p, mode=oracle.FIELD, field=field)
            out.update({e: (A[k], b[k]) for k, e in enumerate(sel)})
    return [out[e] for e in idx]


@pytest.mark.parametrize("prec", ["split_fp16", "fp32"])
def test_mixed_degree_full_size(fem, prec):
    """The 200000-element mixed-degree batch through both strategies (one persistent launch over
    every degree; one launch per degree with the default tiles): 256 seeded elements of each
    against the oracle. With the per-degree launches set to the single launch's tiles, the two
    strategies agree bit for bit on every element."""
    import torch
    w = synth.make(4)
    g, c, f, d = to_dev(w.geom, w.coef, w.field, w.degree)
    code = fem.PRECISIONS[prec]
    saved = {p: fem.fem_get_variant(p, code, fem.FIELD) for p in range(8)}
    idx = sample(w.nel, 256, 7)
    ref = oracle_field_sample(w, w.field, idx)
    try:
        single = None
        for strategy, name in ((0, "single_launch"), (1, "per_degree_launches")):
            fem.fem_set_variant(0, code, fem.FIELD, strategy)
            print(f"[fullsize] mixed prec={prec} strategy={name}", flush=True)
            A, b, a_off, b_off = fem.integrate_mixed(g, c, d, precision=prec, mode=fem.FIELD, field=f)
            torch.cuda.synchronize()
            ea, eb = packed_errors(A, b, a_off.cpu().numpy(), b_off.cpu().numpy(), w, idx, ref)
            log(f"[fullsize] mixed prec={prec} nel={w.nel} strategy={name} errA max={ea:.3e} errb max={eb:.3e}")
            assert ea <= TOL_A[prec] and eb <= TOL_B[prec]
            if strategy == 0:
                single = (A, b)
            del A, b
        for p in range(1, 8):
            fem.fem_set_variant(p, code, fem.FIELD, fem.mixed_tile_variant(p, code, fem.FIELD))
        print(f"[fullsize] mixed prec={prec} per-degree launches with the single launch's tiles", flush=True)
        A, b, _, _ = fem.integrate_mixed(g, c, d, precision=prec, mode=fem.FIELD, field=f)
        torch.cuda.synchronize()
        assert torch.equal(A, single[0]) and torch.equal(b, single[1])
    finally:
        for p, v in saved.items():
            fem.fem_set_variant(p, code, fem.FIELD, v)


def test_time_steps_full_size(fem):
    """The 100000-element, 50-step replay of the time-stepped workload; the 1 % samples of steps
    1, 25 and 50 against the oracle with that step's fields."""
    import torch
    w = synth.make(5)
    nsteps = 50
    deltas = np.stack([synth.phase_shift(w.seed, t) for t in range(1, nsteps + 1)]).reshape(nsteps, 35)
    g, c, f0, d, dl = to_dev(w.geom, w.coef, w.field, w.degree, deltas)
    f = f0.clone()
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = torch.empty(fem.fem_workspace_bytes(w.nel), dtype=torch.uint8, device="cuda")
    a_off, b_off = fem.mixed_offsets(d, workspace=ws)
    torch.cuda.synchronize()
    A = torch.empty(int(a_off[-1].item()), dtype=torch.float32, device="cuda")
    b = torch.empty(int(b_off[-1].item()), dtype=torch.float32, device="cuda")
    a_np, b_np = a_off.cpu().numpy(), b_off.cpu().numpy()

    def one_step(stream=None):
        fem.field_advance(f, dl, step, stream=stream)
        fem.integrate_mixed(g, c, d, precision="split_fp16", mode=fem.FIELD, field=f, a_off=a_off,
                            b_off=b_off, out_A=A, out_b=b, workspace=ws, stream=stream)

    one_step()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            one_step(stream=s)
    torch.cuda.synchronize()
    f.copy_(f0)
    step.zero_()
    torch.cuda.synchronize()
    for t in range(1, nsteps + 1):
        graph.replay()
        if t in (1, 25, 50):
            torch.cuda.synchronize()
            idx = synth.step_sample(w.seed, t, w.nel)[::4]     # a quarter of the 1 % sample
            ea, eb = packed_errors(A, b, a_np, b_np, w, idx,
                                   oracle_field_sample(w, synth.field_at_step(w.field, w.seed, t), idx))
            log(f"[fullsize] time step {t}: {idx.size} elements, errA max={ea:.3e} errb max={eb:.3e}")
            assert ea <= TOL_A["split_fp16"] and eb <= TOL_B["split_fp16"]
    torch.cuda.synchronize()
    assert int(step.item()) == nsteps


def test_output_offsets_beyond_int32(fem):
    """p = 4 with 140000 elements: the output (2.19e9 entries, 8.75 GB) is indexed past 2^31;
    elements on both sides of that boundary and the last one against the oracle."""
    import oracle
    import torch
    base = synth.make(2, p=4, grid=(10, 10, 10))
    reps = 140
    geom = np.tile(base.geom, (reps, 1, 1))
    coef = np.tile(base.coef, (reps, 1))
    nel = geom.shape[0]
    ns2 = 125 * 125
    assert nel * ns2 > 2 ** 31
    g, c = to_dev(geom, coef)
    A = torch.empty((nel, 125, 125), dtype=torch.float32, device="cuda")
    b = torch.empty((nel, 125), dtype=torch.float32, device="cuda")
    fem.integrate(g, c, 4, precision="split_fp16", out_A=A, out_b=b)
    torch.cuda.synchronize()
    cross = 2 ** 31 // ns2
    idx = np.array([0, cross - 1, cross, cross + 1, nel - 1])
    Aref, bref, _ = oracle.integrate(geom[idx], coef[idx], p=4)
    ti = torch.from_numpy(idx).cuda()
    ea = rel_fro(A[ti].double().cpu().numpy(), Aref)
    eb = rel_vec(b[ti].double().cpu().numpy(), bref)
    log(f"[fullsize] p=4 nel={nel} entries={nel * ns2:.3e} errA max={ea.max():.3e} errb max={eb.max():.3e}")
    assert ea.max() <= TOL_A["split_fp16"] and eb.max() <= TOL_B["split_fp16"]


@pytest.mark.parametrize("scale", [1e-4, 1e4])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "split_fp16"])
def test_extreme_element_sizes(fem, scale, prec):
    """Meshes scaled by 1e-4 and 1e4 (detJ ~ 1e-12 and 1e12 per unit element): the per-element
    power-of-two scaling keeps the split products in FP16 range, so relative errors hold."""
    import oracle
    import torch
    w = synth.make(2, p=3, grid=(4, 3, 3))
    geom = w.geom * scale
    A_ref, b_ref, _ = oracle.integrate(geom, w.coef, p=3)
    g, c = to_dev(geom, w.coef)
    status = torch.zeros(2, dtype=torch.int32, device="cuda")
    A, b = fem.integrate(g, c, 3, precision=prec, status=status)
    torch.cuda.synchronize()
    ea = rel_fro(A.double().cpu().numpy(), A_ref)
    eb = rel_vec(b.double().cpu().numpy(), b_ref)
    log(f"[fullsize] scale={scale:g} prec={prec} errA max={ea.max():.3e} errb max={eb.max():.3e}")
    assert status.cpu().tolist() == [0, 0]
    assert ea.max() <= TOL_A[prec] and eb.max() <= TOL_B[prec]
