"""Parity at the workloads' full sizes, in the launch configuration the benchmark times (the
default tile variant of each degree and precision, the default mixed-degree strategy):

* sampled elements (random, plus the first and the last) against the FP64 oracle, one by one;
* on every element, a property exact for the quadrature sums: the shape functions sum to one
  and their gradients to zero, so each row sum of A is c / f times the load-vector entry
  (A 1 = (c / f) b, ELEMENT mode), checked where |f| is not small;
* the mixed-degree batch of 200000 elements and the 50-step time-stepped replay of 100000
  elements on their samples;
* the limits: an output indexed past 2^31 entries, and meshes scaled by 1e-4 and 1e4.
"""
import numpy as np
import pytest

from gpu_cases import TOL_A, TOL_B, log, rel_fro, rel_vec, to_dev
from paper_1310_1191_amd import synth

pytestmark = pytest.mark.gpu

# |sum_j A_ij - (c/f) b_i| / max_i sum_j |A_ij| per element: accumulated rounding of the
# contraction (relative error per entry within TOL_A) summed over a row of Ns entries, plus the
# load vector's own error; bounded by Ns * TOL_A with margin, and an absolute floor for FP64
ROWSUM_TOL = {"fp64": 1e-11, "fp32": 2e-5, "split_fp16": 4e-6, "bf16": 5e-2}


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


def rowsum_error(torch, A, b, coef):
    """Per-element max_i |sum_j A_ij - (c/f) b_i| / max_i sum_j |A_ij| on the device, over
    elements with |f| >= 0.05."""
    c = torch.from_numpy(coef[:, 12]).to(A.device)
    f = torch.from_numpy(coef[:, 13]).to(A.device)
    keep = f.abs() >= 0.05
    Ad = A[keep].double()
    rs = Ad.sum(dim=2)
    ref = (c[keep] / f[keep])[:, None] * b[keep].double()
    scale = Ad.abs().sum(dim=2).amax(dim=1)
    return ((rs - ref).abs().amax(dim=1) / scale).max().item()


def check_uniform(fem, torch, w, p, prec, nsample):
    import oracle
    g, c = to_dev(w.geom, w.coef)
    A, b = fem.integrate(g, c, p, precision=prec)
    torch.cuda.synchronize()
    idx = sample(w.nel, nsample, 100 + p)
    Aref, bref, _ = oracle.integrate(w.geom[idx], w.coef[idx], p=p)
    ti = torch.from_numpy(idx).to(A.device)
    ea = rel_fro(A[ti].double().cpu().numpy(), Aref)
    eb = rel_vec(b[ti].double().cpu().numpy(), bref)
    rs = rowsum_error(torch, A, b, w.coef)
    log(f"[fullsize] p={p} prec={prec} nel={w.nel} sample={idx.size} errA max={ea.max():.3e} "
        f"errb max={eb.max():.3e} rowsum={rs:.3e}")
    assert ea.max() <= TOL_A[prec] and eb.max() <= TOL_B[prec]
    assert rs <= ROWSUM_TOL[prec]
    del A, b
    torch.cuda.empty_cache()


@pytest.mark.parametrize("p", [2, 3, 4])
@pytest.mark.parametrize("prec", ["split_fp16", "fp32"])
def test_plain_method_full_size(fem, p, prec):
    import torch
    check_uniform(fem, torch, synth.make(2, p=p), p, prec, 16)


@pytest.mark.parametrize("p", [5, 6, 7])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "split_fp16", "bf16"])
def test_high_order_full_size(fem, p, prec):
    import torch
    check_uniform(fem, torch, synth.make(3, p=p), p, prec, {5: 6, 6: 3, 7: 2}[p])


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
    import torch
    w = synth.make(4)
    g, c, f, d = to_dev(w.geom, w.coef, w.field, w.degree)
    A, b, a_off, b_off = fem.integrate_mixed(g, c, d, precision=prec, mode=fem.FIELD, field=f)
    torch.cuda.synchronize()
    idx = sample(w.nel, 24, 7)
    ea, eb = packed_errors(A, b, a_off.cpu().numpy(), b_off.cpu().numpy(), w, idx,
                           oracle_field_sample(w, w.field, idx))
    log(f"[fullsize] mixed prec={prec} nel={w.nel} strategy={fem.fem_get_variant(0, fem.PRECISIONS[prec], fem.FIELD)} "
        f"errA max={ea:.3e} errb max={eb:.3e}")
    assert ea <= TOL_A[prec] and eb <= TOL_B[prec]


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
