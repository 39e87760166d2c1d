#!/usr/bin/env python3
"""Throughput of element stiffness-matrix integration on one MI355X.

One step integrates the whole hot path over the plain-method workload at scale: tensor-product
Lagrange hexahedra of degree 2, 3 and 4 (27/64/125 shape functions) on jittered structured
grids of 64x64x64, 64x64x32 and 64x32x32 elements (262144 + 131072 + 65536 elements),
convection-diffusion-reaction coefficients per element, (p+1)^3 Gauss points, FP32 output.
Each step runs every stage of the path on the GPU: FP64 Jacobian prologue, point-matrix fold,
MFMA contraction, load vector and the stores of A and b. Inputs are resident in HBM before
timing starts; outputs stay on the device.

The reported value is element matrices per second for the split-FP16 contraction (three FP16
MFMA products per term, FP32 accumulation, <= 1e-6 relative error against the FP64 oracle).
The same step is also timed with the plain FP32 MFMA path for comparison.

``python bench.py [--steps K] [--warmup W] [--precision split_fp16] [--no-cpu-baseline]
[--no-extras]`` prints one JSON line. Besides the headline it carries, under ``extras``, every
other workload of the build measured in the same run (p = 1 Poisson at 16^3 -- also replayed from
a graph -- and 128^3; p = 5, 6, 7 in five precisions; the 200000-element mixed-degree batch in
both strategies; the 50-step graph-replayed time loop; prisms p = 1..7 and the paper's prism
elastostatics), each with per-element error statistics against the FP64 oracle on samples.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "split_bf16": 2500.0,
               "split_fp16": 2500.0}
PRODUCTS = {"fp64": 1, "fp32": 1, "bf16": 1, "split_bf16": 3, "split_fp16": 3}
WORKLOAD = [(2, (64, 64, 64)), (3, (64, 64, 32)), (4, (64, 32, 32))]


PRISM_TRI_POINTS = {1: 3, 2: 6, 3: 12, 4: 16, 5: 25, 6: 33, 7: 42}


def nq_prism(p: int) -> int:
    return PRISM_TRI_POINTS[p] * (p + 1)


def sizes(p: int, prism: bool = False):
    """(Ns, NQ): (p+1)^3 and (p+1)^3 for the hexahedron; (p+1)^2 (p+2)/2 and Table 1's N_Q for
    the prism."""
    if prism:
        return (p + 1) * (p + 1) * (p + 2) // 2, nq_prism(p)
    return (p + 1) ** 3, (p + 1) ** 3


def flops_per_element(p: int, prism: bool = False) -> float:
    """Algorithmic work of one element: the contraction 8 Ns^2 NQ plus the load vector 2 Ns NQ."""
    ns, nq = sizes(p, prism)
    return 8.0 * ns * ns * nq + 2.0 * ns * nq


def bytes_per_element(p: int, out_bytes: int = 4, prism: bool = False) -> float:
    """Algorithmic HBM bytes of one element: the FP64 vertex coordinates (24, or 18 for a prism),
    a 14-double coefficient record, and the unpadded A (Ns^2) and b (Ns) outputs."""
    ns, _ = sizes(p, prism)
    return (144.0 if prism else 192.0) + 112.0 + (ns * ns + ns) * out_bytes


def log(msg):
    print(msg, file=sys.stderr, flush=True)


KERNEL_SOURCES = ["fem_kernel.h", "fem_launch.h", "fem_layout.h", "fem_geometry.h"]


def kernel_source_hash() -> str:
    """Hash of the kernel sources with comments and whitespace removed (a comment edit keeps a
    counter summary valid; any code change invalidates it)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1310_1191_amd", "csrc", name)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update(re.sub(r"\s+", "", text).encode())
    return h.hexdigest()[:16]


def measured_traffic(p: int, precision: str, variant: int):
    """HBM bytes per launch of the dominant kernel from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by what the counter reads for a copy of known size),
    or None when there is no summary for this kernel or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"k_integrate_p{p}_{precision}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("traffic-record: "):
            rec = json.loads(line[len("traffic-record: "):])
    if not rec or rec.get("sources") != kernel_source_hash() or rec.get("variant") != variant:
        return None
    return rec["bytes_per_launch"]


def _oracle_rate(meshes, threads, budget_s):
    """Seconds per element of the oracle for each degree of ``meshes`` on ``threads`` threads,
    from the first elements of each mesh (about budget_s / len(meshes) of CPU time per degree)."""
    import oracle
    per_el, samples = {}, []
    for p, geom, coef in meshes:
        probe = min(geom.shape[0], max(threads, 8))
        t0 = time.perf_counter()
        oracle.integrate(geom[:probe], coef[:probe], p=p, threads=threads)
        t_probe = time.perf_counter() - t0
        n = int(min(geom.shape[0],
                    max(probe, probe * (budget_s / len(meshes)) / max(t_probe, 1e-6))))
        t0 = time.perf_counter()
        oracle.integrate(geom[:n], coef[:n], p=p, threads=threads)
        dt = time.perf_counter() - t0
        per_el[p] = dt / n
        samples.append(f"p={p}: first {n} elements in {dt:.2f} s")
    return per_el, samples


def cpu_baseline(meshes, budget_s: float = 12.0):
    """The FP64 oracle on the host cores (gcc -O3 -march=native, OpenMP over elements), timed on
    a bounded sample of the same workload, and on one thread."""
    import oracle
    oracle.build(force=False)
    threads = oracle.max_threads()
    total_el = sum(g.shape[0] for _, g, _ in meshes)
    per_el, samples = _oracle_rate(meshes, threads, budget_s)
    total_t = sum(per_el[p] * g.shape[0] for p, g, _ in meshes)
    per1, samples1 = _oracle_rate(meshes, 1, budget_s / 3.0)
    total_1 = sum(per1[p] * g.shape[0] for p, g, _ in meshes)
    return {"value": total_el / total_t, "unit": "element matrices/s", "cores": threads,
            "kind": "oracle", "sample": "; ".join(samples) + " (FP64, OpenMP over elements; "
            "rate scaled to the full step's element mix)",
            "single_thread": {"value": total_el / total_1, "unit": "element matrices/s",
                              "sample": "; ".join(samples1)},
            "gflops_fp64": sum(flops_per_element(p) * g.shape[0] for p, g, _ in meshes) / total_t / 1e9}


def check_fractions(obj, path="line"):
    """Every fraction of a peak in the record (keys "frac..."), at any depth, lies in [0, 1]: a
    value above 1 means the counted work was not the work done."""
    if isinstance(obj, dict):
        for k, v in obj.items():
            if k.startswith("frac") and isinstance(v, (int, float)) and not 0.0 <= v <= 1.0:
                raise ValueError(f"{path}.{k} = {v}: a fraction of a peak outside [0, 1]")
            check_fractions(v, f"{path}.{k}")
    elif isinstance(obj, list):
        for i, v in enumerate(obj):
            check_fractions(v, f"{path}[{i}]")


def err_stats(errs):
    """Max, 99th percentile and median of per-element relative errors."""
    e = np.asarray(errs, dtype=np.float64)
    return {"n": int(e.size), "max": float(e.max()), "p99": float(np.percentile(e, 99)),
            "median": float(np.median(e))}


def rel_fro_rows(A, R):
    """Per-element ||A - R||_F / ||R||_F over all but the first axis."""
    ax = tuple(range(1, A.ndim))
    return np.sqrt(((A - R) ** 2).sum(axis=ax) / (R ** 2).sum(axis=ax))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="split_fp16")
    ap.add_argument("--compare", default="fp32", help="second path timed for comparison ('' = none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only (no other workloads in the line)")
    ap.add_argument("--workload", default="plain",
                    choices=["plain", "high", "mixed", "timestep", "poisson", "elasticity", "nojac",
                             "staged", "degree", "prism", "prism-elastic"],
                    help="plain: p = 2, 3, 4 at scale (the headline, with every other workload under "
                         "'extras'); high: p = 5, 6, 7 in every precision; mixed: 200000 elements of "
                         "degrees 1..7 with coefficient fields, one launch against per-degree launches; "
                         "timestep: 50 graph-replayed steps of 100000 mixed-degree elements; poisson: "
                         "p = 1; elasticity: the vector model problem (linear elastostatics) for "
                         "p = 2..7; nojac: supplied per-point Jacobian terms against computed ones for "
                         "p = 1..7; staged: the plain workload from and to pinned host memory, chunks "
                         "over streams; degree: one degree's benchmark mesh (--degree) in --precision, "
                         "for profilers; prism: prismatic elements p = 1..7; prism-elastic: the "
                         "paper's own benchmark, elastostatics on prisms p = 2..7")
    ap.add_argument("--degree", type=int, default=4, help="degree of the 'degree' workload (1..7)")
    ap.add_argument("--variant", type=int, default=-1,
                    help="'degree' workload: the tile variant to launch (default: the library's choice)")
    ap.add_argument("--nojac", action="store_true",
                    help="timestep workload: read per-point Jacobian terms written once before the "
                         "time loop instead of computing them in every step")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run a plain elementwise copy y = -x of MIB MiB three times (the "
                         "known-size kernel that calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the integration shards "
              "elements across GPUs without communication, and this benchmark measures one GPU's "
              "share.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1310_1191_amd import fem, synth

    assert torch.cuda.is_available(), "no GPU visible"
    dev = torch.device("cuda:0")
    fem.fem_init(0)

    if args.copy_probe > 0:
        n = args.copy_probe * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            torch.neg(x, out=y)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: 3 x (read {n * 4} B + write {n * 4} B)")
        del x, y
        torch.cuda.empty_cache()

    if args.workload != "plain":
        line = WORKLOADS[args.workload](args, torch, fem, synth, dev)
        check_fractions(line)
        print(json.dumps(line), flush=True)
        return

    t0 = time.time()
    meshes = []
    for p, grid in WORKLOAD:
        w = synth.make(2, p=p, grid=grid)
        meshes.append((p, w.geom, w.coef))
    log(f"[bench] generated workload in {time.time() - t0:.1f} s: "
        + ", ".join(f"p={p} nel={g.shape[0]}" for p, g, _ in meshes))

    dev_in = []
    for p, geom, coef in meshes:
        g = torch.from_numpy(geom).to(dev)
        c = torch.from_numpy(coef).to(dev)
        dev_in.append((p, g, c))

    def run_path(precision, steps, warmup, record_events):
        """Time `steps` steps; returns (seconds, per-degree ms, outputs of the last step)."""
        dt = fem.out_dtype(precision)
        outs = []
        for p, g, c in dev_in:
            ns = (p + 1) ** 3
            outs.append((torch.empty((g.shape[0], ns, ns), dtype=dt, device=dev),
                         torch.empty((g.shape[0], ns), dtype=dt, device=dev)))
        stream = torch.cuda.current_stream()
        ev = {p: [] for p, _, _ in dev_in}

        def step(timed):
            for (p, g, c), (A, b) in zip(dev_in, outs):
                if timed and record_events:
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                fem.integrate(g, c, p, precision=precision, out_A=A, out_b=b)
                if timed and record_events:
                    e1.record(stream)
                    ev[p].append((e0, e1))

        for _ in range(warmup):
            step(False)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for k in range(steps):
            step(True)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        per_p = {}
        if record_events:
            for p in ev:
                per_p[p] = float(np.mean([a.elapsed_time(b) for a, b in ev[p]]))  # ms
        return elapsed, per_p, outs

    def sampled_errors(outs, nsample):
        """Per-degree error statistics of the last step's outputs on seeded element samples."""
        import oracle
        res = {}
        for (p, geom, coef), (A, b) in zip(meshes, outs):
            n = min(nsample[p], geom.shape[0])
            idx = np.sort(np.random.default_rng(100 + p).choice(geom.shape[0], n, replace=False))
            Ar, br, _ = oracle.integrate(geom[idx], coef[idx], p=p, threads=oracle_threads())
            it = torch.from_numpy(idx).to(dev)
            Ag = A[it].double().cpu().numpy()
            bg = b[it].double().cpu().numpy()
            res[str(p)] = {"A": err_stats(rel_fro_rows(Ag, Ar)),
                           "b": err_stats(np.linalg.norm(bg - br, axis=1) / np.linalg.norm(br, axis=1))}
        return res

    nsample = {2: 2048, 3: 1024, 4: 512}
    log(f"[bench] {args.precision}: warmup {args.warmup}, timing {args.steps} steps")
    elapsed, per_p, outs = run_path(args.precision, args.steps, args.warmup, True)
    ms_per_step = elapsed / args.steps * 1e3
    total_el = sum(g.shape[0] for _, g, _ in dev_in)
    value = total_el / (elapsed / args.steps)
    log(f"[bench] {args.precision}: {ms_per_step:.3f} ms/step, {value:.4g} el/s")
    errors = sampled_errors(outs, nsample)
    log(f"[bench] {args.precision}: sampled errors " +
        ", ".join(f"p={p} max {e['A']['max']:.2e}" for p, e in errors.items()))
    del outs
    torch.cuda.empty_cache()

    per_degree = {}
    for p, g, _ in dev_in:
        t = per_p[p] * 1e-3
        nel = g.shape[0]
        fl = flops_per_element(p) * nel / t
        by = bytes_per_element(p) * nel / t
        per_degree[str(p)] = {
            "nel": nel, "ms": round(per_p[p], 4), "el_per_s": nel / t,
            "tflops": fl / 1e12, "gbs": by / 1e9,
            "frac_mfma": fl / 1e12 / PEAK_TFLOPS[args.precision],
            "frac_mfma_executed": fl * PRODUCTS[args.precision] / 1e12 / PEAK_TFLOPS[args.precision],
            "frac_hbm": by / 1e9 / HBM_PEAK_GBS,
            "rel_err": errors[str(p)]}

    # dominant kernel: the degree whose launch takes the longest
    pd = max(per_p, key=lambda p: per_p[p])
    nel_d = dict((p, g.shape[0]) for p, g, _ in dev_in)[pd]
    ach_flops = flops_per_element(pd) * nel_d / (per_p[pd] * 1e-3) / 1e12
    ach_bytes = bytes_per_element(pd) * nel_d / (per_p[pd] * 1e-3) / 1e9
    # bound: the matrix cores execute PRODUCTS x the algorithmic flops
    t_mfma = flops_per_element(pd) * PRODUCTS[args.precision] / (PEAK_TFLOPS[args.precision] * 1e12)
    t_hbm = bytes_per_element(pd) / (HBM_PEAK_GBS * 1e9)
    if t_mfma >= t_hbm:
        roof = {"bound": "mfma", "achieved": round(ach_flops, 3),
                "peak": PEAK_TFLOPS[args.precision], "unit": "TFLOP/s",
                "frac": round(ach_flops / PEAK_TFLOPS[args.precision], 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(ach_bytes, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach_bytes / HBM_PEAK_GBS, 4)}
    variant = fem.fem_get_variant(pd, fem.PRECISIONS[args.precision], fem.ELEMENT)
    roof["kernel"] = f"k_integrate p={pd} {args.precision} variant {variant}"
    roof["launch_ms"] = round(per_p[pd], 4)
    roof["traffic"] = measured_traffic(pd, args.precision, variant)

    compare = None
    if args.compare:
        csteps = max(3, args.steps // 4)
        log(f"[bench] comparison path {args.compare}: {csteps} steps")
        ce, cper, couts = run_path(args.compare, csteps, 1, True)
        cerr = sampled_errors(couts, {2: 512, 3: 256, 4: 128})
        del couts
        torch.cuda.empty_cache()
        compare = {"precision": args.compare, "ms_per_step": ce / csteps * 1e3,
                   "el_per_s": total_el / (ce / csteps),
                   "speedup_of_headline": (ce / csteps) / (elapsed / args.steps),
                   "per_degree_ms": {str(p): round(v, 4) for p, v in cper.items()},
                   "rel_err": cerr}

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU baseline (oracle) on a bounded sample")
        cpu = cpu_baseline(meshes)

    extras = None
    if not args.no_extras:
        extras = {}
        for name in EXTRAS:
            t0 = time.time()
            log(f"[bench] extra workload: {name}")
            extras[name] = WORKLOADS[name](args, torch, fem, synth, dev, quick=True)
            extras[name]["wall_s"] = round(time.time() - t0, 1)
            torch.cuda.empty_cache()

    line = {
        "metric": "element matrices/s (split-precision MFMA, <= 1e-6 relative error)",
        "value": value,
        "unit": "element matrices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"split_fp16": "f16x3->f32", "split_bf16": "bf16x3->f32", "fp32": "f32",
                  "fp64": "f64", "bf16": "bf16->f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "cdr-hex p=2,3,4 on 64x64x64/64x64x32/64x32x32 jittered grids "
                               "(262144+131072+65536 elements), FP32 output",
                   "precision": args.precision, "elements_per_step": total_el,
                   "error_sample": "seeded random elements of the last timed step against the "
                                   "FP64 oracle: " + ", ".join(f"p={p}: {n}" for p, n in nsample.items())},
        "roofline": roof,
        "per_degree": per_degree,
        "compare": compare,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    check_fractions(line)
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------------------------------------
# the other workloads (each prints its own JSON line with --workload; the default run collects
# them, with fewer repetitions, under "extras")
# ---------------------------------------------------------------------------------------------
def rel_fro(A, R):
    return float(np.linalg.norm(A - R) / np.linalg.norm(R))


def time_calls(torch, fn, steps, warmup):
    """Mean milliseconds of fn() over `steps` calls on the current stream (HIP events)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def oracle_threads():
    import oracle
    oracle.build(force=False)
    return oracle.max_threads()


def bench_high(args, torch, fem, synth, dev, quick=False):
    """p = 5, 6, 7 (16384 / 8192 / 4096 elements, CDR coefficients per element) in every
    precision; per-element error statistics of a seeded sample against the FP64 oracle."""
    import oracle
    precs = ["fp64", "fp32", "bf16", "split_bf16", "split_fp16"]
    out = {}
    nsample = {5: 48, 6: 24, 7: 16}
    reps = 3 if quick else max(3, args.steps // 4)
    for p in (5, 6, 7):
        w = synth.make(3, p=p)
        g = torch.from_numpy(w.geom).to(dev)
        c = torch.from_numpy(w.coef).to(dev)
        idx = np.sort(np.random.default_rng(p).choice(w.nel, nsample[p], replace=False))
        t0 = time.time()
        Aref, _, _ = oracle.integrate(w.geom[idx], w.coef[idx], p=p, threads=oracle_threads())
        log(f"[bench] high p={p}: oracle sample of {idx.size} in {time.time() - t0:.1f} s")
        ns = (p + 1) ** 3
        res = {"nel": w.nel}
        for prec in precs:
            A = torch.empty((w.nel, ns, ns), dtype=fem.out_dtype(prec), device=dev)
            b = torch.empty((w.nel, ns), dtype=fem.out_dtype(prec), device=dev)
            ms = time_calls(torch, lambda: fem.integrate(g, c, p, precision=prec, out_A=A, out_b=b),
                            reps, 1)
            Ag = A[torch.from_numpy(idx).to(dev)].double().cpu().numpy()
            st = err_stats(rel_fro_rows(Ag, Aref))
            fl = flops_per_element(p) * w.nel / (ms * 1e-3) / 1e12
            res[prec] = {"ms": round(ms, 4), "el_per_s": w.nel / (ms * 1e-3), "tflops": round(fl, 2),
                         "frac_peak": round(fl / PEAK_TFLOPS[prec], 4),
                         "frac_peak_executed": round(fl * PRODUCTS[prec] / PEAK_TFLOPS[prec], 4),
                         "rel_err": st}
            log(f"[bench] high p={p} {prec}: {ms:.3f} ms, {fl:.1f} TFLOP/s, max err {st['max']:.2e}")
            del A, b
            torch.cuda.empty_cache()
        out[str(p)] = res
    tot_el = sum(out[k]["nel"] for k in out)
    tot_ms = sum(out[k]["split_fp16"]["ms"] for k in out)
    return {"metric": "element matrices/s (split-precision MFMA, <= 1e-6 relative error)",
            "value": tot_el / (tot_ms * 1e-3), "unit": "element matrices/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f16x3->f32", "data": "synthetic",
            "config": {"workload": "cdr-hex p=5,6,7 on 32x32x16/32x16x16/16x16x16 jittered grids "
                                   "(16384+8192+4096 elements)",
                       "sample": "seeded random elements against the FP64 oracle: "
                                 + ", ".join(f"p={p}: {n}" for p, n in nsample.items())},
            "per_degree": out}


def mixed_buffers(torch, fem, w, dev, precision):
    g, c = torch.from_numpy(w.geom).to(dev), torch.from_numpy(w.coef).to(dev)
    f = torch.from_numpy(w.field).to(dev)
    d = torch.from_numpy(w.degree).to(dev)
    ws = torch.empty(fem.fem_workspace_bytes(w.nel), dtype=torch.uint8, device=dev)
    a_off, b_off = fem.mixed_offsets(d, workspace=ws)
    torch.cuda.synchronize()
    A = torch.empty(int(a_off[-1].item()), dtype=fem.out_dtype(precision), device=dev)
    b = torch.empty(int(b_off[-1].item()), dtype=fem.out_dtype(precision), device=dev)
    return g, c, f, d, ws, a_off, b_off, A, b


def sample_errors(fem, w, field, idx, A, a_np, precision_results):
    """Relative Frobenius errors of the sampled elements of packed A against oracle results."""
    errs = []
    for k, e in enumerate(idx):
        p = int(w.degree[e])
        ns = (p + 1) ** 3
        Ag = A[a_np[e]:a_np[e + 1]].double().cpu().numpy().reshape(ns, ns)
        errs.append(rel_fro(Ag, precision_results[k]))
    return errs


def oracle_sample(w, field, idx):
    import oracle
    res = []
    for p in range(1, 8):
        sel = [k for k, e in enumerate(idx) if int(w.degree[e]) == p]
        if not sel:
            continue
        ee = idx[sel]
        A, _, _ = oracle.integrate(w.geom[ee], w.coef[ee], p=p, mode=oracle.FIELD, field=field,
                                   threads=oracle_threads())
        res += list(zip(sel, A))
    res.sort(key=lambda t: t[0])
    return [a for _, a in res]


def bench_mixed(args, torch, fem, synth, dev, quick=False):
    """200000 elements, degrees 1..7 with P(p) proportional to 8 - p, coefficient fields per
    quadrature point; the single persistent launch against one launch per degree."""
    w = synth.make(4)
    idx = np.sort(np.random.default_rng(44).choice(w.nel, 256, replace=False))
    t0 = time.time()
    ref = oracle_sample(w, w.field, idx)
    log(f"[bench] mixed: oracle sample of {idx.size} in {time.time() - t0:.1f} s")
    flops = sum(flops_per_element(int(p)) for p in w.degree)
    res = {}
    reps = 3 if quick else max(3, args.steps // 4)
    for prec in ["split_fp16", "fp32"]:
        g, c, f, d, ws, a_off, b_off, A, b = mixed_buffers(torch, fem, w, dev, prec)
        a_np = a_off.cpu().numpy()
        code = fem.PRECISIONS[prec]
        keys = [0] + [fem.mixed(p) for p in range(1, 8)]
        saved = {k: fem.fem_get_variant(k, code, fem.FIELD) for k in keys}
        # the autotuner chooses the tile of every degree inside the single launch (on its own
        # seeded batch of the same size and degree mix), then the strategy
        t0 = time.time()
        tuned, tune_ms = fem.fem_autotune(0, code, fem.FIELD, w.nel, None)
        tiles = {str(p): fem.fem_mixed_variant(p, code, fem.FIELD) for p in range(1, 8)}
        log(f"[bench] mixed {prec}: autotune {time.time() - t0:.1f} s, tiles {tiles}, strategy {tuned} "
            f"(tuning batch ms {['%.2f' % x for x in tune_ms]})")
        for strategy, name in ((0, "single_launch"), (1, "per_degree_launches")):
            fem.fem_set_variant(0, code, fem.FIELD, strategy)
            call = lambda: fem.integrate_mixed(g, c, d, precision=prec, mode=fem.FIELD, field=f,
                                               a_off=a_off, b_off=b_off, out_A=A, out_b=b, workspace=ws)
            ms = time_calls(torch, call, reps, 1)
            st = err_stats(sample_errors(fem, w, w.field, idx, A, a_np, ref))
            fl = flops / (ms * 1e-3) / 1e12
            res[f"{prec}/{name}"] = {"ms": round(ms, 3), "el_per_s": w.nel / (ms * 1e-3),
                                     "tflops": round(fl, 2), "rel_err": st}
            if strategy == 0:
                res[f"{prec}/{name}"]["tiles"] = tiles  # per-degree variant run inside the launch
            log(f"[bench] mixed {prec} {name}: {ms:.3f} ms, {fl:.1f} TFLOP/s, max err {st['max']:.2e}")
        res[f"{prec}/autotuned_strategy"] = ["single_launch", "per_degree_launches"][tuned]
        for k, v in saved.items():  # the choices in force before the benchmark
            fem.fem_set_variant(k, code, fem.FIELD, v)
        del A, b
        torch.cuda.empty_cache()
    best = min(res["split_fp16/single_launch"]["ms"], res["split_fp16/per_degree_launches"]["ms"])
    counts = {str(p): int((w.degree == p).sum()) for p in range(1, 8)}
    return {"metric": "element matrices/s (split-precision MFMA, <= 1e-6 relative error)",
            "value": w.nel / (best * 1e-3), "unit": "element matrices/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f16x3->f32", "data": "synthetic",
            "config": {"workload": "mixed-degree hex p=1..7 (P ~ 8-p), 100x50x40 jittered grid "
                                   "(200000 elements), coefficient fields per quadrature point",
                       "degree_counts": counts, "gflop_per_call": flops / 1e9,
                       "sample": f"{idx.size} seeded random elements against the FP64 oracle"},
            "results": res}


def bench_timestep(args, torch, fem, synth, dev, quick=False):
    """100000 elements of degree 2..6 on a strongly distorted mesh; 50 time steps, each a graph
    replay of {phase update of the coefficient fields, mixed-degree integration}. Every step is
    checked against the FP64 oracle on the first `per_step` elements of that step's 1% sample."""
    w = synth.make(5)
    nsteps = 50
    per_step = 24
    deltas = np.stack([synth.phase_shift(w.seed, t) for t in range(1, nsteps + 1)]).reshape(nsteps, 35)
    refs = {}
    t0 = time.time()
    for t in range(1, nsteps + 1):
        idx = synth.step_sample(w.seed, t, w.nel)[:per_step]
        refs[t] = (idx, oracle_sample(w, synth.field_at_step(w.field, w.seed, t), idx))
    log(f"[bench] timestep: oracle on {per_step} elements of every step's 1% sample in "
        f"{time.time() - t0:.1f} s")
    flops = sum(flops_per_element(int(p)) for p in w.degree)
    res = {}
    for prec in ["split_fp16", "fp32"]:
        g, c, f0, d, ws, a_off, b_off, A, b = mixed_buffers(torch, fem, w, dev, prec)
        a_np = a_off.cpu().numpy()
        f = f0.clone()
        dl = torch.from_numpy(deltas).to(dev)
        step = torch.zeros(1, dtype=torch.int32, device=dev)
        # the geometry is fixed over the steps: with --nojac its Jacobian terms are written once
        jt = fem.jacobian_terms(g, 0, degree=d, b_off=b_off) if args.nojac else None
        # each step's checked elements, gathered on the device at the end of the replayed step
        sel = torch.from_numpy(np.stack([refs[t][0] for t in range(1, nsteps + 1)]).astype(np.int32)).to(dev)
        cap = max(int(sum(a_np[e + 1] - a_np[e] for e in refs[t][0])) for t in range(1, nsteps + 1))
        gathered = torch.empty(cap, dtype=fem.out_dtype(prec), device=dev)

        def one_step(stream=None):
            fem.field_advance(f, dl, step, stream=stream)
            fem.integrate_mixed(g, c, d, precision=prec, mode=fem.FIELD, field=f, a_off=a_off,
                                b_off=b_off, out_A=A, out_b=b, workspace=ws, stream=stream, jac=jt)
            fem.gather_sample(sel, a_off, A, gathered, prec, step=step, stream=stream)

        one_step()  # warm-up outside the capture
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(graph, stream=s):
                one_step(stream=s)
        torch.cuda.synchronize()

        def reset():
            f.copy_(f0)
            step.zero_()
            torch.cuda.synchronize()

        reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(nsteps):
            graph.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / nsteps
        reset()
        maxerr, allerr = {}, []
        for t in range(1, nsteps + 1):
            graph.replay()
            torch.cuda.synchronize()
            idx, ref = refs[t]
            got = gathered.double().cpu().numpy()  # only the sample leaves the device
            errs, at = [], 0
            for k, e in enumerate(idx):
                ns = (int(w.degree[e]) + 1) ** 3
                errs.append(rel_fro(got[at:at + ns * ns].reshape(ns, ns), ref[k]))
                at += ns * ns
            maxerr[str(t)] = max(errs)
            allerr += errs
        torch.cuda.synchronize()
        assert int(step.item()) == nsteps
        fl = flops / (ms * 1e-3) / 1e12
        res[prec] = {"ms_per_step": round(ms, 3), "el_per_s": w.nel / (ms * 1e-3),
                     "tflops": round(fl, 2), "rel_err": err_stats(allerr),
                     "max_rel_err_by_step": maxerr}
        log(f"[bench] timestep {prec}: {ms:.3f} ms/step, {fl:.1f} TFLOP/s, max err {max(allerr):.2e}")
        del graph, A, b
        torch.cuda.empty_cache()
    return {"metric": "element matrices/s (split-precision MFMA, <= 1e-6 relative error)",
            "value": res["split_fp16"]["el_per_s"], "unit": "element matrices/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f16x3->f32", "data": "synthetic",
            "steps": nsteps,
            "config": {"workload": "time-stepped mixed-degree hex p=2..6, 50x50x40 grid jittered "
                                   "+-30% (100000 elements, detJ > 0 by a Bernstein test, "
                                   f"{w.redraws} redraws), phase-shifted coefficient fields, "
                                   "hipGraph replay per step {phase update, integration, sample gather}",
                       "gflop_per_step": flops / 1e9,
                       "jacobian_terms": "supplied (written once)" if args.nojac else "computed",
                       "sample": f"every step: the first {per_step} elements of the step's 1% "
                                 "sample against the FP64 oracle"},
            "results": res, "speedup_split_vs_fp32": res["fp32"]["ms_per_step"] / res["split_fp16"]["ms_per_step"]}


def bench_poisson(args, torch, fem, synth, dev, quick=False):
    """p = 1 Poisson: the 16^3 workload (FP64 output; every element against the oracle), the same
    call replayed from a captured graph (launch cost amortised), and a 128^3 mesh, where the
    outputs are far larger than the last-level cache and HBM bandwidth bounds the kernel."""
    import oracle
    res = {}
    for grid in [(16, 16, 16), (128, 128, 128)]:
        w = synth.make(1, grid=grid)
        g, c = torch.from_numpy(w.geom).to(dev), torch.from_numpy(w.coef).to(dev)
        for prec in ["fp64", "fp32", "split_fp16"]:
            A = torch.empty((w.nel, 8, 8), dtype=fem.out_dtype(prec), device=dev)
            b = torch.empty((w.nel, 8), dtype=fem.out_dtype(prec), device=dev)
            call = lambda: fem.integrate(g, c, 1, precision=prec, out_A=A, out_b=b)
            ms = time_calls(torch, call, args.steps, args.warmup)
            ob = 8 if prec == "fp64" else 4
            gbs = bytes_per_element(1, ob) * w.nel / (ms * 1e-3) / 1e9
            key = f"{'x'.join(map(str, grid))}/{prec}"
            res[key] = {"nel": w.nel, "ms": round(ms, 4), "el_per_s": w.nel / (ms * 1e-3),
                        "gbs": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
            if grid == (16, 16, 16):
                Aref, _, _ = oracle.integrate(w.geom, w.coef, p=1, threads=oracle_threads())
                res[key]["rel_err"] = err_stats(rel_fro_rows(A.double().cpu().numpy(), Aref))
                # graph-amortised: 100 integrations captured in one graph, replayed
                s = torch.cuda.Stream()
                s.wait_stream(torch.cuda.current_stream())
                graph = torch.cuda.CUDAGraph()
                with torch.cuda.stream(s):
                    with torch.cuda.graph(graph, stream=s):
                        for _ in range(100):
                            fem.integrate(g, c, 1, precision=prec, out_A=A, out_b=b, stream=s)
                torch.cuda.synchronize()
                gms = time_calls(torch, graph.replay, 3, 1) / 100
                res[key]["graph_ms"] = round(gms, 5)
                res[key]["graph_el_per_s"] = w.nel / (gms * 1e-3)
                del graph
            log(f"[bench] poisson {key}: {ms:.4f} ms, {gbs:.0f} GB/s")
            del A, b
            torch.cuda.empty_cache()
    return {"metric": "element matrices/s", "value": res["16x16x16/fp64"]["el_per_s"],
            "unit": "element matrices/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "p=1 Poisson, 16^3 (4096 elements, every element against the "
                                   "oracle; graph_ms: 100 calls replayed from one graph) and 128^3 "
                                   "(2097152 elements) jittered grids"},
            "results": res}


def elastic_flops(fem, p_key, prec, p, nel, prism=False):
    """Algorithmic flops of an elastostatics call: the full 3 x 3 block matrix, and the part the
    matrix cores execute (6 or 9 blocks; the others are transposed copies)."""
    blocks = fem.fem_elastic_blocks(p_key, fem.PRECISIONS[prec])
    return 9 * flops_per_element(p, prism) * nel, blocks * flops_per_element(p, prism) * nel


def bench_elasticity(args, torch, fem, synth, dev, quick=False):
    """Linear elastostatics (3 components, isotropic material per element, the paper's model
    problem) on the plain-method grids for p = 2, 3, 4 and the high-order grids for p = 5, 6, 7;
    output 9 Ns^2 + 3 Ns per element; sampled errors against the FP64 oracle."""
    import oracle
    grids = {2: (64, 64, 64), 3: (64, 64, 32), 4: (64, 32, 32), 5: (32, 32, 16), 6: (32, 16, 16),
             7: (16, 16, 16)}
    out = {}
    for p, grid in grids.items():
        rng = np.random.default_rng(70 + p)
        nodes = synth.node_grid(*grid, 0.15, rng)
        geom = synth.element_vertices(nodes)
        coef = synth.elastic_coeffs(geom.shape[0], rng)
        nel = geom.shape[0]
        g, c = torch.from_numpy(geom).to(dev), torch.from_numpy(coef).to(dev)
        idx = np.sort(np.random.default_rng(p).choice(nel, 8 if p <= 5 else 4, replace=False))
        Aref, _, _ = oracle.integrate_elastic(geom[idx], coef[idx], p, threads=oracle_threads(),
                                              with_b=False)
        ns = (p + 1) ** 3
        res = {"nel": nel}
        for prec in ["split_fp16", "fp32"]:
            A = torch.empty((nel, 3, 3, ns, ns), dtype=fem.out_dtype(prec), device=dev)
            b = torch.empty((nel, 3, ns), dtype=fem.out_dtype(prec), device=dev)
            ms = time_calls(torch, lambda: fem.integrate(g, c, p, precision=prec, mode=fem.ELASTIC,
                                                         out_A=A, out_b=b), max(3, args.steps // 5), 1)
            Ag = A[torch.from_numpy(idx).to(dev)].double().cpu().numpy()
            st = err_stats(rel_fro_rows(Ag, Aref))
            f_all, f_exec = elastic_flops(fem, p, prec, p, nel)
            t = ms * 1e-3
            gbs = (192 + 40 + 4 * (9 * ns * ns + 3 * ns)) * nel / t / 1e9
            res[prec] = {"ms": round(ms, 3), "el_per_s": nel / t,
                         "tflops_full_matrix": round(f_all / t / 1e12, 2),
                         "blocks_integrated": fem.fem_elastic_blocks(p, fem.PRECISIONS[prec]),
                         "tflops_executed": round(f_exec / t / 1e12, 2),
                         "frac_peak_executed": round(f_exec * PRODUCTS[prec] / t / 1e12 / PEAK_TFLOPS[prec], 4),
                         "gbs": round(gbs, 1), "rel_err": st}
            log(f"[bench] elasticity p={p} {prec}: {ms:.3f} ms, {f_exec / t / 1e12:.1f} TFLOP/s "
                f"executed, max err {st['max']:.2e}")
            del A, b
            torch.cuda.empty_cache()
        out[str(p)] = res
    tot_el = sum(out[k]["nel"] for k in out)
    tot_ms = sum(out[k]["split_fp16"]["ms"] for k in out)
    return {"metric": "element matrices/s (split-precision MFMA, <= 1e-6 relative error)",
            "value": tot_el / (tot_ms * 1e-3), "unit": "element matrices/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f16x3->f32", "data": "synthetic",
            "config": {"workload": "linear elastostatics hex p=2..7 (3 components, E ~ U[1,10], "
                                   "nu ~ U[0.2,0.4] per element) on the plain and high-order grids",
                       "sample": "8 (p<=5) or 4 seeded random elements per degree against the FP64 oracle"},
            "per_degree": out}


def bench_prism(args, torch, fem, synth, dev, quick=False):
    """Prismatic elements, the paper's reference element (section 2, Tables 1-2), p = 1..7 with
    the CDR coefficient law on jittered grids of cells split into two prisms (524288 ... 8192
    prisms); FP64, FP32 and split FP16; error statistics of seeded samples against the prism
    oracle."""
    import oracle
    out = {}
    precs = ["split_fp16", "fp32", "fp64"]
    reps = 3 if quick else max(3, args.steps // 4)
    for p in range(1, 8):
        w = synth.make_prism("cdr", p)
        g, c = torch.from_numpy(w.geom).to(dev), torch.from_numpy(w.coef).to(dev)
        ns = fem.prism_ns(p)
        n = {1: 256, 2: 256, 3: 128, 4: 64, 5: 32, 6: 16, 7: 12}[p]
        idx = np.sort(np.random.default_rng(200 + p).choice(w.nel, n, replace=False))
        Aref, _, _ = oracle.integrate_prism(w.geom[idx], w.coef[idx], p, threads=oracle_threads())
        res = {"nel": w.nel, "ns": ns, "nq": nq_prism(p)}
        for prec in precs:
            A = torch.empty((w.nel, ns, ns), dtype=fem.out_dtype(prec), device=dev)
            b = torch.empty((w.nel, ns), dtype=fem.out_dtype(prec), device=dev)
            ms = time_calls(torch, lambda: fem.integrate_prism(g, c, p, precision=prec, out_A=A, out_b=b),
                            reps, 1)
            Ag = A[torch.from_numpy(idx).to(dev)].double().cpu().numpy()
            st = err_stats(rel_fro_rows(Ag, Aref))
            t = ms * 1e-3
            fl = flops_per_element(p, prism=True) * w.nel / t / 1e12
            ob = 8 if prec == "fp64" else 4
            gbs = bytes_per_element(p, ob, prism=True) * w.nel / t / 1e9
            res[prec] = {"ms": round(ms, 4), "el_per_s": w.nel / t, "tflops": round(fl, 2),
                         "frac_peak": round(fl / PEAK_TFLOPS[prec], 4),
                         "frac_peak_executed": round(fl * PRODUCTS[prec] / PEAK_TFLOPS[prec], 4),
                         "gbs": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4), "rel_err": st}
            log(f"[bench] prism p={p} {prec}: {ms:.3f} ms, {fl:.1f} TFLOP/s, {gbs:.0f} GB/s, "
                f"max err {st['max']:.2e}")
            del A, b
            torch.cuda.empty_cache()
        out[str(p)] = res
    tot_el = sum(out[k]["nel"] for k in out)
    tot_ms = sum(out[k]["split_fp16"]["ms"] for k in out)
    return {"metric": "element matrices/s (split-precision MFMA, <= 1e-6 relative error)",
            "value": tot_el / (tot_ms * 1e-3), "unit": "element matrices/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f16x3->f32", "data": "synthetic",
            "config": {"workload": "cdr-prism p=1..7 on jittered grids of cells split into two "
                                   "prisms (" + ", ".join(f"p={p}: {out[str(p)]['nel']}" for p in range(1, 8)) + ")",
                       "sample": "seeded random elements per degree against the FP64 prism oracle"},
            "per_degree": out}


# the paper's own per-element kernel times for its elastostatics benchmark on prisms (Table 6,
# GTX580, FP32; the fastest of its four kernels), in microseconds: context only
PAPER_PRISM_ELASTIC_US = {2: 1.21, 3: 17.80, 4: 80.07, 5: 439.9, 6: 1932.0, 7: 6199.0}


def bench_prism_elastic(args, torch, fem, synth, dev, quick=False):
    """The paper's benchmark problem: linear elastostatics on prisms (sections 5.1-5.4), p = 2..7
    on the prism grids; element matrices of 3 x 3 blocks; sampled errors against the prism oracle;
    the paper's per-element kernel time on its GPU quoted as context."""
    import oracle
    out = {}
    reps = 3 if quick else max(3, args.steps // 5)
    for p in range(2, 8):
        w = synth.make_prism("elastic", p)
        g, c = torch.from_numpy(w.geom).to(dev), torch.from_numpy(w.coef).to(dev)
        ns = fem.prism_ns(p)
        n = {2: 64, 3: 32, 4: 16, 5: 8, 6: 6, 7: 4}[p]
        idx = np.sort(np.random.default_rng(300 + p).choice(w.nel, n, replace=False))
        Aref, _, _ = oracle.integrate_prism(w.geom[idx], w.coef[idx], p, mode=oracle.ELASTIC,
                                            threads=oracle_threads(), with_b=False)
        res = {"nel": w.nel, "paper_us_per_element_gtx580": PAPER_PRISM_ELASTIC_US[p]}
        for prec in ["split_fp16", "fp32"]:
            A = torch.empty((w.nel, 3, 3, ns, ns), dtype=fem.out_dtype(prec), device=dev)
            b = torch.empty((w.nel, 3, ns), dtype=fem.out_dtype(prec), device=dev)
            ms = time_calls(torch, lambda: fem.integrate_prism(g, c, p, precision=prec, mode=fem.ELASTIC,
                                                               out_A=A, out_b=b), reps, 1)
            Ag = A[torch.from_numpy(idx).to(dev)].double().cpu().numpy()
            st = err_stats(rel_fro_rows(Ag, Aref))
            t = ms * 1e-3
            blocks = fem.fem_elastic_blocks(fem.prism(p), fem.PRECISIONS[prec])
            f_exec = blocks * flops_per_element(p, prism=True) * w.nel
            res[prec] = {"ms": round(ms, 3), "el_per_s": w.nel / t,
                         "us_per_element": round(ms * 1e3 / w.nel, 5),
                         "blocks_integrated": blocks,
                         "tflops_executed": round(f_exec / t / 1e12, 2),
                         "frac_peak_executed": round(f_exec * PRODUCTS[prec] / t / 1e12 / PEAK_TFLOPS[prec], 4),
                         "rel_err": st}
            log(f"[bench] prism elasticity p={p} {prec}: {ms:.3f} ms ({ms * 1e3 / w.nel:.4f} us per "
                f"element; paper {PAPER_PRISM_ELASTIC_US[p]} us), max err {st['max']:.2e}")
            del A, b
            torch.cuda.empty_cache()
        out[str(p)] = res
    tot_el = sum(out[k]["nel"] for k in out)
    tot_ms = sum(out[k]["split_fp16"]["ms"] for k in out)
    return {"metric": "element matrices/s (split-precision MFMA, <= 1e-6 relative error)",
            "value": tot_el / (tot_ms * 1e-3), "unit": "element matrices/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f16x3->f32", "data": "synthetic",
            "config": {"workload": "linear elastostatics on prisms p=2..7 (the paper's model problem, "
                                   "E ~ U[1,10], nu ~ U[0.2,0.4] per element) on the prism grids",
                       "context": "paper_us_per_element_gtx580: the fastest kernel of Table 6 "
                                  "(NVIDIA GTX580, FP32, 2013), another machine"},
            "per_degree": out}


def bench_nojac(args, torch, fem, synth, dev, quick=False):
    """Supplied per-point Jacobian terms (detJ and J^{-1}, 80 B per point) against the in-kernel
    FP64 computation from the 8 vertices (192 B per element), p = 1..7 on the plain-method and
    high-order grids (p = 1: 128x128x64); the terms writer's own time; sampled errors of the
    supplied-terms path against the FP64 oracle."""
    import oracle
    grids = {1: (128, 128, 64), 2: (64, 64, 64), 3: (64, 64, 32), 4: (64, 32, 32),
             5: (32, 32, 16), 6: (32, 16, 16), 7: (16, 16, 16)}
    out = {}
    for p, grid in grids.items():
        w = synth.make(2 if p <= 4 else 3, p=p, grid=grid) if p > 1 else synth.make(2, p=2, grid=grid)
        geom, coef, nel = w.geom, w.coef, w.nel
        ns = (p + 1) ** 3
        g, c = torch.from_numpy(geom).to(dev), torch.from_numpy(coef).to(dev)
        jt = torch.empty((nel, ns, 10), dtype=torch.float64, device=dev)
        ms_terms = time_calls(torch, lambda: fem.jacobian_terms(g, p, out=jt), max(3, args.steps // 4), 1)
        idx = np.sort(np.random.default_rng(p).choice(nel, 8, replace=False))
        Aref, _, _ = oracle.integrate(geom[idx], coef[idx], p=p, threads=oracle_threads(), with_b=False)
        res = {"nel": nel, "terms_ms": round(ms_terms, 4),
               "terms_gbs": round((192 + 80 * ns) * nel / (ms_terms * 1e-3) / 1e9, 1),
               "extra_bytes_per_element": 80 * ns - 192}
        for prec in ["split_fp16", "fp32"]:
            A = torch.empty((nel, ns, ns), dtype=fem.out_dtype(prec), device=dev)
            b = torch.empty((nel, ns), dtype=fem.out_dtype(prec), device=dev)
            reps = max(3, args.steps // 4)
            ms_jac = time_calls(torch, lambda: fem.integrate(g, c, p, precision=prec, out_A=A, out_b=b), reps, 1)
            ms_sup = time_calls(torch, lambda: fem.integrate(None, c, p, precision=prec, out_A=A, out_b=b,
                                                             jac=jt), reps, 1)
            Ag = A[torch.from_numpy(idx).to(dev)].double().cpu().numpy()
            st = err_stats(rel_fro_rows(Ag, Aref))
            res[prec] = {"ms_computed": round(ms_jac, 4), "ms_supplied": round(ms_sup, 4),
                         "supplied_over_computed": round(ms_sup / ms_jac, 3),
                         "rel_err_supplied": st}
            log(f"[bench] nojac p={p} {prec}: computed {ms_jac:.3f} ms, supplied {ms_sup:.3f} ms "
                f"(terms writer {ms_terms:.3f} ms), max err {st['max']:.2e}")
            del A, b
            torch.cuda.empty_cache()
        out[str(p)] = res
        del jt
        torch.cuda.empty_cache()
    tot_el = sum(out[k]["nel"] for k in out if k != "1")
    tot_ms = sum(out[k]["split_fp16"]["ms_supplied"] for k in out if k != "1")
    return {"metric": "element matrices/s (split-precision MFMA, <= 1e-6 relative error)",
            "value": tot_el / (tot_ms * 1e-3), "unit": "element matrices/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f16x3->f32", "data": "synthetic",
            "config": {"workload": "cdr-hex p=2..7 on the plain and high-order grids with supplied "
                                   "per-point Jacobian terms (value); p=1 on 128x128x64 reported only",
                       "sample": "8 seeded random elements per degree against the FP64 oracle"},
            "per_degree": out}


def bench_staged(args, torch, fem, synth, dev, quick=False):
    """The plain workload (p = 2, 3, 4) with inputs and outputs in pinned host memory: one chunk
    on one stream (copy in, kernel, copy out in sequence) against chunks over three streams
    (copies of one chunk under the kernels of others). Reports the end-to-end rate including the
    host transfers and the per-stage sums."""
    res = {}
    tot = {"serial": 0.0, "pipelined": 0.0}
    nel_all = 0
    for p, grid in WORKLOAD:
        w = synth.make(2, p=p, grid=grid)
        nel = w.nel
        nel_all += nel
        gh = torch.from_numpy(w.geom).pin_memory()
        ch = torch.from_numpy(w.coef).pin_memory()
        ns = (p + 1) ** 3
        A = torch.empty((nel, ns, ns), dtype=torch.float32, pin_memory=True)
        b = torch.empty((nel, ns), dtype=torch.float32, pin_memory=True)
        out = {"nel": nel}
        for name, chunk, nstreams in (("serial", nel, 1), ("pipelined", -(-nel // 16), 3)):
            fem.integrate_staged(gh, ch, p, precision="split_fp16", chunk=chunk, nstreams=nstreams,
                                 out_A=A, out_b=b)  # warm-up (allocates the staging buffers)
            runs = [fem.integrate_staged(gh, ch, p, precision="split_fp16", chunk=chunk,
                                         nstreams=nstreams, out_A=A, out_b=b)[2] for _ in range(3)]
            st = min(runs, key=lambda r: r["total_ms"])
            gbs = (st["h2d_bytes"] + st["d2h_bytes"]) / (st["total_ms"] * 1e-3) / 1e9
            out[name] = {"chunk": chunk, "streams": nstreams, "total_ms": round(st["total_ms"], 3),
                         "h2d_ms": round(st["h2d_ms"], 3), "kernel_ms": round(st["kernel_ms"], 3),
                         "d2h_ms": round(st["d2h_ms"], 3), "el_per_s": nel / (st["total_ms"] * 1e-3),
                         "pcie_gbs": round(gbs, 1)}
            tot[name] += st["total_ms"]
            log(f"[bench] staged p={p} {name}: {st['total_ms']:.2f} ms (h2d {st['h2d_ms']:.2f}, "
                f"kernel {st['kernel_ms']:.2f}, d2h {st['d2h_ms']:.2f}), {gbs:.1f} GB/s over PCIe")
        res[str(p)] = out
        del A, b, gh, ch
    return {"metric": "element matrices/s including host transfers (split-precision MFMA)",
            "value": nel_all / (tot["pipelined"] * 1e-3), "unit": "element matrices/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f16x3->f32", "data": "synthetic",
            "config": {"workload": "cdr-hex p=2,3,4 plain grids (458752 elements) from and to "
                                   "pinned host memory; pipelined = 16 chunks over 3 streams",
                       "serial_ms": round(tot["serial"], 3), "pipelined_ms": round(tot["pipelined"], 3)},
            "per_degree": res}


DEGREE_GRIDS = {1: (128, 128, 64), 2: (64, 64, 64), 3: (64, 64, 32), 4: (64, 32, 32),
                5: (32, 32, 16), 6: (32, 16, 16), 7: (16, 16, 16)}


def bench_degree(args, torch, fem, synth, dev, quick=False):
    """One degree's benchmark mesh (the plain-method grids for p = 2..4, the high-order grids
    for p = 5..7, 128x128x64 for p = 1) integrated --steps times in --precision with the
    default tile: the single-kernel run that the counter profiles are taken on."""
    p = args.degree
    if not 1 <= p <= 7:
        raise SystemExit("--degree must be 1..7")
    w = synth.make(2, p=max(p, 2), grid=DEGREE_GRIDS[p]) if p <= 4 else synth.make(3, p=p)
    g, c = torch.from_numpy(w.geom).to(dev), torch.from_numpy(w.coef).to(dev)
    if args.variant >= 0:
        fem.fem_set_variant(p, fem.PRECISIONS[args.precision], fem.ELEMENT, args.variant)
    ns = (p + 1) ** 3
    A = torch.empty((w.nel, ns, ns), dtype=fem.out_dtype(args.precision), device=dev)
    b = torch.empty((w.nel, ns), dtype=fem.out_dtype(args.precision), device=dev)
    ms = time_calls(torch, lambda: fem.integrate(g, c, p, precision=args.precision, out_A=A, out_b=b),
                    args.steps, args.warmup)
    fl = flops_per_element(p) * w.nel / (ms * 1e-3) / 1e12
    return {"metric": "element matrices/s", "value": w.nel / (ms * 1e-3), "unit": "element matrices/s",
            "n_gpus": 1, "higher_is_better": True, "dtype": args.precision, "data": "synthetic",
            "config": {"workload": f"cdr-hex p={p} on {'x'.join(map(str, DEGREE_GRIDS[p]))} ({w.nel} elements)",
                       "variant": fem.fem_get_variant(p, fem.PRECISIONS[args.precision], fem.ELEMENT)},
            "ms_per_launch": round(ms, 4), "tflops": round(fl, 2)}

WORKLOADS = {"high": bench_high, "mixed": bench_mixed, "timestep": bench_timestep,
             "poisson": bench_poisson, "elasticity": bench_elasticity, "nojac": bench_nojac,
             "staged": bench_staged, "degree": bench_degree, "prism": bench_prism,
             "prism-elastic": bench_prism_elastic}
# measured in the default run as well, under "extras" (fewer repetitions)
EXTRAS = ["poisson", "high", "mixed", "timestep", "prism", "prism-elastic"]


if __name__ == "__main__":
    main()
