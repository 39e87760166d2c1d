"""Shared helpers for the GPU parity tests: seeded cases, cached oracle results, error metrics.

Tolerances are per element, relative Frobenius norm of A against the FP64 oracle: FP64 1e-12,
FP32 1e-5, split products 1e-6 (the targets of the hot path); plain BF16 is measured and only
checked against a loose sanity bound."""
from __future__ import annotations

import functools
import sys

import numpy as np

from paper_1310_1191_amd import synth

# split_bf16 (hi*hi + hi*lo + lo*hi in BF16) keeps ~2^-16 per product and cannot meet 1e-6; its
# measured error is reported and bounded at 1e-5. split_fp16 is the accepted split path.
TOL_A = {"fp64": 1e-12, "fp32": 1e-5, "split_bf16": 1e-5, "split_fp16": 1e-6, "bf16": 3e-2}
TOL_B = {"fp64": 1e-12, "fp32": 1e-6, "split_bf16": 1e-6, "split_fp16": 1e-6, "bf16": 1e-6}

# grids that span several work items and leave ragged tails (element groups of 16/8/4/2)
GRIDS = {1: (10, 10, 10), 2: (9, 8, 7), 3: (6, 5, 4), 4: (5, 4, 3), 5: (4, 3, 1), 6: (3, 2, 1),
         7: (3, 1, 1)}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def cdr_case(p: int, grid: tuple | None = None):
    """Jittered CDR mesh with the per-element coefficient law of the p = 2..7 workloads."""
    cfg = 2 if p <= 4 else 3
    g = grid or GRIDS[p]
    if p == 1:
        # p = 1 with the full CDR coefficient law (the Poisson workload is a separate case)
        rng = np.random.default_rng(11)
        nodes = synth.node_grid(*g, 0.15, rng)
        geom = synth.element_vertices(nodes)
        return geom, synth.cdr_element_coeffs(geom.shape[0], rng)
    w = synth.make(cfg, p=p, grid=g)
    return w.geom, w.coef


@functools.lru_cache(maxsize=None)
def oracle_uniform(p: int, which: str = "cdr", grid: tuple | None = None):
    import oracle
    if which == "cdr":
        geom, coef = cdr_case(p, grid)
        A, b, fl = oracle.integrate(geom, coef, p=p)
        return geom, coef, A, b, fl
    if which == "poisson":
        w = synth.make(1) if grid is None else synth.make(1, grid=grid)
        A, b, fl = oracle.integrate(w.geom, w.coef, p=1)
        return w.geom, w.coef, A, b, fl
    raise ValueError(which)


def rel_fro(A, Aref):
    """Per-element ||A - A*||_F / ||A*||_F over the trailing two axes."""
    num = np.sqrt(((A - Aref) ** 2).sum(axis=(-2, -1)))
    den = np.sqrt((Aref ** 2).sum(axis=(-2, -1)))
    return num / den


def rel_vec(b, bref):
    num = np.sqrt(((b - bref) ** 2).sum(axis=-1))
    den = np.sqrt((bref ** 2).sum(axis=-1))
    den = np.maximum(den, 1e-300)
    return num / den


def to_dev(*arrays, device="cuda"):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).to(device) for a in arrays]
