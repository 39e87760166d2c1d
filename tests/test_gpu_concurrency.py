"""Concurrent use of the library from several host threads (the header's thread-safety claims):
fem_integrate on disjoint outputs from two threads on their own streams, and two concurrent
host-staged calls (serialised inside the library), each equal bit for bit to the same calls
made one after the other."""
import threading

import numpy as np
import pytest

from gpu_cases import cdr_case, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fem():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_1310_1191_amd import fem as F
    F.fem_init(0)
    return F


def run_threads(targets):
    errors = []

    def wrap(fn):
        try:
            fn()
        except Exception as exc:  # re-raised in the main thread
            errors.append(exc)

    threads = [threading.Thread(target=wrap, args=(t,)) for t in targets]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
        assert not t.is_alive(), "a worker thread did not finish"
    if errors:
        raise errors[0]


def test_integrate_from_two_threads(fem):
    import torch
    cases = {}
    for p in (2, 3):
        geom, coef = cdr_case(p)
        cases[p] = to_dev(geom, coef)
    ref = {}
    for p, (g, c) in cases.items():
        ref[p] = fem.integrate(g, c, p, precision="split_fp16")
    torch.cuda.synchronize()
    got = {}

    def worker(p):
        def run():
            s = torch.cuda.Stream()
            g, c = cases[p]
            with torch.cuda.stream(s):
                for _ in range(5):
                    got[p] = fem.integrate(g, c, p, precision="split_fp16", stream=s)
            s.synchronize()
        return run

    run_threads([worker(2), worker(3)])
    torch.cuda.synchronize()
    for p in (2, 3):
        assert torch.equal(got[p][0], ref[p][0]) and torch.equal(got[p][1], ref[p][1])


def test_staged_calls_from_two_threads(fem):
    import torch
    inputs = {}
    for p in (2, 3):
        geom, coef = cdr_case(p)
        inputs[p] = (torch.from_numpy(np.ascontiguousarray(geom)).pin_memory(),
                     torch.from_numpy(np.ascontiguousarray(coef)).pin_memory())
    ref = {p: fem.integrate_staged(*inputs[p], p, precision="fp32", chunk=50, nstreams=2)[:2]
           for p in (2, 3)}
    got = {}

    def worker(p):
        def run():
            for _ in range(3):
                got[p] = fem.integrate_staged(*inputs[p], p, precision="fp32", chunk=50, nstreams=2)[:2]
        return run

    run_threads([worker(2), worker(3)])
    for p in (2, 3):
        assert torch.equal(got[p][0], ref[p][0]) and torch.equal(got[p][1], ref[p][1])
