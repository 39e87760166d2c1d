"""Time-stepped re-integration: the device phase update matches the host recipe, and a captured
{phase update, mixed-degree integration} graph replays step after step, each step matching the
FP64 oracle on a sample of elements and the eager launches bit for bit."""
import numpy as np
import pytest

from gpu_cases import TOL_A, log, rel_fro, to_dev
from paper_1310_1191_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fem():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_1310_1191_amd import fem as F
    F.fem_init(0)
    return F


def test_field_advance_matches_host_recipe(fem):
    import torch
    w = synth.make(5, grid=(3, 3, 2))
    nsteps = 4
    deltas = np.stack([synth.phase_shift(w.seed, t) for t in range(1, nsteps + 1)])
    f, dl = to_dev(w.field, deltas.reshape(nsteps, 35))
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    for t in range(1, nsteps + 2):   # one call past the end leaves everything unchanged
        fem.field_advance(f, dl, step)
        torch.cuda.synchronize()
        ref = synth.field_at_step(w.field, w.seed, min(t, nsteps))
        got = f.cpu().numpy()
        np.testing.assert_allclose(got.reshape(7, 5, 5)[:, :, :4], ref.reshape(7, 5, 5)[:, :, :4], rtol=0, atol=0)
        dth = np.abs(got.reshape(7, 5, 5)[:, :, 4] - ref.reshape(7, 5, 5)[:, :, 4])
        assert np.all(np.minimum(dth, 2 * np.pi - dth) < 1e-12)
        assert int(step.item()) == min(t, nsteps)


def test_graph_replay_time_steps(fem):
    import oracle
    import torch
    w = synth.make(5, grid=(6, 5, 4))
    nsteps = 5
    deltas = np.stack([synth.phase_shift(w.seed, t) for t in range(1, nsteps + 1)]).reshape(nsteps, 35)
    g, c, f0, d, dl = to_dev(w.geom, w.coef, w.field, w.degree, deltas)
    f = f0.clone()
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = torch.empty(fem.fem_workspace_bytes(w.nel), dtype=torch.uint8, device="cuda")
    a_off, b_off = fem.mixed_offsets(d, workspace=ws)
    torch.cuda.synchronize()
    A = torch.empty(int(a_off[-1].item()), dtype=torch.float32, device="cuda")
    b = torch.empty(int(b_off[-1].item()), dtype=torch.float32, device="cuda")
    a_np = a_off.cpu().numpy()

    def one_step(stream=None):
        fem.field_advance(f, dl, step, stream=stream)
        fem.integrate_mixed(g, c, d, precision="split_fp16", mode=fem.FIELD, field=f, a_off=a_off,
                            b_off=b_off, out_A=A, out_b=b, workspace=ws, stream=stream)

    # eager reference run of all steps
    eager = []
    for t in range(nsteps):
        one_step()
        torch.cuda.synchronize()
        eager.append(A.clone())
    # capture one step, replay it nsteps times from the initial phases
    f.copy_(f0)
    step.zero_()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            one_step(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    f.copy_(f0)
    step.zero_()
    torch.cuda.synchronize()
    for t in range(nsteps):
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(A, eager[t]), f"replay {t} differs from the eager step"
        # sampled oracle check of this step's coefficients
        fld = synth.field_at_step(w.field, w.seed, t + 1)
        idx = synth.step_sample(w.seed, t + 1, w.nel)[:3]
        for e in idx:
            p = int(w.degree[e])
            ns = (p + 1) ** 3
            Ar, _, _ = oracle.integrate(w.geom[e:e + 1], w.coef[e:e + 1], p=p, mode=oracle.FIELD,
                                        field=fld)
            Ag = A[a_np[e]:a_np[e + 1]].double().cpu().numpy().reshape(1, ns, ns)
            err = rel_fro(Ag, Ar)[0]
            assert err <= TOL_A["split_fp16"], (t, e, err)
        log(f"[graph] step {t + 1}: replay == eager, sample ok")
