"""The seeded workload generators: determinism, shapes, value ranges, mesh validity."""
import hashlib

import numpy as np
import pytest

from paper_1310_1191_amd import synth


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


@pytest.mark.parametrize("cfg,p", [(1, None), (2, 3), (3, 6), (4, None), (5, None)])
def test_deterministic(cfg, p):
    a = synth.small(cfg, p=p)
    b = synth.small(cfg, p=p)
    assert digest(a.geom, a.coef) == digest(b.geom, b.coef)
    if a.degree is not None:
        assert digest(a.degree, a.field) == digest(b.degree, b.field)


def test_config_sizes_and_ranges():
    w = synth.make(1)
    assert w.nel == 4096 and w.p == 1
    np.testing.assert_array_equal(w.coef[0], [1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 0, 1])
    w = synth.small(2, p=2, scale=4)
    K = w.coef[:, :9].reshape(-1, 3, 3)
    ev = np.linalg.eigvalsh(K)
    assert ev.min() >= 0.1 - 1e-12 and ev.max() <= 10 + 1e-9
    assert np.all(np.abs(w.coef[:, 9:12]) <= 1) and np.all((w.coef[:, 12] >= 0) & (w.coef[:, 12] <= 1))
    w4 = synth.small(4, scale=4)
    Q = w4.coef[:, :9].reshape(-1, 3, 3)
    np.testing.assert_allclose(np.einsum("eij,ekj->eik", Q, Q), np.broadcast_to(np.eye(3), Q.shape),
                               atol=1e-13)
    fd = w4.field.reshape(7, 5, 5)
    np.testing.assert_allclose(np.abs(fd[:, :, 0]).sum(axis=1), 1.0)
    assert set(np.unique(fd[:, :, 1:4])) <= {-2.0, -1.0, 0.0, 1.0, 2.0}
    assert w4.degree.min() >= 1 and w4.degree.max() <= 7


def test_boundary_nodes_fixed_and_jitter_bounded():
    rng = np.random.default_rng(0)
    nodes = synth.node_grid(4, 3, 2, 0.3, rng)
    assert np.all(nodes[0, :, :, 2] == 0.0) and np.all(nodes[-1, :, :, 2] == 1.0)
    assert np.all(nodes[:, 0, :, 1] == 0.0) and np.all(nodes[:, :, -1, 0] == 1.0)
    ref = np.stack(np.meshgrid(np.arange(5) / 4, np.arange(4) / 3, np.arange(3) / 2, indexing="ij"),
                   -1).transpose(2, 1, 0, 3)
    assert np.all(np.abs(nodes - ref) <= 0.3 * np.array([1 / 4, 1 / 3, 1 / 2]) + 1e-15)


def test_bernstein_filter_is_exact_on_boxes_and_catches_inversion():
    box = np.array([[(v & 1) * 2.0, ((v >> 1) & 1) * 3.0, ((v >> 2) & 1) * 0.5] for v in range(8)])
    # undistorted box: the volume form is constant = product of the edge lengths
    assert synth.min_bernstein_volume(box[None])[0] == pytest.approx(3.0, rel=1e-14)
    mirrored = box[[1, 0, 3, 2, 5, 4, 7, 6]]
    assert synth.min_bernstein_volume(mirrored[None])[0] < 0


def test_config5_mesh_is_valid():
    w = synth.small(5, scale=5)
    h = np.array([1 / g for g in w.grid])
    assert synth.min_bernstein_volume(w.geom).min() > 0.05 * h.prod() - 1e-18
    assert w.degree.min() >= 2 and w.degree.max() <= 6


def test_phase_steps_and_samples():
    f0 = synth.make(4, grid=(4, 4, 4)).field
    f2 = synth.field_at_step(f0, 5, 2)
    d = (f2.reshape(7, 5, 5)[:, :, 4] - f0.reshape(7, 5, 5)[:, :, 4]
         - synth.phase_shift(5, 1) - synth.phase_shift(5, 2))
    np.testing.assert_allclose(np.mod(d + np.pi, 2 * np.pi) - np.pi, 0.0, atol=1e-12)
    s = synth.step_sample(5, 3, 100000)
    assert s.size == 1000 and np.unique(s).size == 1000
