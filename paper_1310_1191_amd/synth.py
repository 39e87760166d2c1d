"""Seeded synthetic workloads: meshes, coefficients, coefficient fields and degree mixes.

This module only draws inputs. It holds none of the integration arithmetic and imports nothing
from the HIP binding or from the oracle; both of those consume what it returns.

The paper integrates model problems on meshes it does not publish and states that, for
integration alone, the problem solved does not change the performance (section 5.4). These
generators stand in for its workloads:

* Domain [0,1]^3, structured nx x ny x nz grid, element e = i + nx (j + ny k).
  Node (I, J, K) sits at (I/nx, J/ny, K/nz); interior nodes get an independent uniform jitter in
  [-alpha, alpha] * h_d per coordinate (boundary nodes stay fixed, so the volume is exactly 1).
  Element vertex v = v1 + 2 v2 + 4 v3 is node (i + v1, j + v2, k + v3).
* Draw order from ``numpy.random.default_rng(seed)``: jitter (nz+1, ny+1, nx+1, 3); then per
  element, each as one array over all elements: G ~ N(0,1)^{3x3} (Q = QR(G) with diag(R) > 0),
  log10(lambda) ~ U[-1,1]^3, b ~ U[-1,1]^3, c ~ U[0,1], f ~ U[-1,1]; then degrees; then fields.
* ELEMENT record (14): K = Q diag(lambda) Q^T (row-major), b, c, f.
  FIELD record (10): Q (row-major), f; with a field descriptor of 7 fields x 5 modes x
  (a, k1, k2, k3, theta): a ~ U[-1,1] normalised to sum_m |a_sm| = 1, k ~ U{-2..2}^3,
  theta ~ U[0, 2 pi). Field s is g_s(x) = sum_m a_sm sin(2 pi k_sm . x + theta_sm); the
  coefficients at a point are K = Q diag(10^g0, 10^g1, 10^g2) Q^T, b = (g3, g4, g5),
  c = (1 + g6) / 2 -- the same ranges as the per-element draws.
"""
from __future__ import annotations

from dataclasses import dataclass, field as dc_field

import numpy as np

ELEMENT = 0
FIELD = 1

FIELD_LEN = 7 * 5 * 5


# --------------------------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------------------------
def node_grid(nx: int, ny: int, nz: int, alpha: float, rng: np.random.Generator) -> np.ndarray:
    """Jittered node coordinates, shape (nz+1, ny+1, nx+1, 3)."""
    h = np.array([1.0 / nx, 1.0 / ny, 1.0 / nz])
    jit = rng.uniform(-1.0, 1.0, size=(nz + 1, ny + 1, nx + 1, 3)) * alpha * h
    kk, jj, ii = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    nodes = np.stack([ii / nx, jj / ny, kk / nz], axis=-1).astype(np.float64)
    interior = np.ones((nz + 1, ny + 1, nx + 1), dtype=bool)
    interior[0, :, :] = interior[-1, :, :] = False
    interior[:, 0, :] = interior[:, -1, :] = False
    interior[:, :, 0] = interior[:, :, -1] = False
    nodes[interior] += jit[interior]
    return nodes


def element_vertices(nodes: np.ndarray) -> np.ndarray:
    """Gather [nel][8][3] vertex coordinates (vertex v = v1 + 2 v2 + 4 v3)."""
    nz, ny, nx = (s - 1 for s in nodes.shape[:3])
    out = np.empty((nz, ny, nx, 8, 3))
    for v in range(8):
        v1, v2, v3 = v & 1, (v >> 1) & 1, (v >> 2) & 1
        out[:, :, :, v, :] = nodes[v3:v3 + nz, v2:v2 + ny, v1:v1 + nx, :]
    return np.ascontiguousarray(out.reshape(nx * ny * nz, 8, 3))


def prism_vertices(nodes: np.ndarray) -> np.ndarray:
    """Split every cell of the node grid into two prisms along the diagonal of its xy face and
    gather [2 nel][6][3] vertex coordinates (vertex v = t + 3h: triangle vertex t of the layer
    h = 0 below, h = 1 above). Cell e = i + nx (j + ny k) gives prism 2e with the triangle
    (n00, n10, n01) and prism 2e + 1 with (n11, n01, n10) (both counter-clockwise seen from +z),
    nab being the cell's node (i + a, j + b)."""
    nz, ny, nx = (s - 1 for s in nodes.shape[:3])
    tri = (((0, 0), (1, 0), (0, 1)), ((1, 1), (0, 1), (1, 0)))
    out = np.empty((nz, ny, nx, 2, 6, 3))
    for half in range(2):
        for h in range(2):
            for t, (a, b) in enumerate(tri[half]):
                out[:, :, :, half, t + 3 * h, :] = nodes[h:h + nz, b:b + ny, a:a + nx, :]
    return np.ascontiguousarray(out.reshape(2 * nx * ny * nz, 6, 3))


def random_rotations(nel: int, rng: np.random.Generator) -> np.ndarray:
    g = rng.standard_normal((nel, 3, 3))
    q, r = np.linalg.qr(g)
    s = np.sign(np.diagonal(r, axis1=1, axis2=2))
    s[s == 0] = 1.0
    return q * s[:, None, :]


def cdr_element_coeffs(nel: int, rng: np.random.Generator) -> np.ndarray:
    """ELEMENT records [nel][14] = K (row-major), b, c, f with K = Q diag(10^U[-1,1]) Q^T."""
    q = random_rotations(nel, rng)
    loglam = rng.uniform(-1.0, 1.0, size=(nel, 3))
    bvec = rng.uniform(-1.0, 1.0, size=(nel, 3))
    c = rng.uniform(0.0, 1.0, size=nel)
    f = rng.uniform(-1.0, 1.0, size=nel)
    lam = 10.0 ** loglam
    K = np.einsum("eij,ej,ekj->eik", q, lam, q)
    K = 0.5 * (K + np.transpose(K, (0, 2, 1)))
    rec = np.empty((nel, 14))
    rec[:, 0:9] = K.reshape(nel, 9)
    rec[:, 9:12] = bvec
    rec[:, 12] = c
    rec[:, 13] = f
    return rec


def poisson_coeffs(nel: int) -> np.ndarray:
    """ELEMENT records for K = I, b = 0, c = 0, f = 1."""
    rec = np.zeros((nel, 14))
    rec[:, 0] = rec[:, 4] = rec[:, 8] = 1.0
    rec[:, 13] = 1.0
    return rec


def field_element_records(nel: int, rng: np.random.Generator) -> np.ndarray:
    """FIELD records [nel][10] = Q (row-major), f."""
    q = random_rotations(nel, rng)
    f = rng.uniform(-1.0, 1.0, size=nel)
    rec = np.empty((nel, 10))
    rec[:, 0:9] = q.reshape(nel, 9)
    rec[:, 9] = f
    return rec


def field_descriptor(rng: np.random.Generator) -> np.ndarray:
    """[7][5][5] = (a, k1, k2, k3, theta) per field and mode, flattened to 175 doubles."""
    a = rng.uniform(-1.0, 1.0, size=(7, 5))
    a /= np.abs(a).sum(axis=1, keepdims=True)
    k = rng.integers(-2, 3, size=(7, 5, 3)).astype(np.float64)
    theta = rng.uniform(0.0, 2.0 * np.pi, size=(7, 5))
    d = np.empty((7, 5, 5))
    d[:, :, 0] = a
    d[:, :, 1:4] = k
    d[:, :, 4] = theta
    return d.reshape(-1).copy()


def elastic_coeffs(nel: int, rng: np.random.Generator) -> np.ndarray:
    """Per-element material data of the elastostatics model problem (section 5.1): Young modulus
    E ~ U[1, 10], Poisson ratio nu ~ U[0.2, 0.4], body force f ~ U[-1, 1]^3. [nel, 5]."""
    rec = np.empty((nel, 5))
    rec[:, 0] = rng.uniform(1.0, 10.0, nel)
    rec[:, 1] = rng.uniform(0.2, 0.4, nel)
    rec[:, 2:5] = rng.uniform(-1.0, 1.0, (nel, 3))
    return rec


def phase_shift(seed: int, step: int) -> np.ndarray:
    """The phase increment delta_t ~ U[0, 2 pi)^{7x5} of time step ``step`` (>= 1)."""
    return np.random.default_rng([seed, step]).uniform(0.0, 2.0 * np.pi, size=(7, 5))


def field_at_step(field0: np.ndarray, seed: int, step: int) -> np.ndarray:
    """Descriptor after ``step`` phase updates: theta_t = theta_0 + sum_{s=1..t} delta_s (mod 2 pi)."""
    d = np.array(field0, dtype=np.float64).reshape(7, 5, 5).copy()
    for s in range(1, step + 1):
        d[:, :, 4] = np.mod(d[:, :, 4] + phase_shift(seed, s), 2.0 * np.pi)
    return d.reshape(-1)


def step_sample(seed: int, step: int, nel: int) -> np.ndarray:
    """Sorted 1 % element sample checked at time step ``step``."""
    idx = np.random.default_rng([seed, step, 1]).choice(nel, max(1, nel // 100), replace=False)
    return np.sort(idx)


def degrees_weighted(nel: int, rng: np.random.Generator) -> np.ndarray:
    """i.i.d. p in 1..7 with P(p) proportional to 8 - p."""
    w = np.array([8 - p for p in range(1, 8)], dtype=np.float64)
    return (rng.choice(7, size=nel, p=w / w.sum()) + 1).astype(np.int8)


def degrees_uniform(nel: int, lo: int, hi: int, rng: np.random.Generator) -> np.ndarray:
    return rng.integers(lo, hi + 1, size=nel).astype(np.int8)


# --------------------------------------------------------------------------------------------
# mesh validity: a sufficient condition for detJ > 0 on the whole element
# --------------------------------------------------------------------------------------------
def min_bernstein_volume(geom: np.ndarray) -> np.ndarray:
    """Per element, the smallest Bernstein coefficient of the trilinear map's volume form.

    With u in [0,1]^3, each column of dx/du is bilinear in the two other variables, so the
    determinant is a polynomial of degree <= 2 per variable. Written in the degree-(2,2,2)
    tensor Bernstein basis, every coefficient is an average of scalar triple products of edge
    differences; all coefficients > 0 implies det > 0 everywhere on the element (the basis is
    non-negative and sums to one). This is a mesh-quality filter only.
    """
    X = np.asarray(geom, dtype=np.float64).reshape(-1, 2, 2, 2, 3)  # [e][c][b][a][xyz], v = a+2b+4c
    # E1[b][c] = X[a=1] - X[a=0], E2[a][c] = X[b=1] - X[b=0], E3[a][b] = X[c=1] - X[c=0]
    E1 = X[:, :, :, 1, :] - X[:, :, :, 0, :]   # [e][c][b]
    E2 = X[:, :, 1, :, :] - X[:, :, 0, :, :]   # [e][c][a]
    E3 = X[:, 1, :, :, :] - X[:, 0, :, :, :]   # [e][b][a]
    nel = X.shape[0]
    acc = np.zeros((nel, 3, 3, 3))
    cnt = np.zeros((3, 3, 3))
    for b in range(2):
        for c in range(2):
            e1 = E1[:, c, b, :]
            for a1 in range(2):
                for c1 in range(2):
                    e2 = E2[:, c1, a1, :]
                    for a2 in range(2):
                        for b2 in range(2):
                            e3 = E3[:, b2, a2, :]
                            t = np.einsum("ei,ei->e", e1, np.cross(e2, e3))
                            i, j, k = a1 + a2, b + b2, c + c1
                            acc[:, i, j, k] += t
                            cnt[i, j, k] += 1
    return (acc / cnt).min(axis=(1, 2, 3))


# --------------------------------------------------------------------------------------------
# workload configurations
# --------------------------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    seed: int
    grid: tuple
    alpha: float
    geom: np.ndarray
    mode: int
    coef: np.ndarray
    p: int = 0                      # uniform degree, 0 if mixed
    degree: np.ndarray | None = None
    field: np.ndarray | None = None
    redraws: int = 0
    extra: dict = dc_field(default_factory=dict)

    @property
    def nel(self) -> int:
        return int(self.geom.shape[0])


def _grid_for(cfg: int, p: int | None):
    if cfg == 1:
        return (16, 16, 16)
    if cfg == 2:
        return {2: (64, 64, 64), 3: (64, 64, 32), 4: (64, 32, 32)}[p]
    if cfg == 3:
        return {5: (32, 32, 16), 6: (32, 16, 16), 7: (16, 16, 16)}[p]
    if cfg == 4:
        return (100, 50, 40)
    if cfg == 5:
        return (50, 50, 40)
    raise ValueError(cfg)


def make(cfg: int, p: int | None = None, grid: tuple | None = None) -> Workload:
    """Build workload ``cfg`` (1..5). ``grid`` overrides the grid to get a smaller instance with
    the same seed, jitter, coefficient law and degree law."""
    seed = cfg
    g = tuple(grid) if grid is not None else _grid_for(cfg, p)
    nx, ny, nz = g
    nel = nx * ny * nz
    rng = np.random.default_rng(seed)
    if cfg == 1:
        nodes = node_grid(nx, ny, nz, 0.10, rng)
        return Workload("p1-poisson", seed, g, 0.10, element_vertices(nodes), ELEMENT,
                        poisson_coeffs(nel), p=1)
    if cfg in (2, 3):
        assert p is not None and ((cfg == 2 and 2 <= p <= 4) or (cfg == 3 and 5 <= p <= 7))
        nodes = node_grid(nx, ny, nz, 0.15, rng)
        return Workload(f"cdr-p{p}", seed, g, 0.15, element_vertices(nodes), ELEMENT,
                        cdr_element_coeffs(nel, rng), p=p)
    if cfg == 4:
        nodes = node_grid(nx, ny, nz, 0.15, rng)
        geom = element_vertices(nodes)
        rec = field_element_records(nel, rng)
        deg = degrees_weighted(nel, rng)
        fld = field_descriptor(rng)
        return Workload("mixed-field", seed, g, 0.15, geom, FIELD, rec, degree=deg, field=fld)
    if cfg == 5:
        nodes = node_grid(nx, ny, nz, 0.30, rng)
        nodes, redraws = _fix_inverted(nodes, nx, ny, nz, 0.30, seed)
        geom = element_vertices(nodes)
        rec = field_element_records(nel, rng)
        deg = degrees_uniform(nel, 2, 6, rng)
        fld = field_descriptor(rng)
        return Workload("timestep-field", seed, g, 0.30, geom, FIELD, rec, degree=deg, field=fld,
                        redraws=redraws)
    raise ValueError(cfg)


def _fix_inverted(nodes, nx, ny, nz, alpha, seed, max_iter=200, tol=0.05):
    """Redraw the interior-node jitter of elements that fail the Bernstein volume test until none
    fails. An element passes when every Bernstein coefficient of its volume form exceeds
    ``tol`` times the undistorted cell volume (detJ > 0 everywhere, with a margin that keeps
    elements away from degeneracy). Redraw r uses default_rng([seed, 7, r])."""
    h = np.array([1.0 / nx, 1.0 / ny, 1.0 / nz])
    kk, jj, ii = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    base = np.stack([ii / nx, jj / ny, kk / nz], axis=-1).astype(np.float64)
    interior = np.ones((nz + 1, ny + 1, nx + 1), dtype=bool)
    interior[0, :, :] = interior[-1, :, :] = False
    interior[:, 0, :] = interior[:, -1, :] = False
    interior[:, :, 0] = interior[:, :, -1] = False
    redraws = 0
    for it in range(max_iter):
        vmin = min_bernstein_volume(element_vertices(nodes))
        bad = np.nonzero(vmin <= tol * h[0] * h[1] * h[2])[0]
        if bad.size == 0:
            return nodes, redraws
        redraws += int(bad.size)
        mark = np.zeros_like(interior)
        k = bad // (nx * ny)
        j = (bad // nx) % ny
        i = bad % nx
        for v in range(8):
            mark[k + ((v >> 2) & 1), j + ((v >> 1) & 1), i + (v & 1)] = True
        mark &= interior
        rr = np.random.default_rng([seed, 7, it])
        jit = rr.uniform(-1.0, 1.0, size=nodes.shape) * alpha * h
        nodes = nodes.copy()
        nodes[mark] = base[mark] + jit[mark]
    raise RuntimeError("mesh repair did not converge")


# Prism workloads (the paper's reference element, section 2): jittered grids of cells split into
# two prisms each; per prism the CDR coefficient law of the hexahedral workloads ("prism-cdr",
# seed 6), the elastostatics model problem of section 5.1 ("prism-elastic", seed 7; the paper's
# own benchmark) or FIELD records ("prism-field", seed 8). Draw order: jitter, then records.
PRISM_GRIDS = {1: (64, 64, 64), 2: (64, 64, 32), 3: (64, 32, 32), 4: (32, 32, 32),
               5: (32, 32, 16), 6: (32, 16, 16), 7: (16, 16, 16)}
PRISM_KINDS = {"cdr": 6, "elastic": 7, "field": 8}


def make_prism(kind: str, p: int, grid: tuple | None = None, alpha: float = 0.15) -> Workload:
    """Prism workload ``kind`` ("cdr", "elastic" or "field") of degree p on ``grid`` cells
    (default PRISM_GRIDS[p]; 2 nx ny nz prisms)."""
    seed = PRISM_KINDS[kind]
    g = tuple(grid) if grid is not None else PRISM_GRIDS[p]
    nx, ny, nz = g
    rng = np.random.default_rng(seed)
    geom = prism_vertices(node_grid(nx, ny, nz, alpha, rng))
    nel = geom.shape[0]
    if kind == "cdr":
        return Workload(f"prism-cdr-p{p}", seed, g, alpha, geom, ELEMENT, cdr_element_coeffs(nel, rng), p=p)
    if kind == "elastic":
        return Workload(f"prism-elastic-p{p}", seed, g, alpha, geom, 2, elastic_coeffs(nel, rng), p=p)
    rec = field_element_records(nel, rng)
    return Workload(f"prism-field-p{p}", seed, g, alpha, geom, FIELD, rec, p=p,
                    field=field_descriptor(rng))


def small(cfg: int, p: int | None = None, scale: int = 8) -> Workload:
    """A reduced instance of ``cfg``: each grid dimension divided by ``scale`` (at least 2)."""
    g = _grid_for(cfg, p)
    g = tuple(max(2, d // scale) for d in g)
    return make(cfg, p=p, grid=g)
