"""Python binding of libfem (include/fem.h): argument marshalling only.

Every step of the integration runs in the HIP kernels of ``libfem.so``; this module turns torch
device tensors into pointers and calls the C ABI with the same names. There is no CPU fallback:
if the library is not built, or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfem.so")

FEM_OK = 0
FEM_EINVAL = -1
FEM_EDEGREE = -2
FEM_ENOTINIT = -3
FEM_ENOMEM = -4
FEM_EHIP = -5
FEM_ECONFIG = -6
FEM_EWORKSPACE = -7
FEM_ETOOBIG = -8
NOALLOC_MAX_NEL = 1 << 22

FP64, FP32, BF16, SPLIT_BF16, SPLIT_FP16 = 0, 1, 2, 3, 4
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "split_bf16": SPLIT_BF16,
              "split_fp16": SPLIT_FP16}
ELEMENT, FIELD, ELASTIC = 0, 1, 2


class fem_coeffs(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("elem", ctypes.c_void_p),
        ("field", ctypes.c_void_p),
        ("degree", ctypes.c_void_p),
        ("a_off", ctypes.c_void_p),
        ("b_off", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("jac", ctypes.c_void_p),
    ]


class fem_staged_stats(ctypes.Structure):
    _fields_ = [
        ("total_ms", ctypes.c_double),
        ("h2d_ms", ctypes.c_double),
        ("kernel_ms", ctypes.c_double),
        ("d2h_ms", ctypes.c_double),
        ("h2d_bytes", ctypes.c_int64),
        ("d2h_bytes", ctypes.c_int64),
        ("chunks", ctypes.c_int64),
    ]


STAGED_MAX_STREAMS = 8


class FemError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {fem_strerror(status)} ({status})")
        self.status = status


_lib = None


def load():
    """Load libfem.so (built in-tree by paper_1310_1191_amd.build). Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1310_1191_amd.build` "
                           "(there is no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.fem_init.argtypes = [ctypes.c_int]
    lib.fem_finalize.argtypes = []
    lib.fem_integrate.argtypes = [ctypes.c_int64, ctypes.c_int, vp, ctypes.POINTER(fem_coeffs), vp,
                                  vp, vp]
    lib.fem_integrate_prism.argtypes = [ctypes.c_int64, ctypes.c_int, vp,
                                        ctypes.POINTER(fem_coeffs), vp, vp, vp]
    lib.fem_prism_reference_tables.argtypes = [ctypes.c_int, vp, vp]
    lib.fem_integrate_noalloc.argtypes = [ctypes.c_int64, ctypes.c_int, vp,
                                          ctypes.POINTER(fem_coeffs), vp, vp, vp]
    lib.fem_workspace_bytes.argtypes = [ctypes.c_int64]
    lib.fem_workspace_bytes.restype = ctypes.c_size_t
    lib.fem_mixed_offsets.argtypes = [ctypes.c_int64, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.fem_jacobian_terms.argtypes = [ctypes.c_int64, ctypes.c_int, vp, vp, vp, vp, vp]
    lib.fem_integrate_staged.argtypes = [ctypes.c_int64, ctypes.c_int, vp, ctypes.POINTER(fem_coeffs),
                                         vp, vp, ctypes.c_int64, ctypes.c_int,
                                         ctypes.POINTER(fem_staged_stats)]
    lib.fem_strerror.argtypes = [ctypes.c_int]
    lib.fem_strerror.restype = ctypes.c_char_p
    lib.fem_abi_version.argtypes = []
    dp = ctypes.POINTER(ctypes.c_double)
    lib.fem_reference_tables.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp]
    lib.fem_field_advance.argtypes = [vp, vp, ctypes.c_int32, vp, vp]
    lib.fem_gather_sample.argtypes = [ctypes.c_int64, vp, ctypes.c_int32, vp, ctypes.c_int64, vp, vp,
                                      vp, vp, ctypes.c_int, vp, ctypes.c_int64, vp, ctypes.c_int64, vp]
    lib.fem_variant_count.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.fem_get_variant.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.fem_set_variant.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.fem_autotune.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                 ctypes.c_char_p, ctypes.POINTER(ctypes.c_int), dp]
    lib.fem_load_tuning.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)]
    lib.fem_mixed_variant.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.fem_elastic_blocks.argtypes = [ctypes.c_int, ctypes.c_int]
    _lib = lib
    return lib


def exported_symbols():
    return ["fem_init", "fem_finalize", "fem_integrate", "fem_workspace_bytes",
            "fem_mixed_offsets", "fem_field_advance", "fem_reference_tables", "fem_strerror",
            "fem_abi_version", "fem_variant_count", "fem_get_variant", "fem_set_variant",
            "fem_autotune", "fem_load_tuning", "fem_mixed_variant", "fem_jacobian_terms",
            "fem_integrate_staged", "fem_integrate_noalloc", "fem_integrate_prism",
            "fem_prism_reference_tables", "fem_elastic_blocks", "fem_gather_sample"]


# ---------------------------------------------------------------------------------------------
# the C ABI, one to one
# ---------------------------------------------------------------------------------------------
def fem_strerror(status: int) -> str:
    return load().fem_strerror(int(status)).decode()


def fem_abi_version() -> int:
    return int(load().fem_abi_version())


def fem_reference_tables(p: int):
    """Host copies of the degree-p tables: (gauss_x, gauss_w, lobatto_x, L[q][a], D[q][a])."""
    import numpy as np
    n = p + 1
    gx, gw, lx = np.zeros(n), np.zeros(n), np.zeros(n)
    L, D = np.zeros((n, n)), np.zeros((n, n))
    dp = ctypes.POINTER(ctypes.c_double)
    rc = load().fem_reference_tables(int(p), *(a.ctypes.data_as(dp) for a in (gx, gw, lx, L, D)))
    if rc != FEM_OK:
        raise FemError(rc, "fem_reference_tables")
    return gx, gw, lx, L, D


def fem_init(device: int = 0) -> None:
    rc = load().fem_init(int(device))
    if rc != FEM_OK:
        raise FemError(rc, "fem_init")


def fem_finalize() -> None:
    rc = load().fem_finalize()
    if rc != FEM_OK:
        raise FemError(rc, "fem_finalize")


def fem_workspace_bytes(nel: int) -> int:
    return int(load().fem_workspace_bytes(int(nel)))


def fem_integrate(nel: int, p: int, geom: int, coeffs: fem_coeffs, out_A: int, out_b: int | None,
                  stream: int | None) -> int:
    """Raw call: integer device addresses, returns the status code."""
    return int(load().fem_integrate(int(nel), int(p), geom, ctypes.byref(coeffs), out_A, out_b,
                                    stream))


def fem_integrate_prism(nel: int, p: int, geom: int, coeffs: fem_coeffs, out_A: int,
                        out_b: int | None, stream: int | None) -> int:
    """Raw call for prisms: integer device addresses, returns the status code."""
    return int(load().fem_integrate_prism(int(nel), int(p), geom, ctypes.byref(coeffs), out_A,
                                          out_b, stream))


PRISM_TRI_POINTS = {1: 3, 2: 6, 3: 12, 4: 16, 5: 25, 6: 33, 7: 42}


def prism(p: int) -> int:
    """Variant key of the degree-p prism (FEM_PRISM(p))."""
    return 10 + int(p)


def mixed(p: int) -> int:
    """Variant key of degree p's tile inside the single mixed-degree launch (FEM_MIXED(p))."""
    return 20 + int(p)


def prism_ns(p: int) -> int:
    return (p + 1) * (p + 1) * (p + 2) // 2


def fem_prism_reference_tables(p: int):
    """Host copies of the prism's triangle rule [ntq, 3] = (xi1, xi2, w) and B [Nq, 4, Ns]."""
    import numpy as np
    if not 1 <= p <= 7:
        raise FemError(FEM_EDEGREE, "fem_prism_reference_tables")
    ntq = PRISM_TRI_POINTS[p]
    tri = np.zeros((ntq, 3))
    B = np.zeros((ntq * (p + 1), 4, prism_ns(p)))
    rc = load().fem_prism_reference_tables(int(p), ctypes.c_void_p(tri.ctypes.data),
                                           ctypes.c_void_p(B.ctypes.data))
    if rc != FEM_OK:
        raise FemError(rc, "fem_prism_reference_tables")
    return tri, B


def fem_integrate_noalloc(nel: int, p: int, geom: int, coeffs: fem_coeffs, out_A: int,
                          out_b: int | None, stream: int | None) -> int:
    """Raw call of the allocation-free variant: integer device addresses, returns the status."""
    return int(load().fem_integrate_noalloc(int(nel), int(p), geom, ctypes.byref(coeffs), out_A,
                                            out_b, stream))


def fem_mixed_offsets(nel: int, degree: int, a_off: int, b_off: int, workspace: int,
                      workspace_bytes: int, stream: int | None) -> int:
    return int(load().fem_mixed_offsets(int(nel), degree, a_off, b_off, workspace,
                                         int(workspace_bytes), stream))


def fem_jacobian_terms(nel: int, p: int, geom: int, degree: int | None, b_off: int | None,
                       jac: int, stream: int | None) -> int:
    return int(load().fem_jacobian_terms(int(nel), int(p), geom, degree, b_off, jac, stream))


def fem_integrate_staged(nel: int, p: int, geom: int, coeffs: fem_coeffs, out_A: int,
                         out_b: int | None, chunk: int, nstreams: int,
                         stats: fem_staged_stats | None) -> int:
    """Raw call: integer HOST addresses, returns the status code."""
    return int(load().fem_integrate_staged(int(nel), int(p), geom, ctypes.byref(coeffs), out_A,
                                           out_b, int(chunk), int(nstreams),
                                           ctypes.byref(stats) if stats is not None else None))


def fem_field_advance(field: int, deltas: int, nsteps: int, step: int, stream: int | None) -> int:
    return int(load().fem_field_advance(field, deltas, int(nsteps), step, stream))


def fem_gather_sample(nsel, sel, nrows, step, nel, a_off, b_off, A, b, precision, out_A, cap_A,
                      out_b, cap_b, stream) -> int:
    return int(load().fem_gather_sample(int(nsel), sel, int(nrows), step, int(nel), a_off, b_off, A, b,
                                        int(precision), out_A, int(cap_A), out_b, int(cap_b), stream))


MAX_VARIANTS = 7


def trilinear_variant(precision: int) -> int:
    """FEM_TRILINEAR_VARIANT: the p = 1 vector-ALU variant (ELEMENT mode only)."""
    return 1 if int(precision) == FP64 else 5


def fem_variant_count(p: int, precision: int) -> int:
    rc = int(load().fem_variant_count(int(p), int(precision)))
    if rc < 0:
        raise FemError(rc, "fem_variant_count")
    return rc


MODES = (ELEMENT, FIELD, ELASTIC)


def fem_get_variant(p: int, precision: int, mode: int) -> int:
    rc = int(load().fem_get_variant(int(p), int(precision), int(mode)))
    if rc < 0:
        raise FemError(rc, "fem_get_variant")
    return rc


def fem_set_variant(p: int, precision: int, mode: int, variant: int) -> None:
    rc = int(load().fem_set_variant(int(p), int(precision), int(mode), int(variant)))
    if rc != FEM_OK:
        raise FemError(rc, "fem_set_variant")


def fem_autotune(p: int, precision: int, mode: int, nel: int, json_path: str | None = None):
    """Time every variant of (p, precision, mode) on nel synthetic elements and choose the
    fastest. Returns (chosen variant, [ms per call of each variant])."""
    chosen = ctypes.c_int(-1)
    times = (ctypes.c_double * MAX_VARIANTS)()
    path = None if json_path is None else os.fsencode(json_path)
    rc = int(load().fem_autotune(int(p), int(precision), int(mode), int(nel), path,
                                 ctypes.byref(chosen), times))
    if rc != FEM_OK:
        raise FemError(rc, "fem_autotune")
    return chosen.value, list(times)[:fem_variant_count(p, precision)]


def fem_mixed_variant(p: int, precision: int, mode: int) -> int:
    rc = int(load().fem_mixed_variant(int(p), int(precision), int(mode)))
    if rc < 0:
        raise FemError(rc, "fem_mixed_variant")
    return rc


def fem_elastic_blocks(p: int, precision: int) -> int:
    """Blocks (6 or 9) an ELASTIC call integrates on the matrix cores for (p, precision)."""
    rc = int(load().fem_elastic_blocks(int(p), int(precision)))
    if rc < 0:
        raise FemError(rc, "fem_elastic_blocks")
    return rc


def mixed_tile_variant(p: int, precision: int, mode: int) -> int:
    """The per-degree variant number of the tile degree p runs with in the single launch."""
    return fem_mixed_variant(p, precision, mode)


def fem_load_tuning(json_path: str) -> int:
    applied = ctypes.c_int(0)
    rc = int(load().fem_load_tuning(os.fsencode(json_path), ctypes.byref(applied)))
    if rc != FEM_OK:
        raise FemError(rc, "fem_load_tuning")
    return applied.value


# ---------------------------------------------------------------------------------------------
# torch conveniences (device memory and the current stream only)
# ---------------------------------------------------------------------------------------------
def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libfem needs a ROCm GPU; none is visible")
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check(t, dtype, name, shape=None, min_numel=None):
    """A caller's buffer must be a contiguous device tensor of the kernel's element type and
    size: the kernels write and read by computed offsets, so a short or mistyped buffer would be
    accessed out of bounds. Raises ValueError before anything is launched."""
    if t is None:
        return
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} device tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{name} holds {t.numel()} entries, the call writes {min_numel}")


RECORD_LENGTH = {ELEMENT: 14, FIELD: 10, ELASTIC: 5}


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_coeffs(precision, mode, elem, field=None, degree=None, a_off=None, b_off=None,
                status=None, workspace=None, jac=None) -> fem_coeffs:
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    c = fem_coeffs()
    c.precision = prec
    c.mode = int(mode)
    c.elem = elem.data_ptr()
    c.field = field.data_ptr() if field is not None else None
    c.degree = degree.data_ptr() if degree is not None else None
    c.a_off = a_off.data_ptr() if a_off is not None else None
    c.b_off = b_off.data_ptr() if b_off is not None else None
    c.status = status.data_ptr() if status is not None else None
    c.workspace = workspace.data_ptr() if workspace is not None else None
    c.workspace_bytes = workspace.numel() if workspace is not None else 0
    c.jac = jac.data_ptr() if jac is not None else None
    return c


def out_dtype(precision):
    torch = _torch()
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return torch.float64 if prec == FP64 else torch.float32


def _check_inputs(torch, geom, elem, mode, nel, field, status, jac, jac_rows):
    if mode not in RECORD_LENGTH:
        raise ValueError(f"unknown coefficient mode {mode}")
    _check(elem, torch.float64, "elem", shape=(nel, RECORD_LENGTH[mode]))
    _check(geom, torch.float64, "geom", shape=(nel, 8, 3))
    _check(field, torch.float64, "field", min_numel=175)
    _check(status, torch.int32, "status", min_numel=2)
    _check(jac, torch.float64, "jac", min_numel=None if jac_rows is None else jac_rows * 10)
    if mode == FIELD and field is None:
        raise ValueError("FIELD mode needs the field descriptor")


def integrate(geom, elem, p: int, precision="split_fp16", mode: int = ELEMENT, field=None,
              out_A=None, out_b=None, status=None, with_b: bool = True, stream=None, jac=None):
    """Uniform degree p: returns (A [nel, Ns, Ns], b [nel, Ns] or None) on the device; for
    mode ELASTIC (elem [nel, 5] = E, nu, f1, f2, f3) A is [nel, 3, 3, Ns, Ns], b [nel, 3, Ns].
    ``jac`` ([nel, Ns, 10], see ``jacobian_terms``) supplies the Jacobian terms; ``geom`` may
    then be None outside FIELD mode."""
    torch = _torch()
    if not 1 <= p <= 7:
        raise ValueError(f"degree {p} outside 1..7 (per-element degrees: integrate_mixed)")
    fem_init(elem.device.index or 0)
    nel = elem.shape[0]
    ns = (p + 1) ** 3
    dt = out_dtype(precision)
    _check_inputs(torch, geom, elem, mode, nel, field, status, jac, nel * ns)
    if jac is not None:
        _check(jac, torch.float64, "jac", shape=(nel, ns, 10))
    ashape, bshape = ((nel, 3, 3, ns, ns), (nel, 3, ns)) if mode == ELASTIC else ((nel, ns, ns), (nel, ns))
    if out_A is None:
        out_A = torch.empty(ashape, dtype=dt, device=elem.device)
    if out_b is None and with_b:
        out_b = torch.empty(bshape, dtype=dt, device=elem.device)
    _check(out_A, dt, "out_A", min_numel=nel * (9 if mode == ELASTIC else 1) * ns * ns)
    _check(out_b, dt, "out_b", min_numel=nel * (3 if mode == ELASTIC else 1) * ns)
    c = make_coeffs(precision, mode, elem, field=field, status=status, jac=jac)
    rc = fem_integrate(nel, p, _ptr(geom), c, _ptr(out_A), _ptr(out_b), _stream(stream))
    if rc != FEM_OK:
        raise FemError(rc, "fem_integrate")
    return out_A, out_b


def integrate_prism(geom, elem, p: int, precision="split_fp16", mode: int = ELEMENT, field=None,
                    out_A=None, out_b=None, status=None, with_b: bool = True, stream=None):
    """Prisms of uniform degree p (geom [nel, 6, 3]): returns (A [nel, Ns, Ns], b [nel, Ns] or
    None) on the device; for mode ELASTIC (elem [nel, 5]) A is [nel, 3, 3, Ns, Ns], b [nel, 3, Ns]."""
    torch = _torch()
    if not 1 <= p <= 7:
        raise ValueError(f"degree {p} outside 1..7")
    fem_init(elem.device.index or 0)
    nel = elem.shape[0]
    ns = prism_ns(p)
    dt = out_dtype(precision)
    if mode not in RECORD_LENGTH:
        raise ValueError(f"unknown coefficient mode {mode}")
    _check(elem, torch.float64, "elem", shape=(nel, RECORD_LENGTH[mode]))
    _check(geom, torch.float64, "geom", shape=(nel, 6, 3))
    _check(field, torch.float64, "field", min_numel=175)
    _check(status, torch.int32, "status", min_numel=2)
    if mode == FIELD and field is None:
        raise ValueError("FIELD mode needs the field descriptor")
    ashape, bshape = ((nel, 3, 3, ns, ns), (nel, 3, ns)) if mode == ELASTIC else ((nel, ns, ns), (nel, ns))
    if out_A is None:
        out_A = torch.empty(ashape, dtype=dt, device=elem.device)
    if out_b is None and with_b:
        out_b = torch.empty(bshape, dtype=dt, device=elem.device)
    _check(out_A, dt, "out_A", min_numel=nel * (9 if mode == ELASTIC else 1) * ns * ns)
    _check(out_b, dt, "out_b", min_numel=nel * (3 if mode == ELASTIC else 1) * ns)
    c = make_coeffs(precision, mode, elem, field=field, status=status)
    rc = fem_integrate_prism(nel, p, _ptr(geom), c, _ptr(out_A), _ptr(out_b), _stream(stream))
    if rc != FEM_OK:
        raise FemError(rc, "fem_integrate_prism")
    return out_A, out_b


def mixed_offsets(degree, workspace=None, stream=None):
    """Device exclusive scans of Ns^2 and Ns over the degrees: (a_off, b_off), nel + 1 each."""
    torch = _torch()
    fem_init(degree.device.index or 0)
    nel = degree.shape[0]
    _check(degree, torch.int8, "degree")
    a_off = torch.empty(nel + 1, dtype=torch.int64, device=degree.device)
    b_off = torch.empty(nel + 1, dtype=torch.int64, device=degree.device)
    if workspace is None:
        workspace = torch.empty(fem_workspace_bytes(nel), dtype=torch.uint8, device=degree.device)
    rc = fem_mixed_offsets(nel, _ptr(degree), _ptr(a_off), _ptr(b_off), _ptr(workspace),
                           workspace.numel(), _stream(stream))
    if rc != FEM_OK:
        raise FemError(rc, "fem_mixed_offsets")
    return a_off, b_off


def integrate_mixed(geom, elem, degree, precision="split_fp16", mode: int = ELEMENT, field=None,
                    a_off=None, b_off=None, out_A=None, out_b=None, status=None, workspace=None,
                    with_b: bool = True, stream=None, jac=None):
    """Per-element degrees: returns (A packed, b packed, a_off, b_off) on the device. ``jac``
    (packed by b_off, see ``jacobian_terms``) supplies the Jacobian terms."""
    torch = _torch()
    dev = elem.device
    fem_init(dev.index or 0)
    nel = elem.shape[0]
    if mode == ELASTIC:
        raise ValueError("the elasticity mode takes a uniform degree")
    _check(degree, torch.int8, "degree", shape=(nel,))
    _check_inputs(torch, geom, elem, mode, nel, field, status, None, None)
    _check(a_off, torch.int64, "a_off", shape=(nel + 1,))
    _check(b_off, torch.int64, "b_off", shape=(nel + 1,))
    _check(workspace, torch.uint8, "workspace", min_numel=fem_workspace_bytes(nel))
    if workspace is None:
        workspace = torch.empty(fem_workspace_bytes(nel), dtype=torch.uint8, device=dev)
    if a_off is None or b_off is None:
        a_off, b_off = mixed_offsets(degree, workspace=workspace, stream=stream)
    dt = out_dtype(precision)
    # output sizes are read back only when the outputs are allocated here; with caller-provided
    # outputs the call enqueues work and never synchronises (stream capture is possible)
    if out_A is None:
        out_A = torch.empty(int(a_off[-1].item()), dtype=dt, device=dev)
    if out_b is None and with_b:
        out_b = torch.empty(int(b_off[-1].item()), dtype=dt, device=dev)
    # caller-provided outputs: type and contiguity only (their sizes follow from the device scans,
    # which are not read back so that the call can be captured)
    _check(out_A, dt, "out_A")
    _check(out_b, dt, "out_b")
    _check(jac, torch.float64, "jac")
    c = make_coeffs(precision, mode, elem, field=field, degree=degree, a_off=a_off, b_off=b_off,
                    status=status, workspace=workspace, jac=jac)
    rc = fem_integrate(nel, 0, _ptr(geom), c, _ptr(out_A), _ptr(out_b), _stream(stream))
    if rc != FEM_OK:
        raise FemError(rc, "fem_integrate")
    return out_A, out_b, a_off, b_off


def _host(t, dtype, name):
    if t is None:
        return
    if t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} host tensor")


def integrate_staged(geom, elem, p: int, precision="split_fp16", mode: int = ELEMENT, field=None,
                     chunk: int = 16384, nstreams: int = 3, out_A=None, out_b=None,
                     with_b: bool = True, status=None):
    """Host-resident mesh (CPU tensors; pinned memory lets the copies overlap the kernels):
    returns (A, b, stats) with A, b host tensors (pinned when allocated here) and stats the
    per-stage times of fem_integrate_staged as a dict. ``status``: host int32[2], added to."""
    torch = _torch()
    fem_init(torch.cuda.current_device())
    nel = elem.shape[0]
    ns = (p + 1) ** 3 if 1 <= p <= 7 else 0
    dt = out_dtype(precision)
    _host(geom, torch.float64, "geom")
    _host(elem, torch.float64, "elem")
    _host(field, torch.float64, "field")
    _host(status, torch.int32, "status")
    ashape, bshape = ((nel, 3, 3, ns, ns), (nel, 3, ns)) if mode == ELASTIC else ((nel, ns, ns), (nel, ns))
    if out_A is None:
        out_A = torch.empty(ashape, dtype=dt, pin_memory=True)
    if out_b is None and with_b:
        out_b = torch.empty(bshape, dtype=dt, pin_memory=True)
    _host(out_A, dt, "out_A")
    _host(out_b, dt, "out_b")
    c = make_coeffs(precision, mode, elem, field=field, status=status)
    st = fem_staged_stats()
    rc = fem_integrate_staged(nel, p, _ptr(geom), c, _ptr(out_A), _ptr(out_b), chunk, nstreams, st)
    if rc != FEM_OK:
        raise FemError(rc, "fem_integrate_staged")
    stats = {k: getattr(st, k) for k, _ in fem_staged_stats._fields_}
    return out_A, out_b, stats


def jacobian_terms(geom, p: int = 0, degree=None, b_off=None, out=None, stream=None):
    """Device Jacobian terms of the NOJAC variant: [nel, Ns, 10] for a uniform p, or packed by
    the b_off scan ([b_off[-1], 10]) for per-element degrees (p = 0 with degree, b_off)."""
    torch = _torch()
    fem_init(geom.device.index or 0)
    nel = geom.shape[0]
    _check(geom, torch.float64, "geom")
    if out is None:
        if p > 0:
            ns = (p + 1) ** 3 if p <= 7 else 0
            out = torch.empty((nel, ns, 10), dtype=torch.float64, device=geom.device)
        else:
            out = torch.empty((int(b_off[-1].item()), 10), dtype=torch.float64, device=geom.device)
    rc = fem_jacobian_terms(nel, p, _ptr(geom), _ptr(degree), _ptr(b_off), _ptr(out),
                            _stream(stream))
    if rc != FEM_OK:
        raise FemError(rc, "fem_jacobian_terms")
    return out


def gather_sample(sel, a_off, A, out_A, precision, b_off=None, b=None, out_b=None, step=None,
                  stream=None):
    """Copy the element matrices (and vectors) of one row of `sel` into out_A (out_b), back to back
    in selection order (see fem_gather_sample). sel: int32 [nrows, nsel] (or [nsel]); the row
    used is (step - 1) mod nrows with a step counter, else 0."""
    torch = _torch()
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(sel, torch.int32, "sel")
    _check(a_off, torch.int64, "a_off")
    dt = out_dtype(prec)
    _check(A, dt, "A")
    _check(out_A, dt, "out_A")
    if step is not None:
        _check(step, torch.int32, "step")
    if b is not None:
        _check(b, dt, "b")
        _check(out_b, dt, "out_b")
        _check(b_off, torch.int64, "b_off", shape=tuple(a_off.shape))
    if sel.dim() not in (1, 2):
        raise ValueError("sel: [nsel] or [nrows, nsel] element ids")
    nrows, nsel = (1, sel.shape[0]) if sel.dim() == 1 else (sel.shape[0], sel.shape[1])
    rc = fem_gather_sample(nsel, _ptr(sel), nrows, _ptr(step) if step is not None else None,
                           a_off.shape[0] - 1, _ptr(a_off), _ptr(b_off) if b_off is not None else None,
                           _ptr(A), _ptr(b) if b is not None else None, prec, _ptr(out_A),
                           out_A.numel(), _ptr(out_b) if out_b is not None else None,
                           out_b.numel() if out_b is not None else 0, _stream(stream))
    if rc != FEM_OK:
        raise FemError(rc, "fem_gather_sample")


def field_advance(field, deltas, step, stream=None):
    """One device-side phase step of a FIELD descriptor (see fem_field_advance)."""
    torch = _torch()
    _check(field, torch.float64, "field")
    _check(deltas, torch.float64, "deltas")
    _check(step, torch.int32, "step")
    nsteps = deltas.shape[0]
    rc = fem_field_advance(_ptr(field), _ptr(deltas), nsteps, _ptr(step), _stream(stream))
    if rc != FEM_OK:
        raise FemError(rc, "fem_field_advance")
