"""FP64 CPU oracle for element integration (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package. It wraps ``fem_oracle.c`` (plain C, OpenMP over elements), which follows
Algorithm 2 of the paper (section 2) with the element entry of eq. (sum_int) (section 5.1),
specialised to a scalar convection-diffusion-reaction form, and the paper's vector model problem
(linear elastostatics, section 5.1). It shares no code with the HIP
library; the two meet only in the seeded input generators.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "fem_oracle.c"), os.path.join(_HERE, "fem_oracle_prism.c")]
_LIB_PATH = os.path.join(_HERE, "libfem_oracle.so")
_lib = None

ELEMENT = 0
FIELD = 1
ELASTIC = 2
FLAG_DETJ = 1
FLAG_NONFINITE = 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O3 -march=native, OpenMP) for the host it runs on; the
    library is built on each machine and never copied between them. ISO C11 keeps floating-point
    contraction off, and nothing reassociates sums, so the results do not depend on the flags.
    Returns the library path."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O3", "-march=native", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC",
               "-shared", "-Wall", "-Wextra", "-o", tmp, *_SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_gauss_legendre.argtypes = [ctypes.c_int, dp, dp]
    lib.oracle_gll_nodes.argtypes = [ctypes.c_int, dp]
    lib.oracle_lagrange.argtypes = [ctypes.c_int, dp, ctypes.c_double, dp, dp]
    lib.oracle_lagrange.restype = None
    lib.oracle_field_eval.argtypes = [dp, dp, dp]
    lib.oracle_field_eval.restype = None
    lib.oracle_integrate.argtypes = [
        ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    lib.oracle_integrate_elastic.argtypes = [
        ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    lib.oracle_jacobian_terms.argtypes = [
        ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_int]
    lib.oracle_integrate_nojac.argtypes = [
        ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    lib.oracle_integrate_elastic_nojac.argtypes = [
        ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    lib.oracle_max_threads.restype = ctypes.c_int
    lib.oracle_prism_ns.argtypes = [ctypes.c_int]
    lib.oracle_prism_shape.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, dp]
    lib.oracle_integrate_prism.argtypes = [
        ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_int]
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vp(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def gauss_legendre(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    if _load().oracle_gauss_legendre(n, _dptr(x), _dptr(w)) != 0:
        raise ValueError("bad n")
    return x, w


def gll_nodes(p: int):
    x = np.zeros(p + 1)
    if _load().oracle_gll_nodes(p, _dptr(x)) != 0:
        raise ValueError("bad p")
    return x


def lagrange(nodes, x: float):
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    n = nodes.size
    val = np.zeros(n)
    der = np.zeros(n)
    _load().oracle_lagrange(n, _dptr(nodes), float(x), _dptr(val), _dptr(der))
    return val, der


def field_eval(field, x):
    field = np.ascontiguousarray(field, dtype=np.float64).reshape(-1)
    assert field.size == 175
    x = np.ascontiguousarray(x, dtype=np.float64)
    g = np.zeros(7)
    _load().oracle_field_eval(_dptr(field), _dptr(x), _dptr(g))
    return g


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def mixed_offsets(degree):
    """Exclusive scans of Ns^2 and Ns over a per-element degree array."""
    ns = (np.asarray(degree, dtype=np.int64) + 1) ** 3
    a_off = np.zeros(ns.size + 1, dtype=np.int64)
    b_off = np.zeros(ns.size + 1, dtype=np.int64)
    np.cumsum(ns * ns, out=a_off[1:])
    np.cumsum(ns, out=b_off[1:])
    return a_off, b_off


def integrate(geom, coef, p: int | None = None, degree=None, mode: int = ELEMENT, field=None,
              threads: int = 0, with_b: bool = True):
    """Integrate elements in FP64.

    Uniform degree: returns (A [nel, Ns, Ns], b [nel, Ns], flags [nel]).
    Mixed degree (``degree`` given): returns (A packed, b packed, flags, a_off, b_off).
    """
    geom = np.ascontiguousarray(geom, dtype=np.float64)
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    nel = geom.shape[0]
    assert geom.shape[1:] == (8, 3)
    rec = 14 if mode == ELEMENT else 10
    assert coef.shape == (nel, rec)
    fld = None
    if mode == FIELD:
        fld = np.ascontiguousarray(field, dtype=np.float64).reshape(-1)
        assert fld.size == 175
    flags = np.zeros(nel, dtype=np.int32)
    lib = _load()
    if degree is None:
        if p is None:
            raise ValueError("p or degree is required")
        ns = (p + 1) ** 3 if 1 <= p <= 7 else 1   # the C side rejects other p
        A = np.zeros((nel, ns, ns))
        b = np.zeros((nel, ns)) if with_b else None
        rc = lib.oracle_integrate(nel, p, None, _vp(geom), mode, _vp(coef), _vp(fld), None, None,
                                  _vp(A), _vp(b), _vp(flags), threads)
        if rc != 0:
            raise ValueError("oracle_integrate: bad arguments")
        return A, b, flags
    deg = np.ascontiguousarray(degree, dtype=np.int8)
    a_off, b_off = mixed_offsets(deg)
    A = np.zeros(int(a_off[-1]))
    b = np.zeros(int(b_off[-1])) if with_b else None
    rc = lib.oracle_integrate(nel, 0, _vp(deg), _vp(geom), mode, _vp(coef), _vp(fld), _vp(a_off),
                              _vp(b_off), _vp(A), _vp(b), _vp(flags), threads)
    if rc != 0:
        raise ValueError("oracle_integrate: bad arguments")
    return A, b, flags, a_off, b_off


def integrate_elastic(geom, coef, p: int, threads: int = 0, with_b: bool = True):
    """Linear elastostatics (section 5.1) in FP64: coef [nel, 5] = (E, nu, f1, f2, f3).
    Returns (A [nel, 3, 3, Ns, Ns], b [nel, 3, Ns] or None, flags [nel]); block A[e, i, k]
    couples test component i with trial component k."""
    geom = np.ascontiguousarray(geom, dtype=np.float64)
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    nel = geom.shape[0]
    assert geom.shape[1:] == (8, 3) and coef.shape == (nel, 5)
    ns = (p + 1) ** 3 if 1 <= p <= 7 else 1
    A = np.zeros((nel, 3, 3, ns, ns))
    b = np.zeros((nel, 3, ns)) if with_b else None
    flags = np.zeros(nel, dtype=np.int32)
    rc = _load().oracle_integrate_elastic(nel, p, _vp(geom), _vp(coef), _vp(A), _vp(b), _vp(flags),
                                         threads)
    if rc != 0:
        raise ValueError("oracle_integrate_elastic: bad arguments")
    return A, b, flags


def jacobian_terms(geom, p: int | None = None, degree=None, threads: int = 0):
    """Per-point Jacobian terms of the NOJAC variant (section 4): [.., 10] = detJ, then J^{-1}
    row-major, for q = q1 + n q2 + n^2 q3. Uniform p: shape [nel, Ns, 10]; mixed degree: the
    records packed by the b_off scan, shape [sum Ns, 10]."""
    geom = np.ascontiguousarray(geom, dtype=np.float64)
    nel = geom.shape[0]
    assert geom.shape[1:] == (8, 3)
    lib = _load()
    if degree is None:
        ns = (p + 1) ** 3 if p is not None and 1 <= p <= 7 else 1
        out = np.zeros((nel, ns, 10))
        rc = lib.oracle_jacobian_terms(nel, -1 if p is None else p, None, None, _vp(geom), _vp(out),
                                       threads)
    else:
        deg = np.ascontiguousarray(degree, dtype=np.int8)
        _, b_off = mixed_offsets(deg)
        out = np.zeros((int(b_off[-1]), 10))
        rc = lib.oracle_jacobian_terms(nel, 0, _vp(deg), _vp(b_off), _vp(geom), _vp(out), threads)
    if rc != 0:
        raise ValueError("oracle_jacobian_terms: bad arguments")
    return out


def integrate_nojac(jac, coef, p: int | None = None, degree=None, mode: int = ELEMENT,
                    geom=None, field=None, threads: int = 0, with_b: bool = True):
    """``integrate`` with the Jacobian terms read from ``jac`` (layout of ``jacobian_terms``)
    instead of computed from vertices; ``geom`` is needed only in FIELD mode (for x_q)."""
    jac = np.ascontiguousarray(jac, dtype=np.float64)
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    nel = coef.shape[0]
    rec = 14 if mode == ELEMENT else 10
    assert coef.shape == (nel, rec) and jac.shape[-1] == 10
    if geom is not None:
        geom = np.ascontiguousarray(geom, dtype=np.float64)
        assert geom.shape == (nel, 8, 3)
    fld = None
    if mode == FIELD:
        fld = np.ascontiguousarray(field, dtype=np.float64).reshape(-1)
        assert fld.size == 175
    flags = np.zeros(nel, dtype=np.int32)
    lib = _load()
    if degree is None:
        ns = (p + 1) ** 3 if p is not None and 1 <= p <= 7 else 1
        assert jac.size == nel * ns * 10
        A = np.zeros((nel, ns, ns))
        b = np.zeros((nel, ns)) if with_b else None
        rc = lib.oracle_integrate_nojac(nel, -1 if p is None else p, None, _vp(jac), _vp(geom), mode,
                                        _vp(coef), _vp(fld), None, None, _vp(A), _vp(b), _vp(flags),
                                        threads)
        if rc != 0:
            raise ValueError("oracle_integrate_nojac: bad arguments")
        return A, b, flags
    deg = np.ascontiguousarray(degree, dtype=np.int8)
    a_off, b_off = mixed_offsets(deg)
    assert jac.size == int(b_off[-1]) * 10
    A = np.zeros(int(a_off[-1]))
    b = np.zeros(int(b_off[-1])) if with_b else None
    rc = lib.oracle_integrate_nojac(nel, 0, _vp(deg), _vp(jac), _vp(geom), mode, _vp(coef), _vp(fld),
                                    _vp(a_off), _vp(b_off), _vp(A), _vp(b), _vp(flags), threads)
    if rc != 0:
        raise ValueError("oracle_integrate_nojac: bad arguments")
    return A, b, flags, a_off, b_off


def integrate_elastic_nojac(jac, coef, p: int, threads: int = 0, with_b: bool = True):
    """``integrate_elastic`` with the Jacobian terms read from ``jac`` [nel, Ns, 10]."""
    jac = np.ascontiguousarray(jac, dtype=np.float64)
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    nel = coef.shape[0]
    ns = (p + 1) ** 3 if 1 <= p <= 7 else 1
    assert coef.shape == (nel, 5) and jac.size == nel * ns * 10
    A = np.zeros((nel, 3, 3, ns, ns))
    b = np.zeros((nel, 3, ns)) if with_b else None
    flags = np.zeros(nel, dtype=np.int32)
    rc = _load().oracle_integrate_elastic_nojac(nel, p, _vp(jac), _vp(coef), _vp(A), _vp(b),
                                               _vp(flags), threads)
    if rc != 0:
        raise ValueError("oracle_integrate_elastic_nojac: bad arguments")
    return A, b, flags


# ---- prismatic elements (the reference element of section 2, Tables 1-2) ----
def prism_ns(p: int) -> int:
    return (p + 1) * (p + 1) * (p + 2) // 2


def prism_shape(p: int, xi1: float, xi2: float, zeta: float):
    """[Ns, 4]: value and reference derivatives of every prism shape function at one point."""
    out = np.zeros((prism_ns(p), 4))
    if _load().oracle_prism_shape(int(p), float(xi1), float(xi2), float(zeta), _dptr(out)) != 0:
        raise ValueError("bad p")
    return out


def integrate_prism(geom, coef, p: int, mode: int = ELEMENT, field=None, threads: int = 0,
                    with_b: bool = True, tri=None):
    """Integrate prisms in FP64 (geom [nel, 6, 3]). ELEMENT / FIELD: (A [nel, Ns, Ns],
    b [nel, Ns], flags); ELASTIC (coef [nel, 5]): (A [nel, 3, 3, Ns, Ns], b [nel, 3, Ns], flags).
    The triangle rule is the oracle's own (prism_rule.triangle_rule) unless ``tri`` is given."""
    from . import prism_rule
    geom = np.ascontiguousarray(geom, dtype=np.float64)
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    nel = geom.shape[0]
    assert geom.shape[1:] == (6, 3)
    rec = {ELEMENT: 14, FIELD: 10, ELASTIC: 5}[mode]
    assert coef.shape == (nel, rec)
    if tri is None:
        pts, w = prism_rule.triangle_rule(p)
        tri = np.column_stack([pts, w])
    tri = np.ascontiguousarray(tri, dtype=np.float64)
    fld = None
    if mode == FIELD:
        fld = np.ascontiguousarray(field, dtype=np.float64).reshape(-1)
        assert fld.size == 175
    ns = prism_ns(p) if 1 <= p <= 7 else 1
    blk, comp = (9, 3) if mode == ELASTIC else (1, 1)
    A = np.zeros((nel, 3, 3, ns, ns) if mode == ELASTIC else (nel, ns, ns))
    b = (np.zeros((nel, 3, ns) if mode == ELASTIC else (nel, ns))) if with_b else None
    flags = np.zeros(nel, dtype=np.int32)
    rc = _load().oracle_integrate_prism(nel, p, _vp(geom), mode, _vp(coef), _vp(fld),
                                        tri.shape[0], _vp(tri), _vp(A), _vp(b), _vp(flags), threads)
    if rc != 0:
        raise ValueError("oracle_integrate_prism: bad arguments")
    return A, b, flags
