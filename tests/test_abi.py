"""The C-ABI library: it loads, exports every function include/fem.h declares, and rejects calls
made before fem_init without touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fem.h")
LIB = os.path.join(ROOT, "paper_1310_1191_amd", "libfem.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fem_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libfem.so is not built (run `python -m paper_1310_1191_amd.build`)")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert {"fem_init", "fem_integrate", "fem_finalize", "fem_strerror"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def test_binding_wraps_every_symbol():
    from paper_1310_1191_amd import fem
    assert sorted(fem.exported_symbols()) == declared_functions()


def test_host_only_calls(lib):
    from paper_1310_1191_amd import fem
    assert fem.fem_abi_version() == 4
    assert fem.fem_strerror(0) == "success"
    assert "init" in fem.fem_strerror(fem.FEM_ENOTINIT)
    assert fem.fem_strerror(-99) == "unknown status"
    assert fem.fem_workspace_bytes(-1) == 0
    a, b = fem.fem_workspace_bytes(1000), fem.fem_workspace_bytes(100000)
    assert 0 < a < b and a % 256 == 0


def test_calls_before_init_are_rejected_on_the_host(lib):
    from paper_1310_1191_amd import fem
    c = fem.fem_coeffs()
    assert fem.fem_integrate(10, 3, None, c, None, None, None) == fem.FEM_ENOTINIT
    assert fem.fem_mixed_offsets(10, None, None, None, None, 0, None) == fem.FEM_ENOTINIT
    assert fem.fem_gather_sample(1, None, 1, None, 1, None, None, None, None, 0, None, 0, None, 0,
                                 None) == fem.FEM_ENOTINIT
    assert lib.fem_finalize() == fem.FEM_ENOTINIT


@pytest.mark.parametrize("struct", ["fem_coeffs", "fem_staged_stats"])
def test_c_struct_layout_matches_header(tmp_path, struct):
    """The binding's structs against the C compiler's layout of the header's structs."""
    import subprocess
    from paper_1310_1191_amd import fem
    cls = getattr(fem, struct)
    names = [f[0] for f in cls._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"fem.h\"\nint main(void){\n"
                   f'  printf("%zu\\n", sizeof({struct}));\n'
                   + "".join(f'  printf("%zu\\n", offsetof({struct}, {n}));\n' for n in names)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-std=c11", f"-I{inc}", str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got[0] == ctypes.sizeof(cls)
    assert got[1:] == [getattr(cls, n).offset for n in names]


@pytest.mark.parametrize("p", range(1, 8))
def test_library_reference_tables_vs_numpy(p):
    """The library's own quadrature and Lagrange tables (independent of the oracle's code)
    against numpy's Gauss-Legendre rule and polynomial algebra."""
    import numpy as np
    from numpy.polynomial import legendre as npleg

    from paper_1310_1191_amd import fem
    from polyexact import gll_nodes_numpy, lagrange_polys
    gx, gw, lx, L, D = fem.fem_reference_tables(p)
    xr, wr = npleg.leggauss(p + 1)
    np.testing.assert_allclose(gx, xr, atol=2e-15)
    np.testing.assert_allclose(gw, wr, rtol=2e-14)
    np.testing.assert_allclose(lx, gll_nodes_numpy(p), atol=5e-15)
    polys = lagrange_polys(gll_nodes_numpy(p))
    for q in range(p + 1):
        np.testing.assert_allclose(L[q], [pl(gx[q]) for pl in polys], atol=1e-13)
        np.testing.assert_allclose(D[q], [pl.deriv()(gx[q]) for pl in polys], atol=1e-11)
    assert np.isfinite(D).all()


def test_reference_tables_reject_bad_degree():
    from paper_1310_1191_amd import fem
    with pytest.raises(fem.FemError):
        fem.fem_reference_tables(8)


def test_variant_table_host_calls(lib):
    """Variant counts and choices are host state: they need neither fem_init nor a GPU. Each
    (degree, precision, coefficient mode) has its own choice."""
    from paper_1310_1191_amd import fem
    for p in range(1, 8):
        for prec in range(5):
            n = fem.fem_variant_count(p, prec)
            assert 1 <= n <= fem.MAX_VARIANTS
            v0 = {m: fem.fem_get_variant(p, prec, m) for m in fem.MODES}
            assert all(0 <= v < n for v in v0.values())
            # p = 1: the last variant is the vector-ALU kernel, ELEMENT mode only (its default)
            last = n - 2 if p == 1 else n - 1
            fem.fem_set_variant(p, prec, fem.FIELD, last)
            assert fem.fem_get_variant(p, prec, fem.FIELD) == last
            assert fem.fem_get_variant(p, prec, fem.ELEMENT) == v0[fem.ELEMENT]
            assert fem.fem_get_variant(p, prec, fem.ELASTIC) == v0[fem.ELASTIC]
            fem.fem_set_variant(p, prec, fem.FIELD, v0[fem.FIELD])
            assert lib.fem_set_variant(p, prec, fem.ELEMENT, n) == fem.FEM_ECONFIG
            if p == 1:
                tri = fem.trilinear_variant(prec)
                assert tri == n - 1 and v0[fem.ELEMENT] == tri
                assert v0[fem.FIELD] != tri and v0[fem.ELASTIC] != tri
                assert lib.fem_set_variant(1, prec, fem.FIELD, tri) == fem.FEM_ECONFIG
                assert lib.fem_set_variant(1, prec, fem.ELASTIC, tri) == fem.FEM_ECONFIG
    for p in range(1, 8):  # prisms: keys FEM_PRISM(p) = 10 + p
        for prec in range(5):
            n = fem.fem_variant_count(fem.prism(p), prec)
            assert 1 <= n <= fem.MAX_VARIANTS
            assert 0 <= fem.fem_get_variant(fem.prism(p), prec, fem.ELEMENT) < n
    assert lib.fem_variant_count(8, 0) == fem.FEM_EDEGREE
    assert lib.fem_variant_count(10, 0) == fem.FEM_EDEGREE
    assert lib.fem_variant_count(18, 0) == fem.FEM_EDEGREE
    for prec in range(5):  # p = 0: the mixed-degree strategies
        assert fem.fem_variant_count(0, prec) == 2
        for m in fem.MODES:
            assert fem.fem_get_variant(0, prec, m) in (0, 1)
    for p in range(1, 8):  # keys FEM_MIXED(p) = 20 + p: degree p's tile inside the single launch
        for prec in range(5):
            n = fem.fem_variant_count(fem.mixed(p), prec)
            assert n == (1 if (p == 1 and prec == fem.PRECISIONS["fp64"]) else 2)
            for m in fem.MODES:
                assert fem.fem_get_variant(fem.mixed(p), prec, m) == 0
            tiles = []
            for t in range(n):
                fem.fem_set_variant(fem.mixed(p), prec, fem.FIELD, t)
                v = fem.fem_mixed_variant(p, prec, fem.FIELD)
                assert 0 <= v < fem.fem_variant_count(p, prec)
                assert p != 1 or v != fem.trilinear_variant(prec)  # a tile, not the vector kernel
                tiles.append(v)
            assert len(set(tiles)) == n  # the alternatives are distinct tiles
            assert fem.fem_mixed_variant(p, prec, fem.ELEMENT) == tiles[0]  # per mode
            fem.fem_set_variant(fem.mixed(p), prec, fem.FIELD, 0)
            assert lib.fem_set_variant(fem.mixed(p), prec, fem.FIELD, n) == fem.FEM_ECONFIG
    assert lib.fem_variant_count(20, 0) == fem.FEM_EDEGREE
    assert lib.fem_variant_count(28, 0) == fem.FEM_EDEGREE
    assert lib.fem_mixed_variant(0, 0, 0) == fem.FEM_EDEGREE
    assert lib.fem_mixed_variant(8, 0, 0) == fem.FEM_EDEGREE
    assert lib.fem_mixed_variant(3, 0, 3) == fem.FEM_EINVAL
    assert lib.fem_variant_count(-1, 0) == fem.FEM_EDEGREE
    assert lib.fem_variant_count(3, 5) == fem.FEM_EINVAL
    assert lib.fem_set_variant(8, 0, 0, 0) == fem.FEM_EDEGREE
    assert lib.fem_set_variant(3, 0, 3, 0) == fem.FEM_EINVAL
    assert lib.fem_get_variant(3, 0, -1) == fem.FEM_EINVAL
    assert lib.fem_autotune(3, 0, 0, 100, None, None, None) == fem.FEM_ENOTINIT
    assert lib.fem_load_tuning(b"/nonexistent.json", None) == fem.FEM_ENOTINIT


def test_variant_numbering_is_contiguous():
    """Variants of each (degree, family) are numbered 0..n-1 with no gap, so every index below
    fem_variant_count names a compiled kernel."""
    src = open(os.path.join(ROOT, "paper_1310_1191_amd", "csrc", "fem_launch.h")).read()
    seen = {}
    for p, fam, v in re.findall(r"VariantCfg<(\d+), (MF_\w+), (\d)>", src):
        seen.setdefault((p, fam), []).append(int(v))
    assert seen
    for key, vs in seen.items():
        assert sorted(vs) == list(range(len(vs))), key


def test_every_declaration_cites_the_paper():
    """Each function declared in include/fem.h is preceded by a comment block that names the
    passage of the paper it implements (a section, an algorithm, an equation or a table)."""
    src = open(os.path.join(ROOT, "include", "fem.h")).read()
    decls = list(re.finditer(r"^(?:int|size_t|const char \*)\s*(fem_\w+)\(", src, flags=re.M))
    assert len(decls) >= 17
    cite = re.compile(r"section \d|Algorithm \d|eq\. \(|Table \d", re.I)
    prev_end = 0
    for m in decls:
        # the comments between the previous declaration and this one
        comments = " ".join(re.findall(r"/\*.*?\*/", src[prev_end:m.start()], flags=re.S))
        assert comments, f"{m.group(1)} has no comment block"
        if m.group(1) == "fem_integrate_noalloc":
            # not a step of the method: its comment names the callers it exists for
            assert "cannot allocate" in comments, "fem_integrate_noalloc: callers not named"
        else:
            assert cite.search(comments), f"{m.group(1)}: its comment cites no passage"
        prev_end = m.end()


class _FakeDeviceTensor:
    """Stands in for a device tensor on a machine without a GPU: the binding's checks read only
    these attributes."""

    def __init__(self, shape, dtype, contiguous=True):
        self.shape, self.dtype, self._contiguous = tuple(shape), dtype, contiguous
        self.is_cuda = True

    def is_contiguous(self):
        return self._contiguous

    def numel(self):
        n = 1
        for s in self.shape:
            n *= s
        return n


def test_binding_rejects_mis_sized_buffers():
    """The binding refuses outputs and inputs whose type, contiguity, shape or size differ from
    what the kernels index, before anything is launched (ValueError, no library call)."""
    import torch
    from paper_1310_1191_amd import fem
    T = _FakeDeviceTensor
    nel, ns = 10, 27
    ok_elem, ok_geom = T((nel, 14), torch.float64), T((nel, 8, 3), torch.float64)
    fem._check_inputs(torch, ok_geom, ok_elem, fem.ELEMENT, nel, None, None, None, None)
    bad = [
        dict(geom=T((nel, 8, 2), torch.float64)),                 # wrong geometry shape
        dict(elem=T((nel, 10), torch.float64)),                   # FIELD-width record in ELEMENT mode
        dict(elem=T((nel, 14), torch.float32)),                   # wrong dtype
        dict(elem=T((nel, 14), torch.float64, contiguous=False)),
        dict(status=T((1,), torch.int32)),                        # status needs 2 counters
        dict(status=T((2,), torch.int64)),
        dict(jac=T((nel * ns - 1, 10), torch.float64), rows=nel * ns),
    ]
    for b in bad:
        args = dict(geom=ok_geom, elem=ok_elem, status=None, jac=None, rows=None)
        args.update(b)
        with pytest.raises(ValueError):
            fem._check_inputs(torch, args["geom"], args["elem"], fem.ELEMENT, nel, None,
                              args["status"], args["jac"], args["rows"])
    with pytest.raises(ValueError):  # FIELD mode without its descriptor
        fem._check_inputs(torch, ok_geom, T((nel, 10), torch.float64), fem.FIELD, nel, None, None, None, None)
    # outputs: the element matrices of every element must fit
    fem._check(T((nel, ns, ns), torch.float32), torch.float32, "out_A", min_numel=nel * ns * ns)
    for t in (T((nel, ns, ns - 1), torch.float32), T((nel, ns, ns), torch.float64)):
        with pytest.raises(ValueError):
            fem._check(t, torch.float32, "out_A", min_numel=nel * ns * ns)
    with pytest.raises(ValueError):  # a host tensor is not a device buffer
        fem._check(torch.zeros(3), torch.float32, "out_b")
