"""Build libfem.so in-tree for gfx950 (hipcc cross-compiles without a GPU).

Every translation unit is compiled on its own (in parallel) into ``_build/`` and linked into
``paper_1310_1191_amd/libfem.so``. The device code is built with packed-FP32 instructions
switched off (``-Xclang -target-feature -Xclang -packed-fp32-ops``).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build", "libfem")
LIB = os.path.join(HERE, "libfem.so")
ARCH = os.environ.get("FEM_OFFLOAD_ARCH", "gfx950")

HIP_SOURCES = [
    "fem_api.cpp",
    "fem_mixed.hip",
    "fem_timestep.hip",
    "fem_jacobian.hip",
    "fem_transpose.hip",
    "fem_staged.cpp",
    "fem_k_f64.hip",
    "fem_k_f32.hip",
    "fem_k_bf16.hip",
    "fem_k_split_bf16.hip",
    "fem_k_split_f16.hip",
]
CXX_SOURCES = ["fem_tables.cpp", "fem_prism_tables.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
HIP_FLAGS = ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-ffp-contract=fast", "-Wno-unused-result"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    return r.returncode, out, cmd


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    cmds = []
    objs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        cmds.append([HIPCC, *COMMON, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
    for src in CXX_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        cmds.append(["g++", *COMMON, "-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_run, cmds))
    failed = [(rc, out, cmd) for rc, out, cmd in results if rc != 0]
    for rc, out, cmd in results:
        if verbose or rc != 0:
            if out.strip():
                print(" ".join(cmd[-3:]), "\n", out, file=sys.stderr)
    if failed:
        raise RuntimeError(f"libfem build failed in {len(failed)} translation unit(s)")
    tmp = LIB + ".tmp"
    rc, out, cmd = _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    if rc != 0:
        print(out, file=sys.stderr)
        raise RuntimeError("libfem link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
