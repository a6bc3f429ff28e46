"""Build libcosm.so in-tree with hipcc for gfx950.

The host sources (*.cpp) and the kernels (*.hip) are compiled separately and
linked into one shared library next to this file.  Packed-FP32 instructions
are disabled for every device compilation.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libcosm.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("COSM_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def _jobs() -> int:
    try:
        cap = int(os.environ.get("MAX_JOBS", "0"))
    except ValueError:
        cap = 0
    n = os.cpu_count() or 1
    return max(1, min(8, n, cap if cap > 0 else n))


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cmds, objs = [], []
    for name in sorted(os.listdir(CSRC)):
        src = os.path.join(CSRC, name)
        obj = os.path.join(BUILD, name + ".o")
        if name.endswith(".hip"):
            cmds.append(["hipcc", "-c", *COMMON, *DEVICE, "-x", "hip", src, "-o", obj])
        elif name.endswith(".cpp"):
            # host-only code: plain g++ against the HIP runtime headers
            cmds.append(["g++", "-c", *COMMON, "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
                         src, "-o", obj])
        else:
            continue
        objs.append(obj)
    # the translation units are independent: compile them side by side
    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        for f in [ex.submit(_run, c) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    _run(["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp,
          "-Wl,-rpath,/opt/rocm/lib"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
