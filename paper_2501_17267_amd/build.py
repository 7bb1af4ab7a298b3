"""Build libsgmi.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

python -m paper_2501_17267_amd.build      # compile every source, link the library
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsgmi.so")

ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
# device code: gfx950 only; packed-fp32 instructions disabled
HIPFLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-munsafe-fp-atomics"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    if src.endswith(".hip"):
        cmd = ["hipcc", "-c", "-x", "hip", src, "-o", obj] + COMMON + HIPFLAGS
    else:
        cmd = ["hipcc", "-c", "-x", "c++", src, "-o", obj] + COMMON
    subprocess.check_call(cmd)
    return obj


def _deps(path: str, seen: set) -> set:
    """The file and the project headers it includes, transitively."""
    import re
    if path in seen or not os.path.exists(path):
        return seen
    seen.add(path)
    for name in re.findall(r'^\s*#include\s+"([^"]+)"', open(path).read(), re.M):
        for d in (CSRC, os.path.join(ROOT, "include")):
            if os.path.exists(os.path.join(d, name)):
                _deps(os.path.join(d, name), seen)
                break
    return seen


def _stale(src: str) -> bool:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    if not os.path.exists(obj):
        return True
    return os.path.getmtime(obj) < max(os.path.getmtime(f) for f in _deps(src, set()))


def build(jobs: int | None = None, incremental: bool = False) -> str:
    """Compile every source (incremental: only those older than their object
    or than the newest header) and link the library."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    if incremental:
        todo = [s for s in srcs if _stale(s)]
    else:
        todo = srcs
    jobs = jobs or min(8, len(srcs))
    with cf.ThreadPoolExecutor(jobs) as ex:
        list(ex.map(_compile, todo))
    objs = [os.path.join(OBJ, os.path.basename(s) + ".o") for s in srcs]
    tmp = LIB + ".tmp"
    subprocess.check_call(["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    inc = "--incremental" in sys.argv
    args = [a for a in sys.argv[1:] if a != "--incremental"]
    print(build(int(args[0]) if args else None, incremental=inc))
