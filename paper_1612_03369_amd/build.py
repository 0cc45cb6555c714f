"""Build the HIP library ``libpic.so`` for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpic.so")
SOURCES = ["pic_api.hip"]
DEPENDS = ["pic_api.hip", "pic_kernels.hip", "pic_adjoint.hip", "pic_common.h", "pic_internal.h",
           "pic_octree.inc", "pic_adjoint_api.inc", "pic_batch.inc"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def command(out: str = LIB, extra=()) -> list:
    return [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            # packed FP32 instructions are kept out of the generated code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # contraction only within an expression: identical rounding in every kernel
            "-ffp-contract=on", "-munsafe-fp-atomics", "-fvisibility=hidden",
            "-Wall", "-Wno-unused-value", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable",
            "-I", os.path.join(HERE, "..", "include"),
            *extra, "-o", out, *[os.path.join(CSRC, s) for s in SOURCES]]


def build_variant(out: str, defines: dict) -> str:
    """Compile a copy of the library with -D overrides of the tuning macros."""
    extra = [f"-D{k}={v}" for k, v in defines.items()]
    r = subprocess.run(command(out, extra), capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stderr[-20000:])
    return out


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile libpic.so; with force=False only when a source is newer."""
    if not force and os.path.exists(LIB):
        t = os.path.getmtime(LIB)
        if all(os.path.getmtime(os.path.join(CSRC, d)) <= t for d in DEPENDS) and \
                os.path.getmtime(os.path.join(HERE, "..", "include", "pic.h")) <= t:
            return LIB
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stderr[-20000:])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
