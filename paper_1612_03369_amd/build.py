"""Build the HIP library ``libpic.so`` for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpic.so")
# translation units, compiled in parallel: the API with the non-advect
# kernels, and the advect kernel instances split by dimension and kind
SOURCES = ["pic_api.hip", "pic_adv_blk3f.hip", "pic_adv_blk3d.hip", "pic_adv_blk2.hip", "pic_adv_gen2.hip",
           "pic_adv_gen3.hip"]
DEPENDS = SOURCES + ["pic_kernels.hip", "pic_adjoint.hip", "pic_advect.h", "pic_common.h", "pic_internal.h",
                     "pic_octree.inc", "pic_adjoint_api.inc", "pic_batch.inc"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # packed FP32 instructions are kept out of the generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # contraction only within an expression: identical rounding in every kernel
         "-ffp-contract=on", "-munsafe-fp-atomics", "-fvisibility=hidden",
         "-Wall", "-Wno-unused-value", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable"]


def compile_commands(out: str, extra=()) -> list:
    """One hipcc -c per translation unit, then the link of the shared library."""
    objdir = os.path.join(HERE, "_build", os.path.basename(out).replace(".", "_"))
    objs = [os.path.join(objdir, s.replace(".hip", ".o")) for s in SOURCES]
    cc = [[hipcc(), *FLAGS, "-I", os.path.join(HERE, "..", "include"), *extra, "-c", "-o", o, os.path.join(CSRC, s)]
          for s, o in zip(SOURCES, objs)]
    link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out, *objs]
    return objdir, cc, link


def _run_all(out: str, extra=(), verbose=False) -> str:
    objdir, cc, link = compile_commands(out, extra)
    os.makedirs(objdir, exist_ok=True)
    jobs = max(1, min(len(cc), os.cpu_count() or 1))
    running, errors = [], []
    pending = list(cc)
    while pending or running:
        while pending and len(running) < jobs:
            cmd = pending.pop(0)
            if verbose:
                print(" ".join(cmd), file=sys.stderr)
            running.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
        cmd, proc = running.pop(0)
        _, err = proc.communicate()
        if proc.returncode != 0:
            errors.append(f"{cmd[-1]}:\n{err[-20000:]}")
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
    if verbose:
        print(" ".join(link), file=sys.stderr)
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + r.stderr[-20000:])
    return out


def build_variant(out: str, defines: dict) -> str:
    """Compile a copy of the library with -D overrides of the tuning macros."""
    return _run_all(out, [f"-D{k}={v}" for k, v in defines.items()])


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile libpic.so; with force=False only when a source is newer."""
    if not force and os.path.exists(LIB):
        t = os.path.getmtime(LIB)
        if all(os.path.getmtime(os.path.join(CSRC, d)) <= t for d in DEPENDS) and \
                os.path.getmtime(os.path.join(HERE, "..", "include", "pic.h")) <= t:
            return LIB
    tmp = LIB + ".tmp"
    _run_all(tmp, verbose=verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
