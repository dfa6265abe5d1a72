"""Builds libvgsim.so (the HIP kernels and the C ABI) in-tree for gfx950.

    python -m paper_2406_04177_amd.build        # or: python paper_2406_04177_amd/build.py

hipcc cross-compiles without a GPU.  Flags:
  --offload-arch=gfx950            MI355X (CDNA4) code object only
  -ffp-contract=off                no fused multiply-add: every operation rounds
                                   as written, so the FP64 path reproduces a
                                   plain IEEE implementation bit for bit
  -target-feature -packed-fp32-ops no packed FP32 instructions
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvgsim.so")
SOURCES = ["vg_graph.hip", "vg_step.hip", "vg_cg.hip", "vg_adjoint.hip", "vg_reduce.hip", "vg_pngm.hip", "vg_api.cpp"]
HEADERS = ["vg_internal.h"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def build(verbose: bool = False, out: str = LIB, defines=(), extra_flags=()) -> str:
    """Compile every source to an object (in parallel), then link the library.
    ``extra_flags`` go to every compile (e.g. host-side sanitizers, each
    behind ``-Xarch_host``)."""
    objdir = os.path.join(os.path.dirname(out), "_build") if out != LIB else os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmd = ([hipcc()] + FLAGS + list(extra_flags) + ["-D%s" % d for d in defines] + inc
               + ["-c", os.path.join(CSRC, src), "-o", obj])
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
    failed = [src for src, p in procs if p.wait() != 0]
    if failed:
        raise RuntimeError("hipcc failed for %s" % ", ".join(failed))
    tmp = out + ".tmp%d" % os.getpid()
    link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
