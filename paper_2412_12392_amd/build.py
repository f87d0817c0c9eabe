"""Build libm3s.so (the gfx950 HIP library) in-tree with hipcc.

    python -m paper_2412_12392_amd.build

Flags: gfx950 only; -O3; floating-point contraction limited to single source
expressions (-ffp-contract=on) so that every kernel that inlines the shared
per-query code fuses it the same way; packed-FP32 instruction selection
disabled (-packed-fp32-ops).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libm3s.so")
SOURCES = ["m3s_kernels.hip", "m3s_track.hip", "m3s_backend.hip", "m3s_capi.hip"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags(arch: str = "gfx950"):
    return ["--offload-arch=%s" % arch, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=on",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC]


def build(out: str = LIB, verbose: bool = False, extra=()) -> str:
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *flags(), "-shared", *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp, *extra]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
