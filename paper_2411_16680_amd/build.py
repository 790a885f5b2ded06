"""Build libquark.so in-tree with hipcc for gfx950.

Run as ``python -m paper_2411_16680_amd.build``.  The library is written next
to this file so it travels with the source tree."""

from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libquark.so")
SOURCES = ["k_update_fuse.hip", "k_backward.hip", "k_init.hip", "k_fp8.hip", "k_render.hip",
           "k_views.hip", "k_conv.hip",
           "k_collapse.hip", "k_ray.hip", "k_resample.hip", "capi.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-fvisibility=hidden", "-fvisibility-inlines-hidden",
    # keep the compiler from forming packed float32 vector ops
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, *srcs, "-o", tmp]
    t0 = time.time()
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{out}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s")
        if out.strip():
            print(out)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
