"""Compile the gfx950 HIP library (libvf.so) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "csrc", f) for f in ("vf_device.hip", "vf_api.cpp")]
LIB = os.path.join(HERE, "libvf.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
]


# The same library with the build kernel's stage clocks (vf_stage_clocks),
# for profiling only.
LIB_STAGES = os.path.join(HERE, "libvf_stages.so")


def build(verbose: bool = False, stage_clocks: bool = False) -> str:
    out = LIB_STAGES if stage_clocks else LIB
    tmp = out + ".tmp%d" % os.getpid()
    extra = ["-DVF_STAGE_CLOCKS"] if stage_clocks else []
    cmd = [HIPCC, *FLAGS, *extra, "-x", "hip", SRC[0], "-x", "hip", SRC[1], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, stage_clocks="--stage-clocks" in sys.argv)
