"""Build libsph.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2507_21684_amd.build

Every build compiles from source.  Packed FP32 instructions are disabled for the device
code (-target-feature -packed-fp32-ops); the host pass warns that it does not know the
feature, which is harmless.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "csrc", "sph_api.hip")]
DEPS = [os.path.join(HERE, "csrc", "sph_device.hpp"), os.path.join(ROOT, "include", "sph.h")]
LIB = os.path.join(HERE, "libsph.so")
ARCH = os.environ.get("SPH_OFFLOAD_ARCH", "gfx950")

FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-command-line-argument", "-Wno-unknown-warning-option",
         "-I" + os.path.join(ROOT, "include")]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc"] + FLAGS + SRC + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libsph.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
