"""Builds liblbm.so for gfx950 in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc")

# packed FP32 instructions are disabled for every HIP translation unit
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument"]

LIBRARIES = {
    "liblbm.so": ["lbm.hip"],
    "libsur.so": ["sur.hip"],
    "libprobe.so": ["probe.hip"],
}


def build_library(name: str = "liblbm.so", verbose: bool = False) -> str:
    out = os.path.join(HERE, name)
    tmp = out + ".tmp"
    srcs = [os.path.join(SRC, s) for s in LIBRARIES[name]]
    cmd = ["hipcc", *HIPFLAGS, "-I", os.path.join(ROOT, "include"), "-I", SRC, "-o", tmp, *srcs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {name}:\n{res.stdout}\n{res.stderr}")
    if verbose:
        print(res.stderr)
    os.replace(tmp, out)
    return out


def build_all(verbose: bool = False):
    return [build_library(n, verbose) for n in LIBRARIES]


if __name__ == "__main__":
    for p in build_all(verbose=False):
        print("built", p)
