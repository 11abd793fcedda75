"""Builds libnbody.so (HIP, gfx950) in the package directory with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnbody.so")
SOURCES = ["capi.hip", "pairs.hip", "kick.hip", "kepler.hip", "adjoint.hip", "batched.hip", "groups.hip", "ce.hip", "levels.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # binary64 results must not depend on the compiler fusing multiplies and adds
    "-ffp-contract=off",
    # no packed binary32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def command():
    return ["hipcc"] + FLAGS + ["-o", LIB] + [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose: bool = False) -> str:
    cmd = command()
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libnbody.so")
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
