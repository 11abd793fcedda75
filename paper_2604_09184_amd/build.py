"""Builds libnbody.so (HIP, gfx950) in the package directory with hipcc: every source compiled to an
object in parallel (build/ next to this file), then one shared-library link."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "build")
LIB = os.path.join(HERE, "libnbody.so")
SOURCES = ["capi.hip", "pairs.hip", "kick.hip", "kepler.hip", "adjoint.hip", "batched.hip", "groups.hip", "ce.hip", "levels.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # binary64 results must not depend on the compiler fusing multiplies and adds
    "-ffp-contract=off",
    # no packed binary32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def compile_command(src):
    return ["hipcc"] + FLAGS + ["-c", "-o", os.path.join(OBJ, src + ".o"), os.path.join(CSRC, src)]


def link_command():
    return ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB] + \
        [os.path.join(OBJ, s + ".o") for s in SOURCES]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    return subprocess.run(cmd, capture_output=True, text=True)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, min(os.cpu_count() or 1, 16)))
    with concurrent.futures.ThreadPoolExecutor(jobs) as pool:
        results = list(pool.map(lambda s: _run(compile_command(s), verbose), SOURCES))
    for src, r in zip(SOURCES, results):
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"hipcc failed compiling {src}")
    r = _run(link_command(), verbose)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed linking libnbody.so")
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
