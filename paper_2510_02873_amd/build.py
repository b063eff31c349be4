"""Build the HIP library libpino_collapse.so for gfx950 in-tree, and the
ceiling probes of the benchmark, libpino_probes.so."""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpino_collapse.so")
PROBES = os.path.join(HERE, "libpino_probes.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions in the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # FP32 divide and square root as the hardware approximations (FP32 only
    # feeds starting guesses and the mixed-precision path, polished in FP64)
    "-fno-hip-fp32-correctly-rounded-divide-sqrt",
    # multiply-adds fused only within one source expression, so every kernel
    # that inlines the same device function computes the same bits
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-function",
]


# hipFFT for the Hessian stage (pino_field.h)
LINK = ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lhipfft"]


def _compile(src, out, link, verbose):
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, src, "-o", tmp, *link]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    _compile(os.path.join(CSRC, "pino_collapse.hip"), LIB, LINK, verbose)
    _compile(os.path.join(CSRC, "probes.hip"), PROBES, [], verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
