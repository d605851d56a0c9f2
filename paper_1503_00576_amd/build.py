"""Builds libtc.so (the HIP kernels and the C ABI) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtc.so")
SOURCES = ["sort.hip", "prep.hip", "count.hip", "hub.hip", "api.hip", "batched.hip", "pack.hip",
           "split.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed-FP32 instructions stay off in every device build of this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-command-line-argument",
]


# the yardstick kernels for the ablation of the paper's own design (not the counting path)
ABLATION_SOURCES = ["ablation.hip"]
ABLATION_LIB = os.path.join(HERE, "libtc_ablation.so")


def build(verbose: bool = False, extra: tuple[str, ...] = ()) -> str:
    _compile([os.path.join(CSRC, s) for s in ABLATION_SOURCES], ABLATION_LIB, verbose, extra)
    return _compile([os.path.join(CSRC, s) for s in SOURCES], LIB, verbose, extra)


def _compile(srcs, lib, verbose, extra) -> str:
    tmp = lib + ".tmp"
    cmd = [HIPCC, *FLAGS, *extra, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stderr=subprocess.PIPE, text=True)
    # the host pass does not know the device-only feature flag; that warning is noise
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    if err.strip():
        print(err, file=sys.stderr)
    if r.returncode != 0:
        raise subprocess.CalledProcessError(r.returncode, cmd)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose=True, extra=tuple(sys.argv[1:]))
