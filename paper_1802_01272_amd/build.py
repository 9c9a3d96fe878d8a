"""Build step of the HIP libraries: compiles the stepper (csrc/lbm_kernels.hip,
csrc/lbm_api.hip) for gfx950 into _lib/liblbm.so, and the copy probe used by
bench.py's memory-side measurement (csrc/copy_probe.hip) into
_lib/libprobe.so (in-tree, so they travel with the source tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "csrc", n) for n in ("lbm_kernels.hip", "lbm_api.hip")]
LIB = os.path.join(HERE, "_lib", "liblbm.so")
PROBE_SRC = [os.path.join(HERE, "csrc", "copy_probe.hip")]
PROBE_LIB = os.path.join(HERE, "_lib", "libprobe.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Wall", "-Wno-unused-function",
    # keep the compiler from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
    "-I" + os.path.join(HERE, "csrc"),
]


def _hipcc(sources, lib, verbose):
    os.makedirs(os.path.dirname(lib), exist_ok=True)
    cmd = [HIPCC] + FLAGS + ["-shared"] + sources + ["-o", lib + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + err)
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(lib + ".tmp", lib)
    return lib


def build(verbose: bool = False) -> str:
    _hipcc(PROBE_SRC, PROBE_LIB, verbose)
    return _hipcc(SRC, LIB, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
