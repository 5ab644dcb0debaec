"""Build the HIP library (libfwapsp.so) for gfx950 in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfwapsp.so")

SOURCES = ["fw_kernels.hip", "fw_ooc_kernels.hip", "fw_batched.hip", "fw_backward.hip", "fw_validate.hip", "fw_runtime.cpp", "fw_ooc.cpp"]

# Packed FP32 instructions are kept out of the generated code (the feature is
# disabled, not merely avoided): two scalar adds plus one 3-way min per pair of
# updates is the schedule the kernels are written for.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall", "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(out: str = LIB, extra: list[str] | None = None, verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = out + ".tmp"
    cmd = [hipcc()] + FLAGS + (extra or []) + ["-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True)
