"""Build the HIP library (gfx950) in-tree: paper_2401_11324_amd/_bang.so."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "_bang.so")
SOURCES = [os.path.join(CSRC, f)
           for f in ("bang_kernels.hip", "bang_api.cpp", "bang_server.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=off: no fused multiply-add (fixed FP32 rounding sequence).
# -packed-fp32-ops off: no packed FP32 VALU instructions are generated.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-Wall", "-Wno-unused-function",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False, extra: list | None = None) -> str:
    cmd = [HIPCC, *FLAGS, *(extra or []), *SOURCES, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
