"""Build the HIP library (gfx950) in-tree: paper_2401_11324_amd/_bang.so.

Each translation unit compiles to an object of its own, in parallel (the
search kernel is compiled once per variant from search_variants.hip), then
the objects are linked into the shared library.
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "_bang.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# (source, extra defines): the search variants are host-resident adjacency
# (bit 0) | visited filter << 1 (none, Bloom, seen bitmap) | timed << 3 (the
# timed copies of the device-resident forms without the Bloom filter)
VARIANTS = (0, 1, 2, 3, 4, 5, 8, 12)
UNITS = ([("bang_kernels.hip", []), ("bang_api.cpp", []),
          ("bang_server.cpp", [])] +
         [("search_variants.hip", [f"-DBANG_VARIANT={v}"]) for v in VARIANTS])
SOURCES = sorted({os.path.join(CSRC, f) for f, _ in UNITS} |
                 {os.path.join(CSRC, f) for f in
                  ("search_kernel.h", "internal.h", "api_internal.h")})

# -ffp-contract=off: no fused multiply-add (fixed FP32 rounding sequence).
# -packed-fp32-ops off: no packed FP32 VALU instructions are generated.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-Wall", "-Wno-unused-function",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False, extra: list | None = None,
          jobs: int = 0) -> str:
    jobs = jobs or min(len(UNITS), os.cpu_count() or 1)
    with tempfile.TemporaryDirectory(prefix="bang_build_") as tmp:
        cmds = []
        for i, (src, defs) in enumerate(UNITS):
            obj = os.path.join(tmp, f"{i}_{os.path.splitext(src)[0]}.o")
            cmds.append((obj, [HIPCC, *FLAGS, *(extra or []), *defs, "-c",
                               os.path.join(CSRC, src), "-o", obj]))
        with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
            futs = []
            for _, cmd in cmds:
                if verbose:
                    print(" ".join(cmd), flush=True)
                futs.append(ex.submit(subprocess.run, cmd, check=True))
            for f in futs:
                f.result()
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC",
                *[o for o, _ in cmds], "-o", LIB + ".tmp"]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
