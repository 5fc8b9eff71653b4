"""Builds libpso.so (the HIP kernels and the C ABI of include/pso.h) for
gfx950 with hipcc, in-tree next to this file."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpso.so")
SOURCES = ["pso_kernels.hip", "pso_block.hip", "pso_capi.hip", "pso_server.hip", "pso_f64.hip", "pso_static.hip"]

# IEEE binary32 throughout: no contraction of a*b+c into fma (the fitness
# functions use explicit fmaf), denormals kept, correctly rounded divide and
# square root; packed-FP32 instructions off.
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math", "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(out: str = LIB, extra=()) -> str:
    """Compile every source (in parallel, one object each) and link them into
    `out`; raises on failure."""
    inc = ["-I", os.path.join(ROOT, "include")]
    with tempfile.TemporaryDirectory(prefix="pso_build_") as tmpdir:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(tmpdir, src.replace(".hip", ".o"))
            cmd = [hipcc(), *HIPCC_FLAGS, *extra, *inc, "-c", os.path.join(CSRC, src), "-o", obj]
            procs.append((cmd, subprocess.Popen(cmd)))
            objs.append(obj)
        failed = [cmd for cmd, p in procs if p.wait() != 0]
        if failed:
            raise subprocess.CalledProcessError(1, failed[0])
        tmp = out + ".tmp"
        subprocess.run([hipcc(), *HIPCC_FLAGS, *extra, *objs, "-o", tmp], check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(extra=sys.argv[1:]))
