"""Builds libpso_prims.so (tests/hip/pso_prims.hip: test kernels around the
library's device primitives) for gfx950 with the library's own flags."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2205_01313_amd import build as lib_build  # noqa: E402

LIB = os.path.join(HERE, "libpso_prims.so")


def build(out: str = LIB) -> str:
    inc = ["-I", os.path.join(ROOT, "include"), "-I", lib_build.CSRC]
    tmp = out + ".tmp"
    subprocess.run([lib_build.hipcc(), *lib_build.HIPCC_FLAGS, *inc, os.path.join(HERE, "pso_prims.hip"), "-o", tmp],
                   check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
