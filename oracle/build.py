"""Compile the C oracle into oracle/liboracle.so with gcc (OpenMP, IEEE FP64).

Test infrastructure: the HIP library never links or loads the result.
``extra_defines`` lets a test build a deliberately broken variant elsewhere.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qaoa_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(out: str = LIB, extra_defines=(), quiet: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-fno-fast-math", "-ffp-contract=off", "-Wall", "-Wextra",
           *[f"-D{d}" for d in extra_defines], SRC, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True, capture_output=quiet)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else LIB))
