"""Compile the C oracle with the host compiler (gcc, OpenMP)."""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hisq_oracle.c")
OUT = os.path.join(HERE, "_hisq_oracle.so")


def build(force: bool = True, quiet: bool = False) -> str:
    if not force and os.path.exists(OUT) and os.path.getmtime(OUT) >= os.path.getmtime(SRC):
        return OUT
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", OUT + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True, capture_output=quiet)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(force=True))
    sys.exit(0)
