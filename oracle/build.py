"""Build the C part of the oracle (cellsum.c -> liboracle_cells.so, next to
this file) with the host compiler: plain float64, OpenMP, no contraction
into fused multiply-adds and no reassociation, so the sums are the
definition's operations in the order cellsum.c writes them.

    python -m oracle.build
"""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cellsum.c")
LIB = os.path.join(HERE, "liboracle_cells.so")
FLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math"]


def build() -> str:
    cc = os.environ.get("CC") or shutil.which("gcc") or shutil.which("cc")
    if not cc:
        raise RuntimeError("no C compiler found for the CPU oracle")
    tmp = LIB + ".tmp"
    r = subprocess.run([cc, *FLAGS, SRC, "-o", tmp, "-lm"], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling cellsum.c failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
