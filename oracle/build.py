"""Builds the CPU oracle library (test infrastructure only).

gcc, -ffp-contract=off and no fast-math so that the TwoSum/TwoProduct steps of
the compensated dot product are evaluated exactly as written; -mfma so that
fma() is a single hardware instruction; OpenMP over output rows.
"""

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mg_oracle.c")
OUT = os.path.join(HERE, "libmg_oracle.so")

CFLAGS = ["-O3", "-march=x86-64-v3", "-mfma", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", *CFLAGS, SRC, "-o", OUT + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
