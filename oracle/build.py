"""Compile the C oracle into oracle/_silhouette_oracle.so with gcc (test infrastructure).

binary64 semantics are kept strict: -O2 without fast-math and with floating-point contraction
off, so every sum and product is rounded in the order the source states.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "silhouette_oracle.c")
OUT = os.path.join(HERE, "_silhouette_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", OUT + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
