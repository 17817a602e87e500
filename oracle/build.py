"""Build the FP64 CPU oracle (test infrastructure) into oracle/_pt_oracle.so.

The oracle is plain C compiled with gcc.  Contraction of a*b+c into fused
multiply-adds is switched off so that the cell/wrap arithmetic is the plain
sequence of IEEE-754 double operations it states.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pt_oracle.c")
OUT = os.path.join(HERE, "_pt_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", SRC, "-o", OUT + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
