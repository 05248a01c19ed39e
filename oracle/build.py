"""Compile the FP64 CPU oracle into oracle/liberf_oracle.so (test infrastructure).

Plain gcc, -O2, no fast-math and no FMA contraction, so that every operation
rounds as written in the source.  OpenMP only distributes independent output
points over threads; results do not depend on the thread count.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "erf_oracle.c")
OUT = os.path.join(HERE, "liberf_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-fopenmp", "-Wall", "-Wno-unknown-pragmas", "-o", OUT + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
