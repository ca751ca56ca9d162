"""Build the CPU oracle library ``liberi4_oracle.so`` (test infrastructure only).

Compiled with plain gcc, ``-O2 -ffp-contract=off`` (no fused multiply-add, no
fast-math) so that its rounding is that of the source as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "eri4_oracle.c")
LIB = os.path.join(HERE, "liberi4_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-std=gnu11", "-Wall", "-o", LIB + ".tmp", SRC, "-lquadmath", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
