"""Compile the CPU FP64 oracle (test infrastructure) into oracle/liboracle.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    src = os.path.join(HERE, "oracle.c")
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=gnu11", "-Wall", "-fPIC", "-shared",
           "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
