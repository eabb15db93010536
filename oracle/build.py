"""Build the FP64 CPU oracle (test infrastructure) into oracle/liblbm3_oracle.so.

Plain gcc, no GPU code.  Run as a script or call build().
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liblbm3_oracle.so")
SRC = [os.path.join(HERE, "lbm3_oracle.c")]


def build(verbose=False):
    cmd = ["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", LIB + ".tmp"] + SRC + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
