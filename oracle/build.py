"""Build the C oracle (test infrastructure) into oracle/liboracle.so with gcc.

The oracle is plain C99 + OpenMP.  liboracle.so (the parity checker) is
compiled for generic x86-64 so the library built here also runs on other
hosts; build_native() compiles the same source with -O3 -march=native into
liboracle_native.so on the host that times it (the CPU baseline), with the
same -ffp-contract=off, so its arithmetic is the same.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nested_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_NATIVE = os.path.join(HERE, "liboracle_native.so")
NATIVE_FLAGS = ["-O3", "-march=native"]


def build(verbose=False):
    cmd = ["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
           "-ffp-contract=off", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build_native(verbose=False):
    cmd = ["gcc"] + NATIVE_FLAGS + ["-std=c99", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
                                    "-ffp-contract=off", "-Wall", "-Wextra", "-o", LIB_NATIVE + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB_NATIVE + ".tmp", LIB_NATIVE)
    return LIB_NATIVE


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
