"""Build the CPU oracle's shared library with gcc.

Test infrastructure: the library is loaded only by the tests, the package's
smoke check and the CPU-baseline leg of the benchmark.  The flags keep every
FP64 operation an IEEE operation in the written order (no contraction, no
fast-math); OpenMP only splits independent blocks across threads.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hydro_oracle.c")
LIB = os.path.join(HERE, "libhydro_oracle.so")
FLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
         "-std=c99", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", *FLAGS, "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
