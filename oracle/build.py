"""Build the CPU oracle library (oracle/liboracle.so) with gcc.

Test infrastructure only: the oracle is compiled here so that the tests, the
smoke check and the CPU-baseline leg of the benchmark can call it.  The
product library never links or loads it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "vco.c")
    tmp = f"{LIB}.tmp{os.getpid()}"
    # IEEE semantics: no fast-math, no contraction of a*b+c into FMA
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
