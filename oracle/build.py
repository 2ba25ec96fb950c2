"""Build the FP64 CPU oracle (test infrastructure) into oracle/liblj_oracle.so.

The oracle is plain C built with gcc.  -ffp-contract=off keeps every multiply
and add separately rounded unless the source calls fma() explicitly; -mfma lets
those fma() calls compile to the hardware instruction (same result as libm's
correctly rounded fma, faster).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lj_oracle.c")
LIB = os.path.join(HERE, "liblj_oracle.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-mfma",
           "-fno-fast-math", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def ensure_built() -> str:
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
