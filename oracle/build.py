"""Compile the FP64 C oracle into ``oracle/liboracle.so`` with gcc.

Test infrastructure only: the library it builds is loaded by the test-suite,
the smoke check and the CPU-baseline leg of the benchmark, never by the
product path.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "omt_oracle.c"), os.path.join(HERE, "momt_oracle.c"), os.path.join(HERE, "omt3_oracle.c")]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    # -ffp-contract=off keeps every expression exactly as written (no fused
    # multiply-adds), so the oracle's rounding is that of the plain formula.
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall", "-Wextra", "-o", LIB + ".tmp", *SRCS, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
