"""Build step for the CPU oracle library (test infrastructure only).

Compiles ``rlb_oracle.cpp`` with g++ into ``liboracle.so`` next to this file.
Plain ``-O2`` on the baseline x86-64 target: no fast-math and no fused
multiply-add contraction, so the oracle's arithmetic is plain IEEE FP64.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rlb_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-ffp-contract=off", SRC, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
