"""Builds the FP64 CPU oracle (test infrastructure only) into oracle/liborc.so.

Plain g++ (C++17, OpenMP, -O2, no fast-math, no FP contraction) so that the
oracle's arithmetic is the order written in pinn_oracle.cpp.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liborc.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "pinn_oracle.cpp")
    tmp = LIB + ".tmp"
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", tmp, src]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
