"""Build the FP64 CPU oracle (test infrastructure) into oracle/libmpm_oracle.so.

Plain g++, -O2, no fast-math, no OpenMP: the oracle is the slow, obviously
correct reference, single-threaded by design.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mpm_oracle.cpp")
LIB = os.path.join(HERE, "libmpm_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["g++", "-std=c++17", "-O2", "-fno-fast-math", "-ffp-contract=off",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
