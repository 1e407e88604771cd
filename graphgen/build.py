"""Compiles the generator library (host C++ with OpenMP) in place."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libgraphgen.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "gen.cpp")
    tmp = LIB + ".tmp"
    cmd = ["g++", "-O3", "-march=x86-64-v2", "-std=c++17", "-fopenmp", "-shared", "-fPIC",
           "-Wall", "-Wextra", src, "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
