"""Compiles the multithreaded CPU baseline (plain C, gcc, OpenMP) in place."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libcpubase.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "cpubase.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-march=x86-64-v2", "-std=gnu11", "-fopenmp", "-shared", "-fPIC", "-Wall", "-Wextra",
           src, "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
