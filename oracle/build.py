"""Compile the CPU oracle (plain C + OpenMP) into oracle/liboracle.so.

Test infrastructure only: building the checker is not using it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def build(src: str | None = None, out: str | None = None) -> str:
    src = src or os.path.join(HERE, "oracle.c")
    out = out or os.path.join(HERE, "liboracle.so")
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                           "-o", tmp, src])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(*sys.argv[1:]))
