"""Compile the generators' native helper (plain C, host only)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build() -> str:
    src = os.path.join(HERE, "workloads.c")
    out = os.path.join(HERE, "libworkloads.so")
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, src])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
