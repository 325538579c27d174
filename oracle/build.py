"""Compile the oracle's C arithmetic into oracle/_prims.so.

TEST INFRASTRUCTURE ONLY: the oracle checks the GPU library and is never part
of it.  Built with plain gcc; nothing here touches HIP.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ckks_prims.c")
OUT = os.path.join(HERE, "_prims.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(OUT) and os.path.getmtime(OUT) >= os.path.getmtime(SRC):
        return OUT
    tmp = OUT + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                           "-Wall", "-Wextra", "-o", tmp, SRC])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
