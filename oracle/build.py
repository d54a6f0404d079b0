"""Compile the oracle's C sources into ``oracle/_build/liboracle.so``.

Test infrastructure: the oracle library is built alongside the product but is
never linked into it.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD_DIR, "liboracle.so")
SOURCES = [os.path.join(HERE, "jacobi.c")]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    tmp = LIB + ".tmp"
    # x86-64-v3 (AVX2 + FMA) runs on any recent x86 host; no -ffast-math, so
    # the arithmetic is plain IEEE double.
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fPIC", "-shared", "-std=c11",
           "-o", tmp] + SOURCES + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
