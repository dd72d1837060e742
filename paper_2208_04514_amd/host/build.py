"""Build ``libdawn_host.so`` (the host CPU DAWN, ``include/dawn_host.h``) with g++.

Always rebuilds; run ``python -m paper_2208_04514_amd.host.build``.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
SRC = os.path.join(HERE, "dawn_host.cpp")
LIB = os.path.join(PKG, "libdawn_host.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["g++", "-O3", "-std=c++17", "-fPIC", "-shared", "-pthread", "-Wall",
           f"-I{os.path.join(ROOT, 'include')}", SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
