"""Build the oracle's shared library: ``python -m oracle.build``.

Plain gcc, -O2 without auto-vectorisation, so that the CPU baseline measures the
scalar branching code as written.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CFLAGS = ["-O2", "-fno-tree-vectorize", "-std=c99", "-Wall", "-Wextra", "-Werror", "-fPIC", "-shared"]


def build(extra_flags=(), out_name: str = "liboracle.so") -> str:
    out = os.path.join(HERE, out_name)
    tmp = out + ".tmp"
    cmd = ["gcc", *CFLAGS, *extra_flags, os.path.join(HERE, "oracle.c"), "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(sys.argv[1:]))
