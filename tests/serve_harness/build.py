"""Build the scheduler test harness (host C++, no GPU): ``python -m tests.serve_harness.build``."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
LIB = os.path.join(HERE, "libserve_harness.so")


def build(extra=()) -> str:
    tmp = LIB + ".tmp"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-Wall", "-Wextra", "-Werror",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2109_10433_amd", "csrc"),
           *extra, os.path.join(HERE, "harness.cpp"), "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
