"""Build the gfx950 shared library ``libhiputf.so`` in-tree: ``python -m paper_2109_10433_amd.build``.

One hipcc invocation over csrc/hiputf.hip (kernels and the C ABI),
csrc/variants.hip (non-validating and big-endian kernels) and csrc/serve.hip
(the server, host code). Packed FP32 instruction selection is
disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libhiputf.so")
ARCH = os.environ.get("HIPUTF_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(extra=(), out: str = LIB, verbose: bool = False) -> str:
    tmp = out + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, *extra, "-I", os.path.join(ROOT, "include"),
           os.path.join(PKG, "csrc", "hiputf.hip"), os.path.join(PKG, "csrc", "variants.hip"),
           os.path.join(PKG, "csrc", "serve.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(sys.argv[1:], verbose=True))
