"""The C-ABI library loads and exports every function that include/hiputf.h
declares (no compute calls: runs without a GPU)."""
from __future__ import annotations

import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hiputf.h")
LIB = os.path.join(ROOT, "paper_2109_10433_amd", "libhiputf.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    # prototypes: identifier ( args ) ;
    names = re.findall(r"([A-Za-z_]\w*)\s*\(([^;{}()]*)\)\s*;", src, flags=re.S)
    return sorted(set(n for n, _ in names))


def test_header_declares_the_six_functions():
    names = declared_functions()
    for n in ("validate_utf8", "utf16_length_from_utf8", "convert_utf8_to_utf16le",
              "validate_utf16le", "utf8_length_from_utf16le", "convert_utf16le_to_utf8"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        from paper_2109_10433_amd.build import build
        build()
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_match_header():
    from paper_2109_10433_amd import binding
    assert sorted(binding.EXPORTED) == sorted(n for n in declared_functions() if n in binding.EXPORTED)
    assert set(declared_functions()) <= set(binding.EXPORTED) | set(getattr(binding, "EXPORTED_EXTRA", []))
