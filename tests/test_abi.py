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


def test_detect_bom_on_the_host():
    """Byte-order marks of section 3 (UTF-16: FF FE little endian, FE FF big
    endian) and RFC 3629's EF BB BF; a host-only call, no GPU involved."""
    from paper_2109_10433_amd import binding as hu
    cases = [
        (b"\xef\xbb\xbfabc", (hu.BOM_UTF8, 3)),
        (b"\xff\xfea\x00", (hu.BOM_UTF16LE, 2)),
        (b"\xfe\xff\x00a", (hu.BOM_UTF16BE, 2)),
        (b"\xef\xbb", (hu.BOM_NONE, 0)),          # truncated UTF-8 mark
        (b"\xff", (hu.BOM_NONE, 0)),
        (b"", (hu.BOM_NONE, 0)),
        (b"abc", (hu.BOM_NONE, 0)),
        (b"\xfe\xfe", (hu.BOM_NONE, 0)),
        (b"\xef\xbb\xbe", (hu.BOM_NONE, 0)),
        (b"\xff\xfe\x00\x00", (hu.BOM_UTF16LE, 2)),  # UTF-32LE's mark starts the same way
    ]
    for head, want in cases:
        assert hu.detect_bom(head) == want, head
    r = hu.lib.hu_detect_bom(None, 3)
    assert (r.encoding, r.length) == (hu.BOM_NONE, 0)


def test_tile_bytes_on_the_host():
    """hu_tile_bytes is host-only: tile sizes per operation (conversions: 4 KiB
    sub-tiles per workgroup tile, the UTF-8 -> UTF-16LE conversion taking
    larger tiles from 64 MiB on; validation and length: 1 KiB pieces per wave
    tile), 0 for an unknown op; the workspace of validation and length is the
    header alone."""
    from paper_2109_10433_amd import binding as hu
    sub, piece = 4096, 1024
    want = {0: 2 * piece, 1: 2 * piece, 2: 1 * sub, 3: 2 * piece, 4: 4 * piece, 5: 1 * sub}
    for op in (0, 1, 3, 4):
        assert hu.lib.hu_workspace_bytes(op, 1 << 28) == 256
    for op, tb in want.items():
        assert hu.lib.hu_tile_bytes(op, 1000) == tb
    mib = 1 << 20
    # conversion tiles by input size: UTF-8 (units = bytes) 1, 2, 5, 6 sub-tiles
    # below 4, 24, 64 MiB and above; UTF-16 (units = words) 1, 2, 6 below 8,
    # 48 MiB of input and above
    for n, u in ((4 * mib - 1, 1), (4 * mib, 2), (24 * mib - 1, 2), (24 * mib, 5), (64 * mib - 1, 5),
                 (64 * mib, 6)):
        assert hu.lib.hu_tile_bytes(2, n) == u * sub, n
    for n, u in ((4 * mib - 1, 1), (4 * mib, 2), (24 * mib - 1, 2), (24 * mib, 6)):
        assert hu.lib.hu_tile_bytes(5, n) == u * sub, n

    def tiles(nbytes, tb):
        return (nbytes + 15 + tb - 1) // tb

    # a workspace for n units holds the status words of the most tiles any
    # input of at most n units takes
    assert hu.lib.hu_workspace_bytes(2, mib) == 256 + 128 * tiles(mib, sub)
    n = 256 * mib
    most = max(tiles(4 * mib - 1, sub), tiles(24 * mib - 1, 2 * sub), tiles(64 * mib - 1, 5 * sub), tiles(n, 6 * sub))
    assert hu.lib.hu_workspace_bytes(2, n) == 256 + 128 * most
    most16 = max(tiles(8 * mib - 1, sub), tiles(48 * mib - 1, 2 * sub), tiles(2 * n, 6 * sub))
    assert hu.lib.hu_workspace_bytes(5, n) == 256 + 128 * most16
    assert hu.lib.hu_tile_bytes(6, 10) == 0 and hu.lib.hu_tile_bytes(-1, 10) == 0
