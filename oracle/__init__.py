"""Scalar CPU oracle for validating UTF-8 <-> UTF-16LE transcoding (ctypes binding).

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. The GPU library never
imports it, and it imports nothing from the GPU library.

The arithmetic lives in ``oracle.c`` (plain C, one character at a time, written
from section 3 of Lemire & Mula and RFC 3629 / RFC 2781). This module only
marshals numpy buffers into it. Build with ``python -m oracle.build``.
"""
from __future__ import annotations

import ctypes
import os
from typing import NamedTuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK = 0
BAD_LEAD = 1
TRUNCATED = 2
STRAY_CONTINUATION = 3
OVERLONG = 4
TOO_LARGE = 5
SURROGATE = 6
UNPAIRED_SURROGATE = 7
OUTPUT_TOO_SMALL = 16

KIND_NAMES = {
    OK: "OK",
    BAD_LEAD: "BAD_LEAD",
    TRUNCATED: "TRUNCATED",
    STRAY_CONTINUATION: "STRAY_CONTINUATION",
    OVERLONG: "OVERLONG",
    TOO_LARGE: "TOO_LARGE",
    SURROGATE: "SURROGATE",
    UNPAIRED_SURROGATE: "UNPAIRED_SURROGATE",
    OUTPUT_TOO_SMALL: "OUTPUT_TOO_SMALL",
}


class Result(NamedTuple):
    error: int
    count: int


class _CResult(ctypes.Structure):
    _fields_ = [("error", ctypes.c_int32), ("reserved", ctypes.c_int32), ("count", ctypes.c_uint64)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library not built: {LIB_PATH} (run `python -m oracle.build`)")
        _lib = _configure(ctypes.CDLL(LIB_PATH))
    return _lib


def use_library(path: str | None):
    """Route every call to another build of oracle.c (the pin tests use this to
    check that deliberately broken builds fail them); None restores the default."""
    global _lib
    _lib = None if path is None else _configure(ctypes.CDLL(path))


def _configure(lib):
    p, sz = ctypes.c_void_p, ctypes.c_size_t
    for name, args in [
        ("oracle_validate_utf8", [p, sz]),
        ("oracle_utf16_length_from_utf8", [p, sz]),
        ("oracle_convert_utf8_to_utf16le", [p, sz, p, sz]),
        ("oracle_validate_utf16le", [p, sz]),
        ("oracle_utf8_length_from_utf16le", [p, sz]),
        ("oracle_convert_utf16le_to_utf8", [p, sz, p, sz]),
    ]:
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = _CResult
    for name in ("oracle_many_utf8", "oracle_many_utf16le"):
        f = getattr(lib, name)
        f.argtypes = [ctypes.c_int, p, p, sz, p]
        f.restype = None
    lib.oracle_many_at.argtypes = [ctypes.c_int, ctypes.c_int, p, p, sz, p]
    lib.oracle_many_at.restype = None
    lib.oracle_many_convert_at.argtypes = [ctypes.c_int, p, p, p, p, sz, p]
    lib.oracle_many_convert_at.restype = None
    return lib


def _u8(data) -> np.ndarray:
    if isinstance(data, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(data), dtype=np.uint8)
    a = np.ascontiguousarray(data)
    if a.dtype != np.uint8:
        raise TypeError("UTF-8 input must be bytes or a uint8 array")
    return a


def _u16(data) -> np.ndarray:
    """UTF-16LE input as a uint16 array (host order is little-endian on x86)."""
    if isinstance(data, (bytes, bytearray, memoryview)):
        b = bytes(data)
        if len(b) % 2:
            raise ValueError("UTF-16LE input must have an even number of bytes")
        return np.frombuffer(b, dtype="<u2")
    a = np.ascontiguousarray(data)
    if a.dtype == np.int16:
        a = a.view(np.uint16)
    if a.dtype != np.uint16:
        raise TypeError("UTF-16LE input must be bytes or a uint16 array")
    return a


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a.size else None


def _res(r) -> Result:
    return Result(int(r.error), int(r.count))


def validate_utf8(data) -> Result:
    a = _u8(data)
    return _res(_load().oracle_validate_utf8(_ptr(a), a.size))


def utf16_length_from_utf8(data) -> Result:
    a = _u8(data)
    return _res(_load().oracle_utf16_length_from_utf8(_ptr(a), a.size))


def convert_utf8_to_utf16le(data, cap_words: int | None = None):
    """Returns (uint16 array of the written words, Result).

    With the default capacity (one word per input byte, always enough) the
    array holds exactly ``count`` words on success."""
    a = _u8(data)
    cap = a.size if cap_words is None else int(cap_words)
    out = np.zeros(max(cap, 1), dtype=np.uint16)
    r = _res(_load().oracle_convert_utf8_to_utf16le(_ptr(a), a.size, _ptr(out), cap))
    n_out = min(r.count, cap) if r.error == OK else 0
    return out[:n_out].copy(), r


def validate_utf16le(data) -> Result:
    a = _u16(data)
    return _res(_load().oracle_validate_utf16le(_ptr(a), a.size))


def utf8_length_from_utf16le(data) -> Result:
    a = _u16(data)
    return _res(_load().oracle_utf8_length_from_utf16le(_ptr(a), a.size))


def convert_utf16le_to_utf8(data, cap_bytes: int | None = None):
    """Returns (uint8 array of the written bytes, Result).

    The default capacity, three bytes per input word, is always enough."""
    a = _u16(data)
    cap = 3 * a.size if cap_bytes is None else int(cap_bytes)
    out = np.zeros(max(cap, 1), dtype=np.uint8)
    r = _res(_load().oracle_convert_utf16le_to_utf8(_ptr(a), a.size, _ptr(out), cap))
    n_out = min(r.count, cap) if r.error == OK else 0
    return out[:n_out].copy(), r


def _many(fn_name, op, buf, offsets, itemsize):
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    n_docs = offs.size - 1
    out = np.zeros(n_docs, dtype=[("error", "<i4"), ("reserved", "<i4"), ("count", "<u8")])
    getattr(_load(), fn_name)(op, _ptr(buf), _ptr(offs), n_docs, _ptr(out))
    return out["error"].copy(), out["count"].copy()


def many_validate_utf8(buf, offsets):
    """Validate documents buf[offsets[d]:offsets[d+1]]; returns (errors, counts) arrays."""
    return _many("oracle_many_utf8", 0, _u8(buf), offsets, 1)


def many_utf16_length_from_utf8(buf, offsets):
    return _many("oracle_many_utf8", 1, _u8(buf), offsets, 1)


def many_validate_utf16le(buf, offsets):
    """Offsets are in words."""
    return _many("oracle_many_utf16le", 0, _u16(buf), offsets, 2)


def many_utf8_length_from_utf16le(buf, offsets):
    return _many("oracle_many_utf16le", 1, _u16(buf), offsets, 2)


def many_at(op: int, utf16: bool, src_addrs, n_units):
    """Validation (op 0) or length (op 1) of inputs at host addresses
    src_addrs[i] with n_units[i] code units each (the caller keeps the
    buffers alive); returns (errors, counts) arrays."""
    addrs = np.ascontiguousarray(src_addrs, dtype=np.uint64)
    units = np.ascontiguousarray(n_units, dtype=np.uint64)
    assert addrs.size == units.size
    out = np.zeros(addrs.size, dtype=[("error", "<i4"), ("reserved", "<i4"), ("count", "<u8")])
    _load().oracle_many_at(op, 1 if utf16 else 0, _ptr(addrs), _ptr(units), addrs.size, _ptr(out))
    return out["error"].copy(), out["count"].copy()


def many_convert_at(utf16: bool, src_addrs, n_units, dst_addrs, dst_caps):
    """Conversion of inputs at host addresses src_addrs[i] (n_units[i] code
    units) into buffers at dst_addrs[i] holding dst_caps[i] output code
    units (the caller owns and keeps alive every buffer); returns (errors,
    counts) arrays. UTF-16LE -> UTF-8 if utf16, else UTF-8 -> UTF-16LE."""
    arrs = [np.ascontiguousarray(a, dtype=np.uint64) for a in (src_addrs, n_units, dst_addrs, dst_caps)]
    n = arrs[0].size
    assert all(a.size == n for a in arrs)
    out = np.zeros(n, dtype=[("error", "<i4"), ("reserved", "<i4"), ("count", "<u8")])
    _load().oracle_many_convert_at(1 if utf16 else 0, *[_ptr(a) for a in arrs], n, _ptr(out))
    return out["error"].copy(), out["count"].copy()


def convert_raw(utf16: bool, src_addr: int, n_units: int, dst_addr: int, dst_cap: int) -> Result:
    """One conversion on raw host addresses (the caller owns both buffers):
    the least marshalling per call, for timing many small calls."""
    lib = _load()
    f = lib.oracle_convert_utf16le_to_utf8 if utf16 else lib.oracle_convert_utf8_to_utf16le
    return _res(f(src_addr or None, n_units, dst_addr or None, dst_cap))
