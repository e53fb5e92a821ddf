"""Errors and characters at the kernels' real tile boundaries.

Each kernel cuts its input into tiles of a fixed number of bytes (counted from
the 16-byte aligned address at or below the input); a tile validates and
counts on its own and learns its output offset from the tiles before it, so a
tile boundary is where an ill-formed sequence, or a character split across
two tiles, meets two independent pieces of work (section 4: blocks restart at
character boundaries; the input's tail). The tile sizes are mirrored here and
asserted against the library (hu_tile_bytes); every UTF-8 error kind and
arbitrary byte values are put at -6..+6 bytes around two boundaries of every
UTF-8 kernel, including the conversion kernels of the larger tile classes
that inputs of 4, 24 and 64 MiB and more take (there also around the last
boundary), and the four surrogate values and split surrogate pairs around
two boundaries of every UTF-16 kernel, at two source alignments, and around
the tile boundaries of the larger UTF-16 conversion classes. Results (kind and position) and
outputs are compared with the oracle, bit for bit.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2109_10433_amd import workloads as wl
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2109_10433_amd import binding as hu
    from tests.test_gpu_parity import gpu_u16, gpu_u8

SUB = 4096
PIECE = 1024                 # validate / length: a wave's 1 KiB piece (one 16-byte load per lane)
MIB = 1 << 20
LARGE = 64 * MIB             # UTF-8 inputs of this size and more take the largest convert tiles
# (op, input units, tile bytes): mirrors the kernels' tile choice (convert:
# a workgroup's tile; validate / length: a wave's tile)
TILES = [
    (0, 1000, 2 * PIECE), (1, 1000, 2 * PIECE), (2, 1000, 1 * SUB), (2, 4 * MIB, 2 * SUB),
    (2, 24 * MIB, 5 * SUB), (2, LARGE, 6 * SUB), (3, 1000, 2 * PIECE), (4, 1000, 4 * PIECE), (5, 1000, 1 * SUB),
    (5, 4 * MIB, 2 * SUB), (5, 24 * MIB, 6 * SUB),
]
U8_FN = {0: "validate", 1: "length", 2: "convert"}
U16_FN = {3: "validate", 4: "length", 5: "convert"}


def tile_bytes(op: int, n_units: int) -> int:
    return int(hu.lib.hu_tile_bytes(op, n_units))


def test_tile_sizes_match_the_library():
    for op, n, tb in TILES:
        assert tile_bytes(op, n) == tb, (op, n)


def _expect_u8(fn, data):
    if fn == "validate":
        return tuple(oracle.validate_utf8(data)), None
    if fn == "length":
        return tuple(oracle.utf16_length_from_utf8(data)), None
    ow, orr = oracle.convert_utf8_to_utf16le(data)
    return tuple(orr), ow


def _check_u8(fn, data, offset):
    er, ew = _expect_u8(fn, data)
    r, out, dev_out = gpu_u8(fn, data, offset, out_offset=2)
    assert r == er, (fn, r, er)
    if ew is not None:
        h, words = out
        if er[0] == 0:
            assert np.array_equal(words[:er[1]], ew)
            dev_out.check_guards(h, 2 * er[1])
        else:
            dev_out.check_guards(h)
    return er


@pytest.mark.parametrize("op", [0, 1, 2])
def test_utf8_errors_at_tile_boundaries(op):
    fn = U8_FN[op]
    text = wl.make_text("mix", 110_000, wl.rng_for("tile-boundaries", "utf8"))
    T = tile_bytes(op, text.u8.size)
    assert 2 * T + 6 < text.u8.size
    starts = text.char_starts_u8
    rng = np.random.default_rng(op)
    n_err = 0
    for offset in (0, 5):
        for k in (1, 2):
            b = k * T - offset                    # tile boundary in input coordinates
            say("utf8", fn, "tile", T, "boundary", k, "offset", offset)
            for d in range(-6, 7):
                for kind in wl.UTF8_ERROR_KINDS:
                    i = int(np.searchsorted(starts, b + d))
                    pos = int(starts[min(i, starts.size - 2)])
                    data, _ = wl.inject_utf8_error(text.u8, starts, kind, rng, position=pos)
                    n_err += _check_u8(fn, data, offset)[0] != 0
                for val in (0x80, 0xBF, 0xC2, 0xE4, 0xED, 0xF0, 0xF4, 0xF8, 0x41):
                    data = text.u8.copy()
                    data[b + d] = val
                    _check_u8(fn, data, offset)
            # characters of every length split across the boundary, valid text
            for ch in ("é", "中", "\U0001F600"):
                e = np.frombuffer(ch.encode(), np.uint8)
                for back in range(1, e.size):
                    data = text.u8.copy()
                    p = int(starts[np.searchsorted(starts, b - back - 4)])
                    data[p:b - back] = 0x20
                    data[b - back:b - back + e.size] = e
                    j = b - back + e.size
                    while (data[j] & 0xC0) == 0x80:
                        data[j] = 0x20
                        j += 1
                    assert _check_u8(fn, data, offset)[0] == 0
    assert n_err > 0


# UTF-8 inputs (bytes) in the larger conversion tile classes: 2 sub-tiles
# from 4 MiB, 5 from 24 MiB, 6 from 64 MiB
U8_CLASSES = [(4 * MIB + 70_000, 2), (24 * MIB + 70_000, 5), (LARGE + 70_000, 6)]
# UTF-16 inputs (words) in the larger classes: 2 sub-tiles from 8 MiB of
# input, 6 from 48 MiB
U16_CLASSES = [(4 * MIB + 35_000, 2), (24 * MIB + 35_000, 6)]


@pytest.fixture(scope="module", params=U8_CLASSES, ids=lambda c: f"{c[0] >> 20}MiB")
def u8_class_text(request):
    n, u = request.param
    say("generating", n, "bytes of mixed text")
    return wl.make_text("mix", n, wl.rng_for("tile-boundaries", "large", n), encode16=False), u


def test_utf8_errors_at_convert_tiles_of_large_inputs(u8_class_text):
    """The conversion kernels of the larger tile classes: every error kind at
    -6..+6 around the first two tile boundaries and the last one; the device
    copy of the text is patched in place for each case."""
    t, u = u8_class_text
    n = t.u8.size
    T = tile_bytes(2, n)
    assert T == u * SUB
    starts = t.char_starts_u8
    clean = t.u8
    dev = torch.from_numpy(clean.copy()).cuda()
    out = torch.zeros(n, dtype=torch.int16, device="cuda")
    rng = np.random.default_rng(99)
    last = ((n - 1) // T) * T
    for b in (T, 2 * T, last):
        say("utf8 convert, tile", T, "boundary at", b, "of", n)
        for d in range(-6, 7):
            for kind in wl.UTF8_ERROR_KINDS:
                i = int(np.searchsorted(starts, b + d))
                pos = int(starts[min(i, starts.size - 2)])
                data, _ = wl.inject_utf8_error(clean, starts, kind, rng, position=pos)
                lo = pos
                hi = pos + 8
                while hi < n and data[hi] != clean[hi]:
                    hi += 1
                assert np.array_equal(data[:lo], clean[:lo]) and np.array_equal(data[hi:], clean[hi:])
                dev[lo:hi] = torch.from_numpy(data[lo:hi].copy()).cuda()
                r = hu.lib.convert_utf8_to_utf16le(dev.data_ptr(), n, out.data_ptr(), n, hu.stream_handle())
                dev[lo:hi] = torch.from_numpy(clean[lo:hi].copy()).cuda()
                er = tuple(oracle.convert_utf8_to_utf16le(data)[1])
                assert (int(r.error), int(r.count)) == er, (b, d, kind, er)
    # the clean text: whole output against the oracle
    r = hu.lib.convert_utf8_to_utf16le(dev.data_ptr(), n, out.data_ptr(), n, hu.stream_handle())
    ow, orr = oracle.convert_utf8_to_utf16le(clean)
    assert (int(r.error), int(r.count)) == tuple(orr)
    assert np.array_equal(out[:orr[1]].cpu().numpy().view(np.uint16), ow)


@pytest.fixture(scope="module", params=U16_CLASSES, ids=lambda c: f"{c[0] >> 19}MiB")
def u16_class_text(request):
    n_words, u = request.param
    say("generating", n_words, "words of mixed text")
    t = wl.make_text("mix", 2 * n_words, wl.rng_for("tile-boundaries", "large16", n_words))
    return t.u16, u


def test_utf16_surrogates_at_convert_tiles_of_large_inputs(u16_class_text):
    """The UTF-16 conversion kernels of the larger tile classes: the four
    surrogate values at -6..+6 around the first two tile boundaries and the
    last one, the device copy patched in place; then the clean text's whole
    output against the oracle."""
    w, u = u16_class_text
    n = w.size
    T = tile_bytes(5, n) // 2                    # words per tile
    assert T == u * SUB // 2
    dev = torch.from_numpy(w.view(np.int16).copy()).cuda()
    out = torch.zeros(3 * n + 64, dtype=torch.uint8, device="cuda")
    last = ((n - 1) // T) * T
    for b in (T, 2 * T, last):
        say("utf16 convert, tile", T, "words, boundary at", b, "of", n)
        for d in range(-6, 7):
            if not 0 <= b + d < n:
                continue
            for val in (0xD800, 0xDBFF, 0xDC00, 0xDFFF):
                data = w.copy()
                data[b + d] = val
                dev[b + d] = int(np.array([val], np.uint16).view(np.int16)[0])
                r = hu.lib.convert_utf16le_to_utf8(dev.data_ptr(), n, out.data_ptr(), out.numel(), hu.stream_handle())
                dev[b + d] = int(w[b + d : b + d + 1].view(np.int16)[0])
                er = tuple(oracle.convert_utf16le_to_utf8(data)[1])
                assert (int(r.error), int(r.count)) == er, (b, d, hex(val), er)
    r = hu.lib.convert_utf16le_to_utf8(dev.data_ptr(), n, out.data_ptr(), out.numel(), hu.stream_handle())
    ob, orr = oracle.convert_utf16le_to_utf8(w)
    assert (int(r.error), int(r.count)) == tuple(orr)
    assert np.array_equal(out[:orr[1]].cpu().numpy(), ob)


def _expect_u16(fn, words):
    if fn == "validate":
        return tuple(oracle.validate_utf16le(words)), None
    if fn == "length":
        return tuple(oracle.utf8_length_from_utf16le(words)), None
    ob, orr = oracle.convert_utf16le_to_utf8(words)
    return tuple(orr), ob


def _check_u16(fn, words, offset):
    er, eb = _expect_u16(fn, words)
    r, out, dev_out = gpu_u16(fn, words, offset, out_offset=1)
    assert r == er, (fn, r, er)
    if eb is not None:
        h, b = out
        if er[0] == 0:
            assert np.array_equal(b[:er[1]], eb)
            dev_out.check_guards(h, er[1])
        else:
            dev_out.check_guards(h)
    return er


@pytest.mark.parametrize("op", [3, 4, 5])
def test_utf16_surrogates_at_tile_boundaries(op):
    fn = U16_FN[op]
    text = wl.make_text("mix", 150_000, wl.rng_for("tile-boundaries", "utf16"))
    w = text.u16
    T = tile_bytes(op, w.size) // 2              # words per tile
    assert 2 * T + 6 < w.size
    for offset in (0, 6):                        # bytes
        for k in (1, 2):
            b = k * T - offset // 2
            say("utf16", fn, "tile", T, "words, boundary", k, "offset", offset)
            for d in range(-6, 7):
                for val in (0xD800, 0xDBFF, 0xDC00, 0xDFFF):
                    data = w.copy()
                    data[b + d] = val
                    _check_u16(fn, data, offset)
            # a valid pair in every position around the boundary
            for d in range(-3, 3):
                data = w.copy()
                lo, hi = b + d - 3, b + d + 5        # ASCII around the pair, no surrogate halves cut
                data[lo:hi] = 0x41
                if 0xD800 <= data[lo - 1] < 0xDC00:
                    data[lo - 1] = 0x42
                if 0xDC00 <= data[hi] < 0xE000:
                    data[hi] = 0x42
                data[b + d] = 0xD83D
                data[b + d + 1] = 0xDE00
                assert _check_u16(fn, data, offset)[0] == 0
