"""Regression test: the call that wraps a workspace's 22-bit epoch back to 0.

Status words of the single-buffer kernels carry the epoch of the call that
wrote them, so a workspace is reused without clearing, except when the epoch
wraps: then the status words are cleared, and that must not happen while any
tile of the wrapping call still reads them in its look-back. The workspace's
epoch is preset to the largest value, and its status words are filled with
words tagged epoch 0 that claim an inclusive prefix, which the next call (at
epoch 0) would take for its own if the wrapping call had not cleared them.
Every result and output is compared with the oracle, on the wrapping call and
on the call after it, for every kernel family: both convert directions (also
the UTF-8 input of 64 MiB and more, which takes the largest tiles), the
non-validating and big-endian converts, and the validate / length kernels.
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

EPOCH_MAX = (1 << 22) - 1
HEADER_BYTES = 256
EPOCH_OFFSET = 24                  # WsHeader: three 64-bit fields, then the epoch
STALE = (2 << 40) | 0x12345        # tag 0, inclusive flag, a wrong prefix


def _preset(ws: torch.Tensor, wp: int, wb: int):
    off = wp - ws.data_ptr()
    h = np.zeros(wb, np.uint8)
    h[EPOCH_OFFSET:EPOCH_OFFSET + 4] = np.frombuffer(np.uint32(EPOCH_MAX).tobytes(), np.uint8)
    n_words = (wb - HEADER_BYTES) // 8
    h[HEADER_BYTES:HEADER_BYTES + 8 * n_words].view("<u8")[:] = STALE
    ws[off:off + wb].copy_(torch.from_numpy(h).cuda())
    torch.cuda.synchronize()


def _state(ws: torch.Tensor, wp: int, wb: int):
    off = wp - ws.data_ptr()
    h = ws[off:off + wb].cpu().numpy()
    epoch = int(h[EPOCH_OFFSET:EPOCH_OFFSET + 4].view("<u4")[0])
    n_words = (wb - HEADER_BYTES) // 8
    status = h[HEADER_BYTES:HEADER_BYTES + 8 * n_words].view("<u8")
    return epoch, status


def _inject_late(u8: np.ndarray, starts: np.ndarray) -> np.ndarray:
    """A stray continuation byte at a character start near the end (in the
    last tiles, whose look-backs are the ones still running at the end)."""
    bad = u8.copy()
    p = int(starts[starts.size - 300])
    bad[p] = 0x80
    return bad


def _run_u8(fn, src: np.ndarray, ws, wp, wb, be=False):
    """One async call on UTF-8 input; returns (result, output words or None)."""
    s = torch.from_numpy(src.copy()).cuda()
    rec = torch.zeros(16, dtype=torch.uint8, device="cuda")
    if fn in ("validate_utf8_async", "utf16_length_from_utf8_async"):
        rc = getattr(hu.lib, fn)(s.data_ptr(), s.numel(), rec.data_ptr(), wp, wb, hu.stream_handle())
        out = None
    else:
        out = torch.zeros(max(s.numel(), 1), dtype=torch.int16, device="cuda")
        rc = getattr(hu.lib, fn)(s.data_ptr(), s.numel(), out.data_ptr(), s.numel(), rec.data_ptr(), wp, wb,
                                 hu.stream_handle())
    assert rc == 0
    torch.cuda.synchronize()
    r = hu.result_from_device(rec)
    words = None
    if out is not None and r.error == 0:
        words = out.cpu().numpy().view(np.uint16)[:r.count]
        if be:
            words = words.byteswap()
    return r, words


def _run_u16(fn, src: np.ndarray, ws, wp, wb, be=False):
    w = src.astype("<u2")
    if be:
        w = w.byteswap()
    s = torch.from_numpy(w.view(np.int16).copy()).cuda()
    rec = torch.zeros(16, dtype=torch.uint8, device="cuda")
    if fn in ("validate_utf16le_async", "utf8_length_from_utf16le_async"):
        rc = getattr(hu.lib, fn)(s.data_ptr(), s.numel(), rec.data_ptr(), wp, wb, hu.stream_handle())
        out = None
    else:
        out = torch.zeros(max(3 * s.numel(), 1), dtype=torch.uint8, device="cuda")
        rc = getattr(hu.lib, fn)(s.data_ptr(), s.numel(), out.data_ptr(), 3 * s.numel(), rec.data_ptr(), wp, wb,
                                 hu.stream_handle())
    assert rc == 0
    torch.cuda.synchronize()
    r = hu.result_from_device(rec)
    data = out.cpu().numpy()[:r.count] if out is not None and r.error == 0 else None
    return r, data


def _expect_u8(fn, data):
    if fn == "validate_utf8_async":
        return tuple(oracle.validate_utf8(data)), None
    if fn == "utf16_length_from_utf8_async":
        return tuple(oracle.utf16_length_from_utf8(data)), None
    ow, orr = oracle.convert_utf8_to_utf16le(data)
    return tuple(orr), ow


def _expect_u16(fn, words):
    if fn == "validate_utf16le_async":
        return tuple(oracle.validate_utf16le(words)), None
    if fn == "utf8_length_from_utf16le_async":
        return tuple(oracle.utf8_length_from_utf16le(words)), None
    ob, orr = oracle.convert_utf16le_to_utf8(words)
    return tuple(orr), ob


@pytest.fixture(scope="module")
def texts():
    say("generating texts for the epoch-wrap test")
    small = wl.make_text("mix", 1 << 20, wl.rng_for("epoch-wrap", "small"))
    large = wl.make_text("mix", (64 << 20) + 4096, wl.rng_for("epoch-wrap", "large"), encode16=False)
    return small, large


CASES_U8 = [
    # (entry point, op for the workspace size, which text, big endian output)
    ("convert_utf8_to_utf16le_async", 2, "small", False),
    ("convert_utf8_to_utf16le_async", 2, "large", False),
    ("convert_valid_utf8_to_utf16le_async", 2, "small", False),
    ("convert_utf8_to_utf16be_async", 2, "small", True),
    ("validate_utf8_async", 0, "small", False),
    ("utf16_length_from_utf8_async", 1, "small", False),
]
CASES_U16 = [
    ("convert_utf16le_to_utf8_async", 5, False),
    ("convert_valid_utf16le_to_utf8_async", 5, False),
    ("convert_utf16be_to_utf8_async", 5, True),
    ("validate_utf16le_async", 3, False),
    ("utf8_length_from_utf16le_async", 4, False),
]


@pytest.mark.parametrize("fn,op,which,be", CASES_U8)
@pytest.mark.parametrize("bad_first", [False, True])
def test_epoch_wrap_utf8_input(texts, fn, op, which, be, bad_first):
    t = texts[0] if which == "small" else texts[1]
    good = t.u8
    bad = _inject_late(good, t.char_starts_u8)
    seq = [bad, good] if bad_first else [good, bad]
    if fn == "convert_valid_utf8_to_utf16le_async":
        seq = [good, good]     # no validation: valid input only
    ws = hu.workspace(op, good.size)
    wp, wb = hu.workspace_ptr(ws)
    _preset(ws, wp, wb)
    for k, data in enumerate(seq):
        say("epoch wrap", fn, which, "call", k, "bad" if data is bad else "good", data.size, "bytes")
        r, words = _run_u8(fn, data, ws, wp, wb, be)
        er, ew = _expect_u8(fn, data)
        assert tuple(r) == er, (fn, k)
        if ew is not None and er[0] == 0:
            assert np.array_equal(words, ew), (fn, k)
        epoch, status = _state(ws, wp, wb)
        assert epoch == k, (fn, k, epoch)
        if k == 0:
            # the wrapping call cleared every status word, or the next call
            # would have read the stale ones
            assert not np.any(status), "status words left after the epoch wrapped"


@pytest.mark.parametrize("fn,op,be", CASES_U16)
@pytest.mark.parametrize("bad_first", [False, True])
def test_epoch_wrap_utf16_input(texts, fn, op, be, bad_first):
    t = texts[0]
    good = t.u16
    bad = good.copy()
    bad[good.size - 701] = 0x41          # a lone low surrogate after an ASCII word
    bad[good.size - 700] = 0xDC00
    seq = [bad, good] if bad_first else [good, bad]
    if fn == "convert_valid_utf16le_to_utf8_async":
        seq = [good, good]
    ws = hu.workspace(op, good.size)
    wp, wb = hu.workspace_ptr(ws)
    _preset(ws, wp, wb)
    for k, data in enumerate(seq):
        say("epoch wrap", fn, "call", k, "bad" if data is bad else "good", data.size, "words")
        r, out = _run_u16(fn, data, ws, wp, wb, be)
        er, eb = _expect_u16(fn, data)
        assert tuple(r) == er, (fn, k)
        if eb is not None and er[0] == 0:
            assert np.array_equal(out, eb), (fn, k)
        epoch, status = _state(ws, wp, wb)
        assert epoch == k, (fn, k, epoch)
        if k == 0:
            assert not np.any(status), "status words left after the epoch wrapped"
