"""GPU parity of the UTF-16 big-endian calls (section 3: UTF-16's two byte
orders): the oracle's little-endian results with every UTF-16 word byte
swapped on the host, bit-exact, through the C ABI."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2109_10433_amd import workloads as wl
from tests.gpu_util import DeviceBytes, DeviceOut, say

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2109_10433_amd import binding as hu


def _r(res):
    return (int(res.error), int(res.count))


def be_u16(words: np.ndarray, offset: int = 0, cap_bytes: int | None = None, out_offset: int = 0):
    """UTF-16BE validate, length and convert of `words` (values, stored most
    significant byte first at `offset`)."""
    src = DeviceBytes(words.astype(">u2"), offset)
    s = hu.stream_handle()
    n = words.size
    v = _r(hu.lib.validate_utf16be(src.ptr, n, s))
    ln = _r(hu.lib.utf8_length_from_utf16be(src.ptr, n, s))
    cap = 3 * n if cap_bytes is None else cap_bytes
    out = DeviceOut(cap, out_offset)
    c = _r(hu.lib.convert_utf16be_to_utf8(src.ptr, n, out.ptr, cap, s))
    h = out.host()
    return v, ln, c, out, h


def be_u8(data: np.ndarray, offset: int = 0, cap_words: int | None = None, out_offset: int = 0):
    """UTF-8 -> UTF-16BE; returns the result and the output word values."""
    src = DeviceBytes(data, offset)
    cap = data.size if cap_words is None else cap_words
    out = DeviceOut(2 * cap, out_offset)
    c = _r(hu.lib.convert_utf8_to_utf16be(src.ptr, data.size, out.ptr, cap, hu.stream_handle()))
    h = out.host()
    words = out.region(h).view(">u2").astype(np.uint16) if cap else np.zeros(0, np.uint16)
    return c, words, out, h


def check_u16be(words: np.ndarray, offset: int = 0, out_offset: int = 0):
    ov = tuple(oracle.validate_utf16le(words))
    ol = tuple(oracle.utf8_length_from_utf16le(words))
    ob, oc = oracle.convert_utf16le_to_utf8(words)
    v, ln, c, out, h = be_u16(words, offset, out_offset=out_offset)
    assert v == ov
    assert ln == ol
    assert c == tuple(oc)
    if c[0] == 0:
        assert np.array_equal(out.region(h)[:c[1]], ob)
        out.check_guards(h, c[1])
    else:
        out.check_guards(h)
    return ov


def check_u8_to_be(data: np.ndarray, offset: int = 0, out_offset: int = 0):
    ow, oc = oracle.convert_utf8_to_utf16le(data)
    c, words, out, h = be_u8(data, offset, out_offset=out_offset)
    assert c == tuple(oc)
    if c[0] == 0:
        assert np.array_equal(words[:c[1]], ow)
        out.check_guards(h, 2 * c[1])
    else:
        out.check_guards(h)


@pytest.mark.parametrize("profile", ["mix", "latin", "cyrillic", "cjk", "emoji"])
def test_profiles_both_directions(profile):
    text = wl.make_text(profile, 1 << 20, wl.rng_for("be", profile))
    say("UTF-16BE, 1 MiB", profile)
    assert check_u16be(text.u16) == (0, text.u16.size)
    check_u8_to_be(text.u8)
    for n in (1, 17, 4097, 24577, 100_003):
        say("UTF-16BE prefix", n, profile)
        check_u16be(text.u16[:n], offset=2 * (n % 8), out_offset=n % 5)
        check_u8_to_be(text.u8[:n], offset=n % 16, out_offset=2 * (n % 3))


def test_small_sizes_and_offsets():
    text = wl.make_text("mix", 4096, wl.rng_for("be-small"))
    for offset in (0, 2, 14):
        say("utf16be sizes 0..200 at offset", offset)
        for n in range(0, 201):
            check_u16be(text.u16[:n], offset, out_offset=offset % 5)
    for offset in (0, 7):
        say("utf8 -> utf16be sizes 0..200 at offset", offset)
        for n in range(0, 201):
            check_u8_to_be(text.u8[:n], offset, out_offset=2 * (offset % 3))


def test_unpaired_surrogates_around_tile_boundaries():
    """Word tiles of the UTF-16 convert are 12288 words; the validate and
    length kernels walk 2048-word sub-tiles."""
    text = wl.make_text("mix", 60_000, wl.rng_for("be-surrogates"))
    w = text.u16
    for boundary in (2048, 12288, 24576):
        for d in range(-2, 3):
            for val in (0xD800, 0xDBFF, 0xDC00, 0xDFFF):
                if boundary + d >= w.size:
                    continue
                data = w.copy()
                data[boundary + d] = val
                say("utf16be surrogate", hex(val), "at", boundary + d)
                check_u16be(data, offset=6 if d & 1 else 0)


def test_random_short_strings():
    w_alpha = np.array([0x41, 0x7F, 0x80, 0x7FF, 0x800, 0xD7FF, 0xD800, 0xDBFF, 0xDC00, 0xDFFF, 0xE000,
                        0xFEFF, 0xFFFE, 0xFFFF], dtype=np.uint16)
    rng = np.random.default_rng(12)
    say("random short UTF-16BE strings")
    for _ in range(600):
        n = int(rng.integers(1, 20))
        check_u16be(w_alpha[rng.integers(0, w_alpha.size, size=n)], offset=2 * int(rng.integers(0, 8)))


def test_utf8_errors_still_reported():
    text = wl.make_text("mix", 50_000, wl.rng_for("be-u8err"))
    rng = np.random.default_rng(5)
    for kind in wl.UTF8_ERROR_KINDS:
        data, p = wl.inject_utf8_error(text.u8, text.char_starts_u8, kind, rng)
        say("utf8 -> utf16be with", kind, "at", p)
        check_u8_to_be(data, offset=3)


def test_capacity_and_guards():
    text = wl.make_text("emoji", 10_000, wl.rng_for("be-cap"))
    n16 = text.u16.size
    for cap in (n16, n16 - 1, 1, 0):
        say("utf8 -> utf16be capacity", cap, "of", n16)
        c, words, out, h = be_u8(text.u8, 3, cap_words=cap, out_offset=2)
        if cap >= n16:
            assert c == (0, n16) and np.array_equal(words[:n16], text.u16)
            out.check_guards(h, 2 * n16)
        else:
            assert c == (oracle.OUTPUT_TOO_SMALL, n16)
            out.check_guards(h)
    n8 = text.u8.size
    for cap in (n8, n8 - 1, 0):
        say("utf16be -> utf8 capacity", cap, "of", n8)
        _, _, c, out, h = be_u16(text.u16, 0, cap_bytes=cap, out_offset=1)
        if cap >= n8:
            assert c == (0, n8) and np.array_equal(out.region(h)[:n8], text.u8)
        else:
            assert c == (oracle.OUTPUT_TOO_SMALL, n8)
        out.check_guards(h)


def test_async_calls_share_the_little_endian_workspace():
    text = wl.make_text("cjk", 200_000, wl.rng_for("be-async"))
    src8 = torch.from_numpy(text.u8.copy()).cuda()
    src16 = torch.from_numpy(text.u16.astype(">u2").view(np.uint8).copy()).cuda()
    rec = torch.zeros(16, dtype=torch.uint8, device="cuda")
    s = hu.stream_handle()
    ws = hu.workspace(hu.OP_CONVERT_UTF8_TO_UTF16LE, src8.numel())
    wp, wb = hu.workspace_ptr(ws)
    dst = torch.zeros(src8.numel(), dtype=torch.int16, device="cuda")
    say("async utf8 -> utf16be")
    assert hu.lib.convert_utf8_to_utf16be_async(src8.data_ptr(), src8.numel(), dst.data_ptr(), src8.numel(),
                                                rec.data_ptr(), wp, wb, s) == 0
    torch.cuda.synchronize()
    r = hu.result_from_device(rec)
    assert r == (0, text.u16.size)
    assert np.array_equal(dst.cpu().numpy().view(">u2")[:r.count].astype(np.uint16), text.u16)
    n = text.u16.size
    for op, fn in ((hu.OP_VALIDATE_UTF16LE, hu.lib.validate_utf16be_async),
                   (hu.OP_UTF8_LENGTH_FROM_UTF16LE, hu.lib.utf8_length_from_utf16be_async)):
        ws = hu.workspace(op, n)
        wp, wb = hu.workspace_ptr(ws)
        say("async", fn.__name__)
        assert fn(src16.data_ptr(), n, rec.data_ptr(), wp, wb, s) == 0
        torch.cuda.synchronize()
        want = (0, n) if op == hu.OP_VALIDATE_UTF16LE else (0, text.u8.size)
        assert hu.result_from_device(rec) == want
    ws = hu.workspace(hu.OP_CONVERT_UTF16LE_TO_UTF8, n)
    wp, wb = hu.workspace_ptr(ws)
    out = torch.zeros(3 * n, dtype=torch.uint8, device="cuda")
    say("async utf16be -> utf8")
    assert hu.lib.convert_utf16be_to_utf8_async(src16.data_ptr(), n, out.data_ptr(), 3 * n, rec.data_ptr(),
                                                wp, wb, s) == 0
    torch.cuda.synchronize()
    r = hu.result_from_device(rec)
    assert r == (0, text.u8.size)
    assert np.array_equal(out.cpu().numpy()[:r.count], text.u8)


def test_bom_then_convert():
    """A buffer opening with FE FF: detect it on the host, skip it, convert
    the rest as UTF-16BE."""
    text = wl.make_text("emoji", 5000, wl.rng_for("be-bom"))
    raw = np.concatenate([np.array([0xFE, 0xFF], np.uint8), text.u16.astype(">u2").view(np.uint8)])
    enc, skip = hu.detect_bom(raw[:4].tobytes())
    assert (enc, skip) == (hu.BOM_UTF16BE, 2)
    body = raw[skip:].view(">u2").astype(np.uint16)
    say("BOM + utf16be")
    check_u16be(body)
