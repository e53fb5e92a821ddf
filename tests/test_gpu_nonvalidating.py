"""GPU parity of the non-validating conversions (section 4's non-validating
transcoder and its UTF-16 counterpart): on valid input the same words/bytes
and count as the oracle, bit-exact; on invalid input the call completes and
writes nothing outside its capacity."""
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


def nv_u8(data: np.ndarray, offset: int = 0, cap_words: int | None = None, out_offset: int = 0):
    src = DeviceBytes(data, offset)
    cap = data.size if cap_words is None else cap_words
    out = DeviceOut(2 * cap, out_offset)
    r = hu.lib.convert_valid_utf8_to_utf16le(src.ptr, data.size, out.ptr, cap, hu.stream_handle())
    h = out.host()
    return (int(r.error), int(r.count)), out.region(h).view(np.uint16) if cap else np.zeros(0, np.uint16), out, h


def nv_u16(words: np.ndarray, offset: int = 0, cap_bytes: int | None = None, out_offset: int = 0):
    src = DeviceBytes(words.astype("<u2"), offset)
    cap = 3 * words.size if cap_bytes is None else cap_bytes
    out = DeviceOut(cap, out_offset)
    r = hu.lib.convert_valid_utf16le_to_utf8(src.ptr, words.size, out.ptr, cap, hu.stream_handle())
    h = out.host()
    return (int(r.error), int(r.count)), out.region(h), out, h


def check_valid(text, offset=0, out_offset=0):
    ow, oc = oracle.convert_utf8_to_utf16le(text.u8)
    assert oc.error == 0
    r, words, out, h = nv_u8(text.u8, offset, out_offset=2 * (out_offset % 3))
    assert r == (0, int(oc.count))
    assert np.array_equal(words[:r[1]], ow)
    out.check_guards(h, 2 * r[1])
    ob, oc16 = oracle.convert_utf16le_to_utf8(text.u16)
    r, b, out, h = nv_u16(text.u16, 2 * (offset % 8), out_offset=out_offset % 5)
    assert r == (0, int(oc16.count))
    assert np.array_equal(b[:r[1]], ob)
    out.check_guards(h, r[1])


@pytest.mark.parametrize("profile", ["mix", "latin", "cyrillic", "cjk", "emoji"])
def test_valid_input_matches_the_oracle(profile):
    text = wl.make_text(profile, 1 << 20, wl.rng_for("nv", profile))
    say("non-validating, 1 MiB", profile)
    check_valid(text)
    starts8 = text.char_starts_u8
    for n in (0, 1, 15, 16, 17, 1023, 4097, 20479, 20480, 20481, 24575, 24576, 24577, 65541, 300_001):
        m = int(starts8[np.searchsorted(starts8, n, side="right") - 1])
        for off in (0, 7):
            check_valid(wl.Text(text.cps[:np.searchsorted(starts8, m)], text.utf8_len[:np.searchsorted(starts8, m)],
                                text.u8[:m], text.u16[:int(text.char_starts_u16[np.searchsorted(starts8, m)])]),
                        off, out_offset=off)


def test_invalid_input_stays_inside_the_output():
    """Counts inflated by invalid input (every byte a four-byte lead, counted
    as two words; every word a high surrogate, counted as two bytes, against
    one byte per word) exceed the capacities: OUTPUT_TOO_SMALL, and no write
    outside [dst, dst + cap); random garbage: completes, guards intact."""
    rng = np.random.default_rng(4)
    for n in (1, 100, 4096, 20480 + 7, 1 << 20):
        say("non-validating on invalid input, n =", n)
        r, _, out, h = nv_u8(np.full(n, 0xF8, np.uint8))
        assert r == (hu.OUTPUT_TOO_SMALL, 2 * n)
        out.check_guards(h)
        r, _, out, h = nv_u16(np.full(n, 0xD800, np.uint16), cap_bytes=n)
        assert r == (hu.OUTPUT_TOO_SMALL, 2 * n)
        out.check_guards(h)
        r, _, out, h = nv_u16(np.full(n, 0xDC00, np.uint16))
        assert r == (0, 2 * n)
        out.check_guards(h)
        for _ in range(3):
            r, _, out, h = nv_u8(rng.integers(0, 256, n, dtype=np.uint8), int(rng.integers(0, 16)))
            out.check_guards(h)
            r, _, out, h = nv_u16(rng.integers(0, 65536, n, dtype=np.uint16), 2 * int(rng.integers(0, 8)))
            out.check_guards(h)
