"""GPU parity: the HIP library against the CPU oracle, through the C ABI,
element by element (all results are integers: bit-exact)."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2109_10433_amd import workloads as wl
from tests.gpu_util import DeviceBytes, DeviceOut, say

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2109_10433_amd import binding as hu

SUB = 4096       # sub-tile bytes: one 16-byte load per thread of a 256-thread workgroup


def _stream():
    return hu.stream_handle()


def gpu_u8(op: str, data: np.ndarray, offset: int = 0, cap_words: int | None = None, out_offset: int = 0):
    """Run one UTF-8 entry point; returns (Result, output words or None, DeviceOut)."""
    src = DeviceBytes(data, offset)
    n = data.size
    if op == "validate":
        return _r(hu.lib.validate_utf8(src.ptr, n, _stream())), None, None
    if op == "length":
        return _r(hu.lib.utf16_length_from_utf8(src.ptr, n, _stream())), None, None
    cap = n if cap_words is None else cap_words
    out = DeviceOut(2 * cap, out_offset)
    r = _r(hu.lib.convert_utf8_to_utf16le(src.ptr, n, out.ptr, cap, _stream()))
    h = out.host()
    words = out.region(h).view(np.uint16) if cap else np.zeros(0, np.uint16)
    return r, (h, words), out


def gpu_u16(op: str, words: np.ndarray, offset: int = 0, cap_bytes: int | None = None, out_offset: int = 0):
    src = DeviceBytes(words.astype("<u2"), offset)
    n = words.size
    if op == "validate":
        return _r(hu.lib.validate_utf16le(src.ptr, n, _stream())), None, None
    if op == "length":
        return _r(hu.lib.utf8_length_from_utf16le(src.ptr, n, _stream())), None, None
    cap = 3 * n if cap_bytes is None else cap_bytes
    out = DeviceOut(cap, out_offset)
    r = _r(hu.lib.convert_utf16le_to_utf8(src.ptr, n, out.ptr, cap, _stream()))
    h = out.host()
    return r, (h, out.region(h)), out


def _r(res):
    return (int(res.error), int(res.count))


def check_u8_all(data: np.ndarray, offset: int = 0, out_offset: int = 0):
    """All three UTF-8 entry points against the oracle."""
    ov = tuple(oracle.validate_utf8(data))
    ol = tuple(oracle.utf16_length_from_utf8(data))
    ow, oc = oracle.convert_utf8_to_utf16le(data)
    assert gpu_u8("validate", data, offset)[0] == ov
    assert gpu_u8("length", data, offset)[0] == ol
    r, (h, words), out = gpu_u8("convert", data, offset, out_offset=out_offset)
    assert r == tuple(oc)
    if r[0] == 0:
        assert np.array_equal(words[:r[1]], ow)
        out.check_guards(h, 2 * r[1])
    else:
        out.check_guards(h)
    return ov


def check_u16_all(words: np.ndarray, offset: int = 0, out_offset: int = 0):
    ov = tuple(oracle.validate_utf16le(words))
    ol = tuple(oracle.utf8_length_from_utf16le(words))
    ob, oc = oracle.convert_utf16le_to_utf8(words)
    assert gpu_u16("validate", words, offset)[0] == ov
    assert gpu_u16("length", words, offset)[0] == ol
    r, (h, b), out = gpu_u16("convert", words, offset, out_offset=out_offset)
    assert r == tuple(oc)
    if r[0] == 0:
        assert np.array_equal(b[:r[1]], ob)
        out.check_guards(h, r[1])
    else:
        out.check_guards(h)
    return ov


# ---------------------------------------------------------------- 1 MiB buffer

@pytest.fixture(scope="module")
def mix1m():
    return wl.single_buffer(1 << 20)


def test_mixed_1mib_all_functions(mix1m):
    say("mixed 1 MiB, all six functions")
    assert check_u8_all(mix1m.u8) == (0, mix1m.u8.size)
    assert check_u16_all(mix1m.u16) == (0, mix1m.u16.size)


def test_mixed_1mib_injected_errors(mix1m):
    for kind, data, pos in wl.single_buffer_with_errors(mix1m):
        say("mixed 1 MiB with", kind, "at", pos)
        assert check_u8_all(data) == (getattr(oracle, kind), pos)


# ---------------------------------------------------------------- sizes and alignment

def test_small_sizes_and_offsets():
    text = wl.make_text("mix", 4096, wl.rng_for("small"))
    for offset in (0, 1, 7, 15):
        say("utf8 sizes 0..300 at offset", offset)
        for n in range(0, 301):
            check_u8_all(text.u8[:n], offset, out_offset=2 * (offset % 3))
    for offset in (0, 2, 14):
        say("utf16 sizes 0..300 at offset", offset)
        for n in range(0, 301):
            check_u16_all(text.u16[:n], offset, out_offset=offset % 5)


@pytest.mark.parametrize("profile", ["latin", "cyrillic", "cjk", "emoji", "mix"])
def test_decode_paths_at_edges(profile):
    """Each decode path (waves of one/two-byte characters, of up to three
    bytes, with four-byte characters) at the input's edges: sizes around
    chunk, wave, sub-tile and tile boundaries, cut at character starts,
    unaligned starts."""
    text = wl.make_text(profile, 70_000, wl.rng_for("paths", profile))
    sizes = (0, 1, 2, 3, 15, 16, 17, 255, 1023, 1024, 1025, 4095, 4096, 4097,
             16383, 16384, 16385, 24575, 24576, 24577, 65533, 65541)
    s8, s16 = text.char_starts_u8, text.char_starts_u16
    for offset in (0, 5, 15):
        say(profile, "utf8 edge sizes at offset", offset)
        for n in sizes:
            m = int(s8[np.searchsorted(s8, n, side="right") - 1]) if n < text.u8.size else text.u8.size
            check_u8_all(text.u8[:m], offset, out_offset=2 * (offset % 3))
    for offset in (0, 6, 14):
        say(profile, "utf16 edge sizes at offset", offset)
        for n in sizes:
            m = int(s16[np.searchsorted(s16, n, side="right") - 1]) if n < text.u16.size else text.u16.size
            check_u16_all(text.u16[:m], offset, out_offset=offset % 5)


def test_characters_split_across_wave_boundaries():
    """A three- or four-byte character that starts in the last chunk of a wave
    and ends in the next wave, whose own characters are all shorter (that wave
    decodes on a path for short characters and must still leave the split
    character's words alone), at wave, sub-tile and tile boundaries."""
    fillers = {"ascii": "abcdefgh", "two-byte": "aжbвcд", "three-byte": "a中b文"}
    for boundary in (1024, 4096, 16384):
        for ch in ("中", "😀"):
            for back in range(1, len(ch.encode()) ):
                for name, fill in fillers.items():
                    if len(ch.encode()) <= max(len(c.encode()) for c in fill):
                        continue
                    head = "x" * (boundary - back)
                    text = head + ch + (fill * (3000 // len(fill)))
                    u8 = np.frombuffer(text.encode("utf-8"), np.uint8)
                    u16 = np.frombuffer(text.encode("utf-16-le"), np.uint16)
                    say("split", repr(ch), "at", boundary, "-", back, "then", name)
                    check_u8_all(u8)
                    check_u16_all(u16)


def test_surrogate_pairs_split_across_utf16_boundaries():
    """A surrogate pair whose high word ends a chunk (8 words), a wave (512),
    a sub-tile (2048) or a tile (2048 and 4096 for inputs of this size) and
    whose low word starts the next: the low word's two UTF-8 bytes take two
    bits of the high word, read across the boundary. The words after it are
    of one kind (ASCII, two-byte, three-byte, more pairs), so the next
    chunk's wave takes each encoder path in turn; a lone high or low word at
    the same places must be flagged there."""
    fillers = {"ascii": "abcdefgh", "two-byte": "aжbвcд", "three-byte": "a中b文", "pairs": "😀a🎉b"}
    for boundary in (8, 512, 2048, 4096):
        for name, fill in fillers.items():
            for ch in ("😀", "\U0010FFFF", "\U00010000"):
                text = "x" * (boundary - 1) + ch + (fill * (6000 // len(fill)))
                u16 = np.frombuffer(text.encode("utf-16-le"), np.uint16)
                assert u16[boundary - 1] >> 10 == 0x36 and u16[boundary] >> 10 == 0x37
                say("pair split at word", boundary, repr(ch), "then", name)
                assert check_u16_all(u16)[0] == 0
            for w in (0xD83D, 0xDE00):
                bad = np.frombuffer(("x" * (boundary - 1) + "y" + fill * (6000 // len(fill))).encode("utf-16-le"),
                                    np.uint16).copy()
                bad[boundary - 1 if w < 0xDC00 else boundary] = w
                say("lone", hex(w), "at word", boundary, "then", name)
                assert check_u16_all(bad)[0] == 7   # UNPAIRED_SURROGATE


def test_four_byte_waves_with_one_short_lead():
    """Text of ASCII and four-byte characters only (a wave class whose decode
    leaves out the two- and three-byte forms) with one two- or three-byte
    character inserted at chunk positions of the first wave and around the
    first wave boundary: that wave must take the general four-byte decode and
    its neighbours the reduced one, with the same words either way."""
    base = "a\U0001F600b\U0001F30D" * 700
    for ch in ("\u00e9", "\u4e2d"):
        for k in list(range(0, 40, 3)) + list(range(400, 420, 2)):
            text = base[:k] + ch + base[k:]
            u8 = np.frombuffer(text.encode("utf-8"), np.uint8)
            u16 = np.frombuffer(text.encode("utf-16-le"), np.uint16)
            say("four-byte waves with", repr(ch), "at character", k)
            check_u8_all(u8)
            check_u16_all(u16)


@pytest.mark.parametrize("profile", ["latin", "cyrillic", "cjk"])
def test_errors_in_short_character_waves(profile):
    """Errors inside text of one/two-byte (Latin, Cyrillic) or up to
    three-byte (CJK) characters, where whole waves take the table-free checks:
    each ill-formed sequence must send its wave to the general check and come
    out with the oracle's kind and position, at chunk and wave boundaries."""
    text = wl.make_text(profile, 32 * 1024, wl.rng_for("short-waves", profile))
    seqs = [[0xC0, 0x80], [0xC1, 0xBF], [0xC3, 0x41], [0x80], [0xBF, 0x80], [0xC3, 0xA9, 0xA9],
            [0xE0, 0x80, 0x80], [0xE0, 0x9F, 0xBF], [0xED, 0xA0, 0x80], [0xED, 0xBF, 0xBF],
            [0xE4, 0xB8, 0x41], [0xE4, 0x41], [0xE4, 0xB8, 0xAD, 0x80], [0xEF, 0xBF]]
    starts = text.char_starts_u8[:-1]
    rng = np.random.default_rng(11)
    spots = [1024 * k + d for k in (3, 7, 19) for d in (-3, -1, 0, 1, 2)] + [16 * 5 + 15]
    spots += [int(x) for x in rng.integers(0, text.u8.size - 8, 6)]
    for seq in seqs:
        say(profile, "error sequence", bytes(seq).hex())
        for spot in spots:
            p = int(starts[np.searchsorted(starts, spot)])      # a character start at or after the spot
            data = text.u8.copy()
            data[p:p + len(seq)] = seq
            j = p + len(seq)
            while j < data.size and (data[j] & 0xC0) == 0x80:  # no leftover continuations
                data[j] = 0x20
                j += 1
            check_u8_all(data)


def test_power_of_two_sizes():
    text = wl.make_text("mix", (1 << 17) + 64, wl.rng_for("pow2"))
    for k in range(4, 18):
        for d in (-1, 0, 1):
            n = (1 << k) + d
            say("utf8/utf16 size", n)
            check_u8_all(text.u8[:n], offset=k % 16)
            check_u16_all(text.u16[:n], offset=2 * (k % 8))


# ---------------------------------------------------------------- errors near sub-tile boundaries
# (tile boundaries proper: tests/test_gpu_tile_boundaries.py)

def test_errors_around_sub_tile_boundaries():
    text = wl.make_text("mix", 3 * SUB + 100, wl.rng_for("tiles"))
    rng = np.random.default_rng(3)
    starts = text.char_starts_u8
    for offset in (0, 5):
        for boundary in (SUB, 2 * SUB):
            b = boundary - offset       # tile boundaries in input coordinates
            for d in range(-6, 7):
                for kind in wl.UTF8_ERROR_KINDS:
                    i = int(np.searchsorted(starts, b + d))
                    pos = int(starts[min(i, starts.size - 2)])
                    data, p = wl.inject_utf8_error(text.u8, starts, kind, rng, position=pos)
                    say("sub-tile boundary", boundary, "offset", offset, "delta", d, kind, "at", p)
                    ov = tuple(oracle.validate_utf8(data))
                    assert gpu_u8("validate", data, offset)[0] == ov
                    if ov[0] != 0:
                        assert gpu_u8("length", data, offset)[0] == ov
                    assert gpu_u8("convert", data, offset)[0] == tuple(oracle.convert_utf8_to_utf16le(data)[1])
                # arbitrary byte overwrites, not only at character boundaries
                for val in (0x80, 0xBF, 0xC2, 0xE4, 0xF0, 0xF4, 0xF8, 0x41):
                    data = text.u8.copy()
                    data[b + d] = val
                    ov = tuple(oracle.validate_utf8(data))
                    assert gpu_u8("validate", data, offset)[0] == ov, (boundary, d, hex(val))
    # UTF-16: unpaired surrogates around word tile boundaries
    w = text.u16
    for offset in (0, 6):
        for boundary in (SUB // 2, SUB):
            b = boundary - offset // 2
            for d in range(-3, 4):
                for val in (0xD800, 0xDBFF, 0xDC00, 0xDFFF):
                    data = w.copy()
                    data[b + d] = val
                    say("utf16 sub-tile boundary", boundary, "delta", d, hex(val))
                    check_u16_all(data, offset)


# ---------------------------------------------------------------- random short strings

def test_random_short_strings():
    alphabet = np.array([0x00, 0x41, 0x7F, 0x80, 0x8F, 0x90, 0x9F, 0xA0, 0xBF, 0xC0, 0xC1, 0xC2, 0xDF,
                         0xE0, 0xE1, 0xED, 0xEF, 0xF0, 0xF1, 0xF4, 0xF5, 0xF8, 0xFF], dtype=np.uint8)
    rng = np.random.default_rng(11)
    say("random short UTF-8 strings")
    for i in range(1500):
        n = int(rng.integers(1, 40))
        data = alphabet[rng.integers(0, alphabet.size, size=n)]
        if i % 3 == 0:   # embed in valid context
            data = np.concatenate([np.frombuffer(b"ab\xc3\xa9", np.uint8), data, np.frombuffer(b"z", np.uint8)])
        check_u8_all(data, offset=int(rng.integers(0, 16)))
    w_alpha = np.array([0x41, 0x7F, 0x80, 0x7FF, 0x800, 0xD7FF, 0xD800, 0xDBFF, 0xDC00, 0xDFFF, 0xE000,
                        0xFFFF], dtype=np.uint16)
    say("random short UTF-16 strings")
    for _ in range(800):
        n = int(rng.integers(1, 20))
        check_u16_all(w_alpha[rng.integers(0, w_alpha.size, size=n)], offset=2 * int(rng.integers(0, 8)))


# ---------------------------------------------------------------- capacity

def test_capacity_and_guards():
    text = wl.make_text("emoji", 10_000, wl.rng_for("cap"))
    n16 = text.u16.size
    for cap in (n16, n16 + 7, n16 - 1, n16 // 2, 1, 0):
        say("utf8->16 capacity", cap, "of", n16)
        r, (h, words), out = gpu_u8("convert", text.u8, 3, cap_words=cap, out_offset=2)
        if cap >= n16:
            assert r == (0, n16)
            assert np.array_equal(words[:n16], text.u16)
            out.check_guards(h, 2 * n16)
        else:
            assert r == (oracle.OUTPUT_TOO_SMALL, n16)
            out.check_guards(h)
    n8 = text.u8.size
    for cap in (n8, n8 + 1, n8 - 1, 100, 0):
        say("utf16->8 capacity", cap, "of", n8)
        r, (h, b), out = gpu_u16("convert", text.u16, 0, cap_bytes=cap, out_offset=1)
        if cap >= n8:
            assert r == (0, n8) and np.array_equal(b[:n8], text.u8)
            out.check_guards(h, n8)
        else:
            assert r == (oracle.OUTPUT_TOO_SMALL, n8)
            out.check_guards(h)


def test_invalid_arguments():
    say("invalid arguments")
    s = hu.stream_handle()
    assert _r(hu.lib.validate_utf8(None, 10, s)) == (hu.INVALID_ARGUMENT, 0)
    assert _r(hu.lib.validate_utf8(None, 0, s)) == (0, 0)
    buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
    assert _r(hu.lib.validate_utf16le(buf.data_ptr() + 1, 4, s)) == (hu.INVALID_ARGUMENT, 0)
    assert _r(hu.lib.convert_utf8_to_utf16le(buf.data_ptr(), 4, None, 4, s)) == (hu.INVALID_ARGUMENT, 0)
    assert _r(hu.lib.convert_utf8_to_utf16le(buf.data_ptr(), 4, buf.data_ptr() + 1, 4, s)) == \
        (hu.INVALID_ARGUMENT, 0)
    assert _r(hu.lib.convert_utf16le_to_utf8(buf.data_ptr(), 0, None, 0, s)) == (0, 0)


# ---------------------------------------------------------------- async entry points

def test_async_workspace_reuse():
    text = wl.make_text("cjk", 300_000, wl.rng_for("async"))
    src = torch.from_numpy(text.u8.copy()).cuda()
    ws = hu.workspace(hu.OP_CONVERT_UTF8_TO_UTF16LE, src.numel())
    wp, wb = hu.workspace_ptr(ws)
    rec = torch.zeros(16, dtype=torch.uint8, device="cuda")
    for n in (src.numel(), 1000, 77_777, src.numel()):
        say("async convert n =", n)
        dst = torch.zeros(n, dtype=torch.int16, device="cuda")
        rc = hu.lib.convert_utf8_to_utf16le_async(src.data_ptr(), n, dst.data_ptr(), n, rec.data_ptr(), wp, wb,
                                                  hu.stream_handle())
        assert rc == 0
        torch.cuda.synchronize()
        r = hu.result_from_device(rec)
        ow, orr = oracle.convert_utf8_to_utf16le(text.u8[:n])
        assert r == tuple(orr)
        if r.error == 0:
            assert np.array_equal(dst.cpu().numpy().view(np.uint16)[:r.count], ow)
    say("async calls with too-small workspaces")
    # validation needs the 256-byte header only, conversion also status words
    rc = hu.lib.validate_utf8_async(src.data_ptr(), src.numel(), rec.data_ptr(), wp, 128, hu.stream_handle())
    assert rc == hu.INVALID_ARGUMENT
    dst = torch.zeros(src.numel(), dtype=torch.int16, device="cuda")
    rc = hu.lib.convert_utf8_to_utf16le_async(src.data_ptr(), src.numel(), dst.data_ptr(), src.numel(),
                                              rec.data_ptr(), wp, 256, hu.stream_handle())
    assert rc == hu.INVALID_ARGUMENT
    assert hu.lib.hu_workspace_bytes(hu.OP_VALIDATE_UTF8, src.numel()) == 256
    rc = hu.lib.validate_utf8_async(src.data_ptr(), src.numel(), rec.data_ptr(), wp, 256, hu.stream_handle())
    assert rc == 0
    torch.cuda.synchronize()
    assert hu.result_from_device(rec) == tuple(oracle.validate_utf8(text.u8))


def test_repeat_determinism():
    text = wl.make_text("mix", 3_000_000, wl.rng_for("repeat"))
    src = torch.from_numpy(text.u8.copy()).cuda()
    say("repeat determinism x20")
    first = None
    for _ in range(20):
        words, r = hu.convert_utf8_to_utf16le(src)
        h = words.cpu().numpy()
        if first is None:
            first = h
            assert np.array_equal(h.view(np.uint16), text.u16)
        else:
            assert np.array_equal(h, first)


# ---------------------------------------------------------------- full-size profiles

@pytest.mark.parametrize("profile", wl.LARGE_PROFILES)
def test_large_profile_both_directions(profile):
    say("generating 256 MiB", profile)
    t = wl.large_profile(profile)
    src = torch.from_numpy(t.u8).cuda()
    say("256 MiB", profile, "utf8 -> utf16")
    words, r = hu.convert_utf8_to_utf16le(src)
    ow, orr = oracle.convert_utf8_to_utf16le(t.u8)
    assert r == tuple(orr) == (0, t.u16.size)
    assert np.array_equal(words.cpu().numpy().view(np.uint16), ow)        # the oracle's whole output
    assert hu.validate_utf8(src) == tuple(oracle.validate_utf8(t.u8))
    assert hu.utf16_length_from_utf8(src) == tuple(oracle.utf16_length_from_utf8(t.u8))
    say("256 MiB", profile, "utf16 -> utf8")
    back, r2 = hu.convert_utf16le_to_utf8(words)
    ob, orr2 = oracle.convert_utf16le_to_utf8(ow)
    assert r2 == tuple(orr2) == (0, t.u8.size)
    assert np.array_equal(back.cpu().numpy(), ob)
    assert hu.validate_utf16le(words) == tuple(oracle.validate_utf16le(ow))
    assert hu.utf8_length_from_utf16le(words) == tuple(oracle.utf8_length_from_utf16le(ow))
    del ow, ob
    starts = t.char_starts_u8
    # one error late in the buffer
    bad = src.clone()
    p = int(starts[starts.size - 1000])
    bad[p] = 0xFF
    say("256 MiB", profile, "bad lead at", p)
    assert hu.validate_utf8(bad) == (hu.BAD_LEAD, p)
    assert hu.convert_utf8_to_utf16le(bad)[1] == (hu.BAD_LEAD, p)
    del src, words, back, bad
    torch.cuda.empty_cache()
