"""Pins for the CPU oracle, against sources other than the oracle itself:
values printed in the paper (tests/golden), CPython's codecs, an independently
written table classifier, closed-form counts and brute force on tiny inputs."""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
from tests.table_classifier import (all_strings, utf16_valid_prefix, utf8_valid_prefix,
                                    valid_count_recurrence)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
KIND = {v: k for k, v in oracle.KIND_NAMES.items()}


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line.split()


# ------------------------------------------------------------------ paper values

def test_worked_example_section3():
    rows = list(_rows("worked_example.txt"))
    assert rows
    for row in rows:
        cp = int(row[0], 16)
        u8 = bytes(int(x, 16) for x in row[1:])
        words, r = oracle.convert_utf8_to_utf16le(u8)
        assert r == (oracle.OK, 1) and words.tolist() == [cp]
        out, r = oracle.convert_utf16le_to_utf8(np.array([cp], dtype=np.uint16))
        assert r == (oracle.OK, len(u8)) and out.tobytes() == u8


def test_table_utfsummary_lengths():
    rows = list(_rows("utfsummary.txt"))
    assert len(rows) == 10
    for cp_hex, n8, n16, _name in rows:
        cp, n8, n16 = int(cp_hex, 16), int(n8), int(n16)
        u8 = chr(cp).encode("utf-8")
        u16 = chr(cp).encode("utf-16-le")
        assert (len(u8), len(u16)) == (n8, n16)          # the table agrees with CPython
        assert oracle.utf16_length_from_utf8(u8) == (oracle.OK, n16 // 2)
        assert oracle.utf8_length_from_utf16le(u16) == (oracle.OK, n8)
        assert oracle.validate_utf8(u8) == (oracle.OK, n8)
        assert oracle.validate_utf16le(u16) == (oracle.OK, n16 // 2)


@pytest.mark.parametrize("name", ["error_kinds.txt"])
def test_utf8_error_kinds_golden(name):
    rows = list(_rows(name))
    per_kind = {}
    for row in rows:
        *hexes, pos, kind = row
        data = bytes(int(x, 16) for x in hexes)
        expect = (KIND[kind], int(pos))
        assert oracle.validate_utf8(data) == expect, (hexes, kind)
        assert oracle.utf16_length_from_utf8(data) == expect
        assert oracle.convert_utf8_to_utf16le(data)[1] == expect
        # the position is the end of the longest valid prefix (brute force)
        P = max(p for p in range(len(data) + 1) if _cpython_valid8(data[:p]))
        assert P == int(pos)
        per_kind[kind] = per_kind.get(kind, 0) + 1
    assert all(per_kind.get(k, 0) >= 3 for k in
               ("BAD_LEAD", "TRUNCATED", "STRAY_CONTINUATION", "OVERLONG", "TOO_LARGE", "SURROGATE"))


def test_utf16_errors_golden():
    for row in _rows("utf16_errors.txt"):
        *hexes, pos, kind = row
        words = np.array([int(x, 16) for x in hexes], dtype=np.uint16)
        expect = (KIND[kind], int(pos))
        assert oracle.validate_utf16le(words) == expect
        assert oracle.utf8_length_from_utf16le(words) == expect
        assert oracle.convert_utf16le_to_utf8(words)[1] == expect
        with pytest.raises(UnicodeDecodeError) as ei:
            words.astype("<u2").tobytes().decode("utf-16-le")
        assert ei.value.start == int(pos)


def _cpython_valid8(b: bytes) -> bool:
    try:
        b.decode("utf-8")
        return True
    except UnicodeDecodeError:
        return False


# ------------------------------------------------------------------ every scalar value

def _all_scalars():
    cps = np.arange(0x110000, dtype=np.uint32)
    return cps[(cps < 0xD800) | (cps > 0xDFFF)]


def test_roundtrip_every_scalar_value():
    cps = _all_scalars()
    assert cps.size == 1_112_064 == 128 + 1920 + 61440 + 1048576
    s = cps.astype("<u4").tobytes().decode("utf-32-le")
    u8 = np.frombuffer(s.encode("utf-8"), dtype=np.uint8)
    u16 = np.frombuffer(s.encode("utf-16-le"), dtype="<u2")
    words, r = oracle.convert_utf8_to_utf16le(u8)
    assert r == (oracle.OK, u16.size)
    assert np.array_equal(words, u16)
    back, r = oracle.convert_utf16le_to_utf8(u16)
    assert r == (oracle.OK, u8.size)
    assert np.array_equal(back, u8)
    assert oracle.validate_utf8(u8) == (oracle.OK, u8.size)
    assert oracle.validate_utf16le(u16) == (oracle.OK, u16.size)
    assert oracle.utf16_length_from_utf8(u8) == (oracle.OK, u16.size)
    assert oracle.utf8_length_from_utf16le(u16) == (oracle.OK, u8.size)


def test_each_scalar_alone_per_range():
    # one call per character at the ends of each range and a sample inside:
    # catches errors that a concatenation could hide
    rng = np.random.default_rng(7)
    cps = _all_scalars()
    pick = np.unique(np.concatenate([
        [0, 0x7F, 0x80, 0x7FF, 0x800, 0xD7FF, 0xE000, 0xFFFF, 0x10000, 0x10FFFF],
        rng.choice(cps, 4000, replace=False)]))
    for cp in pick:
        ch = chr(int(cp))
        u8, u16 = ch.encode("utf-8"), ch.encode("utf-16-le")
        w, r = oracle.convert_utf8_to_utf16le(u8)
        assert r.error == oracle.OK and w.astype("<u2").tobytes() == u16
        b, r = oracle.convert_utf16le_to_utf8(u16)
        assert r.error == oracle.OK and b.tobytes() == u8


# ------------------------------------------------------------------ exhaustive short strings

def _oracle_prefix8(S):
    N, L = S.shape
    errs, counts = oracle.many_validate_utf8(S.reshape(-1), np.arange(N + 1, dtype=np.uint64) * L)
    return np.where(errs == 0, L, counts).astype(np.int64), errs


@pytest.mark.parametrize("L", [1, 2, 3])
def test_exhaustive_utf8_strings(L):
    S = all_strings(L)
    P_tab = utf8_valid_prefix(S)
    P_or, errs = _oracle_prefix8(S)
    assert np.array_equal(P_tab, P_or)
    assert int((errs == 0).sum()) == valid_count_recurrence(L) == {1: 128, 2: 18_304, 3: 2_650_112}[L]
    # every kind that fits in L bytes occurs (a value above U+10FFFF needs 4 bytes)
    kinds = {1: {0, 1, 2, 3}, 2: {0, 1, 2, 3, 4}, 3: {0, 1, 2, 3, 4, 6}}[L]
    assert set(np.unique(errs).tolist()) == kinds
    # length function agrees with validation on every string
    e2, c2 = oracle.many_utf16_length_from_utf8(S.reshape(-1), np.arange(S.shape[0] + 1, dtype=np.uint64) * L)
    assert np.array_equal(e2, errs)
    bad = errs != 0
    assert np.array_equal(c2[bad], P_or[bad])


def test_structured_4byte_strings():
    edge = np.array([0x00, 0x7F, 0x80, 0x8F, 0x90, 0x9F, 0xA0, 0xBF, 0xC0, 0xF4, 0xF5, 0xFF], dtype=np.uint8)
    b01 = all_strings(2)
    b23 = np.stack(np.meshgrid(edge, edge, indexing="ij"), axis=-1).reshape(-1, 2)
    S = np.concatenate([np.repeat(b01, b23.shape[0], axis=0), np.tile(b23, (b01.shape[0], 1))], axis=1)
    P_tab = utf8_valid_prefix(S)
    P_or, errs = _oracle_prefix8(S)
    assert np.array_equal(P_tab, P_or)
    assert set(np.unique(errs).tolist()) == {0, 1, 2, 3, 4, 5, 6}


def test_utf16_single_words_and_pairs():
    W1 = np.arange(65536, dtype=np.uint16).reshape(-1, 1)
    errs, counts = oracle.many_validate_utf16le(W1.reshape(-1), np.arange(65537, dtype=np.uint64))
    assert int((errs == 0).sum()) == 63_488
    assert np.array_equal(np.where(errs == 0, 1, counts // 2), utf16_valid_prefix(W1))
    edge = np.array([0, 0x7F, 0x80, 0x7FF, 0x800, 0xD7FF, 0xD800, 0xDBFF, 0xDC00, 0xDFFF, 0xE000, 0xFFFF],
                    dtype=np.uint16)
    allw = np.arange(65536, dtype=np.uint16)
    W2 = np.concatenate([
        np.stack([np.repeat(allw, edge.size), np.tile(edge, allw.size)], axis=1),
        np.stack([np.repeat(edge, allw.size), np.tile(allw, edge.size)], axis=1)])
    N = W2.shape[0]
    errs, counts = oracle.many_validate_utf16le(W2.reshape(-1), np.arange(N + 1, dtype=np.uint64) * 2)
    P_or = np.where(errs == 0, 2, counts // 2)
    assert np.array_equal(P_or, utf16_valid_prefix(W2))
    assert set(np.unique(errs).tolist()) == {0, 7}
    # valid two-word strings: BMP x BMP non-surrogates, or one surrogate pair
    assert 63_488 ** 2 + 1024 ** 2 == 4_031_774_720


# ------------------------------------------------------------------ CPython cross-checks

def _random_mutations(rng, base: bytes, n: int):
    out = []
    for _ in range(n):
        b = bytearray(base)
        for _ in range(int(rng.integers(1, 4))):
            op = rng.integers(0, 3)
            p = int(rng.integers(0, len(b) + 1))
            if op == 0:
                b[p:p] = bytes([int(rng.integers(0, 256))])
            elif op == 1 and p < len(b):
                b[p] = int(rng.integers(0, 256))
            elif p < len(b):
                del b[p]
        out.append(bytes(b))
    return out


def test_first_error_matches_cpython_utf8():
    rng = np.random.default_rng(2109)
    base = "aé中\U0001F600z߿ࠀ￿\U0010FFFF\u0080".encode()
    seen_bad = 0
    for data in _random_mutations(rng, base, 4000):
        r = oracle.validate_utf8(data)
        try:
            s = data.decode("utf-8")
        except UnicodeDecodeError as e:
            seen_bad += 1
            assert r.error != oracle.OK and r.count == e.start, data.hex()
            continue
        assert r == (oracle.OK, len(data))
        w, r2 = oracle.convert_utf8_to_utf16le(data)
        assert r2.error == oracle.OK and w.astype("<u2").tobytes() == s.encode("utf-16-le")
    assert seen_bad > 1000


def test_first_error_matches_cpython_utf16():
    rng = np.random.default_rng(10433)
    pool = np.array([0x41, 0x7F, 0x80, 0x7FF, 0x800, 0xD7FF, 0xE000, 0xFFFF, 0xD800, 0xDBFF, 0xDC00, 0xDFFF,
                     0xD83D, 0xDE00], dtype=np.uint16)
    seen_bad = 0
    for _ in range(4000):
        words = pool[rng.integers(0, pool.size, size=int(rng.integers(1, 9)))]
        data = words.astype("<u2").tobytes()
        r = oracle.validate_utf16le(words)
        try:
            s = data.decode("utf-16-le")
        except UnicodeDecodeError as e:
            seen_bad += 1
            assert r == (oracle.UNPAIRED_SURROGATE, e.start)
            continue
        assert r == (oracle.OK, words.size)
        b, r2 = oracle.convert_utf16le_to_utf8(words)
        assert r2.error == oracle.OK and b.tobytes() == s.encode("utf-8")
    assert seen_bad > 1000


# ------------------------------------------------------------------ invariants and edges

def test_empty_inputs():
    assert oracle.validate_utf8(b"") == (oracle.OK, 0)
    assert oracle.utf16_length_from_utf8(b"") == (oracle.OK, 0)
    assert oracle.convert_utf8_to_utf16le(b"")[1] == (oracle.OK, 0)
    e16 = np.zeros(0, np.uint16)
    assert oracle.validate_utf16le(e16) == (oracle.OK, 0)
    assert oracle.utf8_length_from_utf16le(e16) == (oracle.OK, 0)
    assert oracle.convert_utf16le_to_utf8(e16)[1] == (oracle.OK, 0)


def test_truncation_respects_input_length():
    # the bytes that would complete the character sit in memory just past the
    # end of the input: they must not be read as part of it
    buf = np.frombuffer(b"A\xe4\xb8\xadA\xf0\x9f\x98\x80", dtype=np.uint8)
    assert oracle.validate_utf8(buf[:3]) == (oracle.TRUNCATED, 1)
    assert oracle.validate_utf8(buf[:2]) == (oracle.TRUNCATED, 1)
    assert oracle.validate_utf8(buf[:7]) == (oracle.TRUNCATED, 5)
    assert oracle.utf16_length_from_utf8(buf[:8]) == (oracle.TRUNCATED, 5)
    assert oracle.convert_utf8_to_utf16le(buf[:3])[1] == (oracle.TRUNCATED, 1)
    w = np.frombuffer("A\U0001F600".encode("utf-16-le"), dtype="<u2")
    assert oracle.validate_utf16le(w[:2]) == (oracle.UNPAIRED_SURROGATE, 2)
    assert oracle.convert_utf16le_to_utf8(w[:2])[1] == (oracle.UNPAIRED_SURROGATE, 2)


def test_capacity_rules():
    data = "a\U0001F600".encode()            # 3 words
    assert oracle.convert_utf8_to_utf16le(data, 3)[1] == (oracle.OK, 3)
    assert oracle.convert_utf8_to_utf16le(data, 2)[1] == (oracle.OUTPUT_TOO_SMALL, 3)
    assert oracle.convert_utf8_to_utf16le(data, 0)[1] == (oracle.OUTPUT_TOO_SMALL, 3)
    w = np.frombuffer("中中".encode("utf-16-le"), dtype="<u2")
    assert oracle.convert_utf16le_to_utf8(w, 6)[1] == (oracle.OK, 6)
    assert oracle.convert_utf16le_to_utf8(w, 5)[1] == (oracle.OUTPUT_TOO_SMALL, 6)
    # a validation error wins over a capacity shortfall
    assert oracle.convert_utf8_to_utf16le(b"aaaa\x80", 1)[1] == (oracle.STRAY_CONTINUATION, 4)


def test_lengths_equal_converted_lengths_and_roundtrip():
    from paper_2109_10433_amd import workloads as wl
    for prof in wl.PROFILES:
        t = wl.make_text(prof, 200_003, wl.rng_for("pins", prof))
        w, r = oracle.convert_utf8_to_utf16le(t.u8)
        assert r == (oracle.OK, t.u16.size) and np.array_equal(w, t.u16)
        assert oracle.utf16_length_from_utf8(t.u8) == (oracle.OK, t.u16.size)
        b, r = oracle.convert_utf16le_to_utf8(w)
        assert r == (oracle.OK, t.u8.size) and np.array_equal(b, t.u8)
        assert oracle.utf8_length_from_utf16le(w) == (oracle.OK, t.u8.size)


def test_many_input_helpers_equal_single_calls():
    """The batch helpers (inputs anywhere in host memory) return what the
    single calls return, input by input, and convert into the given buffers."""
    from paper_2109_10433_amd import workloads as wl
    rng = np.random.default_rng(21)
    text = wl.make_text("mix", 50_000, wl.rng_for("many-helpers"))
    docs8, docs16 = [], []
    for k in range(60):
        a, b = sorted(int(x) for x in rng.integers(0, text.u8.size, 2))
        d = text.u8[a:b].copy()
        if k % 3 == 0 and d.size:
            d[int(rng.integers(0, d.size))] = rng.choice([0x80, 0xC0, 0xED, 0xF8])
        docs8.append(d)
        a, b = sorted(int(x) for x in rng.integers(0, text.u16.size, 2))
        w = text.u16[a:b].copy()
        if k % 4 == 0 and w.size:
            w[int(rng.integers(0, w.size))] = 0xDC00
        docs16.append(w)
    for utf16, docs, single in ((False, docs8, (oracle.validate_utf8, oracle.utf16_length_from_utf8)),
                                (True, docs16, (oracle.validate_utf16le, oracle.utf8_length_from_utf16le))):
        addrs = [d.ctypes.data for d in docs]
        units = [d.size for d in docs]
        for op in (0, 1):
            errs, counts = oracle.many_at(op, utf16, addrs, units)
            assert [tuple(single[op](d)) for d in docs] == list(zip(errs.tolist(), counts.tolist()))
        caps = [3 * d.size if utf16 else d.size for d in docs]
        outs = [np.full(max(c, 1), 0xEE, np.uint8 if utf16 else np.uint16) for c in caps]
        errs, counts = oracle.many_convert_at(utf16, addrs, units, [o.ctypes.data for o in outs], caps)
        for d, o, e, c in zip(docs, outs, errs, counts):
            ref, r = (oracle.convert_utf16le_to_utf8 if utf16 else oracle.convert_utf8_to_utf16le)(d)
            assert (int(e), int(c)) == tuple(r)
            if r.error == 0:
                assert np.array_equal(o[:r.count], ref)
