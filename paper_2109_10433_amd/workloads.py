"""Seeded synthetic text for tests and benchmarks.

Holds none of the transcoding arithmetic: characters are drawn as code points
from fixed ranges (each range has a known UTF-8 length class), and encoded to
UTF-8 / UTF-16LE with CPython's built-in codecs. Both the GPU parity tests and
the CPU oracle consume what this module produces; expected results always come
from the oracle, never from here.

The profiles stand in for the paper's data files (section 6.3, Table "data"),
which are not available: their per-length character mixes follow that table
(Latin ~ lipsum Latin / English, Cyrillic ~ lipsum and Mars Russian, CJK ~
lipsum Chinese / Japanese, Emoji ~ lipsum Emoji).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

BASE_SEED = 210910433
MIB = 1 << 20

_ASCII_PRINTABLE = np.arange(0x20, 0x7F, dtype=np.uint32)
_ASCII_SPACE_PUNCT = np.array([ord(c) for c in " ,.;:!?-'\"()"], dtype=np.uint32)


@dataclass(frozen=True)
class CharClass:
    prob: float
    utf8_len: int          # by construction of the ranges below
    ranges: tuple          # inclusive (lo, hi) code point ranges, drawn uniformly over their union
    alphabet: tuple = ()   # explicit list instead of ranges


def _cls(prob, utf8_len, *ranges):
    return CharClass(prob, utf8_len, tuple(ranges))


PROFILES = {
    # 70/10/15/5 % of characters by encoded length, uniform within each range
    "mix": (
        _cls(0.70, 1, (0x20, 0x7E)),
        _cls(0.10, 2, (0x80, 0x7FF)),
        _cls(0.15, 3, (0x800, 0xD7FF), (0xE000, 0xFFFF)),
        _cls(0.05, 4, (0x10000, 0x10FFFF)),
    ),
    "latin": (
        _cls(0.98, 1, (0x20, 0x7E)),
        _cls(0.02, 2, (0xC0, 0x17F)),
    ),
    "cyrillic": (
        CharClass(0.45, 1, (), tuple(int(c) for c in _ASCII_SPACE_PUNCT)),
        _cls(0.55, 2, (0x400, 0x4FF)),
    ),
    "cjk": (
        _cls(0.10, 1, (0x20, 0x7E)),
        _cls(0.90, 3, (0x4E00, 0x9FFF)),
    ),
    "emoji": (
        _cls(0.10, 1, (0x20, 0x7E)),
        _cls(0.90, 4, (0x1F300, 0x1FAFF)),
    ),
}
LARGE_PROFILES = ("latin", "cyrillic", "cjk", "emoji")
BATCH_PROFILES = ("mix", "latin", "cyrillic", "cjk", "emoji")

# error kinds injected into UTF-8 text (names match the library's error kinds)
UTF8_ERROR_KINDS = ("OVERLONG", "SURROGATE", "TOO_LARGE", "TRUNCATED", "STRAY_CONTINUATION", "BAD_LEAD")


def rng_for(*key) -> np.random.Generator:
    """PCG64 stream for a (config, purpose, ...) key under the base seed."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([BASE_SEED, *[hash_key(k) for k in key]])))


def hash_key(k) -> int:
    if isinstance(k, int):
        return k & 0xFFFFFFFF
    h = 2166136261
    for ch in str(k).encode():
        h = ((h ^ ch) * 16777619) & 0xFFFFFFFF
    return h


def _draw_class(rng, cc: CharClass, n: int) -> np.ndarray:
    if cc.alphabet:
        alpha = np.asarray(cc.alphabet, dtype=np.uint32)
        return alpha[rng.integers(0, alpha.size, size=n, dtype=np.uint32)]
    if len(cc.ranges) == 1:
        lo, hi = cc.ranges[0]
        return rng.integers(lo, hi + 1, size=n, dtype=np.uint32)
    sizes = np.array([hi - lo + 1 for lo, hi in cc.ranges], dtype=np.int64)
    k = rng.integers(0, int(sizes.sum()), size=n, dtype=np.uint32)
    out = k.copy()
    base = 0
    for (lo, hi), sz in zip(cc.ranges, sizes):
        sel = (k >= base) & (k < base + sz)
        out[sel] = lo + (k[sel] - base)
        base += sz
    return out


@dataclass
class Text:
    """A synthetic text: code points plus their encodings (CPython codecs)."""
    cps: np.ndarray        # uint32 code points
    utf8_len: np.ndarray   # uint8 per character (by construction)
    u8: np.ndarray         # uint8 UTF-8 bytes
    u16: np.ndarray        # uint16 UTF-16LE code units

    @property
    def char_starts_u8(self) -> np.ndarray:
        """Byte offset of every character (plus the end)."""
        return np.concatenate([[0], np.cumsum(self.utf8_len, dtype=np.int64)])

    @property
    def char_starts_u16(self) -> np.ndarray:
        """Word offset of every character (plus the end); 4-byte UTF-8 characters are pairs."""
        return np.concatenate([[0], np.cumsum(1 + (self.utf8_len == 4), dtype=np.int64)])


def encode_utf8(cps: np.ndarray) -> np.ndarray:
    s = np.ascontiguousarray(cps, dtype="<u4").tobytes().decode("utf-32-le")
    return np.frombuffer(s.encode("utf-8"), dtype=np.uint8)


def encode_utf16le(cps: np.ndarray) -> np.ndarray:
    s = np.ascontiguousarray(cps, dtype="<u4").tobytes().decode("utf-32-le")
    return np.frombuffer(s.encode("utf-16-le"), dtype="<u2")


def _make_codepoints(profile: str, n_bytes: int, rng: np.random.Generator):
    classes = PROFILES[profile]
    probs = np.array([c.prob for c in classes])
    cdf = np.cumsum(probs / probs.sum())
    lens = np.array([c.utf8_len for c in classes], dtype=np.uint8)
    mean = float((probs / probs.sum() * lens).sum())
    cps_parts, len_parts, total = [], [], 0
    while total < n_bytes:
        m = int((n_bytes - total) / mean * 1.01) + 16
        cls = np.searchsorted(cdf, rng.random(m, dtype=np.float32), side="right").astype(np.uint8)
        np.minimum(cls, len(classes) - 1, out=cls)
        cps = np.empty(m, dtype=np.uint32)
        for i, cc in enumerate(classes):
            sel = cls == i
            cps[sel] = _draw_class(rng, cc, int(np.count_nonzero(sel)))
        clen = lens[cls]
        cps_parts.append(cps)
        len_parts.append(clen)
        total += int(clen.sum(dtype=np.int64))
    cps = np.concatenate(cps_parts) if len(cps_parts) > 1 else cps_parts[0]
    clen = np.concatenate(len_parts) if len(len_parts) > 1 else len_parts[0]
    cum = np.cumsum(clen, dtype=np.int64)
    k = int(np.searchsorted(cum, n_bytes, side="right"))
    used = int(cum[k - 1]) if k else 0
    pad = n_bytes - used
    cps = np.concatenate([cps[:k], np.full(pad, 0x20, dtype=np.uint32)])
    clen = np.concatenate([clen[:k], np.ones(pad, dtype=np.uint8)])
    return cps, clen


_PIECE = 16 * MIB


def make_text(profile: str, n_bytes: int, rng: np.random.Generator, encode16: bool = True) -> Text:
    """Text of exactly ``n_bytes`` UTF-8 bytes: characters drawn from the
    profile. Large texts are drawn as independent 16 MiB pieces (each cut at
    its last whole character and padded with U+0020), in parallel threads."""
    if n_bytes <= _PIECE:
        cps, clen = _make_codepoints(profile, n_bytes, rng)
    else:
        from concurrent.futures import ThreadPoolExecutor
        seeds = rng.integers(0, 2**63 - 1, size=(n_bytes + _PIECE - 1) // _PIECE)
        sizes = [min(_PIECE, n_bytes - i * _PIECE) for i in range(seeds.size)]
        with ThreadPoolExecutor(max_workers=8) as ex:
            parts = list(ex.map(lambda a: _make_codepoints(profile, a[1], np.random.Generator(np.random.PCG64(int(a[0])))),
                                zip(seeds, sizes)))
        cps = np.concatenate([p[0] for p in parts])
        clen = np.concatenate([p[1] for p in parts])
    u8 = encode_utf8(cps)
    assert u8.size == n_bytes
    u16 = encode_utf16le(cps) if encode16 else np.zeros(0, dtype=np.uint16)
    return Text(cps, clen, u8, u16)


# ---------------------------------------------------------------- error injection

def _cont(rng, lo=0x80, hi=0xBF, n=1):
    return [int(x) for x in rng.integers(lo, hi + 1, size=n)]


def utf8_error_sequence(kind: str, rng: np.random.Generator) -> list:
    """A short ill-formed byte sequence of the named kind (the kind that the
    first-error rules assign is checked against the oracle by the tests)."""
    if kind == "OVERLONG":
        v = int(rng.integers(0, 3))
        if v == 0:
            return [int(rng.integers(0xC0, 0xC2))] + _cont(rng)
        if v == 1:
            return [0xE0] + _cont(rng, 0x80, 0x9F) + _cont(rng)
        return [0xF0] + _cont(rng, 0x80, 0x8F) + _cont(rng, n=2)
    if kind == "SURROGATE":
        return [0xED] + _cont(rng, 0xA0, 0xBF) + _cont(rng)
    if kind == "TOO_LARGE":
        if rng.integers(0, 2) == 0:
            return [0xF4] + _cont(rng, 0x90, 0xBF) + _cont(rng, n=2)
        return [int(rng.integers(0xF5, 0xF8))] + _cont(rng, n=3)
    if kind == "TRUNCATED":
        ln = int(rng.integers(2, 5))
        seq = encode_utf8(np.array([{2: 0x4A9, 3: 0x6F22, 4: 0x1F600}[ln]], dtype=np.uint32)).tolist()
        return seq[: int(rng.integers(1, ln))]
    if kind == "STRAY_CONTINUATION":
        return _cont(rng)
    if kind == "BAD_LEAD":
        return [int(rng.integers(0xF8, 0x100))]
    raise ValueError(kind)


def inject_utf8_error(u8: np.ndarray, char_starts: np.ndarray, kind: str, rng: np.random.Generator,
                      position: int | None = None):
    """Copy of ``u8`` (same length) with an ill-formed sequence written at a
    character boundary. Continuation bytes left over from overwritten characters
    are replaced by U+0020 so that the injected sequence is what it claims.
    Returns (bytes, boundary position used)."""
    seq = utf8_error_sequence(kind, rng)
    n = u8.size
    starts = char_starts[:-1]
    starts = starts[starts + len(seq) + 1 <= n]
    if position is None:
        position = int(starts[rng.integers(0, starts.size)])
    out = u8.copy()
    out[position:position + len(seq)] = seq
    j = position + len(seq)
    while j < n and (out[j] & 0xC0) == 0x80:
        out[j] = 0x20
        j += 1
    return out, position


def inject_utf16_error(u16: np.ndarray, char_starts: np.ndarray, rng: np.random.Generator,
                       position: int | None = None):
    """Copy of ``u16`` with a lone high surrogate (followed by a non-low word) or
    a lone low surrogate (not preceded by a high word) at a character boundary.
    Returns (words, word index used)."""
    out = u16.copy()
    n = u16.size
    starts = char_starts[:-1]
    if position is None:
        position = int(starts[rng.integers(0, starts.size)])
    high = bool(rng.integers(0, 2))
    if high:
        out[position] = int(rng.integers(0xD800, 0xDC00))
        if position + 1 < n and 0xDC00 <= out[position + 1] <= 0xDFFF:
            out[position + 1] = 0x20
    else:
        # overwrite a whole character so no high word precedes the low one
        out[position] = int(rng.integers(0xDC00, 0xE000))
        if position + 1 < n and 0xDC00 <= out[position + 1] <= 0xDFFF:
            out[position + 1] = 0x20
    return out, position


# ---------------------------------------------------------------- configurations

def single_buffer(n_bytes: int = MIB, profile: str = "mix", seed_key="cfg1") -> Text:
    """One buffer of exactly n_bytes UTF-8 (default: the 1 MiB mixed buffer)."""
    return make_text(profile, n_bytes, rng_for(seed_key, profile, n_bytes))


def single_buffer_with_errors(text: Text, seed_key="cfg1-errors"):
    """One copy per UTF-8 error kind: list of (kind, bytes, injected position)."""
    rng = rng_for(seed_key, text.u8.size)
    starts = text.char_starts_u8
    out = []
    for kind in UTF8_ERROR_KINDS:
        b, pos = inject_utf8_error(text.u8, starts, kind, rng)
        out.append((kind, b, pos))
    return out


def large_profile(profile: str, n_bytes: int = 256 * MIB) -> Text:
    return make_text(profile, n_bytes, rng_for("cfg2", profile, n_bytes))


@dataclass
class DocBatch:
    data: np.ndarray        # concatenated documents (uint8 for UTF-8, uint16 for UTF-16LE)
    offsets: np.ndarray     # int64, n_docs + 1, in input units
    profiles: np.ndarray    # profile index per document (into BATCH_PROFILES)
    injected: np.ndarray    # bool per document: carries an injected error


def _lognormal_lengths(rng, n, median, sigma, lo, hi):
    x = np.exp(np.log(median) + sigma * rng.standard_normal(n))
    return np.clip(np.round(x), lo, hi).astype(np.int64)


def utf8_documents(n_docs: int = 100_000, median: int = 2048, sigma: float = 1.5,
                   lo: int = 16, hi: int = MIB, error_frac: float = 0.01,
                   pool_bytes: int | None = None, seed_key="cfg3") -> DocBatch:
    """Many UTF-8 documents with log-normal byte lengths, each a character-
    aligned slice of one profile's text pool; a fraction carry one injected
    error of a uniformly drawn kind."""
    rng = rng_for(seed_key, n_docs)
    want = _lognormal_lengths(rng, n_docs, median, sigma, lo, hi)
    prof = rng.integers(0, len(BATCH_PROFILES), size=n_docs)
    if pool_bytes is None:
        pool_bytes = int(min(max(4 * hi, 2 * want.sum() // len(BATCH_PROFILES)), 256 * MIB))
    pools = [make_text(p, pool_bytes, rng_for(seed_key, "pool", p, pool_bytes), encode16=False)
             for p in BATCH_PROFILES]
    pool_starts = [t.char_starts_u8 for t in pools]
    parts, lens = [], np.zeros(n_docs, dtype=np.int64)
    inj = rng.random(n_docs) < error_frac
    for d in range(n_docs):
        t, cs = pools[prof[d]], pool_starts[prof[d]]
        max_start = cs.size - 1
        i = int(rng.integers(0, max_start))
        b0 = int(cs[i])
        j = int(np.searchsorted(cs, b0 + want[d], side="right")) - 1
        j = max(j, i)
        doc = t.u8[b0:int(cs[j])]
        if inj[d] and doc.size >= 8:
            kind = UTF8_ERROR_KINDS[int(rng.integers(0, len(UTF8_ERROR_KINDS)))]
            doc, _ = inject_utf8_error(doc, cs[i:j + 1] - b0, kind, rng)
        else:
            inj[d] = False
        parts.append(doc)
        lens[d] = doc.size
    offsets = np.concatenate([[0], np.cumsum(lens)])
    return DocBatch(np.concatenate(parts) if parts else np.zeros(0, np.uint8), offsets, prof, inj)


@dataclass
class DocSpec16:
    """UTF-16LE documents described by reference: each is a slice of one
    profile's pool with at most two words replaced (the injected error), so a
    multi-GiB batch can be assembled on the device from the pools without a
    host copy of the whole batch."""
    pools: list             # per profile (BATCH_PROFILES order): Text with u16
    profiles: np.ndarray    # profile index per document
    start: np.ndarray       # int64 word offset of the slice in its pool
    length: np.ndarray      # int64 words
    inj_pos: np.ndarray     # int64 word index of the injected error in the document, -1 if none
    inj_words: np.ndarray   # uint16 (n, 2): words at inj_pos, inj_pos + 1 after injection

    @property
    def injected(self) -> np.ndarray:
        return self.inj_pos >= 0

    @property
    def offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.length)]).astype(np.int64)

    def doc(self, d: int) -> np.ndarray:
        """Words of document d (a fresh array)."""
        t = self.pools[self.profiles[d]]
        w = t.u16[self.start[d]:self.start[d] + self.length[d]].copy()
        p = int(self.inj_pos[d])
        if p >= 0:
            w[p] = self.inj_words[d, 0]
            if p + 1 < w.size:
                w[p + 1] = self.inj_words[d, 1]
        return w

    def utf8_bytes(self, d: int) -> int:
        """UTF-8 length of document d when it carries no injected error."""
        t = self.pools[self.profiles[d]]
        cs16 = self._starts16[self.profiles[d]]
        i = int(np.searchsorted(cs16, self.start[d]))
        j = int(np.searchsorted(cs16, self.start[d] + self.length[d]))
        cs8 = self._starts8[self.profiles[d]]
        return int(cs8[j] - cs8[i])

    def __post_init__(self):
        self._starts16 = [t.char_starts_u16 for t in self.pools]
        self._starts8 = [t.char_starts_u8 for t in self.pools]

    def materialize(self) -> DocBatch:
        parts = [self.doc(d) for d in range(self.length.size)]
        data = np.concatenate(parts) if parts else np.zeros(0, np.uint16)
        return DocBatch(data, self.offsets, self.profiles, self.injected)


def utf16_document_spec(n_docs: int = 10_000, lo_bytes: int = 64, hi_bytes: int = 4 * MIB,
                        error_frac: float = 0.005, pool_bytes: int | None = None,
                        seed_key="cfg4") -> DocSpec16:
    """Many UTF-16LE documents with byte lengths uniform in [lo, hi] (even),
    character-aligned slices of per-profile pools; a fraction carry one
    unpaired surrogate."""
    rng = rng_for(seed_key, n_docs)
    want_words = rng.integers(lo_bytes // 2, hi_bytes // 2 + 1, size=n_docs)
    prof = rng.integers(0, len(BATCH_PROFILES), size=n_docs)
    if pool_bytes is None:
        pool_bytes = int(min(max(2 * hi_bytes, want_words.sum()), 128 * MIB))
    pools = [make_text(p, pool_bytes, rng_for(seed_key, "pool", p, pool_bytes)) for p in BATCH_PROFILES]
    pool_starts = [t.char_starts_u16 for t in pools]
    start = np.zeros(n_docs, dtype=np.int64)
    length = np.zeros(n_docs, dtype=np.int64)
    inj_pos = np.full(n_docs, -1, dtype=np.int64)
    inj_words = np.zeros((n_docs, 2), dtype=np.uint16)
    inj = rng.random(n_docs) < error_frac
    for d in range(n_docs):
        t, cs = pools[prof[d]], pool_starts[prof[d]]
        total = int(cs[-1])
        w = int(min(want_words[d], total))
        i = int(rng.integers(0, max(1, int(np.searchsorted(cs, total - w, side="right")))))
        b0 = int(cs[i])
        j = int(np.searchsorted(cs, b0 + w, side="right")) - 1
        j = max(j, i)
        start[d], length[d] = b0, int(cs[j]) - b0
        if inj[d] and length[d] >= 4:
            doc, pos = inject_utf16_error(t.u16[b0:int(cs[j])], cs[i:j + 1] - b0, rng)
            inj_pos[d] = pos
            inj_words[d, 0] = doc[pos]
            inj_words[d, 1] = doc[pos + 1] if pos + 1 < doc.size else 0
    return DocSpec16(pools, prof, start, length, inj_pos, inj_words)


def utf16_documents(n_docs: int = 10_000, lo_bytes: int = 64, hi_bytes: int = 4 * MIB,
                    error_frac: float = 0.005, pool_bytes: int | None = None, seed_key="cfg4") -> DocBatch:
    """utf16_document_spec, materialised as one concatenated host array."""
    return utf16_document_spec(n_docs, lo_bytes, hi_bytes, error_frac, pool_bytes, seed_key).materialize()


@dataclass
class RequestTrace:
    """An open-loop request trace: arrival offsets (ns), operations, and each
    request's input as a slice of a profile pool (or its own copy when it
    carries an injected error)."""
    arrival_ns: np.ndarray          # int64, non-decreasing
    ops: np.ndarray                 # uint32: 2 (UTF-8 -> UTF-16LE) or 5 (UTF-16LE -> UTF-8)
    inputs: list                    # per request: uint8 or uint16 array
    invalid: np.ndarray             # bool: carries an injected error
    expect_count: np.ndarray        # uint64: output units when valid (0 for invalid ones)


_POOL_CACHE = {}


def _trace_pools(pool_bytes: int, seed_key):
    """Per-profile text pools of a trace (kept for later traces of the same key)."""
    k = (pool_bytes, seed_key)
    if k not in _POOL_CACHE:
        pools = [make_text(p, pool_bytes, rng_for(seed_key, "pool", p, pool_bytes)) for p in BATCH_PROFILES]
        _POOL_CACHE.clear()
        _POOL_CACHE[k] = (pools, [t.char_starts_u8 for t in pools], [t.char_starts_u16 for t in pools])
    return _POOL_CACHE[k]


def request_trace(rate_per_s: float, duration_s: float, median: int = 4096, sigma: float = 1.5,
                  lo: int = 16, hi: int = 16 * MIB, frac_8to16: float = 0.7, invalid_frac: float = 0.01,
                  pool_bytes: int = 32 * MIB, seed_key="cfg5") -> RequestTrace:
    """Poisson arrivals at `rate_per_s` for `duration_s`; request sizes
    log-normal (median 4 KiB, sigma 1.5, clipped 16 B - 16 MiB, in UTF-8 bytes
    of the text); 70% UTF-8 -> UTF-16LE and 30% the reverse; 1% invalid. Inputs
    are character-aligned slices of mixed-profile pools."""
    rng = rng_for(seed_key, rate_per_s, duration_s)
    n = max(1, int(rng.poisson(rate_per_s * duration_s)))
    gaps = rng.exponential(1e9 / rate_per_s, size=n)
    arrival = np.cumsum(gaps).astype(np.int64)
    arrival -= arrival[0]
    want = _lognormal_lengths(rng, n, median, sigma, lo, hi)
    ops = np.where(rng.random(n) < frac_8to16, 2, 5).astype(np.uint32)
    prof = rng.integers(0, len(BATCH_PROFILES), size=n)
    bad = rng.random(n) < invalid_frac
    pools, starts8, starts16 = _trace_pools(max(pool_bytes, 2 * hi), seed_key)
    first = np.zeros(n, dtype=np.int64)          # character index range [first, last) in the pool
    last = np.zeros(n, dtype=np.int64)
    for p in range(len(BATCH_PROFILES)):
        sel = np.nonzero(prof == p)[0]
        cs8 = starts8[p]
        total = int(cs8[-1])
        w = np.minimum(want[sel], total)
        upper = np.maximum(1, np.searchsorted(cs8, total - w, side="right"))
        i = np.minimum((rng.random(sel.size) * upper).astype(np.int64), upper - 1)
        j = np.maximum(np.searchsorted(cs8, cs8[i] + w, side="right") - 1, i)
        first[sel], last[sel] = i, j
    inputs, expect = [], np.zeros(n, dtype=np.uint64)
    for k in range(n):
        t = pools[prof[k]]
        cs8, cs16 = starts8[prof[k]], starts16[prof[k]]
        i, j = int(first[k]), int(last[k])
        if ops[k] == 2:
            doc = t.u8[int(cs8[i]):int(cs8[j])]
            expect[k] = int(cs16[j] - cs16[i])
            if bad[k] and doc.size >= 8:
                kind = UTF8_ERROR_KINDS[int(rng.integers(0, len(UTF8_ERROR_KINDS)))]
                doc, _ = inject_utf8_error(doc, cs8[i:j + 1] - cs8[i], kind, rng)
            else:
                bad[k] = False
        else:
            doc = t.u16[int(cs16[i]):int(cs16[j])]
            expect[k] = int(cs8[j] - cs8[i])
            if bad[k] and doc.size >= 4:
                doc, _ = inject_utf16_error(doc, cs16[i:j + 1] - cs16[i], rng)
            else:
                bad[k] = False
        inputs.append(doc)
    expect[bad] = 0
    return RequestTrace(arrival, ops, inputs, bad, expect)
