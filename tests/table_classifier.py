"""Independent well-formedness classifiers used to pin the oracle.

Written separately from the oracle: instead of decoding values and testing the
six rules, they walk the per-lead table of well-formed byte sequences (RFC 3629
section 4; equivalently the lead byte / first continuation byte ranges that the
six rules of section 3 of Lemire & Mula allow), vectorised over many strings
with numpy. They return the longest valid prefix of each string, not the error
kind.
"""
from __future__ import annotations

import numpy as np

# (first lead, last lead, sequence length, allowed range of the second byte)
# later bytes are always 80..BF
WELL_FORMED_ROWS = [
    (0x00, 0x7F, 1, None),
    (0xC2, 0xDF, 2, (0x80, 0xBF)),
    (0xE0, 0xE0, 3, (0xA0, 0xBF)),
    (0xE1, 0xEC, 3, (0x80, 0xBF)),
    (0xED, 0xED, 3, (0x80, 0x9F)),
    (0xEE, 0xEF, 3, (0x80, 0xBF)),
    (0xF0, 0xF0, 4, (0x90, 0xBF)),
    (0xF1, 0xF3, 4, (0x80, 0xBF)),
    (0xF4, 0xF4, 4, (0x80, 0x8F)),
]

LEAD_LEN = np.zeros(256, dtype=np.int64)
SECOND_LO = np.zeros(256, dtype=np.int64)
SECOND_HI = np.zeros(256, dtype=np.int64)
for lo, hi, ln, second in WELL_FORMED_ROWS:
    LEAD_LEN[lo:hi + 1] = ln
    if second is not None:
        SECOND_LO[lo:hi + 1] = second[0]
        SECOND_HI[lo:hi + 1] = second[1]


def utf8_valid_prefix(S: np.ndarray) -> np.ndarray:
    """S: (N, L) uint8, N strings of L bytes. Returns the length of the longest
    valid (whole-character) prefix of each string."""
    N, L = S.shape
    pos = np.zeros(N, dtype=np.int64)
    done = np.zeros(N, dtype=bool)
    for _ in range(L):
        idx = np.nonzero(~done & (pos < L))[0]
        if idx.size == 0:
            break
        p = pos[idx]
        b = S[idx, p].astype(np.int64)
        ln = LEAD_LEN[b]
        ok = (ln > 0) & (p + ln <= L)
        for k in (1, 2, 3):
            need = ok & (ln > k)
            c = S[idx, np.minimum(p + k, L - 1)].astype(np.int64)
            lo = SECOND_LO[b] if k == 1 else 0x80
            hi = SECOND_HI[b] if k == 1 else 0xBF
            ok &= ~need | ((c >= lo) & (c <= hi))
        pos[idx[ok]] += ln[ok]
        done[idx[~ok]] = True
    return pos


def utf16_valid_prefix(W: np.ndarray) -> np.ndarray:
    """W: (N, L) uint16 words. Longest valid prefix in words: a word in
    D800..DBFF must be followed by one in DC00..DFFF, a word in DC00..DFFF must
    be preceded by one in D800..DBFF."""
    N, L = W.shape
    pos = np.zeros(N, dtype=np.int64)
    done = np.zeros(N, dtype=bool)
    for _ in range(L):
        idx = np.nonzero(~done & (pos < L))[0]
        if idx.size == 0:
            break
        p = pos[idx]
        w = W[idx, p].astype(np.int64)
        nxt = W[idx, np.minimum(p + 1, L - 1)].astype(np.int64)
        is_high = (w >= 0xD800) & (w <= 0xDBFF)
        is_low = (w >= 0xDC00) & (w <= 0xDFFF)
        pair = is_high & (p + 1 < L) & (nxt >= 0xDC00) & (nxt <= 0xDFFF)
        single = ~is_high & ~is_low
        step = np.where(single, 1, np.where(pair, 2, 0))
        ok = step > 0
        pos[idx[ok]] += step[ok]
        done[idx[~ok]] = True
    return pos


def all_strings(L: int) -> np.ndarray:
    """Every byte string of length L, shape (256**L, L), first byte slowest."""
    n = 256 ** L
    k = np.arange(n, dtype=np.int64)
    cols = [((k >> (8 * (L - 1 - i))) & 0xFF).astype(np.uint8) for i in range(L)]
    return np.stack(cols, axis=1)


def valid_count_recurrence(L: int) -> int:
    """Number of valid UTF-8 strings of exactly L bytes: 128, 1920, 61440 and
    1048576 scalar values take 1, 2, 3 and 4 bytes (Table utfsummary ranges,
    minus the 2048 surrogates), so V(L) = 128 V(L-1) + 1920 V(L-2) +
    61440 V(L-3) + 1048576 V(L-4), V(0) = 1."""
    V = [1]
    for m in range(1, L + 1):
        v = 0
        for k, c in ((1, 128), (2, 1920), (3, 61440), (4, 1048576)):
            if m - k >= 0:
                v += c * V[m - k]
        V.append(v)
    return V[L]
