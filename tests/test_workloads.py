"""Seeded input generators: exact sizes, reproducibility, character mixes, and
injected errors that the oracle classifies as intended."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2109_10433_amd import workloads as wl


@pytest.mark.parametrize("profile", list(wl.PROFILES))
def test_exact_size_and_reproducible(profile):
    a = wl.make_text(profile, 100_001, wl.rng_for("t", profile))
    b = wl.make_text(profile, 100_001, wl.rng_for("t", profile))
    assert a.u8.size == 100_001
    assert np.array_equal(a.u8, b.u8) and np.array_equal(a.u16, b.u16)
    assert oracle.validate_utf8(a.u8) == (oracle.OK, a.u8.size)
    assert int(a.char_starts_u8[-1]) == a.u8.size
    assert int(a.char_starts_u16[-1]) == a.u16.size


@pytest.mark.parametrize("profile", list(wl.PROFILES))
def test_profile_mix(profile):
    t = wl.make_text(profile, 400_000, wl.rng_for("mix", profile))
    classes = wl.PROFILES[profile]
    n = t.utf8_len.size
    for cc in classes:
        frac = float((t.utf8_len == cc.utf8_len).sum()) / n
        assert abs(frac - cc.prob) < 0.02 + 0.01, (profile, cc.utf8_len, frac)
    # lengths by construction agree with CPython's encoding per character
    sample = np.random.default_rng(0).choice(n, 2000, replace=False)
    for i in sample:
        assert len(chr(int(t.cps[i])).encode()) == int(t.utf8_len[i])


def test_mix_bytes_per_char():
    t = wl.single_buffer(1 << 20)
    assert t.u8.size == 1 << 20
    chars = t.cps.size
    assert 1.50 < t.u8.size / chars < 1.60            # 0.7 + 0.2 + 0.45 + 0.2 = 1.55
    assert 2.05 < 2 * t.u16.size / chars < 2.15       # 2 + 2 x 0.05 = 2.10


def test_injected_utf8_errors_have_their_kind():
    t = wl.single_buffer(1 << 16, seed_key="inj")
    for kind, data, pos in wl.single_buffer_with_errors(t, seed_key="inj-e"):
        assert data.size == t.u8.size
        r = oracle.validate_utf8(data)
        assert r == (getattr(oracle, kind), pos), (kind, r, pos)


def test_injected_utf16_errors():
    t = wl.make_text("mix", 1 << 15, wl.rng_for("inj16"))
    rng = wl.rng_for("inj16-e")
    for _ in range(50):
        data, pos = wl.inject_utf16_error(t.u16, t.char_starts_u16, rng)
        r = oracle.validate_utf16le(data)
        assert r.error == oracle.UNPAIRED_SURROGATE
        assert r.count == 2 * pos


def test_document_batches_small():
    b = wl.utf8_documents(n_docs=300, error_frac=0.1, pool_bytes=1 << 20, seed_key="docs-t")
    assert b.offsets.size == 301 and b.offsets[-1] == b.data.size
    lens = np.diff(b.offsets)
    assert lens.min() >= 0 and lens.max() <= 1 << 20
    errs, _ = oracle.many_validate_utf8(b.data, b.offsets)
    assert np.array_equal(errs != 0, b.injected)
    b16 = wl.utf16_documents(n_docs=100, hi_bytes=1 << 14, error_frac=0.2, pool_bytes=1 << 18, seed_key="d16")
    errs, counts = oracle.many_validate_utf16le(b16.data, b16.offsets)
    assert np.array_equal(errs != 0, b16.injected)


def test_utf16_document_spec():
    spec = wl.utf16_document_spec(n_docs=80, hi_bytes=1 << 13, error_frac=0.25, pool_bytes=1 << 17, seed_key="spec16")
    b = spec.materialize()
    offs = spec.offsets
    assert np.array_equal(offs, b.offsets)
    le, lc = oracle.many_utf8_length_from_utf16le(b.data, offs)
    assert np.array_equal(le != 0, spec.injected)
    for d in range(80):
        assert np.array_equal(spec.doc(d), b.data[offs[d]:offs[d + 1]])
        if not spec.injected[d]:
            text = spec.doc(d).tobytes().decode("utf-16-le")
            assert spec.utf8_bytes(d) == len(text.encode("utf-8")) == lc[d]
