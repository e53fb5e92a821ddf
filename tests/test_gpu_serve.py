"""GPU tests of the server (hu_server_*): every request's result and output
equal the oracle's, and equal whether the request runs alone or in a mix of
concurrent traffic (bit-exact, tolerance 0)."""
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


@pytest.fixture(scope="module")
def text():
    return wl.make_text("mix", 4 << 20, wl.rng_for("serve-text"))


def make_requests(text, rng, n, sizes, tag0=0, invalid_frac=0.05):
    """(records, inputs, outputs, ops): inputs are slices of the text (some
    with an injected error), outputs sized to the worst case or less."""
    reqs, keep = [], []
    for k in range(n):
        op = int(rng.choice([2, 2, 2, 5, 5, 0, 1, 3, 4]))
        size = int(sizes[rng.integers(0, len(sizes))])
        if op < 3:
            a = int(rng.integers(0, text.u8.size - size))
            data = text.u8[a:a + size].copy()
            if size and rng.random() < invalid_frac:
                data[int(rng.integers(0, size))] = int(rng.integers(0x80, 0x100))
            cap = size if rng.random() < 0.9 else int(size * rng.random())
            dst = np.full(cap + 8, 0xA5A5, np.uint16) if op == 2 else None
        else:
            a = int(rng.integers(0, text.u16.size - size))
            data = text.u16[a:a + size].copy()
            if size and rng.random() < invalid_frac:
                data[int(rng.integers(0, size))] = int(rng.integers(0xD800, 0xE000))
            cap = 3 * size if rng.random() < 0.9 else int(size * rng.random())
            dst = np.full(cap + 8, 0xA5, np.uint8) if op == 5 else None
        rec = hu.Server.request(tag0 + k, op, data, dst, dst_cap=cap if dst is not None else None)
        reqs.append(rec)
        keep.append((op, data, dst, cap))
    return np.array(reqs, dtype=hu.REQUEST_DTYPE), keep


def expected(op, data, cap):
    if op == 0:
        return (*oracle.validate_utf8(data), None)
    if op == 1:
        return (*oracle.utf16_length_from_utf8(data), None)
    if op == 2:
        w, r = oracle.convert_utf8_to_utf16le(data, cap)
        return r.error, r.count, w
    if op == 3:
        return (*oracle.validate_utf16le(data), None)
    if op == 4:
        return (*oracle.utf8_length_from_utf16le(data), None)
    b, r = oracle.convert_utf16le_to_utf8(data, cap)
    return r.error, r.count, b


def check_against_oracle(comps, keep, label):
    by_tag = {int(c["tag"]): c for c in comps}
    for k, (op, data, dst, cap) in enumerate(keep):
        c = by_tag[k]
        e, n, out = expected(op, data, cap)
        assert (int(c["error"]), int(c["count"])) == (e, n), (label, k, op, data.size, cap)
        if dst is not None:
            if e == 0:
                assert np.array_equal(dst[:n], out), (label, k)
                assert np.all(dst[n:] == dst.dtype.type(0xA5A5 if dst.dtype == np.uint16 else 0xA5)), (label, k)
            else:
                assert np.all(dst == dst.dtype.type(0xA5A5 if dst.dtype == np.uint16 else 0xA5)), (label, k)


SIZES = [0, 1, 2, 3, 15, 16, 17, 100, 1000, 4095, 4096, 4097, 20000, 70000, 300000]


def test_server_alone_vs_in_the_mix(text):
    rng = np.random.default_rng(11)
    probe, keep = make_requests(text, rng, 60, SIZES)
    with hu.Server(pool_bytes=1 << 30, batch_bytes=64 << 20) as srv:
        # alone: one request at a time, waiting for each
        alone = []
        for k in range(probe.size):
            assert srv.submit(probe[k]) == 0
            got = srv.poll(1, timeout_s=30)
            assert got.size == 1 and int(got[0]["tag"]) == k
            alone.append(got[0].copy())
        say("server alone done")
        check_against_oracle(alone, keep, "alone")
        outs_alone = [None if d is None else d.copy() for (_, _, d, _) in keep]
        for (_, _, d, _) in keep:
            if d is not None:
                d[:] = 0xA5A5 if d.dtype == np.uint16 else 0xA5
        # in the mix: the same requests interleaved with 3000 others arriving at
        # ~300k/s, so they share batches with other traffic
        bg, bg_keep = make_requests(text, rng, 3000, [10, 100, 2000, 9000, 50000], tag0=10_000)
        allr = np.concatenate([bg, probe])
        order = rng.permutation(allr.size)
        allr = allr[order]
        arrival = np.cumsum(rng.exponential(3_300, size=allr.size)).astype(np.int64)
        comps = srv.replay(allr, arrival)
        st = srv.stats()
        say("server mix", st)
        assert st["mean_batch"] > 1.5, "requests were not batched together"
        mix = [c for c in comps if int(c["tag"]) < 10_000]
        check_against_oracle(mix, keep, "mix")
        by_tag = {int(c["tag"]): c for c in mix}
        for k in range(probe.size):
            assert (int(by_tag[k]["error"]), int(by_tag[k]["count"])) == (int(alone[k]["error"]), int(alone[k]["count"]))
            if outs_alone[k] is not None:
                assert np.array_equal(outs_alone[k], keep[k][2])
        # background traffic is right too
        bg_by = {int(c["tag"]) - 10_000: c for c in comps if int(c["tag"]) >= 10_000}
        check_against_oracle([dict(tag=k, error=v["error"], count=v["count"]) for k, v in bg_by.items()],
                             bg_keep, "background")


def test_server_plain_mode_agrees(text):
    rng = np.random.default_rng(12)
    reqs, keep = make_requests(text, rng, 120, SIZES)
    with hu.Server(pool_bytes=1 << 28, batch_bytes=32 << 20, plain=True) as srv:
        arrival = np.arange(reqs.size, dtype=np.int64) * 20_000
        comps = srv.replay(reqs, arrival)
        st = srv.stats()
        assert st["batches"] == reqs.size and st["mean_batch"] == 1.0
    check_against_oracle(comps, keep, "plain")


def test_server_small_pool_admission(text):
    """A 2 MiB pool with requests up to ~600 KiB regions: requests wait for
    memory at the head of the queue; all finish, right, in arrival order of
    launch."""
    rng = np.random.default_rng(13)
    reqs, keep = make_requests(text, rng, 200, [100, 30000, 100000, 200000], invalid_frac=0.02)
    with hu.Server(pool_bytes=2 << 20, batch_bytes=2 << 20, slots=3) as srv:
        arrival = np.zeros(reqs.size, dtype=np.int64)
        comps = srv.replay(reqs, arrival)
        st = srv.stats()
    assert st["completed"] == reqs.size
    check_against_oracle(comps, keep, "small pool")


def test_server_rejects_and_poll(text):
    rng = np.random.default_rng(14)
    good, keep = make_requests(text, rng, 20, [10, 1000])
    with hu.Server(pool_bytes=1 << 26, batch_bytes=1 << 20) as srv:
        big = np.zeros(2 << 20, np.uint8)
        bad = [hu.Server.request(100, 9, text.u8[:10]),          # unknown op
               hu.Server.request(101, 0, big)]                   # larger than a batch
        for r in bad:
            assert srv.submit(r) == 0
        for r in good:
            assert srv.submit(r) == 0
        got = []
        while len(got) < 22:
            c = srv.poll(64, timeout_s=30)
            assert c.size > 0
            got.extend(c)
        st = srv.stats()
    by = {int(c["tag"]): c for c in got}
    assert by[100]["error"] == hu.INVALID_ARGUMENT and by[101]["error"] == hu.INVALID_ARGUMENT
    assert st["rejected"] == 2 and st["completed"] == 22 and st["submitted"] == 22
    check_against_oracle([by[k] for k in range(20)], keep, "poll")
