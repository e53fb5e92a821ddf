"""Host logic of the server (scheduler, device pool, latency statistics) on the
CPU: the scheduler runs with a fake executor on a virtual clock (each batch
takes a fixed virtual time plus a per-byte time and returns count = n_units),
so admission, slot and memory limits, FIFO order, continuous batching and
error isolation are checked deterministically."""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import pytest

from tests.serve_harness import build as hb

OK, INVALID_ARGUMENT, DEVICE = 0, 17, 18
U8U16, U16U8, VAL8 = 2, 5, 0


def _lib():
    if not os.path.exists(hb.LIB) or os.path.getmtime(hb.LIB) < max(
            os.path.getmtime(p) for p in (os.path.join(hb.HERE, "harness.cpp"),
                                          os.path.join(hb.ROOT, "paper_2109_10433_amd", "csrc", "serve_core.hpp"))):
        hb.build()
    lib = ctypes.CDLL(hb.LIB)
    u64, i64, u32, vp = ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p
    lib.h_create.restype = vp
    lib.h_create.argtypes = [u64, u64, u32, ctypes.c_int, u32, u32, i64, i64]
    lib.h_destroy.argtypes = [vp]
    lib.h_submit.argtypes = [vp, u64, u32, u64, u64, i64, ctypes.c_int]
    lib.h_fail_next_launch.argtypes = [vp]
    lib.h_step.restype = ctypes.c_int
    lib.h_step.argtypes = [vp, i64, ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(u64),
                           ctypes.POINTER(i64), u32, ctypes.POINTER(u32)]
    for f in ("h_pool_used", "h_in_flight", "h_queued", "h_running", "h_batches"):
        getattr(lib, f).restype = u64
        getattr(lib, f).argtypes = [vp]
    lib.h_idle.restype = ctypes.c_int
    lib.h_idle.argtypes = [vp]
    lib.h_last_batch.restype = u32
    lib.h_last_batch.argtypes = [vp, ctypes.POINTER(u64), u32]
    lib.h_percentile.restype = i64
    lib.h_percentile.argtypes = [ctypes.POINTER(i64), u64, ctypes.c_double]
    lib.h_region_bytes.restype = u64
    lib.h_region_bytes.argtypes = [u64, u64, u64]
    lib.rp_create.restype = vp
    lib.rp_create.argtypes = [u64]
    lib.rp_destroy.argtypes = [vp]
    lib.rp_reserve.restype = ctypes.c_int
    lib.rp_reserve.argtypes = [vp, u64, ctypes.POINTER(u64)]
    lib.rp_release.argtypes = [vp, u64]
    lib.rp_largest.restype = u64
    lib.rp_largest.argtypes = [vp]
    lib.rp_used.restype = u64
    lib.rp_used.argtypes = [vp]
    return lib


LIB = _lib()


class Sim:
    """The scheduler with a fake executor; time is virtual (ns)."""

    def __init__(self, pool=1 << 30, slot_bytes=64 << 20, slot_requests=4096, slots=3, max_batch=4096,
                 max_in_flight=65536, latency=1000, ps_per_byte=0):
        self.h = LIB.h_create(pool, slot_bytes, slot_requests, slots, max_batch, max_in_flight, latency, ps_per_byte)
        self.done = {}
        self.order = []

    def __del__(self):
        LIB.h_destroy(self.h)

    def submit(self, tag, op=U8U16, n=100, t=0, cap=None, src=True):
        LIB.h_submit(self.h, tag, op, n, n if cap is None else cap, t, 1 if src else 0)

    def step(self, now):
        m = 4096
        tags = (ctypes.c_uint64 * m)()
        errs = (ctypes.c_int32 * m)()
        counts = (ctypes.c_uint64 * m)()
        lat = (ctypes.c_int64 * m)()
        n = ctypes.c_uint32()
        launched = LIB.h_step(self.h, now, tags, errs, counts, lat, m, ctypes.byref(n))
        assert launched >= 0
        for i in range(n.value):
            assert tags[i] not in self.done, "completed twice"
            self.done[tags[i]] = (errs[i], counts[i], lat[i])
            self.order.append(tags[i])
        return launched

    def last_batch(self):
        buf = (ctypes.c_uint64 * 8192)()
        k = LIB.h_last_batch(self.h, buf, 8192)
        return list(buf[:min(k, 8192)])

    def __getattr__(self, name):
        f = getattr(LIB, "h_" + name)
        return lambda: f(self.h)


def region(n, ins, outs):
    """Expected region size: 40-byte document entries (256-aligned block),
    16-byte aligned inputs and outputs, 16-byte results, 256-aligned total."""
    a = lambda x, k: (x + k - 1) // k * k
    return a(a(40 * n, 256) + sum(a(x, 16) for x in ins) + sum(a(x, 16) for x in outs) + 16 * n, 256)


def test_region_layout():
    for n, ins, outs in [(1, [100], [200]), (3, [1, 17, 33], [2, 34, 66]), (7, [4096] * 7, [0] * 7)]:
        assert LIB.h_region_bytes(n, sum((x + 15) // 16 * 16 for x in ins),
                                  sum((x + 15) // 16 * 16 for x in outs)) == region(n, ins, outs)


def test_percentile_nearest_rank():
    def pct(v, p):
        a = (ctypes.c_int64 * max(len(v), 1))(*v)
        return LIB.h_percentile(a, len(v), p)
    v = list(range(1, 101))
    rng = np.random.default_rng(0)
    rng.shuffle(v)
    assert pct(v, 50) == 50 and pct(v, 99) == 99 and pct(v, 100) == 100
    assert pct([7], 50) == 7 and pct([7], 99) == 7
    assert pct([], 50) == 0
    # nearest rank: the smallest value with at least p% of the sample at or below it
    for n in (1, 2, 3, 10, 37, 1000):
        w = rng.integers(0, 10**9, size=n).tolist()
        s = sorted(w)
        for p in (1, 50, 90, 99, 99.9):
            k = max(1, math.ceil(p / 100 * n))
            assert pct(w, p) == s[k - 1]


def test_ring_pool_against_model():
    rng = np.random.default_rng(1)
    cap = 1 << 20
    p = LIB.rp_create(cap)
    try:
        live = []            # (off, bytes) in allocation order
        freed = set()
        for it in range(20000):
            if live and rng.random() < 0.45:
                k = int(rng.integers(0, len(live)))
                off, b = live[k]
                if off in freed:
                    continue
                LIB.rp_release(p, off)
                freed.add(off)
                while live and live[0][0] in freed:
                    freed.discard(live[0][0])
                    live.pop(0)
            else:
                b = int(rng.integers(1, cap // 6))
                largest = LIB.rp_largest(p)
                off = ctypes.c_uint64()
                ok = LIB.rp_reserve(p, b, ctypes.byref(off))
                assert ok == (b <= largest), (it, b, largest)
                if ok:
                    o = off.value
                    assert o + b <= cap
                    for lo, lb in live:
                        if lo not in freed:
                            assert o + b <= lo or lo + lb <= o, "overlap"
                    live.append((o, b))
            used = sum(b for o, b in live if o not in freed)
            assert LIB.rp_used(p) == used
        # empty ring hands out the whole capacity
        for o, b in list(live):
            if o not in freed:
                LIB.rp_release(p, o)
        assert LIB.rp_used(p) == 0 and LIB.rp_largest(p) == cap
    finally:
        LIB.rp_destroy(p)


def test_continuous_batching_joins_next_step():
    s = Sim(slots=2, latency=100)
    for i in range(10):
        s.submit(i, t=0)
    assert s.step(0) == 1 and s.last_batch() == list(range(10))
    # arrivals while batch 1 runs go out in batch 2 at once, on the free slot
    for i in range(10, 15):
        s.submit(i, t=10)
    assert s.step(10) == 1 and s.last_batch() == list(range(10, 15))
    assert s.running() == 2
    s.step(99)
    assert not s.done
    s.step(100)
    assert sorted(s.done) == list(range(10))
    assert all(v == (OK, 100, 100) for v in s.done.values())
    s.step(110)
    assert sorted(s.done) == list(range(15))
    assert all(s.done[t][2] == 100 for t in range(10, 15))
    assert s.idle() == 1 and s.pool_used() == 0 and s.in_flight() == 0


def test_slot_limit_and_wait():
    s = Sim(slots=1, latency=50)
    s.submit(0, t=0)
    s.step(0)
    s.submit(1, t=5)
    s.submit(2, t=6)
    assert s.step(10) == 0 and s.queued() == 2      # the only slot is busy
    assert s.step(50) == 1                          # batch 1 done, 1 and 2 launched together
    assert s.last_batch() == [1, 2]
    assert s.done[0][2] == 50
    s.step(100)
    assert s.done[1][2] == 95 and s.done[2][2] == 94


def test_batch_request_cap():
    s = Sim(slots=3, max_batch=4, latency=10)
    for i in range(10):
        s.submit(i)
    assert s.step(0) == 3
    assert s.batches() == 3
    s.step(10)
    assert sorted(s.done) == list(range(10))


def test_in_flight_limit():
    s = Sim(slots=4, max_in_flight=5, latency=10)
    for i in range(12):
        s.submit(i)
    s.step(0)
    assert s.in_flight() == 5 and s.queued() == 7
    s.step(10)
    assert len(s.done) == 5 and s.in_flight() == 5
    s.step(20)
    s.step(30)
    assert sorted(s.done) == list(range(12))


def test_pool_admission_fifo_no_starvation():
    # pool fits one large request or many small ones: the large one at the head
    # waits for memory and nothing behind it overtakes it
    pool = 64 << 10
    s = Sim(pool=pool, slot_bytes=pool, slots=3, latency=100)
    s.submit(0, n=4000, t=0)                 # ~12 KiB region
    s.step(0)
    s.submit(1, n=21000, t=1)                # ~62 KiB region: does not fit beside request 0
    s.submit(2, n=1000, t=2)                 # ~3 KiB each: would fit beside 0, but may not overtake 1
    s.submit(3, n=1000, t=3)
    s.step(5)
    assert s.queued() == 3 and s.pool_used() > 0
    s.step(100)                              # 0 done, 1 now fits; 2 and 3 do not fit beside it
    assert 0 in s.done and s.last_batch() == [1]
    assert s.queued() == 2
    s.step(200)
    assert 1 in s.done and s.last_batch() == [2, 3]
    s.step(300)
    assert sorted(s.done) == [0, 1, 2, 3]
    assert s.order == [0, 1, 2, 3]


def test_invalid_requests_isolated():
    s = Sim(slot_bytes=1 << 20, latency=10)
    s.submit(0)
    s.submit(1, op=9)                        # unknown operation
    s.submit(2, n=1 << 20)                   # larger than a batch can hold
    s.submit(3, n=10, src=False)             # no input
    s.submit(4)
    s.step(0)
    assert s.done[1][0] == INVALID_ARGUMENT and s.done[2][0] == INVALID_ARGUMENT
    assert s.done[3][0] == INVALID_ARGUMENT
    assert s.last_batch() == [0, 4]
    s.step(10)
    assert s.done[0] == (OK, 100, 10) and s.done[4] == (OK, 100, 10)


def test_launch_failure_fails_only_its_batch():
    s = Sim(slots=1, latency=10)
    s.submit(0)
    s.submit(1)
    LIB.h_fail_next_launch(s.h)
    s.step(0)
    s.submit(2, t=1)
    s.step(1)                                # failed batch completes, its slot is free again
    assert s.done[0][0] == DEVICE and s.done[1][0] == DEVICE
    s.step(2)
    s.step(20)
    assert s.done[2][0] == OK
    assert s.pool_used() == 0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_trace_invariants(seed):
    rng = np.random.default_rng(seed)
    pool = 4 << 20
    max_in_flight = 300
    s = Sim(pool=pool, slot_bytes=1 << 20, slots=3, max_batch=64, max_in_flight=max_in_flight,
            latency=20_000, ps_per_byte=500)
    n = 3000
    gaps = rng.exponential(2_000, size=n).astype(np.int64)
    t_arr = np.cumsum(gaps)
    sizes = np.clip(np.exp(np.log(2000) + 1.5 * rng.standard_normal(n)), 16, 200_000).astype(np.int64)
    ops = np.where(rng.random(n) < 0.7, U8U16, U16U8)
    bad = rng.random(n) < 0.01
    now, i = 0, 0
    launched_tags = []
    while len(s.done) < n:
        while i < n and t_arr[i] <= now:
            s.submit(i, op=9 if bad[i] else int(ops[i]), n=int(sizes[i]), t=int(t_arr[i]))
            i += 1
        if s.step(now):
            launched_tags.extend(s.last_batch())
        assert s.pool_used() <= pool
        assert s.in_flight() <= max_in_flight
        now += 1_000
        assert now < 10**12
    # every request completed once, launched in arrival order (rejected ones never launched)
    assert launched_tags == [t for t in range(n) if not bad[t]]
    for t in range(n):
        e, c, lat = s.done[t]
        if bad[t]:
            assert e == INVALID_ARGUMENT
        else:
            assert (e, c) == (OK, sizes[t]) and lat >= 20_000
    assert s.idle() == 1 and s.pool_used() == 0
