"""GPU parity of the batch entry point (hu_batch_run), its HIP-graph replay
and the autotuner, against the CPU oracle per document (bit-exact)."""
from __future__ import annotations

import os

import numpy as np
import pytest
import torch

import oracle
from paper_2109_10433_amd import workloads as wl
from tests.gpu_util import say
from tests.table_classifier import all_strings

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2109_10433_amd import binding as hu

U8_OPS = (0, 1, 2)
U16_OPS = (3, 4, 5)


def expected(op: int, data: np.ndarray, cap: int):
    """(error, count, output or None) from the oracle for one document."""
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


def lay_out(items, rng):
    """items: list of (op, input array, cap). Inputs go to one byte buffer at
    random offsets (UTF-16 inputs even), outputs to another with a gap after
    each capacity. Returns (docs, src bytes, dst size, out offsets)."""
    docs = np.zeros(len(items), dtype=hu.DOC_DTYPE)
    src_parts, pos = [], 0
    dpos = 0
    for i, (op, data, cap) in enumerate(items):
        gap = int(rng.integers(0, 16))
        if op >= 3:
            gap += (pos + gap) & 1
        src_parts.append(np.zeros(gap, np.uint8))
        pos += gap
        raw = np.ascontiguousarray(data).view(np.uint8).reshape(-1)
        docs[i]["src_off"] = pos
        docs[i]["n_units"] = data.size
        src_parts.append(raw)
        pos += raw.size
        docs[i]["op"] = op
        if op in (2, 5):
            unit = 2 if op == 2 else 1
            dpos += int(rng.integers(0, 8)) * unit
            dpos += dpos & (unit - 1)          # UTF-16 output at an even offset
            docs[i]["dst_off"] = dpos
            docs[i]["dst_cap"] = cap
            dpos += cap * unit + 16
    src = np.concatenate(src_parts + [np.zeros(64, np.uint8)]) if src_parts else np.zeros(64, np.uint8)
    return docs, src, dpos + 64


def run_and_check(items, rng, tuning=None, label=""):
    docs, src, dst_size = lay_out(items, rng)
    src_t = torch.from_numpy(src).cuda()
    dst_t = torch.full((dst_size,), 0xA5, dtype=torch.uint8, device="cuda")
    b = hu.Batch(docs, src_t, dst_t)
    say("batch", label, "docs", len(items), "tuning", None if tuning is None else (tuning.sub_tiles, tuning.groups_per_cu))
    assert b.run(tuning) == 0
    errs, counts = b.results_host()
    dst = dst_t.cpu().numpy()
    for i, (op, data, cap) in enumerate(items):
        e, c, out = expected(op, data, cap)
        assert (int(errs[i]), int(counts[i])) == (e, c), (label, i, op, data.size, (errs[i], counts[i]), (e, c))
        if out is not None and e == 0:
            o = int(docs[i]["dst_off"])
            got = dst[o:o + out.nbytes]
            assert np.array_equal(got, out.view(np.uint8)), (label, i)
            unit = 2 if op == 2 else 1
            tail = dst[o + out.nbytes:o + cap * unit]
            assert np.all(tail == 0xA5), (label, i, "write past the count")
    return b


def random_items(rng, n, text8, text16, sizes):
    items = []
    for _ in range(n):
        op = int(rng.integers(0, 6))
        size = int(sizes[rng.integers(0, len(sizes))])
        if op < 3:
            start = int(rng.integers(0, text8.size - size))
            data = text8[start:start + size].copy()
            if size and rng.random() < 0.3:
                data[int(rng.integers(0, size))] = int(rng.integers(0x80, 0x100))
            cap = size
            if op == 2 and rng.random() < 0.2:
                cap = int(size * rng.random())
        else:
            start = int(rng.integers(0, text16.size - size))
            data = text16[start:start + size].copy()
            if size and rng.random() < 0.3:
                data[int(rng.integers(0, size))] = int(rng.integers(0xD800, 0xE000))
            cap = 3 * size
            if op == 5 and rng.random() < 0.2:
                cap = int(size * rng.random())
        items.append((op, data, cap))
    return items


@pytest.fixture(scope="module")
def texts():
    t = wl.make_text("mix", 1 << 20, wl.rng_for("batch-text"))
    return t.u8, t.u16


def test_batch_mixed_ops(texts):
    rng = np.random.default_rng(101)
    sizes = [0, 1, 2, 3, 5, 15, 16, 17, 100, 4095, 4096, 4097, 8191, 8192, 8193, 16383, 16385, 20000, 70000]
    items = random_items(rng, 700, texts[0], texts[1], sizes)
    run_and_check(items, rng, label="mixed")


@pytest.mark.parametrize("sub_tiles,groups", [(1, 1), (2, 2), (4, 0), (1, 0), (4, 6), (6, 0), (6, 3)])
def test_batch_tunings_agree(texts, sub_tiles, groups):
    rng = np.random.default_rng(7 + sub_tiles * 10 + groups)
    sizes = [0, 1, 7, 64, 4096, 5000, 9000, 40000]
    items = random_items(rng, 200, texts[0], texts[1], sizes)
    run_and_check(items, rng, tuning=hu.HuTuning(sub_tiles, groups), label=f"tuning {sub_tiles}/{groups}")


def test_batch_utf8_documents():
    b = wl.utf8_documents(n_docs=4000, pool_bytes=4 << 20, seed_key="gpu-batch8")
    rng = np.random.default_rng(8)
    items = []
    for d in range(4000):
        data = b.data[b.offsets[d]:b.offsets[d + 1]]
        items.append((2 if d % 3 else 0, data, data.size))
    run_and_check(items, rng, label="utf8 documents")


def test_batch_utf16_documents():
    b = wl.utf16_documents(n_docs=400, hi_bytes=1 << 18, error_frac=0.05, pool_bytes=1 << 20, seed_key="gpu-b16")
    rng = np.random.default_rng(16)
    items = []
    for d in range(400):
        data = b.data[b.offsets[d]:b.offsets[d + 1]]
        items.append((5 if d % 2 else 4, data, 3 * data.size))
    run_and_check(items, rng, label="utf16 documents")


def test_batch_exhaustive_short_strings():
    """Every UTF-8 string of 1, 2 and 3 bytes as its own document (16.8 M
    documents): device validation and length against the oracle."""
    for L in (1, 2, 3):
        S = all_strings(L)
        n = S.shape[0]
        src = torch.from_numpy(S.reshape(-1).copy()).cuda()
        offs = np.arange(n + 1, dtype=np.uint64) * L
        oe, oc = oracle.many_validate_utf8(S.reshape(-1), offs)
        le, lc = oracle.many_utf16_length_from_utf8(S.reshape(-1), offs)
        for op, (ee, ec) in ((0, (oe, oc)), (1, (le, lc))):
            docs = np.zeros(n, dtype=hu.DOC_DTYPE)
            docs["src_off"] = offs[:-1]
            docs["n_units"] = L
            docs["op"] = op
            say("exhaustive strings of", L, "bytes, op", op, "docs", n)
            b = hu.Batch(docs, src)
            assert b.run() == 0
            errs, counts = b.results_host()
            assert np.array_equal(errs, ee)
            assert np.array_equal(counts, ec)
            del b
        del src
        torch.cuda.empty_cache()


def test_batch_invalid_arguments(texts):
    rng = np.random.default_rng(5)
    t8, t16 = texts
    docs = np.zeros(6, dtype=hu.DOC_DTYPE)
    src = torch.from_numpy(t8[:1000].copy()).cuda()
    dst = torch.full((256,), 0xA5, dtype=torch.uint8, device="cuda")
    docs[0] = (1, 10, 0, 0, 3, 0)      # UTF-16 at an odd address
    docs[1] = (0, 10, 0, 0, 9, 0)      # unknown op
    docs[2] = (0, 100, 0, 0, 0, 0)     # fine
    docs[3] = (0, 0, 0, 0, 2, 0)       # empty convert
    docs[4] = (0, 10, 1, 10, 2, 0)     # UTF-16 output at an odd address
    docs[5] = (0, 10, 64, 10, 2, 0)    # fine
    say("batch invalid arguments")
    b = hu.Batch(docs, src, dst)
    assert b.run() == 0
    errs, counts = b.results_host()
    assert errs[0] == hu.INVALID_ARGUMENT and errs[1] == hu.INVALID_ARGUMENT
    assert (errs[2], counts[2]) == tuple(oracle.validate_utf8(t8[:100]))
    assert (errs[3], counts[3]) == (0, 0)
    assert errs[4] == hu.INVALID_ARGUMENT
    w, r = oracle.convert_utf8_to_utf16le(t8[:10], 10)
    assert (errs[5], counts[5]) == (r.error, r.count)
    out = dst.cpu().numpy()
    assert np.all(out[:64] == 0xA5)
    if r.error == 0:
        assert np.array_equal(out[64:64 + w.nbytes], w.view(np.uint8))
    # a workspace sized for fewer work items than the documents need: every
    # document reports it (capacity for total 0 bytes is 2 items per document
    # + 1; two 60000-byte documents need 8 items each at 8 KiB tiles)
    big = torch.from_numpy(t8[:120000].copy()).cuda()
    docs2 = np.zeros(2, dtype=hu.DOC_DTYPE)
    docs2[0] = (0, 60000, 0, 0, 0, 0)
    docs2[1] = (60000, 60000, 0, 0, 1, 0)
    small = hu.Batch(docs2, big, total_input_bytes=0)
    assert small.run() == 0
    errs, _ = small.results_host()
    assert list(errs) == [hu.INVALID_ARGUMENT, hu.INVALID_ARGUMENT]
    # the same documents with a right-sized workspace
    ok = hu.Batch(docs2, big)
    assert ok.run() == 0
    errs, counts = ok.results_host()
    assert (errs[0], counts[0]) == tuple(oracle.validate_utf8(t8[:60000]))
    assert (errs[1], counts[1]) == tuple(oracle.utf16_length_from_utf8(t8[60000:120000]))
    # the same check with more documents than one planning block (1024):
    # 1500 documents of 20000 bytes need 3 items each, the workspace for
    # total 0 bytes holds 3001
    many = np.zeros(1500, dtype=hu.DOC_DTYPE)
    many["src_off"] = (np.arange(1500) % 5) * 20000
    many["n_units"] = 20000
    many["op"] = np.arange(1500) % 2
    say("batch capacity exceeded, 1500 documents")
    over = hu.Batch(many, big, total_input_bytes=0)
    assert over.run() == 0
    errs, _ = over.results_host()
    assert np.all(errs == hu.INVALID_ARGUMENT)
    fits = hu.Batch(many, big)
    assert fits.run() == 0
    errs, counts = fits.results_host()
    for i in (0, 1, 1023, 1024, 1499):
        data = t8[int(many["src_off"][i]):int(many["src_off"][i]) + 20000]
        want = oracle.validate_utf8(data) if i % 2 == 0 else oracle.utf16_length_from_utf8(data)
        assert (errs[i], counts[i]) == tuple(want), i


def test_batch_graph_replay(texts):
    rng = np.random.default_rng(42)
    t8, t16 = texts
    sizes = [0, 3, 100, 5000, 20000]
    items = random_items(rng, 150, t8, t16, sizes)
    docs, src, dst_size = lay_out(items, rng)
    src_t = torch.from_numpy(src).cuda()
    dst_t = torch.zeros(dst_size, dtype=torch.uint8, device="cuda")
    b = hu.Batch(docs, src_t, dst_t)
    g = b.graph()
    try:
        for replay in range(4):
            # change the inputs in place between replays (inject one error)
            if replay:
                k = int(rng.integers(0, len(items)))
                op, data, cap = items[k]
                if data.size:
                    j = int(rng.integers(0, data.size))
                    data = data.copy()
                    data[j] = 0xFF if op < 3 else 0xDC00
                    items[k] = (op, data, cap)
                    raw = data.view(np.uint8).reshape(-1)
                    off = int(docs[k]["src_off"])
                    src_t[off:off + raw.size] = torch.from_numpy(raw.copy()).cuda()
            say("graph replay", replay)
            assert hu.graph_launch(g) == 0
            errs, counts = b.results_host()
            # eager run of the same batch, then compare both with the oracle
            assert b.run() == 0
            errs2, counts2 = b.results_host()
            assert np.array_equal(errs, errs2) and np.array_equal(counts, counts2)
            for i, (op, data, cap) in enumerate(items):
                e, c, _ = expected(op, data, cap)
                assert (int(errs[i]), int(counts[i])) == (e, c), (replay, i)
    finally:
        hu.graph_destroy(g)


def test_batch_tuner_and_cache(texts, tmp_path, monkeypatch):
    rng = np.random.default_rng(3)
    items = random_items(rng, 300, texts[0], texts[1], [10, 2000, 6000, 30000])
    docs, src, dst_size = lay_out(items, rng)
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("HIPUTF_TUNE_CACHE", str(cache))
    b = hu.Batch(docs, torch.from_numpy(src).cuda(), torch.zeros(dst_size, dtype=torch.uint8, device="cuda"))
    say("tuner")
    best, us = b.tune("test-mix")
    assert best.sub_tiles in (1, 2, 4, 6) and best.groups_per_cu in (0, 2, 4, 6) and us > 0
    got = hu.tuning_lookup("test-mix")
    assert got is not None and (got.sub_tiles, got.groups_per_cu) == (best.sub_tiles, best.groups_per_cu)
    assert hu.tuning_lookup("no-such-key") is None
    # results after tuning runs are still right
    errs, counts = b.results_host()
    for i, (op, data, cap) in enumerate(items):
        e, c, _ = expected(op, data, cap)
        assert (int(errs[i]), int(counts[i])) == (e, c)


def test_workspace_reused_across_batch_shapes(texts):
    """One workspace for batches of different document counts and sizes
    (growing and shrinking): the per-document arrays move with the shape, and
    earlier calls' data must never be read as error keys or status words."""
    rng = np.random.default_rng(77)
    t8, t16 = texts
    shapes = [(40, [100, 5000]), (3, [60000]), (300, [10, 200]), (1, [3]), (120, [9000, 30000]),
              (2500, [1, 400]), (500, [1, 50]), (20, [100000])]
    max_docs = max(n for n, _ in shapes)
    max_total = 4 << 20
    ws = torch.zeros(hu.lib.hu_batch_workspace_bytes(max_docs, max_total) + 256, dtype=torch.uint8, device="cuda")
    wsp, wsb = hu.workspace_ptr(ws)
    for rep in range(2):
        for n, sizes in shapes:
            items = random_items(rng, n, t8, t16, sizes)
            docs, src, dst_size = lay_out(items, rng)
            total = int(sum(d.view(np.uint8).size for _, d, _ in items))
            assert total <= max_total
            src_t = torch.from_numpy(src).cuda()
            dst_t = torch.full((dst_size,), 0xA5, dtype=torch.uint8, device="cuda")
            docs_t = torch.from_numpy(docs.view(np.uint8).copy()).cuda()
            res = torch.zeros((n, 16), dtype=torch.uint8, device="cuda")
            say("shared workspace", rep, n, total)
            rc = hu.lib.hu_batch_run(docs_t.data_ptr(), n, total, src_t.data_ptr(), dst_t.data_ptr(), res.data_ptr(),
                                     None, wsp, wsb, hu.stream_handle())
            assert rc == 0
            torch.cuda.synchronize()
            rec = res.cpu().numpy().reshape(-1).view([("error", "<i4"), ("reserved", "<i4"), ("count", "<u8")])
            for i, (op, data, cap) in enumerate(items):
                e, c, _ = expected(op, data, cap)
                assert (int(rec["error"][i]), int(rec["count"][i])) == (e, c), (rep, n, i, op)
