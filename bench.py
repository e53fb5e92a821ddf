"""Benchmark: validating UTF-8 -> UTF-16LE (and the rest of the hot path) on
one MI355X.

A step is one pass of the whole single-buffer hot path over the large-buffer
workload: for each of four 256 MiB UTF-8 profiles (Latin, Cyrillic, CJK,
Emoji) convert UTF-8 -> UTF-16LE, convert UTF-16LE -> UTF-8, both length
functions and both validations (and the non-validating and big-endian
conversions), each one kernel launch of the library's async entry points with
caller-owned workspaces (no allocation in the timed region). Inputs are
resident in HBM before timing starts; each profile has two input copies that
successive steps use in turn, and every operation writes its own output
buffer. After the timed steps every result and every output is compared with
the CPU oracle's, whose single-thread timings on the same inputs are the CPU
baseline legs (both directions, length, validation; GB/s and Gchar/s).
Per operation and profile: minimum, median and mean over the steps, and
whether the mean lies within 1 % of the minimum.

The 1 MiB mixed buffer and its six copies with one injected error each are
timed 2000 times each (per-launch HIP events), results against the oracle.

`value` is the validating UTF-8 -> UTF-16LE throughput in GB/s of algorithmic
bytes (input bytes read + output bytes written), aggregated over the four
profiles, from HIP events around each launch on the launch stream.

Two batched workloads are timed after the step loop, each against the same
documents run as one launch per document (the plain path):
  * 100 000 UTF-8 documents (log-normal lengths, median 2 KiB, 16 B - 1 MiB,
    mixed profiles, 1% with one injected error) converted to UTF-16LE in one
    batch call, with sub-tile count and workgroups per CU from the autotuner;
  * 10 000 UTF-16LE documents (uniform 64 B - 4 MiB, mixed profiles, 0.5% with
    an unpaired surrogate) converted to UTF-8 by replaying a captured HIP graph.
Every document's result (and the output of every UTF-8 document, of a
seeded sample of 1000 UTF-16 ones) is compared with the oracle's, run over
the documents on up to 16 host threads (the CPU figure for the batches).
Then open-loop Poisson request traces of 10 s (10k, 50k and 200k requests/s; sizes
log-normal, median 4 KiB, 16 B - 16 MiB; 70% UTF-8 -> UTF-16LE, 30% the
reverse; 1% invalid) are replayed from host memory through the continuous-
batching server (8 GiB device pool) and through the plain path (one request at
a time: copy in, one launch, copy out, wait), with p50/p99 latency from arrival
to output in host memory; every request's result (error kind and position
included) is compared with the oracle's, and the oracle's own per-request
latency is sampled beside it.
Last, an input-size sweep (1 B - 256 MiB of the mixed profile, both
directions) times single calls back to back and one synchronous call at a
time, with the CPU oracle on the same inputs up to 16 MiB.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, AMD published peak
METRIC = "validating UTF-8→UTF-16 GB/s and % HBM peak; batched docs/s vs plain; p99"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_u8_to_u16_256mib.json")


def kernel_source_digest() -> str:
    """Digest of the device sources: counters taken on other sources are stale."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2109_10433_amd", "csrc")
    for name in sorted(os.listdir(d)):
        if name.endswith((".hpp", ".hip", ".h")):
            h.update(name.encode())
            h.update(open(os.path.join(d, name), "rb").read())
    return h.hexdigest()[:16]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _time_on_stream(fn, stream, reps):
    """Mean seconds of fn() over reps calls, from HIP events on `stream`."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def _per_launch_times(fn, stream, reps):
    """Seconds of each of reps calls of fn(), from a HIP event pair around
    each launch on `stream` (numpy array)."""
    import numpy as np
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    ev[-1][1].synchronize()
    return np.array([a.elapsed_time(b) * 1e-3 for a, b in ev])


def _timing_stats(ts) -> dict:
    """Minimum, median and mean of repeated timings (microseconds), and the
    repeatability check of the paper's protocol: the mean within 1 % of the
    minimum."""
    import numpy as np
    ts = np.asarray(ts, dtype=np.float64)
    mn, md, mean = float(ts.min()), float(np.median(ts)), float(ts.mean())
    return {"reps": int(ts.size), "us_min": round(mn * 1e6, 2), "us_median": round(md * 1e6, 2),
            "us_mean": round(mean * 1e6, 2), "mean_over_min_pct": round(100 * (mean / mn - 1), 2),
            "mean_within_1pct_of_min": bool(mean <= 1.01 * mn)}


def _workers() -> int:
    """Host threads for the oracle's parallel legs: the cores the process may
    use, at most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _pool_map(fn, chunks, workers):
    """fn over chunks in a thread pool (the oracle's C calls release the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, chunks))


def _chunks(n, parts):
    step = max(1, -(-n // parts))
    return [(a, min(a + step, n)) for a in range(0, n, step)]


def _cpu_info() -> dict:
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    from oracle.build import CFLAGS
    return {"cpu_model": model, "host_cores_visible": os.cpu_count(), "oracle_compiler": "gcc",
            "oracle_flags": " ".join(CFLAGS)}


def bench_single_1mib(args, hu, wl, dev, stream):
    """One 1 MiB buffer of mixed text (70/10/15/5 % one- to four-byte
    characters) and six copies with one injected error of each kind:
    validating UTF-8 -> UTF-16LE, R repetitions each (per-launch HIP events,
    minimum / median / mean), every result and the clean copy's words checked
    against the oracle."""
    import numpy as np
    import torch

    import oracle
    text = wl.single_buffer(wl.MIB)
    copies = [("clean", text.u8, None)] + list(wl.single_buffer_with_errors(text))
    n = text.u8.size
    ws = hu.workspace(hu.OP_CONVERT_UTF8_TO_UTF16LE, n, dev)
    wsp, wsb = hu.workspace_ptr(ws)
    dst = torch.empty(n, dtype=torch.int16, device=dev)
    rec = torch.zeros(16, dtype=torch.uint8, device=dev)
    sh = hu.stream_handle(stream)
    out = {"workload": "1 MiB mixed text (70/10/15/5 % of characters with 1/2/3/4 UTF-8 bytes) and six copies "
                       "with one injected error each, validating UTF-8 -> UTF-16LE",
           "bytes": n, "copies": {}}
    for kind, data, pos in copies:
        src = torch.from_numpy(data.copy()).to(dev)
        call = (lambda src=src: hu.lib.convert_utf8_to_utf16le_async(src.data_ptr(), n, dst.data_ptr(), n,
                                                                      rec.data_ptr(), wsp, wsb, sh))
        for _ in range(50):
            if call() != 0:
                raise RuntimeError("1 MiB buffer: enqueue failed")
        ts = _per_launch_times(call, stream, args.reps_1mib)
        t_b2b = _time_on_stream(call, stream, args.reps_1mib)
        r = hu.result_from_device(rec)
        ow, orr = oracle.convert_utf8_to_utf16le(data)
        if tuple(r) != tuple(orr):
            raise RuntimeError(f"1 MiB buffer {kind}: result {tuple(r)} != oracle {tuple(orr)}")
        if orr.error == 0 and not np.array_equal(dst[:orr.count].cpu().numpy().view(np.uint16), ow):
            raise RuntimeError("1 MiB buffer: words differ from the oracle's")
        e = _timing_stats(ts)
        e["us_back_to_back_mean"] = round(t_b2b * 1e6, 2)
        e["result"] = {"error": hu.error_name(r.error), "count": int(r.count)}
        if kind == "clean":
            moved = n + 2 * int(r.count)
            e["GBps_at_min"] = round(moved / (e["us_min"] * 1e-6) / 1e9, 1)
            e["GBps_at_median"] = round(moved / (e["us_median"] * 1e-6) / 1e9, 1)
        else:
            e["injected_at"] = int(pos)
        out["copies"][kind.lower()] = e
    out["oracle_agrees"] = True
    log("1 MiB buffer: " + ", ".join(f"{k} {v['us_median']} us" for k, v in out["copies"].items()))
    return out


def _plain_launches(hu, fns, stream, passes):
    """One library launch per document (fns: one callable each); mean seconds
    per pass over all documents, HIP events on the stream."""
    def one_pass():
        for f in fns:
            rc = f()
            if rc != 0:
                raise RuntimeError(f"per-document launch failed: {hu.error_name(rc)}")
    one_pass()
    return _time_on_stream(one_pass, stream, passes)


def bench_utf8_documents(args, hu, wl, dev, stream):
    """100k UTF-8 documents -> UTF-16LE: autotuned batch vs per-document launches."""
    import numpy as np
    import torch
    t_gen = time.time()
    b = wl.utf8_documents(n_docs=args.docs8, pool_bytes=32 * wl.MIB)
    n = b.offsets.size - 1
    lens = np.diff(b.offsets).astype(np.uint64)
    total = int(b.offsets[-1])
    src = torch.from_numpy(b.data).to(dev)
    dst = torch.zeros(2 * total + 64, dtype=torch.uint8, device=dev)
    docs = np.zeros(n, dtype=hu.DOC_DTYPE)
    docs["src_off"] = b.offsets[:-1]
    docs["n_units"] = lens
    docs["dst_off"] = 2 * b.offsets[:-1]
    docs["dst_cap"] = lens
    docs["op"] = hu.OP_CONVERT_UTF8_TO_UTF16LE
    batch = hu.Batch(docs, src, dst)
    log(f"utf8 documents: {n} docs, {total} B, generated in {time.time() - t_gen:.1f}s")
    best, best_us = batch.tune(f"utf8-documents-{n}", stream)
    log(f"utf8 documents: tuned sub_tiles={best.sub_tiles} groups_per_cu={best.groups_per_cu} ({best_us:.0f} us)")

    t_batch = _time_on_stream(lambda: batch.run(best, stream), stream, args.steps)
    g = batch.graph(best)
    try:
        hu.graph_launch(g, stream)
        t_graph = _time_on_stream(lambda: hu.graph_launch(g, stream), stream, args.steps)
    finally:
        torch.cuda.synchronize()
        hu.graph_destroy(g)
    errs, counts = batch.results_host()
    bad = errs != 0
    out_bytes = int(2 * counts[~bad].sum())
    oracle_check, cpu_leg = _oracle_utf8_documents(b, lens, errs, counts, dst)

    # plain: one async convert launch per document, results to their own records
    recs = torch.zeros((n, 16), dtype=torch.uint8, device=dev)
    ws = hu.workspace(hu.OP_CONVERT_UTF8_TO_UTF16LE, int(lens.max()), dev)
    wsp, wsb = hu.workspace_ptr(ws)
    sh = hu.stream_handle(stream)
    sp, dp, rp = src.data_ptr(), dst.data_ptr(), recs.data_ptr()
    f = hu.lib.convert_utf8_to_utf16le_async
    offs = [int(x) for x in b.offsets[:-1]]
    ls = [int(x) for x in lens]
    fns = [(lambda i=i: f(sp + offs[i], ls[i], dp + 2 * offs[i], ls[i], rp + 16 * i, wsp, wsb, sh)) for i in range(n)]
    t_plain = _plain_launches(hu, fns, stream, args.plain_passes)
    torch.cuda.synchronize()
    h = recs.cpu().numpy().reshape(-1).view([("error", "<i4"), ("reserved", "<i4"), ("count", "<u8")])
    if not (np.array_equal(h["error"], errs) and np.array_equal(h["count"], counts)):
        raise RuntimeError("utf8 documents: batched and per-document results differ")
    # naive use: one synchronous call per document, on a prefix of the batch
    n_sync = min(n, args.sync_docs)
    fs = hu.lib.convert_utf8_to_utf16le
    t0 = time.perf_counter()
    for i in range(n_sync):
        r = fs(sp + offs[i], ls[i], dp + 2 * offs[i], ls[i], sh)
        if (r.error, r.count) != (int(errs[i]), int(counts[i])):
            raise RuntimeError(f"utf8 documents: synchronous call {i} disagrees with the batch")
    t_sync = (time.perf_counter() - t0) / n_sync * n
    algo = total + out_bytes
    return {
        "workload": f"{n} UTF-8 documents -> UTF-16LE, log-normal lengths (median 2 KiB, 16 B-1 MiB), "
                    f"mixed profiles, 1% injected errors",
        "docs": n, "input_bytes": total, "docs_with_errors": int(bad.sum()),
        "tuning": {"sub_tiles": best.sub_tiles, "groups_per_cu": best.groups_per_cu, "tile_bytes": 4096 * best.sub_tiles},
        "batched": {"ms": round(t_batch * 1e3, 3), "docs_per_s": round(n / t_batch, 1),
                    "GBps": round(algo / t_batch / 1e9, 1)},
        "batched_graph": {"ms": round(t_graph * 1e3, 3), "docs_per_s": round(n / t_graph, 1),
                          "GBps": round(algo / t_graph / 1e9, 1)},
        "plain_per_document_launches": {"ms": round(t_plain * 1e3, 3), "docs_per_s": round(n / t_plain, 1),
                                        "GBps": round(algo / t_plain / 1e9, 2)},
        "plain_per_document_sync_calls": {"docs_timed": n_sync, "ms_for_all_docs": round(t_sync * 1e3, 1),
                                          "docs_per_s": round(n / t_sync, 1)},
        "speedup_batched_vs_plain": round(t_plain / t_batch, 1),
        "speedup_batched_vs_sync_calls": round(t_sync / t_batch, 1),
        "oracle_agrees": oracle_check,
        "cpu_oracle": cpu_leg,
    }


def _oracle_utf8_documents(b, lens, errs, counts, dst):
    """Every document of the UTF-8 batch through the oracle (host threads,
    each a run of documents): (error, count) of each, and the words of every
    document without an error, compared with the batch's results and output.
    Returns (check record, CPU timing of the oracle pass)."""
    import numpy as np

    import oracle
    n = lens.size
    offs = b.offsets[:-1].astype(np.uint64)
    total = int(b.offsets[-1])
    ref = np.zeros(total + 8, dtype=np.uint16)        # the batch's layout: document d at word offs[d]
    src_addr = b.data.ctypes.data + offs
    dst_addr = ref.ctypes.data + 2 * offs
    workers = _workers()
    parts = _chunks(n, 8 * workers)

    def run(ab):
        a, e = ab
        return oracle.many_convert_at(False, src_addr[a:e], lens[a:e], dst_addr[a:e], lens[a:e])
    t0 = time.perf_counter()
    res = _pool_map(run, parts, workers)
    t_cpu = time.perf_counter() - t0
    oe = np.concatenate([r[0] for r in res])
    oc = np.concatenate([r[1] for r in res])
    if not (np.array_equal(oe, errs) and np.array_equal(oc, counts)):
        k = int(np.nonzero((oe != errs) | (oc != counts))[0][0])
        raise RuntimeError(f"utf8 documents: doc {k}: batch {(errs[k], counts[k])} != oracle {(oe[k], oc[k])}")
    got = dst[:2 * total].cpu().numpy().view(np.uint16).copy()
    for d in np.nonzero(oe != 0)[0]:              # output of a failed call is unspecified
        a, e = int(offs[d]), int(offs[d] + lens[d])
        got[a:e] = 0
        ref[a:e] = 0
    if not np.array_equal(got, ref[:total]):
        k = int(np.nonzero(got != ref[:total])[0][0])
        raise RuntimeError(f"utf8 documents: output word {k} differs from the oracle's")
    moved = total + int(2 * oc[oe == 0].sum())
    check = {"docs_checked": int(n), "results_equal": True, "docs_with_output_compared": int((oe == 0).sum()),
             "output_words_compared": int(oc[oe == 0].sum())}
    cpu = {"docs_per_s": round(n / t_cpu, 1), "GBps": round(moved / t_cpu / 1e9, 3), "threads": workers,
           "seconds": round(t_cpu, 3)}
    return check, cpu


def bench_utf16_documents(args, hu, wl, dev, stream):
    """10k UTF-16LE documents -> UTF-8: graph-replayed tuned batch vs per-document launches."""
    import numpy as np
    import torch
    t_gen = time.time()
    spec = wl.utf16_document_spec(n_docs=args.docs16, pool_bytes=32 * wl.MIB)
    n = spec.length.size
    offs = spec.offsets
    total_w = int(offs[-1])
    # assemble the batch on the device from the profile pools
    pools = [torch.from_numpy(t.u16.view(np.int16).copy()).to(dev) for t in spec.pools]
    src = torch.empty(total_w + 32, dtype=torch.int16, device=dev)
    for d in range(n):
        a, l = int(spec.start[d]), int(spec.length[d])
        src[int(offs[d]):int(offs[d]) + l].copy_(pools[spec.profiles[d]][a:a + l])
    inj = np.nonzero(spec.injected)[0]
    for d in inj:
        p = int(offs[d] + spec.inj_pos[d])
        src[p] = int(np.int16(spec.inj_words[d, 0].view(np.int16)))
        if spec.inj_pos[d] + 1 < spec.length[d]:
            src[p + 1] = int(spec.inj_words[d, 1].view(np.int16))
    del pools
    # exact output capacity for clean documents, 3 bytes per word otherwise
    expect = np.array([spec.utf8_bytes(d) if not spec.injected[d] else 0 for d in range(n)], dtype=np.uint64)
    cap = np.where(spec.injected, 3 * spec.length, expect).astype(np.uint64)
    dst_off = np.concatenate([[0], np.cumsum(cap)])[:-1].astype(np.uint64)
    dst = torch.zeros(int(cap.sum()) + 64, dtype=torch.uint8, device=dev)
    docs = np.zeros(n, dtype=hu.DOC_DTYPE)
    docs["src_off"] = 2 * offs[:-1]
    docs["n_units"] = spec.length
    docs["dst_off"] = dst_off
    docs["dst_cap"] = cap
    docs["op"] = hu.OP_CONVERT_UTF16LE_TO_UTF8
    batch = hu.Batch(docs, src, dst)
    log(f"utf16 documents: {n} docs, {2 * total_w} B, assembled in {time.time() - t_gen:.1f}s")
    best, best_us = batch.tune(f"utf16-documents-{n}", stream)
    log(f"utf16 documents: tuned sub_tiles={best.sub_tiles} groups_per_cu={best.groups_per_cu} ({best_us:.0f} us)")
    g = batch.graph(best)
    try:
        hu.graph_launch(g, stream)
        t_graph = _time_on_stream(lambda: hu.graph_launch(g, stream), stream, args.steps)
    finally:
        torch.cuda.synchronize()
        hu.graph_destroy(g)
    errs, counts = batch.results_host()
    oracle_check, cpu_leg = _oracle_utf16_documents(args, spec, cap, dst_off, errs, counts, dst)
    out_bytes = int(counts[errs == 0].sum())

    recs = torch.zeros((n, 16), dtype=torch.uint8, device=dev)
    ws = hu.workspace(hu.OP_CONVERT_UTF16LE_TO_UTF8, int(spec.length.max()), dev)
    wsp, wsb = hu.workspace_ptr(ws)
    sh = hu.stream_handle(stream)
    sp, dp, rp = src.data_ptr(), dst.data_ptr(), recs.data_ptr()
    f = hu.lib.convert_utf16le_to_utf8_async
    so = [int(2 * x) for x in offs[:-1]]
    ls = [int(x) for x in spec.length]
    do = [int(x) for x in dst_off]
    cp = [int(x) for x in cap]
    fns = [(lambda i=i: f(sp + so[i], ls[i], dp + do[i], cp[i], rp + 16 * i, wsp, wsb, sh)) for i in range(n)]
    t_plain = _plain_launches(hu, fns, stream, args.plain_passes)
    torch.cuda.synchronize()
    h = recs.cpu().numpy().reshape(-1).view([("error", "<i4"), ("reserved", "<i4"), ("count", "<u8")])
    if not (np.array_equal(h["error"], errs) and np.array_equal(h["count"], counts)):
        raise RuntimeError("utf16 documents: batched and per-document results differ")
    algo = 2 * total_w + out_bytes
    return {
        "workload": f"{n} UTF-16LE documents -> UTF-8, lengths uniform 64 B-4 MiB, mixed profiles, "
                    f"0.5% unpaired surrogates, HIP graph replay",
        "docs": n, "input_bytes": 2 * total_w, "docs_with_errors": int(spec.injected.sum()),
        "tuning": {"sub_tiles": best.sub_tiles, "groups_per_cu": best.groups_per_cu, "tile_bytes": 4096 * best.sub_tiles},
        "batched_graph": {"ms": round(t_graph * 1e3, 3), "docs_per_s": round(n / t_graph, 1),
                          "GBps": round(algo / t_graph / 1e9, 1),
                          "pct_peak": round(100 * algo / t_graph / 1e9 / PEAK_HBM_GBS, 1)},
        "plain_per_document_launches": {"ms": round(t_plain * 1e3, 3), "docs_per_s": round(n / t_plain, 1),
                                        "GBps": round(algo / t_plain / 1e9, 1)},
        "speedup_batched_vs_plain": round(t_plain / t_graph, 2),
        "oracle_agrees": oracle_check,
        "cpu_oracle": cpu_leg,
    }


def _oracle_utf16_documents(args, spec, cap, dst_off, errs, counts, dst):
    """Every document of the UTF-16 batch converted by the oracle with the
    batch's capacity (host threads, runs of documents, each into its own
    scratch output): (error, count) of each compared with the batch's; the
    output bytes of a seeded sample of documents compared with the batch's
    output. Returns (check record, CPU timing of the oracle pass)."""
    import numpy as np

    import oracle
    n = spec.length.size
    lens = spec.length.astype(np.uint64)
    injected = np.nonzero(spec.injected)[0]
    own = {int(d): spec.doc(int(d)) for d in injected}    # documents with an injected error: own copies
    src_addr = np.zeros(n, dtype=np.uint64)
    for d in range(n):
        if d in own:
            src_addr[d] = own[d].ctypes.data
        else:
            src_addr[d] = spec.pools[spec.profiles[d]].u16.ctypes.data + 2 * int(spec.start[d])
    rng = np.random.default_rng(wl_seed_sample(spec))
    sample = np.sort(rng.choice(n, size=min(n, args.docs16_sample), replace=False))
    in_sample = np.zeros(n, dtype=bool)
    in_sample[sample] = True
    gpu_out = {int(d): dst[int(dst_off[d]):int(dst_off[d]) + int(counts[d])].cpu().numpy()
               for d in sample if errs[d] == 0}
    workers = _workers()
    parts = _chunks(n, 64 * workers)
    mismatched = []

    def run(ab):
        a, e = ab
        caps = cap[a:e].astype(np.uint64)
        buf = np.empty(int(caps.sum()) + 1, dtype=np.uint8)
        offs = np.concatenate([[0], np.cumsum(caps)[:-1]]).astype(np.uint64)
        r = oracle.many_convert_at(True, src_addr[a:e], lens[a:e], buf.ctypes.data + offs, caps)
        for k in range(e - a):
            d = a + k
            if in_sample[d] and r[0][k] == 0 and d in gpu_out:
                o = int(offs[k])
                if not np.array_equal(buf[o:o + int(r[1][k])], gpu_out[d]):
                    mismatched.append(d)
        return r
    t0 = time.perf_counter()
    res = _pool_map(run, parts, workers)
    t_cpu = time.perf_counter() - t0
    oe = np.concatenate([r[0] for r in res])
    oc = np.concatenate([r[1] for r in res])
    if not (np.array_equal(oe, errs) and np.array_equal(oc, counts)):
        k = int(np.nonzero((oe != errs) | (oc != counts))[0][0])
        raise RuntimeError(f"utf16 documents: doc {k}: batch {(errs[k], counts[k])} != oracle {(oe[k], oc[k])}")
    if mismatched:
        raise RuntimeError(f"utf16 documents: output of doc {mismatched[0]} differs from the oracle's")
    moved = 2 * int(lens.sum()) + int(oc[oe == 0].sum())
    check = {"docs_checked": int(n), "results_equal": True, "docs_with_errors": int((oe != 0).sum()),
             "output_sample_docs": int(len(gpu_out)),
             "output_sample_bytes": int(sum(v.size for v in gpu_out.values()))}
    cpu = {"docs_per_s": round(n / t_cpu, 1), "GBps": round(moved / t_cpu / 1e9, 3), "threads": workers,
           "seconds": round(t_cpu, 3)}
    return check, cpu


def wl_seed_sample(spec) -> int:
    """Seed of the output sample of the UTF-16 batch (fixed per batch size)."""
    return 210910433 + 4 + int(spec.length.size)


def _trace_records(hu, tr, arena):
    """REQUEST_DTYPE records of a trace; outputs go to a host arena used as a ring."""
    import numpy as np
    n = tr.arrival_ns.size
    rec = np.zeros(n, dtype=hu.REQUEST_DTYPE)
    rec["tag"] = np.arange(n)
    rec["op"] = tr.ops
    rec["src"] = [x.ctypes.data for x in tr.inputs]
    units = np.array([x.size for x in tr.inputs], dtype=np.uint64)
    rec["n_units"] = units
    cap = np.where(tr.ops == 2, units, 3 * units).astype(np.uint64)
    out_bytes = np.where(tr.ops == 2, 2 * cap, cap).astype(np.uint64)
    span = arena.nbytes - int(out_bytes.max()) - 16
    assert span > 0
    start = (np.concatenate([[0], np.cumsum((out_bytes + 15) // 16 * 16)[:-1]]) % span).astype(np.uint64)
    rec["dst"] = arena.ctypes.data + start
    rec["dst_cap"] = cap
    return rec


def _oracle_requests(tr, rec):
    """The oracle's result for every request of a trace: with the capacity of
    the worst case (one word per UTF-8 byte, three bytes per UTF-16 word) a
    conversion's result is its length function's (the same first error, the
    same count), which the oracle computes for each request where it lies in
    host memory (host threads, runs of requests). Returns (errors, counts,
    CPU seconds)."""
    import numpy as np

    import oracle
    n = rec.size
    errs = np.zeros(n, dtype=np.int32)
    counts = np.zeros(n, dtype=np.uint64)
    workers = _workers()
    t0 = time.perf_counter()
    for utf16 in (False, True):
        idx = np.nonzero((tr.ops == 5) == utf16)[0]
        addrs, units = rec["src"][idx], rec["n_units"][idx]

        def run(ab, addrs=addrs, units=units, utf16=utf16):
            a, e = ab
            return oracle.many_at(1, utf16, addrs[a:e], units[a:e])
        res = _pool_map(run, _chunks(idx.size, 16 * workers), workers)
        if res:
            errs[idx] = np.concatenate([r[0] for r in res])
            counts[idx] = np.concatenate([r[1] for r in res])
    return errs, counts, time.perf_counter() - t0


def _oracle_request_latency(tr, rec, n_sample):
    """Host time of single oracle conversions, one request at a time (the
    first n_sample requests of the trace): the CPU beside the served path."""
    import numpy as np

    import oracle
    m = min(n_sample, rec.size)
    cap = int(max(rec["dst_cap"][:m].max(), 1))
    scratch = np.empty(2 * cap, dtype=np.uint8)
    lat = np.zeros(m, dtype=np.int64)
    for k in range(m):
        utf16 = bool(tr.ops[k] == 5)
        t0 = time.perf_counter_ns()
        oracle.convert_raw(utf16, int(rec["src"][k]), int(rec["n_units"][k]), scratch.ctypes.data,
                           int(rec["dst_cap"][k]))
        lat[k] = time.perf_counter_ns() - t0
    return {"requests": int(m), "threads": 1, "p50_us": round(float(np.percentile(lat, 50)) * 1e-3, 2),
            "p99_us": round(float(np.percentile(lat, 99)) * 1e-3, 2),
            "mean_us": round(float(lat.mean()) * 1e-3, 2)}


def _serve_once(hu, srv, tr, rec, n_use, label, want_err, want_cnt):
    """Replays the first n_use requests of the trace; checks every result
    (kind and position of errors included) against the oracle's."""
    import numpy as np
    srv.reset_stats()
    t0 = time.perf_counter()
    comps = srv.replay(rec[:n_use], tr.arrival_ns[:n_use])
    wall = time.perf_counter() - t0
    st = srv.stats()
    err = comps["error"]
    cnt = comps["count"]
    bad = (err != want_err[:n_use]) | (cnt != want_cnt[:n_use])
    if np.any(bad):
        k = int(np.nonzero(bad)[0][0])
        raise RuntimeError(f"{label}: request {k}: result ({err[k]}, {cnt[k]}) != oracle "
                           f"({want_err[k]}, {want_cnt[k]})")
    lat = comps["latency_ns"].astype(np.float64)
    ends = tr.arrival_ns[:n_use] + comps["latency_ns"]
    makespan = float(ends.max() - tr.arrival_ns[0]) * 1e-9
    moved = st["input_bytes"] + st["output_bytes"]
    offered = n_use / max(float(tr.arrival_ns[n_use - 1] - tr.arrival_ns[0]) * 1e-9, 1e-9)
    done_rate = n_use / makespan
    return {
        "requests": int(n_use),
        "p50_ms": round(st["p50_ns"] * 1e-6, 3), "p99_ms": round(st["p99_ns"] * 1e-6, 3),
        "mean_ms": round(float(lat.mean()) * 1e-6, 3),
        "GBps": round(moved / makespan / 1e9, 2),
        "completed_per_s": round(done_rate, 1),
        "saturated": bool(done_rate < 0.95 * offered),
        "mean_batch": round(st["mean_batch"], 1),
        "device_busy_frac": round(st["device_ns"] * 1e-9 / makespan, 3),
        "replay_wall_s": round(wall, 2),
        "oracle_agrees": True,
        "requests_with_errors": int((err != 0).sum()),
    }


SWEEP_SIZES = (1, 16, 256, 4096, 65536, 1 << 20, 16 << 20, 256 << 20)


def _prefix8(text, n):
    """The longest character-aligned UTF-8 prefix of at most n bytes (at least
    one character) and its UTF-16LE words."""
    import numpy as np
    if not hasattr(text, "_starts"):
        text._starts = (text.char_starts_u8, text.char_starts_u16)
    cs8, cs16 = text._starts
    k = max(int(np.searchsorted(cs8, n, side="right")) - 1, 1)   # at least one character
    return text.u8[:int(cs8[k])], text.u16[:int(cs16[k])]


def bench_size_sweep(args, hu, wl, dev, stream, text):
    """Single-buffer calls from 1 B to 256 MiB of the mixed profile, both
    directions: per-call time back to back (async, HIP events) and one
    synchronous call at a time (host clock)."""
    import torch
    out = {}
    sh = hu.stream_handle(stream)
    # the UTF-16 side of the largest prefix has the most tiles (2 bytes per word)
    ws = hu.workspace(hu.OP_CONVERT_UTF16LE_TO_UTF8, max(SWEEP_SIZES), dev)
    wsp, wsb = hu.workspace_ptr(ws)
    rec = torch.zeros(16, dtype=torch.uint8, device=dev)
    for size in SWEEP_SIZES:
        u8, u16 = _prefix8(text, size)
        s8 = torch.from_numpy(u8.copy()).to(dev)
        s16 = torch.from_numpy(u16.view("<i2").copy()).to(dev)
        d16 = torch.empty(max(u8.size, 1), dtype=torch.int16, device=dev)
        d8 = torch.empty(max(3 * u16.size, 1), dtype=torch.uint8, device=dev)
        reps = max(5, min(1000, int(2e8 // max(u8.size, 1))))
        entry = {"utf8_bytes": int(u8.size), "utf16_words": int(u16.size)}
        for name, call, scall, moved in (
            ("u8u16", lambda: hu.lib.convert_utf8_to_utf16le_async(s8.data_ptr(), u8.size, d16.data_ptr(), u8.size,
                                                                   rec.data_ptr(), wsp, wsb, sh),
             lambda: hu.lib.convert_utf8_to_utf16le(s8.data_ptr(), u8.size, d16.data_ptr(), u8.size, sh),
             u8.size + 2 * u16.size),
            ("u16u8", lambda: hu.lib.convert_utf16le_to_utf8_async(s16.data_ptr(), u16.size, d8.data_ptr(),
                                                                   3 * u16.size, rec.data_ptr(), wsp, wsb, sh),
             lambda: hu.lib.convert_utf16le_to_utf8(s16.data_ptr(), u16.size, d8.data_ptr(), 3 * u16.size, sh),
             2 * u16.size + u8.size)):
            rc = call()
            if rc != 0:
                raise RuntimeError(f"size sweep {size} {name}: enqueue failed with {hu.error_name(rc)}")
            t_async = _time_on_stream(call, stream, reps)
            srep = max(3, min(200, reps))
            scall()
            t0 = time.perf_counter()
            for _ in range(srep):
                r = scall()
            t_sync = (time.perf_counter() - t0) / srep
            if r.error != 0:
                raise RuntimeError(f"size sweep {size} {name}: error {r.error}")
            entry[name] = {"async_us": round(t_async * 1e6, 2), "sync_us": round(t_sync * 1e6, 2),
                           "GBps_async": round(moved / t_async / 1e9, 2)}
        out[str(size)] = entry
        log(f"size sweep {size} B: " + ", ".join(f"{k} {v['async_us']} us" for k, v in entry.items()
                                                  if isinstance(v, dict)))
    return out


def bench_serving(args, hu, wl):
    """Open-loop Poisson request traces through the continuous-batching server
    and through the plain one-request-at-a-time path."""
    import numpy as np
    rates = [float(r) for r in args.serve_rates.split(",") if r]
    arena = np.empty(1 << 30, dtype=np.uint8)
    arena[::4096] = 0                      # touch the pages before timing
    out = {"pool_bytes": 8 << 30, "duration_s": args.serve_seconds, "rates": {}}
    srv = hu.Server(pool_bytes=8 << 30, batch_bytes=256 << 20, slots=3)
    plain = hu.Server(pool_bytes=1 << 30, batch_bytes=64 << 20, plain=True)
    try:
        for rate in rates:
            t_gen = time.time()
            tr = wl.request_trace(rate, args.serve_seconds)
            rec = _trace_records(hu, tr, arena)
            n = rec.size
            log(f"serving {rate:.0f}/s: {n} requests, {sum(x.nbytes for x in tr.inputs) / 1e9:.2f} GB input, "
                f"generated in {time.time() - t_gen:.1f}s")
            want_err, want_cnt, t_or = _oracle_requests(tr, rec)
            log(f"serving {rate:.0f}/s: oracle results of all requests in {t_or:.1f}s")
            served = _serve_once(hu, srv, tr, rec, n, f"served {rate:.0f}/s", want_err, want_cnt)
            log(f"serving {rate:.0f}/s: served p50 {served['p50_ms']} ms p99 {served['p99_ms']} ms "
                f"{served['GBps']} GB/s")
            n_plain = min(n, args.serve_plain_max)
            pl = _serve_once(hu, plain, tr, rec, n_plain, f"plain {rate:.0f}/s", want_err, want_cnt)
            log(f"serving {rate:.0f}/s: plain p50 {pl['p50_ms']} ms p99 {pl['p99_ms']} ms {pl['GBps']} GB/s")
            out["rates"][f"{rate:.0f}"] = {
                "requests": int(n),
                "offered_input_GBps": round(sum(x.nbytes for x in tr.inputs) / args.serve_seconds / 1e9, 3),
                "served": served,
                "plain_per_request": pl,
                "oracle_requests_checked": int(n),
            }
            if "oracle_latency" not in out:
                out["oracle_latency"] = _oracle_request_latency(tr, rec, args.serve_oracle_sample)
    finally:
        srv.close()
        plain.close()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size-mib", type=int, default=256, help="UTF-8 bytes per profile (MiB)")
    ap.add_argument("--profiles", default="latin,cyrillic,cjk,emoji")
    ap.add_argument("--copies", type=int, default=2,
                    help="input copies per profile, used in turn by successive steps (no repetition re-reads "
                         "an input the one before it left in the Infinity Cache)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", default="", help="comma list of ops to run (default all): "
                    "u8u16,u16u8,len8,len16,val8,val16,nv8u16,nv16u8,u8u16be,u16beu8 "
                    "(nv: non-validating conversions; be: UTF-16 big endian)")
    ap.add_argument("--no-1mib", action="store_true", help="skip the 1 MiB single-buffer workload")
    ap.add_argument("--reps-1mib", type=int, default=2000, help="repetitions of each 1 MiB call")
    ap.add_argument("--no-batched", action="store_true", help="skip the two batched document workloads")
    ap.add_argument("--docs8", type=int, default=100_000, help="UTF-8 documents in the batched workload")
    ap.add_argument("--docs16", type=int, default=10_000, help="UTF-16LE documents in the batched workload")
    ap.add_argument("--docs16-sample", type=int, default=1000,
                    help="UTF-16 documents whose output bytes are compared with the oracle's")
    ap.add_argument("--plain-passes", type=int, default=2, help="timed passes of the per-document launches")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving traces")
    ap.add_argument("--no-sweep", action="store_true", help="skip the input-size sweep")
    ap.add_argument("--sync-docs", type=int, default=10_000,
                    help="documents of the UTF-8 batch also run as synchronous calls (a prefix)")
    ap.add_argument("--serve-rates", default="10000,50000,200000", help="Poisson arrival rates (requests/s)")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="length of each arrival trace")
    ap.add_argument("--serve-plain-max", type=int, default=100_000,
                    help="requests of each trace replayed through the plain path (a prefix)")
    ap.add_argument("--serve-oracle-sample", type=int, default=20_000,
                    help="requests timed one at a time through the oracle (latency context)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build is single-GPU (got --gpus {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2109_10433_amd import binding as hu
    from paper_2109_10433_amd import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    sh = hu.stream_handle(stream)
    profiles = [p for p in args.profiles.split(",") if p]
    n_bytes = args.size_mib * wl.MIB
    ops_all = ["u8u16", "u16u8", "len8", "len16", "val8", "val16", "nv8u16", "nv16u8", "u8u16be", "u16beu8"]
    ops = [o for o in (args.only.split(",") if args.only else ops_all) if o]
    copies = max(1, args.copies)
    # ops with an output, and the buffer each writes (never shared: every
    # output is checked after the timed steps)
    out16_ops = [o for o in ("u8u16", "nv8u16", "u8u16be") if o in ops]
    out8_ops = [o for o in ("u16u8", "nv16u8", "u16beu8") if o in ops]

    # ---------------------------------------------------------------- inputs
    data = {}
    t_gen = time.time()
    for p in profiles:
        t = wl.large_profile(p, n_bytes)
        n8, n16 = int(t.u8.size), int(t.u16.size)
        src8 = [torch.from_numpy(t.u8.copy()).to(dev) for _ in range(copies)]
        src16 = [torch.from_numpy(t.u16.view(np.int16).copy()).to(dev) for _ in range(copies)]
        d = dict(text=t, src8=src8, src16=src16, n8=n8, n16=n16, out={})
        if {"u8u16be", "u16beu8"} & set(ops):
            # the same text in UTF-16BE: each word's two bytes swapped
            d["src16be"] = [x.view(torch.uint8).view(-1, 2).flip(1).contiguous().view(torch.int16).view(-1)
                            for x in src16]
        for o in out16_ops:
            d["out"][o] = torch.empty(n8, dtype=torch.int16, device=dev)
        for o in out8_ops:
            d["out"][o] = torch.empty(n8 + 64, dtype=torch.uint8, device=dev)
        data[p] = d
        log(f"{p}: {n8} B UTF-8, {n16} words UTF-16, {copies} input copies")
    log(f"inputs generated and uploaded in {time.time() - t_gen:.1f}s")

    max8 = max(d["n8"] for d in data.values())
    max16 = max(d["n16"] for d in data.values())
    ws8 = hu.workspace(hu.OP_CONVERT_UTF8_TO_UTF16LE, max8, dev)
    ws16 = hu.workspace(hu.OP_CONVERT_UTF16LE_TO_UTF8, max16, dev)
    w8p, w8b = hu.workspace_ptr(ws8)
    w16p, w16b = hu.workspace_ptr(ws16)

    def profile_calls(p, c):
        """The launches of profile p on its input copy c: (op, profile, fn(rec), algorithmic bytes)."""
        d = data[p]
        n8, n16 = d["n8"], d["n16"]
        s8, s16 = d["src8"][c].data_ptr(), d["src16"][c].data_ptr()
        s16be = d["src16be"][c].data_ptr() if "src16be" in d else 0
        o = {k: v.data_ptr() for k, v in d["out"].items()}
        spec = {
            "u8u16": (lambda rec: hu.lib.convert_utf8_to_utf16le_async(
                s8, n8, o["u8u16"], n8, rec, w8p, w8b, sh), n8 + 2 * n16),
            "nv8u16": (lambda rec: hu.lib.convert_valid_utf8_to_utf16le_async(
                s8, n8, o["nv8u16"], n8, rec, w8p, w8b, sh), n8 + 2 * n16),
            "u16u8": (lambda rec: hu.lib.convert_utf16le_to_utf8_async(
                s16, n16, o["u16u8"], n8 + 64, rec, w16p, w16b, sh), 2 * n16 + n8),
            "nv16u8": (lambda rec: hu.lib.convert_valid_utf16le_to_utf8_async(
                s16, n16, o["nv16u8"], n8 + 64, rec, w16p, w16b, sh), 2 * n16 + n8),
            "u8u16be": (lambda rec: hu.lib.convert_utf8_to_utf16be_async(
                s8, n8, o["u8u16be"], n8, rec, w8p, w8b, sh), n8 + 2 * n16),
            "u16beu8": (lambda rec: hu.lib.convert_utf16be_to_utf8_async(
                s16be, n16, o["u16beu8"], n8 + 64, rec, w16p, w16b, sh), 2 * n16 + n8),
            "len8": (lambda rec: hu.lib.utf16_length_from_utf8_async(s8, n8, rec, w8p, w8b, sh), n8),
            "len16": (lambda rec: hu.lib.utf8_length_from_utf16le_async(s16, n16, rec, w16p, w16b, sh), 2 * n16),
            "val8": (lambda rec: hu.lib.validate_utf8_async(s8, n8, rec, w8p, w8b, sh), n8),
            "val16": (lambda rec: hu.lib.validate_utf16le_async(s16, n16, rec, w16p, w16b, sh), 2 * n16),
        }
        return [(op, p) + spec[op] for op in ops]

    calls = [[x for p in profiles for x in profile_calls(p, c)] for c in range(copies)]
    n_calls = len(calls[0])
    recs = torch.zeros((copies, n_calls, 16), dtype=torch.uint8, device=dev)
    rec_ptrs = [[recs[c, i].data_ptr() for i in range(n_calls)] for c in range(copies)]

    def run_step(s, events=None):
        c = s % copies
        for i, (op, p, fn, _) in enumerate(calls[c]):
            if events is not None:
                events[i][0].record(stream)
            rc = fn(rec_ptrs[c][i])
            if rc != 0:
                raise RuntimeError(f"{op} {p}: enqueue failed with {hu.error_name(rc)}")
            if events is not None:
                events[i][1].record(stream)

    for s in range(args.warmup):
        run_step(s)
    torch.cuda.synchronize()

    ev = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(n_calls)]
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        run_step(s, ev[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    # ---------------------------------------------------------------- timings
    per = {}
    for i, (op, p, _, nbytes) in enumerate(calls[0]):
        ts = np.array([ev[s][i][0].elapsed_time(ev[s][i][1]) * 1e-3 for s in range(args.steps)])
        per[(op, p)] = dict(bytes=nbytes, mean_s=float(ts.mean()), min_s=float(ts.min()),
                            median_s=float(np.median(ts)), stats=_timing_stats(ts))

    # ---------------------------------------------------------------- oracle: results, outputs, CPU legs
    # Every result of the timed steps and every output buffer against the
    # oracle's, which also gives the single-thread CPU figures (each leg timed
    # on its own: the same inputs, one pass).
    host = recs.cpu().numpy()
    # input copies that some warm-up or timed step used (the others' records
    # were never written)
    ran = sorted({s % copies for s in range(args.warmup)} | {s % copies for s in range(args.steps)})
    cpu_legs = {op: {"bytes": 0, "chars": 0, "s": 0.0, "profiles": {}} for op in
                ("u8u16", "u16u8", "len8", "len16", "val8", "val16")}
    oracle_checked = {"results": 0, "outputs": 0, "output_units": 0}
    import oracle

    def timed(fn, *a):
        t1 = time.perf_counter()
        r = fn(*a)
        return r, time.perf_counter() - t1

    for p in profiles:
        d = data[p]
        t = d["text"]
        n8, n16, chars = d["n8"], d["n16"], int(t.cps.size)
        (ow, r8), s_u8u16 = timed(oracle.convert_utf8_to_utf16le, t.u8)
        (ob, r16), s_u16u8 = timed(oracle.convert_utf16le_to_utf8, t.u16)
        rl8, s_len8 = timed(oracle.utf16_length_from_utf8, t.u8)
        rl16, s_len16 = timed(oracle.utf8_length_from_utf16le, t.u16)
        rv8, s_val8 = timed(oracle.validate_utf8, t.u8)
        rv16, s_val16 = timed(oracle.validate_utf16le, t.u16)
        for op, sec, nb in (("u8u16", s_u8u16, n8 + 2 * n16), ("u16u8", s_u16u8, 2 * n16 + n8),
                            ("len8", s_len8, n8), ("len16", s_len16, 2 * n16),
                            ("val8", s_val8, n8), ("val16", s_val16, 2 * n16)):
            leg = cpu_legs[op]
            leg["bytes"] += nb
            leg["chars"] += chars
            leg["s"] += sec
            leg["profiles"][p] = {"GBps": round(nb / sec / 1e9, 3), "Gchar_per_s": round(chars / sec / 1e9, 3)}
        want = {"u8u16": r8, "nv8u16": r8, "u8u16be": r8, "u16u8": r16, "nv16u8": r16, "u16beu8": r16,
                "len8": rl8, "len16": rl16, "val8": rv8, "val16": rv16}
        for c in ran:
            for i, (op, pp, _, _) in enumerate(calls[c]):
                if pp != p:
                    continue
                r = hu.HuResult.from_buffer_copy(host[c, i].tobytes())
                if (r.error, r.count) != tuple(want[op]):
                    raise RuntimeError(f"{op} {p}: result {(r.error, r.count)} != oracle {tuple(want[op])}")
                oracle_checked["results"] += 1
        if r8.error != 0 or r16.error != 0:
            raise RuntimeError(f"{p}: the oracle rejects the profile text")
        ow_t = torch.from_numpy(ow.view(np.int16)).to(dev)
        for o in out16_ops:
            ref = ow_t if o != "u8u16be" else ow_t.view(torch.uint8).view(-1, 2).flip(1).contiguous().view(torch.int16).view(-1)
            if not torch.equal(d["out"][o][:r8.count], ref):
                raise RuntimeError(f"{o} {p}: output differs from the oracle's")
            oracle_checked["outputs"] += 1
            oracle_checked["output_units"] += int(r8.count)
        del ow_t, ow
        ob_t = torch.from_numpy(ob).to(dev)
        for o in out8_ops:
            if not torch.equal(d["out"][o][:r16.count], ob_t):
                raise RuntimeError(f"{o} {p}: output differs from the oracle's")
            oracle_checked["outputs"] += 1
            oracle_checked["output_units"] += int(r16.count)
        del ob_t, ob
    log(f"large buffers: {oracle_checked['results']} results and {oracle_checked['outputs']} outputs "
        f"equal to the oracle's")

    def agg(op):
        keys = [k for k in per if k[0] == op]
        b = sum(per[k]["bytes"] for k in keys)
        t = sum(per[k]["mean_s"] for k in keys)
        return b / t / 1e9 if t > 0 else 0.0

    detail = {}
    for (op, p), v in per.items():
        detail.setdefault(op, {})[p] = {
            "GBps": round(v["bytes"] / v["mean_s"] / 1e9, 1),
            "GBps_best": round(v["bytes"] / v["min_s"] / 1e9, 1),
            "GBps_median": round(v["bytes"] / v["median_s"] / 1e9, 1),
            "pct_peak": round(100 * v["bytes"] / v["mean_s"] / 1e9 / PEAK_HBM_GBS, 1),
            **{k: v["stats"][k] for k in ("us_min", "us_median", "us_mean", "mean_over_min_pct",
                                           "mean_within_1pct_of_min")},
        }
    for op in ops:
        detail[op]["aggregate_GBps"] = round(agg(op), 1)
    # share of the validating conversion's time that validation costs (the
    # non-validating call of the same direction beside it)
    validation_cost = {}
    for full, nv, name in (("u8u16", "nv8u16", "utf8_to_utf16le"), ("u16u8", "nv16u8", "utf16le_to_utf8")):
        if full in ops and nv in ops:
            validation_cost[name] = {p: round(1 - per[(nv, p)]["mean_s"] / per[(full, p)]["mean_s"], 3)
                                     for p in profiles}
    # extra time of the big-endian conversions over the little-endian ones
    big_endian_overhead = {}
    for le, be, name in (("u8u16", "u8u16be", "utf8_to_utf16be"), ("u16u8", "u16beu8", "utf16be_to_utf8")):
        if le in ops and be in ops:
            big_endian_overhead[name] = {p: round(per[(be, p)]["mean_s"] / per[(le, p)]["mean_s"] - 1, 3)
                                         for p in profiles}

    headline_op = "u8u16" if "u8u16" in ops else ops[0]
    value = agg(headline_op)
    launches = [k for k in per if k[0] == headline_op]
    avg_bytes = sum(per[k]["bytes"] for k in launches) / len(launches)
    avg_dur = sum(per[k]["mean_s"] for k in launches) / len(launches)
    achieved = avg_bytes / avg_dur / 1e9

    # practical ceiling: device-to-device copy of the profile size (read + write)
    cbuf_a = torch.empty(n_bytes, dtype=torch.uint8, device=dev)
    cbuf_b = torch.empty(n_bytes, dtype=torch.uint8, device=dev)
    cbuf_a.fill_(1)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        cbuf_b.copy_(cbuf_a)
    e0.record(stream)
    for _ in range(10):
        cbuf_b.copy_(cbuf_a)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * n_bytes * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del cbuf_a, cbuf_b

    traffic = None
    traffic_note = "no counter file"
    if os.path.exists(TRAFFIC_FILE):
        tf = json.load(open(TRAFFIC_FILE))
        if tf.get("kernel_sources") == kernel_source_digest() and tf.get("size_mib") == args.size_mib:
            traffic = tf.get("hbm_bytes_per_launch")
            traffic_note = tf.get("note", "")
        else:
            traffic_note = "counters taken on other kernel sources: stale"

    del data, ws8, ws16, recs, calls
    torch.cuda.empty_cache()

    # ---------------------------------------------------------------- 1 MiB buffer
    single = None
    if not args.no_1mib:
        single = bench_single_1mib(args, hu, wl, dev, stream)
        torch.cuda.empty_cache()

    # ---------------------------------------------------------------- batched documents
    batched = None
    if not args.no_batched:
        batched = {"utf8_documents": bench_utf8_documents(args, hu, wl, dev, stream)}
        torch.cuda.empty_cache()
        batched["utf16_documents"] = bench_utf16_documents(args, hu, wl, dev, stream)
        torch.cuda.empty_cache()

    serving = None
    if not args.no_serving:
        serving = bench_serving(args, hu, wl)

    sweep, sweep_text = None, None
    if not args.no_sweep:
        sweep_text = wl.make_text("mix", max(SWEEP_SIZES), wl.rng_for("size-sweep"))
        sweep = bench_size_sweep(args, hu, wl, dev, stream, sweep_text)

    # ---------------------------------------------------------------- CPU oracle
    cpu = None
    if not args.no_cpu_baseline:
        if sweep is not None:
            # the oracle on the same prefixes (up to 16 MiB): where the host catches up
            for size in SWEEP_SIZES:
                if size > (16 << 20):
                    continue
                u8, u16 = _prefix8(sweep_text, size)
                reps = max(3, min(1000, int(2e7 // max(u8.size, 1))))
                t1 = time.perf_counter()
                for _ in range(reps):
                    oracle.convert_utf8_to_utf16le(u8)
                sweep[str(size)]["u8u16"]["cpu_oracle_us"] = round((time.perf_counter() - t1) / reps * 1e6, 2)
        head = cpu_legs["u8u16"]
        cpu = {"value": round(head["bytes"] / head["s"] / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"validating UTF-8->UTF-16LE of the same {len(profiles)} x {args.size_mib} MiB profiles, "
                         f"one pass each, single thread ({head['s']:.1f} s)",
               "legs": {op: {"GBps": round(v["bytes"] / v["s"] / 1e9, 3),
                             "Gchar_per_s": round(v["chars"] / v["s"] / 1e9, 3),
                             "seconds": round(v["s"], 2), "threads": 1, "profiles": v["profiles"]}
                        for op, v in cpu_legs.items() if v["s"] > 0},
               **_cpu_info()}
        if batched is not None:
            cpu["utf8_documents"] = batched["utf8_documents"]["cpu_oracle"]
            cpu["utf16_documents"] = batched["utf16_documents"]["cpu_oracle"]
        if serving is not None and "oracle_latency" in serving:
            cpu["serving_per_request"] = serving["oracle_latency"]

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"large-buffer transcoding, {args.size_mib} MiB UTF-8 per profile",
                   "profiles": profiles, "ops_per_step": ops, "input_copies": copies,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "kernel": "hu::k_convert_u8<6, 2, false>", "traffic_note": traffic_note},
        "cpu_baseline": cpu,
        "copy_ceiling_GBps": round(copy_gbs, 1),
        "oracle_agrees": {"large_buffers": oracle_checked,
                          "single_1mib": single["oracle_agrees"] if single else None,
                          "utf8_documents": batched["utf8_documents"]["oracle_agrees"] if batched else None,
                          "utf16_documents": batched["utf16_documents"]["oracle_agrees"] if batched else None,
                          "serving_requests": ({r: v["oracle_requests_checked"] for r, v in serving["rates"].items()}
                                               if serving else None)},
        "single_1mib": single,
        "batched": batched,
        "serving": serving,
        "size_sweep": sweep,
        "detail": detail,
        "validation_cost": validation_cost or None,
        "big_endian_overhead": big_endian_overhead or None,
        "kernel_sources": kernel_source_digest(),
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
