#!/usr/bin/env python3
"""Throughput benchmark of the seed-count + approximate-edit-distance path.

Headline workload (the largest single-GPU configuration, dense candidates):
2,000 synthetic genomes = 400 random roots x 5 substitution-only strains
(1-5% divergence) x 2 Mbp = 4 Gbp, taxon = strain; 10M reads of 150 bp at 1%
error (0.9% substitutions, 0.1% indels); k=21, w=11, >= 3 seed hits, top 3,
E = 7.  One step is one classification of the whole read batch (seeding,
lookup, hit counting, top-N, filter, per-taxon counts).  `value` is measured
with the reads and the index already in HBM; `end_to_end` adds the upload of
the reads from pinned host memory and the download of every output into
pinned host memory.

Also measured (same JSON line): the plain one-launch-per-stage and graph
forms of the headline workload; the served headline workload under a memory
budget (admission control); the 500 Mbp batched workload across the E sweep
{0, 3, 7, 15} fused and per-stage, with stage 1, the Table 1 filters, both
strands and abundance; the uneven workload (2M reads up to 10 kbp,
autotuned); the served workload (Poisson traces on the 500 Mbp index).  The
CPU baseline is the plain C oracle on the machine's host cores, single-threaded
and on all cores, each the median of 3 runs on a seeded sample of the
headline reads (its index build is not timed).

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "read×candidate pairs/s and reads/s at E=5%, bit-exact; p50/p99 latency served"
HBM_PEAK_GBS = 8000.0
# Integer VALU peak of the MI355X: 256 CUs x 4 SIMD16 units x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s,
# i.e. one wave64 VALU instruction per CU per cycle.
VALU_WAVE_INSTR_PEAK = 256 * 2.4e9
VALU_LANE_OPS_PEAK = VALU_WAVE_INSTR_PEAK * 64

# Algorithmic bytes per work unit of the fused kernel (see the design notes):
#   per read          its ASCII bases in + 11 B out (read flag, E, candidate count)
#   per minimizer     its 16 B table slot
#   per occurrence    8 B from the multi-occurrence array (k-mers with several occurrences)
#   per window block  16 B of reference planes per 64 window bases
#   per candidate     19 B out
FUSED_MODEL = "bases + 16*minimizers + 8*occurrences + 16*window_blocks + 19*candidates + 11*reads"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def fused_alg_bytes(stats: dict) -> int:
    return int(stats["fused_bases"] + 16 * stats["fused_minimizers"] + 8 * stats.get("fused_occ", 0)
               + 16 * stats["fused_window_blocks"] + 19 * stats["fused_cands"] + 11 * stats["fused_reads"])


def counter_record(name: str):
    """A committed rocprofv3 counter record under profiles/, or None when it is
    missing or was taken on a different kernel source (sha256 of the sources)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for src in rec["kernel_sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return rec if h.hexdigest() == rec["source_sha256"] else None


def useful_ops(host: dict, lengths) -> np.ndarray:
    """Useful int32 lane-ops of the obstacle filter per pair: building the (2E+1)
    rows of ceil(m/64) mismatch words at 6 ops a word, plus 8 ops per row for
    each step of the walk (min(approx, E) + 1 steps)."""
    co = np.asarray(host["cand_offsets"], dtype=np.int64)
    pr = np.repeat(np.arange(len(co) - 1), np.diff(co))
    E = np.asarray(host["read_E"], dtype=np.int64)[pr]
    m = np.asarray(lengths, dtype=np.int64)[pr]
    ap = np.asarray(host["approx"], dtype=np.int64)
    rows = 2 * E + 1
    return 6 * rows * ((m + 63) // 64) + 8 * rows * (np.minimum(ap, E) + 1)


def pair_bucket(host: dict, lengths) -> np.ndarray:
    """The filter bucket of every pair of a result, as the per-stage filter
    forms them: 0 E<=7, 1 E<=15, 2 E<=31, 3..6 long bins by the 64-base blocks
    of read and window staged (<= 96, 192, 384, 768), 7 general."""
    co = np.asarray(host["cand_offsets"], dtype=np.int64)
    pr = np.repeat(np.arange(len(co) - 1), np.diff(co))
    E = np.asarray(host["read_E"], dtype=np.int64)[pr]
    m = np.asarray(lengths, dtype=np.int64)[pr]
    blocks = (m + 63) // 64 + 1 + ((m + 2 * E + 190) >> 6) + 2
    b = np.full(len(pr), 7, np.int64)
    for i, cap in reversed(list(enumerate((96, 192, 384, 768)))):
        b = np.where((E > 31) & (blocks <= cap), 3 + i, b)
    b = np.where(E <= 31, 2, b)
    b = np.where(E <= 15, 1, b)
    b = np.where(E <= 7, 0, b)
    return b


BUCKET_NAMES = ("E<=7", "E<=15", "E<=31", "long<=96", "long<=192", "long<=384", "long<=768", "general")


def _pct(v, q):
    return float(np.percentile(np.asarray(v, dtype=np.float64), q)) if len(v) else None


def time_form(mt, ix, dreads, q, steps, warmup, timing=True):
    """Warm-up steps, then `steps` timed classifications (wall clock between two
    device synchronizations); per-stage HIP-event timings averaged per step."""
    import torch
    for _ in range(warmup):
        ix.classify(dreads, **q).free()
    mt.mt_set_timing(timing)
    stage = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_cands = 0
    for _ in range(steps):
        r = ix.classify(dreads, **q)
        n_cands = r.n_cands
        r.free()
        if timing:
            for name, ms in mt.last_timings():
                stage[name] = stage.get(name, 0.0) + ms
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    mt.mt_set_timing(False)
    stats = mt.last_stats()
    return {"ms_per_step": round(dt * 1000, 4), "reads_per_s": round(dreads.n / dt, 1),
            "pairs_per_s": round(n_cands / dt, 1), "pairs": int(n_cands),
            "stages_ms": {k: round(v / steps, 4) for k, v in stage.items()}}, stats


def end_to_end(mt, ix, reads, q, steps, warmup):
    """Host reads in pinned memory -> device -> classification -> every output
    back in pinned host memory, one step after the other on one stream."""
    import ctypes as C
    import torch
    seq = torch.from_numpy(np.ascontiguousarray(reads.seq)).pin_memory()
    off = torch.from_numpy(np.ascontiguousarray(reads.offsets).view(np.int64)).pin_memory()
    n = reads.n
    cap = n * max(q.get("top_n", 3), 1)
    out = {"cand_offsets": torch.empty(n + 1, dtype=torch.int64).pin_memory(),
           "read_accepted": torch.empty(n, dtype=torch.uint8).pin_memory(),
           "read_E": torch.empty(n, dtype=torch.int16).pin_memory(),
           "genome": torch.empty(cap, dtype=torch.int32).pin_memory(),
           "diag": torch.empty(cap, dtype=torch.int64).pin_memory(),
           "hits": torch.empty(cap, dtype=torch.int32).pin_memory(),
           "approx": torch.empty(cap, dtype=torch.int16).pin_memory(),
           "accept": torch.empty(cap, dtype=torch.uint8).pin_memory()}
    hip = mt._hip()
    hip.hipMemcpyAsync.restype = C.c_int
    hip.hipMemcpyAsync.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
    stream = torch.cuda.current_stream()
    sp = C.c_void_p(stream.cuda_stream)

    def step():
        dseq = seq.to("cuda", non_blocking=True)
        doff = off.to("cuda", non_blocking=True)
        dr = mt.DeviceSeqs(dseq, doff, n, int(reads.offsets[-1]))
        r = ix.classify(dr, **q)
        nr, co, ra, re = r._reads()
        nc, (g, d, h, a, ac) = r._cands()
        assert nc <= cap
        for name, ptr, cnt in (("cand_offsets", co, nr + 1), ("read_accepted", ra, nr), ("read_E", re, nr),
                               ("genome", g, nc), ("diag", d, nc), ("hits", h, nc), ("approx", a, nc),
                               ("accept", ac, nc)):
            t = out[name]
            rc = hip.hipMemcpyAsync(C.c_void_p(t.data_ptr()), C.c_void_p(ptr), C.c_size_t(cnt * t.element_size()),
                                    2, sp)
            assert rc == 0, rc
        stream.synchronize()
        r.free()
        return nc

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        nc = step()
    dt = (time.perf_counter() - t0) / steps
    bytes_in = int(reads.offsets[-1]) + 8 * (n + 1)
    bytes_out = 8 * (n + 1) + 3 * n + 19 * nc
    return {"ms_per_step": round(dt * 1000, 3), "reads_per_s": round(n / dt, 1), "pairs_per_s": round(nc / dt, 1),
            "bytes_in": bytes_in, "bytes_out": bytes_out,
            "note": "reads uploaded from pinned host memory and every per-read and per-candidate output downloaded "
                    "into pinned host memory inside each timed step (one stream, no overlap)"}


def end_to_end_overlapped(mt, ix, reads, q, chunks: int = 32, threads: int = 4, reps: int = 3) -> dict:
    """Host to host with overlap: the batch in `chunks` pieces, each uploaded from
    pinned host memory, classified and its outputs downloaded into pinned host
    memory by one of `threads` host threads on its own stream, so that one
    piece's copies run while another's kernels do; timed from the first upload
    to the last download, the best of `reps` runs."""
    import ctypes as C
    import threading
    import torch
    n = reads.n
    offs = np.asarray(reads.offsets, dtype=np.uint64)
    bounds = [(n * i // chunks, n * (i + 1) // chunks) for i in range(chunks)]
    top = max(q.get("top_n", 3), 1)
    hip = mt._hip()
    hip.hipMemcpyAsync.restype = C.c_int
    hip.hipMemcpyAsync.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
    pieces = []
    for lo, hi in bounds:
        m = hi - lo
        seq = torch.from_numpy(np.ascontiguousarray(reads.seq[int(offs[lo]):int(offs[hi])])).pin_memory()
        off = torch.from_numpy((offs[lo:hi + 1] - offs[lo]).view(np.int64)).pin_memory()
        out = {"cand_offsets": torch.empty(m + 1, dtype=torch.int64).pin_memory(),
               "read_accepted": torch.empty(m, dtype=torch.uint8).pin_memory(),
               "read_E": torch.empty(m, dtype=torch.int16).pin_memory(),
               "genome": torch.empty(m * top, dtype=torch.int32).pin_memory(),
               "diag": torch.empty(m * top, dtype=torch.int64).pin_memory(),
               "hits": torch.empty(m * top, dtype=torch.int32).pin_memory(),
               "approx": torch.empty(m * top, dtype=torch.int16).pin_memory(),
               "accept": torch.empty(m * top, dtype=torch.uint8).pin_memory()}
        pieces.append((m, int(offs[hi] - offs[lo]), seq, off, out))
    streams = [torch.cuda.Stream() for _ in range(threads)]

    def piece(i, stream):
        m, total, seq, off, out = pieces[i]
        with torch.cuda.stream(stream):
            dr = mt.DeviceSeqs(seq.to("cuda", non_blocking=True), off.to("cuda", non_blocking=True), m, total)
            r = ix.classify(dr, stream=stream, **q)
        nr, co, ra, re = r._reads()
        nc, (g, d, h, a, ac) = r._cands()
        assert nc <= m * top
        sp = C.c_void_p(stream.cuda_stream)
        for name, ptr, cnt in (("cand_offsets", co, nr + 1), ("read_accepted", ra, nr), ("read_E", re, nr),
                               ("genome", g, nc), ("diag", d, nc), ("hits", h, nc), ("approx", a, nc),
                               ("accept", ac, nc)):
            t = out[name]
            rc = hip.hipMemcpyAsync(C.c_void_p(t.data_ptr()), C.c_void_p(ptr), C.c_size_t(cnt * t.element_size()),
                                    2, sp)
            assert rc == 0, rc
        stream.synchronize()
        r.free()
        return nc

    def run():
        pairs = [0] * chunks
        errs = []

        def worker(k):
            try:
                for i in range(k, chunks, threads):
                    pairs[i] = piece(i, streams[k])
            except Exception as e:  # noqa: BLE001
                errs.append(e)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ts = [threading.Thread(target=worker, args=(k,)) for k in range(threads)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if errs:
            raise errs[0]
        return dt, sum(pairs)

    run()  # warm-up
    gc.collect()
    gc.disable()  # the harness's garbage collection stays out of the timed runs
    try:
        runs = [run() for _ in range(reps)]
    finally:
        gc.enable()
    dt, pairs = min(runs)
    return {"ms_per_step": round(dt * 1e3, 3), "reads_per_s": round(n / dt, 1), "pairs_per_s": round(pairs / dt, 1),
            "runs_ms": [round(x * 1e3, 3) for x, _ in runs], "chunks": chunks, "threads": threads,
            "note": f"the batch in {chunks} pieces, each uploaded from pinned host memory, classified and its outputs "
                    f"downloaded into pinned host memory by one of {threads} host threads on its own stream, so "
                    "copies of one piece overlap the kernels of another"}


def serving_bench(mt, ix, pool, seconds: float, loads=(0.5, 0.8, 0.95), runs: int = 2, threads: int = 8,
                  baseline_s: float = 4.0, n_streams: int = 0, max_batch_reads: int = 0, mem_budget: int = 0,
                  q=None, workload: str = "", reads_fn=None, mean_reads: float = 25_000.5) -> dict:
    """Served requests: the server's saturated reads/s (clients submitting back
    to back), then p50 / p99 request latency (completion minus scheduled
    arrival) on Poisson traces offering each fraction in `loads` of that rate,
    `runs` traces of `seconds` each per load; then, if baseline_s > 0, the 80%
    trace served by sequential per-request solves (upload, mt_classify,
    download, one request at a time) in the per-stage and fused forms."""
    import threading
    import synth

    q = q or dict(min_hits=3, top_n=3, e_mode=mt.MT_E_CEIL_PERMILLE, e_value=50)
    reads_fn = reads_fn or (lambda n, m: synth.request_reads(pool, n, m))

    def trace(seed, n, qps):
        return synth.request_trace(seed, n, qps, lengths=synth.SERVED_LENGTHS)

    def run_served(tr, paced: bool, stop_after: float | None = None):
        # the harness's own garbage collection stays out of the measured latencies
        gc.collect()
        gc.disable()
        try:
            return run_served_(tr, paced, stop_after)
        finally:
            gc.enable()

    def run_served_(tr, paced: bool, stop_after: float | None = None):
        recs = [None] * len(tr)
        ids = [None] * len(tr)
        errs = []
        with mt.Server(ix, mem_budget_bytes=mem_budget, pinned_arena_bytes=4 << 30, max_queued_requests=8192,
                       n_streams=n_streams, max_batch_reads=max_batch_reads) as sv:
            t0 = time.monotonic_ns()
            stop_at = None if stop_after is None else t0 + int(stop_after * 1e9)
            avail = [threading.Semaphore(0) for _ in range(threads)]

            def client(k):
                try:
                    for i in range(k, len(tr), threads):
                        arr_ns = t0 + int(tr[i][0] * 1e9) if paced else time.monotonic_ns()
                        if stop_at is not None and time.monotonic_ns() >= stop_at:
                            break
                        if paced:
                            while True:
                                d = (arr_ns - time.monotonic_ns()) / 1e9
                                if d <= 0:
                                    break
                                time.sleep(min(d, 0.002))
                        reads = reads_fn(tr[i][1], tr[i][2])
                        while True:
                            try:
                                rid = sv.submit(reads, **q)
                                break
                            except mt.MTError as e:
                                if e.status != mt._abi.MT_EAGAIN:
                                    raise
                                time.sleep(0.0002)
                        ids[i] = (rid, arr_ns)
                        avail[k].release()
                    avail[k].release()  # end marker
                except Exception as e:  # noqa: BLE001
                    errs.append(e)
                    avail[k].release()

            def waiter(k):
                try:
                    i = k
                    while True:
                        avail[k].acquire()
                        if i >= len(tr) or ids[i] is None:
                            return
                        rid, arr_ns = ids[i]
                        res = sv.wait(rid)
                        s_ns, d_ns = res.times_ns()
                        res.free()
                        recs[i] = (arr_ns, s_ns, d_ns, tr[i][1])
                        i += threads
                except Exception as e:  # noqa: BLE001
                    errs.append(e)

            ts = [threading.Thread(target=client, args=(k,)) for k in range(threads)]
            ws = [threading.Thread(target=waiter, args=(k,)) for k in range(threads)]
            for x in ts + ws:
                x.start()
            for x in ts + ws:
                x.join()
            st = sv.stats()
        if errs:
            raise errs[0]
        return [r for r in recs if r is not None], st

    def concurrency(st):
        """Mean number of batches whose kernels ran at once while any ran, and the
        fraction of that time with two or more (HIP events on the worker streams)."""
        u = st.get("kernel_ms_union", 0.0)
        if u <= 0:
            return None
        return {"mean_batches_running": round(st["kernel_ms_sum"] / u, 3),
                "frac_time_two_or_more": round(st["kernel_ms_overlap"] / u, 3)}

    def summarize(recs):
        if not recs:
            return None
        lat = [(d - a) / 1e6 for a, _, d, _ in recs]
        reads = sum(r[3] for r in recs)
        span = (max(r[2] for r in recs) - min(r[0] for r in recs)) / 1e9
        return {"requests": len(recs), "reads": int(reads), "reads_per_s": round(reads / span, 1),
                "p50_ms": round(_pct(lat, 50), 3), "p99_ms": round(_pct(lat, 99), 3),
                "mean_ms": round(float(np.mean(lat)), 3)}

    out = {"workload": workload, "threads": threads, "n_streams": n_streams or 4,
           "max_batch_reads": max_batch_reads or 1 << 18, "trace_seconds": seconds, "runs_per_load": runs}
    run_served(trace(99, 64, 1.0), paced=False)  # warm-up
    recs, st = run_served(trace(3, 1_000_000, 1.0), paced=False, stop_after=min(seconds, 10.0))
    out["saturated"] = summarize(recs)
    out["saturated"]["server"] = st
    out["saturated"]["kernel_concurrency"] = concurrency(st)
    out["mem_budget_bytes"] = st["mem_budget_bytes"]
    log(f"[serve] saturated: {out['saturated']}")
    sat_rps = out["saturated"]["reads_per_s"]
    out["traces"] = []
    for i, load in enumerate(loads):
        qps = load * sat_rps / mean_reads
        per = []
        for k in range(runs):
            recs, st = run_served(trace(3 + i + 10 * k, max(20, int(qps * seconds)), qps), paced=True)
            sm = summarize(recs)
            sm["server"] = st
            sm["kernel_concurrency"] = concurrency(st)
            per.append(sm)
        p50 = [x["p50_ms"] for x in per]
        p99 = [x["p99_ms"] for x in per]
        agg = {"offered_load": load, "qps": round(qps, 1), "runs": per,
               "reads_per_s": round(float(np.mean([x["reads_per_s"] for x in per])), 1),
               "p50_ms": round(float(np.median(p50)), 3), "p99_ms": round(float(np.median(p99)), 3),
               "p50_spread_ms": [min(p50), max(p50)], "p99_spread_ms": [min(p99), max(p99)]}
        out["traces"].append(agg)
        log(f"[serve] load {load}: p50 {agg['p50_ms']} ms (spread {agg['p50_spread_ms']}), "
            f"p99 {agg['p99_ms']} ms (spread {agg['p99_spread_ms']}), {agg['reads_per_s']:.3e} reads/s")
    if baseline_s <= 0:
        return out
    qps = 0.8 * sat_rps / mean_reads
    tr = trace(4, max(20, int(qps * baseline_s * 4)), qps)
    for name, mode in (("sequential_per_stage", mt.MT_MODE_PER_STAGE), ("sequential_fused", mt.MT_MODE_FUSED)):
        recs = []
        t0 = time.monotonic_ns()
        stop_at = t0 + int(baseline_s * 1e9)
        for arr_s, n, m in tr:
            arr_ns = t0 + int(arr_s * 1e9)
            now = time.monotonic_ns()
            if now >= stop_at:
                break
            if arr_ns > now:
                time.sleep((arr_ns - now) / 1e9)
            reads = reads_fn(n, m)
            res = ix.classify(mt.to_device(reads), mode=mode, **q)
            res.to_host()
            res.free()
            recs.append((arr_ns, arr_ns, time.monotonic_ns(), n))
        sm = summarize(recs)
        sm.update({"offered_load": 0.8, "qps": round(qps, 1), "of_trace_requests": len(tr)})
        out[name] = sm
        log(f"[serve] {name}: {sm}")
    return out


def trace_overlap(path: str, kernel: str = "k_fused") -> dict:
    """From a rocprofv3 kernel-trace CSV: the dispatches of `kernel`, the queues
    they ran on, the time during which dispatches of two or more different
    queues were running at once, and how many dispatches overlapped one of
    another queue."""
    import csv
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if kernel in r.get("Kernel_Name", ""):
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r.get("Queue_Id", r.get("Stream_Id"))))
    rows.sort()
    queues = sorted(set(q for _, _, q in rows))
    overlapped = 0
    for i, (s0, e0, q0) in enumerate(rows):
        for j in range(max(0, i - 64), min(len(rows), i + 64)):
            s1, e1, q1 = rows[j]
            if j != i and q1 != q0 and s1 < e0 and s0 < e1:
                overlapped += 1
                break
    ev = sorted([(s, 1, q) for s, _, q in rows] + [(e, -1, q) for _, e, q in rows])
    active, busy, multi, last = {}, 0, 0, None
    for t, d, q in ev:
        if last is not None:
            n_q = sum(1 for v in active.values() if v > 0)
            if n_q >= 1:
                busy += t - last
            if n_q >= 2:
                multi += t - last
        active[q] = active.get(q, 0) + d
        last = t
    return {"kernel": kernel, "dispatches": len(rows), "queues": len(queues),
            "dispatches_overlapping_another_queue": overlapped,
            "busy_ns": busy, "ns_with_two_or_more_queues_running": multi,
            "share_of_busy_time_overlapped": round(multi / busy, 4) if busy else 0.0}


def counter_summary(paths) -> dict:
    """rocprofv3 --pmc CSVs -> {kernel [lds bytes]: {counter: mean per dispatch, dispatches: n}}.  Launches of
    one kernel with different dynamic LDS sizes (the long-read filter's bins) are kept apart."""
    import csv
    acc = {}
    for path in paths:
        with open(path) as f:
            for r in csv.DictReader(f):
                name = r["Kernel_Name"].split("(")[0]
                lds = r.get("LDS_Block_Size", "")
                wg = r.get("Workgroup_Size", "")
                key = f"{name} [lds {lds}, wg {wg}]" if "k_filter_long" in name else name
                d = acc.setdefault(key, {})
                c = d.setdefault(r["Counter_Name"], {})
                did = r.get("Dispatch_Id", r.get("Correlation_Id"))
                c[did] = c.get(did, 0.0) + float(r["Counter_Value"])  # rows of one dispatch add up
    out = {}
    for key, d in sorted(acc.items()):
        out[key] = {cn: round(sum(v.values()) / len(v), 1) for cn, v in sorted(d.items())}
        out[key]["dispatches"] = max(len(v) for v in d.values())
    return out


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(ga, reads, q, single_reads: int, all_reads: int, runs: int = 3) -> dict:
    """The oracle on a seeded sample of the headline reads: single-threaded and
    on every core it may use (OMP_NUM_THREADS), each the median of `runs`."""
    import oracle
    oracle.set_threads(0)
    t = time.time()
    oix = oracle.Index(ga, 21, 11)
    log(f"[cpu] oracle index built in {time.time() - t:.1f}s (not timed)")
    rng = np.random.default_rng(7)
    out = {}
    for leg, threads, size in (("single", 1, single_reads), ("all", 0, all_reads)):
        used = oracle.set_threads(threads)
        idx = np.sort(rng.choice(reads.n, min(size, reads.n), replace=False))
        sample = reads.subset(idx)
        times, pairs = [], 0
        for _ in range(runs):
            t = time.perf_counter()
            res = oix.classify(sample, q["min_hits"], q["top_n"], q["e_mode"], q["e_value"])
            times.append(time.perf_counter() - t)
            pairs = len(res["genome"])
        med = float(np.median(times))
        out[leg] = {"value": round(pairs / med, 1), "unit": "pairs/s", "reads_per_s": round(sample.n / med, 1),
                    "cores": used, "runs_s": [round(x, 3) for x in times],
                    "sample": f"{sample.n} reads drawn uniformly (seed 7) from the headline batch"}
        log(f"[cpu] {leg}: {out[leg]}")
    oracle.set_threads(0)
    del oix
    a = out["all"]
    return {"value": a["value"], "unit": "pairs/s", "cores": a["cores"], "kind": "oracle",
            "sample": a["sample"] + f", median of {runs} runs on {a['cores']} threads",
            "reads_per_s": a["reads_per_s"], "runs_s": a["runs_s"], "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count(), "single_thread": out["single"]}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="strains", choices=["strains", "batched", "uneven"],
                    help="the headline workload (default: the strain database, the largest configuration)")
    ap.add_argument("--mode", default="fused", choices=["fused", "graph", "per_stage"])
    ap.add_argument("--reads", type=int, default=0, help="reads of the headline workload (0: its full size)")
    ap.add_argument("--extras", type=int, default=1,
                    help="1: also the other workloads, forms, serving and the CPU baseline; 0: the headline only")
    ap.add_argument("--cpu", type=int, default=1, help="0 skips the CPU baseline")
    ap.add_argument("--cpu-single-reads", type=int, default=150_000)
    ap.add_argument("--cpu-all-reads", type=int, default=2_000_000)
    ap.add_argument("--serve-seconds", type=float, default=20.0, help="length of each served trace")
    ap.add_argument("--serve-runs", type=int, default=2, help="traces per offered load")
    ap.add_argument("--serve-streams", type=int, default=0, help="server worker streams (0: the library default)")
    ap.add_argument("--serve-max-batch", type=int, default=0,
                    help="server batch cap in reads (0: the library default)")
    ap.add_argument("--serve-baseline-s", type=float, default=4.0,
                    help="seconds of sequential per-request solves on the 80%% trace (0 skips them)")
    ap.add_argument("--only", default="", help="comma list of extras to run (strains_forms, e2e, cpu, "
                                                 "strains_served, batched, uneven, serving); empty: all")
    ap.add_argument("--extra-steps", type=int, default=10, help="timed steps of each extra measurement")
    ap.add_argument("--autotune", type=int, default=1,
                    help="1: autotune the filter variants of the uneven workload first; 0: built-in defaults")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 times), to scale HBM byte counters")
    ap.add_argument("--counter-summary", nargs="+", default=[], metavar="CSV",
                    help="only summarise rocprofv3 --pmc counter CSVs: per kernel (and dynamic LDS size), the mean "
                         "of every counter per dispatch")
    ap.add_argument("--trace-overlap", default="", metavar="CSV",
                    help="only summarise a rocprofv3 kernel-trace CSV: how often k_fused dispatches of different "
                         "queues (the server's worker streams) ran at the same time")
    args = ap.parse_args()
    if args.trace_overlap:
        print(json.dumps(trace_overlap(args.trace_overlap)), flush=True)
        return 0
    if args.counter_summary:
        print(json.dumps(counter_summary(args.counter_summary), indent=1), flush=True)
        return 0
    if args.calibrate_copy:
        import torch
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "copies": 3}), flush=True)
        return 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(reads are independent; see the design notes for how it would shard).", file=sys.stderr)
        return 2
    only = set(x for x in args.only.split(",") if x)

    def want(name):
        return args.extras and (not only or name in only)

    import torch
    import paper_2311_02029_amd as mt
    import synth

    torch.cuda.set_device(0)
    t_start = time.time()
    mode = {"fused": mt.MT_MODE_FUSED, "graph": mt.MT_MODE_FUSED_GRAPH, "per_stage": mt.MT_MODE_PER_STAGE}[args.mode]
    extras = {}

    def guarded(name, fn):
        t = time.time()
        try:
            extras[name] = fn()
        except Exception as e:  # noqa: BLE001  (an extra must not lose the headline)
            extras[name] = {"error": f"{type(e).__name__}: {e}"}
        log(f"[bench] {name} done in {time.time() - t:.1f}s")

    # ------------------------------------------------------------ headline --
    t = time.time()
    if args.workload == "strains":
        db = synth.workload_strains_db()
        reads = synth.workload_strain_reads(db, args.reads or 10_000_000)
        q = dict(min_hits=3, top_n=3, e_mode=mt.MT_E_FIXED, e_value=7)
        workload = (f"dense-candidate strains: 2,000 genomes (400 random roots x 5 substitution-only strains, "
                    f"1-5% divergence) x 2 Mbp = 4 Gbp, taxon = strain; {reads.n} reads x 150 bp at 1% error; "
                    f"k=21 w=11, min_hits=3, top_n=3, E=7")
    elif args.workload == "uneven":
        db = synth.workload_batched_db()
        reads = synth.workload_uneven_reads(db, args.reads or 2_000_000)
        q = dict(min_hits=3, top_n=3, e_mode=mt.MT_E_CEIL_PERMILLE, e_value=50)
        workload = (f"uneven: 500 Mbp / 200 genomes, {reads.n} reads (95% of 75-300 bp, 5% of 1-10 kbp), k=21 w=11, "
                    f"min_hits=3, top_n=3, E=ceil(5% of length)")
    else:
        db = synth.workload_batched_db()
        reads = synth.workload_batched_reads(db, args.reads or 1_000_000)
        q = dict(min_hits=3, top_n=3, e_mode=mt.MT_E_FIXED, e_value=7)
        workload = f"batched: 500 Mbp / 200 genomes, {reads.n} x 150 bp reads, k=21 w=11, min_hits=3, top_n=3, E=7"
    ga = db.ascii()
    del db
    log(f"[bench] headline data generated in {time.time() - t:.1f}s: {ga.n} genomes, {reads.n} reads")
    dreads = mt.to_device(reads)
    t = time.time()
    ix = mt.Index(mt.to_device(ga), 21, 11)
    torch.cuda.synchronize()
    index_s = time.time() - t
    info = ix.info()
    log(f"[bench] index built in {index_s:.2f}s: {info['n_minimizers']} minimizers, {info['n_keys']} keys, "
        f"{info['device_bytes'] / 2**30:.2f} GiB")
    if args.workload == "uneven":
        ix.autotune(dreads, reps=3, **q)
    qm = dict(q, mode=mode)
    head, stats = time_form(mt, ix, dreads, qm, args.steps, args.warmup, timing=True)
    log(f"[bench] headline {args.mode}: {head['ms_per_step']} ms/step, {head['pairs_per_s']:.3e} pairs/s, "
        f"{head['reads_per_s']:.3e} reads/s; stages {head['stages_ms']}")
    # the same steps without event timing: the figure the line reports
    plain, _ = time_form(mt, ix, dreads, qm, args.steps, 1, timing=False)
    log(f"[bench] headline without event timing: {plain['ms_per_step']} ms/step")

    # roofline of the dominant kernel (the fused kernel) from its live HIP-event time
    roofline = None
    stages = head["stages_ms"]
    if "fused" in stages and stats.get("fused_reads"):
        dur_s = stages["fused"] / 1000.0
        alg = fused_alg_bytes(stats)
        ach = alg / dur_s / 1e9
        recname = {"strains": "k_fused_hbm_counters_4gbp_10m.json",
                   "batched": "k_fused_hbm_counters_500mbp_1m.json"}.get(args.workload)
        rec = counter_record(recname) if recname and not args.reads else None
        roofline = {"kernel": "k_fused", "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                    "traffic": int(rec["traffic_bytes_per_dispatch"]) if rec else None,
                    "avg_ms": round(stages["fused"], 4), "algorithmic_bytes": alg, "model": FUSED_MODEL,
                    "units": {k: int(stats[k]) for k in ("fused_reads", "fused_bases", "fused_minimizers", "fused_occ",
                                                         "fused_window_blocks", "fused_cands") if k in stats}}
        if rec:
            roofline["traffic_gbs"] = round(rec["traffic_bytes_per_dispatch"] / dur_s / 1e9, 1)
            roofline["traffic_frac"] = round(roofline["traffic_gbs"] / HBM_PEAK_GBS, 4)
        vrec = counter_record({"strains": "k_fused_valu_counters_4gbp_10m.json",
                               "batched": "k_fused_valu_counters_500mbp_1m.json"}.get(args.workload, "-"))
        if vrec and not args.reads:
            vi = float(vrec["per_dispatch"]["SQ_INSTS_VALU"])
            roofline["valu"] = {"wave_instructions": int(vi), "peak_lane_ops_per_s": VALU_LANE_OPS_PEAK,
                                "issue_frac": round(vi / (dur_s * VALU_WAVE_INSTR_PEAK), 4),
                                "per_read": {k: round(float(v) / stats["fused_reads"], 1)
                                             for k, v in vrec["per_dispatch"].items()}}
        r = ix.classify(dreads, **qm)
        host = r.to_host()
        r.free()
        uo = int(useful_ops(host, reads.lengths()).sum())
        roofline["filter_useful_ops"] = {
            "lane_ops": uo, "model": "per pair 6*(2E+1)*ceil(m/64) + 8*(2E+1)*(min(approx,E)+1) int32 ops",
            "frac_of_peak_over_kernel_time": round(uo / (dur_s * VALU_LANE_OPS_PEAK), 5)}
    log(f"[bench] roofline: {json.dumps(roofline)}")

    # ------------------------------------------------------ other forms --
    if want("strains_forms"):
        def forms():
            out = {}
            for name, m in (("per_stage", mt.MT_MODE_PER_STAGE), ("graph", mt.MT_MODE_FUSED_GRAPH),
                            ("fused", mt.MT_MODE_FUSED)):
                if m == mode:
                    continue
                res, _ = time_form(mt, ix, dreads, dict(q, mode=m), max(3, args.steps // 4), 1, timing=False)
                res.pop("stages_ms")
                out[name] = res
                log(f"[bench] headline {name}: {res}")
            out[args.mode] = {k: v for k, v in plain.items() if k != "stages_ms"}
            # every candidate kept (top_n = 0): the same reads, all locations with >= min_hits filtered
            res, _ = time_form(mt, ix, dreads, dict(q, mode=mode, top_n=0), max(3, args.steps // 4), 1, timing=False)
            res.pop("stages_ms")
            out["keep_all_fused"] = res
            log(f"[bench] headline keep-all: {res}")
            return out
        guarded("forms", forms)
    if want("e2e"):
        guarded("end_to_end", lambda: end_to_end(mt, ix, reads, qm, max(3, args.steps // 4), 1))
        log(f"[bench] end to end: {extras.get('end_to_end')}")
        guarded("end_to_end_overlapped", lambda: end_to_end_overlapped(mt, ix, reads, qm))
        log(f"[bench] end to end, overlapped: {extras.get('end_to_end_overlapped')}")
    if want("cpu") and args.cpu:
        guarded("cpu_baseline", lambda: cpu_baseline(ga, reads, q, args.cpu_single_reads, args.cpu_all_reads))
    if want("strains_served") and args.workload == "strains":
        def strains_served():
            # requests of the headline's reads (the first n of the batch), a tight memory budget
            rq = dict(q)

            def reads_fn(n, m):
                return synth.SeqSet(seq=reads.seq[:n * 150], offsets=reads.offsets[:n + 1])
            budget = 256 << 20
            return serving_bench(mt, ix, None, seconds=args.serve_seconds / 2, loads=(0.8,), runs=2,
                                 baseline_s=0, mem_budget=budget, max_batch_reads=1 << 18, q=rq,
                                 reads_fn=reads_fn,
                                 workload="the headline database resident; Poisson requests of U{1..50,000} reads "
                                          "of the headline batch (150 bp, 1% error), E=7; admission by a "
                                          f"{budget >> 20} MiB device-memory budget")
        guarded("strains_served", strains_served)
    del ix, dreads
    torch.cuda.empty_cache()

    # ------------------------------------------------- batched workload --
    bdb = None
    if want("batched") or want("serving") or want("uneven"):
        t = time.time()
        bdb = synth.workload_batched_db()
        bga = bdb.ascii()
        bix = mt.Index(mt.to_device(bga), 21, 11)
        log(f"[bench] 500 Mbp database and index in {time.time() - t:.1f}s")
    if want("batched"):
        def batched():
            breads = synth.workload_batched_reads(bdb, 1_000_000)
            dr = mt.to_device(breads)
            out = {"workload": "batched: 500 Mbp / 200 genomes (GC ~ U(0.3, 0.7)), 1M x 150 bp, 0.1-1% "
                               "substitutions, 0.01-0.1% indels, k=21 w=11, min_hits=3, top_n=3", "E_sweep": {}}
            for E in (0, 3, 7, 15):
                row = {}
                for name, m in (("fused", mt.MT_MODE_FUSED), ("per_stage", mt.MT_MODE_PER_STAGE)):
                    res, st = time_form(mt, bix, dr, dict(min_hits=3, top_n=3, e_value=E, mode=m),
                                        args.extra_steps, 2, timing=True)
                    row[name] = res
                    if name == "fused" and "fused" in res["stages_ms"]:
                        d = res["stages_ms"]["fused"] / 1000.0
                        alg = fused_alg_bytes(st)
                        row["fused_roofline"] = {"kernel": "k_fused", "bound": "hbm", "achieved": round(alg / d / 1e9, 1),
                                                 "frac": round(alg / d / 1e9 / HBM_PEAK_GBS, 4), "avg_ms": round(d * 1e3, 4),
                                                 "algorithmic_bytes": alg}
                    if name == "per_stage":
                        r = bix.classify(dr, min_hits=3, top_n=3, e_value=E, mode=m)
                        host = r.to_host()
                        r.free()
                        uo = useful_ops(host, breads.lengths())
                        bk = pair_bucket(host, breads.lengths())
                        per = {}
                        for b in np.unique(bk):
                            key = "filter " + BUCKET_NAMES[b]
                            if key in res["stages_ms"]:
                                ms = res["stages_ms"][key]
                                per[BUCKET_NAMES[b]] = {"pairs": int((bk == b).sum()), "ms": ms,
                                                        "useful_ops_frac": round(float(uo[bk == b].sum()) /
                                                                                 (ms / 1e3 * VALU_LANE_OPS_PEAK), 4)}
                        row["per_stage_filter"] = per
                        # the index gather alone (per-stage k_lookup): per read minimizer its 8 B key in, its
                        # 16 B table slot, 8 B value and 4 B count out
                        lk = res["stages_ms"].get("lookup")
                        if lk and st.get("n_minimizers"):
                            gb = 36 * int(st["n_minimizers"]) / (lk / 1e3) / 1e9
                            row["per_stage_lookup_roofline"] = {
                                "kernel": "k_lookup", "bound": "hbm", "achieved": round(gb, 1), "unit": "GB/s",
                                "frac": round(gb / HBM_PEAK_GBS, 4), "lookups": int(st["n_minimizers"]),
                                "ms": lk, "model": "36 B per lookup: 8 B key in, 16 B slot, 12 B out"}
                row["fused_over_per_stage"] = round(row["per_stage"]["ms_per_step"] / row["fused"]["ms_per_step"], 3)
                out["E_sweep"][str(E)] = row
                log(f"[bench] batched E={E}: fused {row['fused']['ms_per_step']} ms, per-stage "
                    f"{row['per_stage']['ms_per_step']} ms")
            res, _ = time_form(mt, bix, dr, dict(min_hits=3, top_n=3, e_value=7, mode=mt.MT_MODE_FUSED_GRAPH),
                               args.extra_steps, 2, timing=False)
            res.pop("stages_ms")
            out["graph_E7"] = res
            # E = 31 per stage: the rows-in-lanes filter with one 64-lane group per pair
            res, _ = time_form(mt, bix, dr, dict(min_hits=3, top_n=3, e_value=31, mode=mt.MT_MODE_PER_STAGE),
                               args.extra_steps, 2, timing=True)
            r = bix.classify(dr, min_hits=3, top_n=3, e_value=31, mode=mt.MT_MODE_PER_STAGE)
            host = r.to_host()
            r.free()
            uo = float(useful_ops(host, breads.lengths()).sum())
            ms = res["stages_ms"].get("filter E<=31")
            res["filter_useful_ops_frac"] = round(uo / (ms / 1e3 * VALU_LANE_OPS_PEAK), 4) if ms else None
            out["per_stage_E31"] = res
            # stage 1 on the same index and batch
            hits = bix.containment(dr)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(5):
                hits = bix.containment(dr)
                sel, mx = mt.select_genomes(hits, 1, 10_000)
            torch.cuda.synchronize()
            c_ms = (time.perf_counter() - t0) * 1000.0 / 5
            total = int(hits.cpu().numpy().view(np.uint64).sum())
            out["containment"] = {"ms": round(c_ms, 3), "reads_per_s": round(breads.n / (c_ms / 1000.0), 1),
                                  "seed_hits_per_s": round(total / (c_ms / 1000.0), 1), "seed_hits": total,
                                  "kept_at_1e-4": int(sel.numel()), "max_hits": mx}
            # Table 1's filters on the batch's own pair stream
            r = bix.classify(dr, min_hits=3, top_n=3, e_value=7, mode=mt.MT_MODE_FUSED)
            h = r.to_host()
            co = np.asarray(h["cand_offsets"], dtype=np.int64)
            pr = np.repeat(np.arange(len(co) - 1, dtype=np.int64), np.diff(co)).astype(np.int32)
            pe = np.asarray(h["read_E"], dtype=np.uint16)[pr]
            dev = [torch.from_numpy(x).cuda() for x in (pr, np.asarray(h["genome"]).view(np.int32),
                                                        np.asarray(h["diag"], dtype=np.int64), pe.view(np.int16))]
            filters = {}
            for name, kind in (("obstacle", mt.MT_FILTER_OBSTACLE), ("hamming", mt.MT_FILTER_HAMMING),
                               ("base_count", mt.MT_FILTER_BASE_COUNT), ("qgram", mt.MT_FILTER_QGRAM),
                               ("shd", mt.MT_FILTER_SHD)):
                bix.filter_pairs(dr, *dev, kind=kind)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(5):
                    _, acc = bix.filter_pairs(dr, *dev, kind=kind)
                torch.cuda.synchronize()
                f_ms = (time.perf_counter() - t0) * 1000.0 / 5
                filters[name] = {"ms": round(f_ms, 3), "pairs_per_s": round(len(pr) / (f_ms / 1000.0), 1),
                                 "accepted": round(float(acc.float().mean().item()), 4)}
            filters["pairs"] = int(len(pr))
            out["filters"] = filters
            # stage 3b on the classification result
            bix.abundance(r)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(5):
                counts, ab, kept = bix.abundance(r)
            torch.cuda.synchronize()
            a_ms = (time.perf_counter() - t0) * 1000.0 / 5
            out["abundance"] = {"ms": round(a_ms, 3), "kept_taxa": kept, "max_abundance": round(float(ab.max().item()), 6)}
            r.free()
            # both strands: half the reads taken from the reverse strand
            flipped = synth.from_reverse_strand(np.random.default_rng(77), breads, 0.5)
            dflip = mt.to_device(flipped)
            st = {}
            for name, m in (("fused", mt.MT_MODE_FUSED), ("per_stage", mt.MT_MODE_PER_STAGE)):
                res, _ = time_form(mt, bix, dflip, dict(min_hits=3, top_n=3, e_value=7, mode=m, strands=2), 3, 1,
                                   timing=False)
                res.pop("stages_ms")
                st[name] = res
            out["strands"] = st
            return out
        guarded("batched", batched)
    if want("serving"):
        def serving():
            pool = synth.served_read_pool(bdb)
            return serving_bench(mt, bix, pool, seconds=args.serve_seconds, runs=args.serve_runs,
                                 n_streams=args.serve_streams, max_batch_reads=args.serve_max_batch,
                                 baseline_s=args.serve_baseline_s,
                                 workload="requests of U{1..50,000} reads x one length in {100..250} bp (16 lengths), "
                                          "0.5% error, E=ceil(5% of length), min_hits=3, top_n=3, 500 Mbp index "
                                          "resident; Poisson arrivals")
        guarded("serving", serving)
    if want("uneven"):
        def uneven():
            ur = synth.workload_uneven_reads(bdb, 2_000_000)
            dr = mt.to_device(ur)
            uq = dict(min_hits=3, top_n=3, e_mode=mt.MT_E_CEIL_PERMILLE, e_value=50)
            t0 = time.time()
            mt.tune_reset()
            tune = bix.autotune(dr, reps=3, **uq) if args.autotune else mt.tune_info()
            out = {"workload": "uneven: 500 Mbp; 2M reads, 95% of U{75..300} bp, 5% of U{1000..10000} bp at 2% "
                               "substitutions + 3% indels; E=ceil(5% of length); autotuned",
                   "autotune_s": round(time.time() - t0, 1),
                   "tuning": {b["name"]: b["current"] for b in tune if b["pairs"]}}
            for name, m in (("fused", mt.MT_MODE_FUSED), ("per_stage", mt.MT_MODE_PER_STAGE),
                            ("graph", mt.MT_MODE_FUSED_GRAPH)):
                res, _ = time_form(mt, bix, dr, dict(uq, mode=m), max(1, min(3, args.extra_steps)), 1,
                                   timing=(name != "graph"))
                out[name] = res
            out["fused_over_per_stage"] = round(out["per_stage"]["ms_per_step"] / out["fused"]["ms_per_step"], 3)
            r = bix.classify(dr, mode=mt.MT_MODE_PER_STAGE, **uq)
            host = r.to_host()
            r.free()
            uo = useful_ops(host, ur.lengths())
            bk = pair_bucket(host, ur.lengths())
            per = {}
            for b in np.unique(bk):
                key = "filter " + BUCKET_NAMES[b]
                ms = out["per_stage"]["stages_ms"].get(key)
                if ms:
                    per[BUCKET_NAMES[b]] = {"pairs": int((bk == b).sum()), "ms": ms,
                                            "useful_ops_frac": round(float(uo[bk == b].sum()) /
                                                                     (ms / 1e3 * VALU_LANE_OPS_PEAK), 4)}
            out["per_stage_filter"] = per
            return out
        guarded("uneven", uneven)

    line = {
        "metric": METRIC, "value": plain["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": plain["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": workload, "reads": reads.n, "bases": int(reads.offsets[-1]),
                   "pairs_per_step": plain["pairs"], "mode": args.mode, "parallelism": "single GPU",
                   "inputs": "reads and index resident in HBM"},
        "reads_per_s": plain["reads_per_s"],
        "index_build_s": round(index_s, 3),
        "stages_ms": head["stages_ms"],
        "roofline": roofline,
        "cpu_baseline": extras.pop("cpu_baseline", None),
        "end_to_end": extras.pop("end_to_end", None),
        "forms": extras.pop("forms", None),
    }
    line.update(extras)
    line["bench_wall_s"] = round(time.time() - t_start, 1)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
