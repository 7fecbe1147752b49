#!/usr/bin/env python3
"""Throughput benchmark of the seed-count + approximate-edit-distance path.

Workload: 200 synthetic genomes totalling 500 Mbp (per-genome GC ~ U(0.3, 0.7)),
1M reads of 150 bp with 0.1-1% substitutions and 0.01-0.1% indels, k=21,
w=11, >= 3 seed hits, top 3 locations, E = 7 (5% of 150).  One step is one
classification of the whole read batch (seeding, lookup, hit counting, top-N,
filter, per-taxon counts) with the reads and the index already in HBM.

Prints one JSON line.  The CPU baseline is the plain C oracle timed on a
bounded sample of the same reads (its index build is not timed).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "read×candidate pairs/s and reads/s at E=5%, bit-exact; p50/p99 latency served"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per work unit of each stage (see the design notes):
#   lookup: per minimizer  8 B k-mer in + 16 B table slot + 8 B value out + 4 B count out
#   fused:  per read       its ASCII bases + 16 B slot per minimizer + 16 B reference
#                          planes per 64 window bases + 19 B per candidate out + 11 B per read out
LOOKUP_BYTES_PER_MIN = 8 + 16 + 8 + 4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(kernel: str):
    """HBM bytes per dispatch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    record of this kernel (scaled by the plain-copy calibration), or None when
    the record is missing or was taken on a different kernel source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_fused_hbm_counters_500mbp_1m.json")
    if kernel != "fused" or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for src in rec["kernel_sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    return int(rec["traffic_bytes_per_dispatch"])


def filter_useful_ops(host: dict, lengths) -> int:
    """Useful int32 lane-ops of the filter over a result's pairs: building
    the (2E+1) rows of ceil(m/64) mismatch words at 6 ops a word, plus 8 ops
    per row for each step of the obstacle walk (min(approx, E) + 1 steps)."""
    co = np.asarray(host["cand_offsets"], dtype=np.int64)
    pr = np.repeat(np.arange(len(co) - 1), np.diff(co))
    E = np.asarray(host["read_E"], dtype=np.int64)[pr]
    m = np.asarray(lengths, dtype=np.int64)[pr]
    ap = np.asarray(host["approx"], dtype=np.int64)
    rows = 2 * E + 1
    return int((6 * rows * ((m + 63) // 64) + 8 * rows * (np.minimum(ap, E) + 1)).sum())


def _pct(v, q):
    return float(np.percentile(np.asarray(v, dtype=np.float64), q)) if len(v) else None


def serving_bench(mt, ix, pool, seconds: float = 2.0, loads=(0.5, 0.8, 0.95), threads: int = 8,
                  baseline_s: float = 4.0, n_streams: int = 0, max_batch_reads: int = 0) -> dict:
    """The served workload: requests of U{1..50,000} reads of one length in
    100-250 bp at 0.5% error, E = ceil(5% of length), against the resident
    index.  Measures
      * the server's saturated reads/s (closed loop: `threads` clients submit
        back to back for `seconds`);
      * p50 / p99 request latency (completion minus scheduled arrival) on
        Poisson traces offering each fraction in `loads` of that rate;
      * the same trace served by sequential per-request solves (upload,
        mt_classify, download, one request at a time), plain per-stage form
        and fused form, for at most `baseline_s` seconds each.
    """
    import threading
    import synth
    from collections import deque

    q = dict(min_hits=3, top_n=3, e_mode=mt.MT_E_CEIL_PERMILLE, e_value=50)
    mean_reads = 25_000.5

    def trace(seed, n, qps):
        return synth.request_trace(seed, n, qps, lengths=synth.SERVED_LENGTHS)

    def run_served(tr, paced: bool, stop_after: float | None = None):
        """Submits tr (paced by arrival, or back to back); returns per-request
        (arrival_ns, submit_ns, done_ns, reads) and the wall interval."""
        recs = [None] * len(tr)
        ids = [None] * len(tr)
        errs = []
        with mt.Server(ix, pinned_arena_bytes=4 << 30, max_queued_requests=8192, n_streams=n_streams,
                       max_batch_reads=max_batch_reads) as sv:
            t0 = time.monotonic_ns()
            stop_at = None if stop_after is None else t0 + int(stop_after * 1e9)
            avail = [threading.Semaphore(0) for _ in range(threads)]
            done_n = [0] * threads

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
                        reads = synth.request_reads(pool, tr[i][1], tr[i][2])
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
                        done_n[k] += 1
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
        if errs:
            raise errs[0]
        recs = [r for r in recs if r is not None]
        return recs, t0

    def summarize(recs, t0):
        if not recs:
            return None
        lat = [(d - a) / 1e6 for a, _, d, _ in recs]
        reads = sum(r[3] for r in recs)
        first = min(r[0] for r in recs)
        last = max(r[2] for r in recs)
        span = (last - first) / 1e9
        return {"requests": len(recs), "reads": int(reads), "reads_per_s": round(reads / span, 1),
                "p50_ms": round(_pct(lat, 50), 3), "p99_ms": round(_pct(lat, 99), 3),
                "mean_ms": round(float(np.mean(lat)), 3)}

    out = {"workload": "requests of U{1..50,000} reads x one length in {100..250} bp (16 lengths), 0.5% error, "
                       "E=ceil(5% of length), min_hits=3, top_n=3, 500 Mbp index resident; Poisson arrivals",
           "threads": threads, "n_streams": n_streams or 4, "max_batch_reads": max_batch_reads or 1 << 18}
    # warm up the server path (allocator, pinned buffers)
    recs, t0 = run_served(trace(99, 64, 1.0), paced=False)
    # saturation: back to back for `seconds`
    recs, t0 = run_served(trace(3, 100_000, 1.0), paced=False, stop_after=seconds)
    sat = summarize(recs, t0)
    out["saturated"] = sat
    log(f"[serve] saturated: {sat}")
    sat_rps = sat["reads_per_s"]
    out["traces"] = []
    for i, load in enumerate(loads):
        qps = load * sat_rps / mean_reads
        n = max(20, int(qps * seconds))
        recs, t0 = run_served(trace(3 + i, n, qps), paced=True)
        sm = summarize(recs, t0)
        sm.update({"offered_load": load, "qps": round(qps, 1)})
        out["traces"].append(sm)
        log(f"[serve] load {load}: {sm}")

    if baseline_s <= 0:
        return out
    # sequential per-request solves on the 80% trace
    qps = 0.8 * sat_rps / mean_reads
    tr = trace(4, max(20, int(qps * seconds)), qps)
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
            reads = synth.request_reads(pool, n, m)
            res = ix.classify(mt.to_device(reads), mode=mode, **q)
            res.to_host()
            res.free()
            recs.append((arr_ns, arr_ns, time.monotonic_ns(), n))
        sm = summarize(recs, t0)
        sm.update({"offered_load": 0.8, "qps": round(qps, 1), "of_trace_requests": len(tr)})
        out[name] = sm
        log(f"[serve] {name}: {sm}")
    return out


def measured_valu(kernel: str):
    """VALU wave-instructions per dispatch from the committed rocprofv3 SQ_INSTS_VALU
    record of this kernel, or None when it is missing or was taken on a different
    kernel source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_fused_valu_counters_500mbp_1m.json")
    if kernel != "fused" or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for src in rec["kernel_sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    return float(rec["per_dispatch"]["SQ_INSTS_VALU"])


# Integer VALU peak of the MI355X: 256 CUs x 4 SIMD16 units x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s,
# i.e. one wave64 VALU instruction per CU per cycle.
VALU_WAVE_INSTR_PEAK = 256 * 2.4e9


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="fused", choices=["fused", "graph", "per_stage"],
                    help="fused: the fused kernel (launched eagerly); graph: the same launches replayed as one "
                         "HIP graph; per_stage: one launch per step")
    ap.add_argument("--E", type=int, default=7)
    ap.add_argument("--reads", type=int, default=1_000_000)
    ap.add_argument("--top-n", type=int, default=3, help="candidates kept per read (0 keeps all)")
    ap.add_argument("--workload", default="batched", choices=["batched", "uneven", "strains"],
                    help="batched: 500 Mbp, 1M x 150 bp, E=7 (the metric's workload); uneven: same database, "
                         "2M reads of 75-300 bp plus 5%% of 1-10 kbp, E=ceil(5%% of length); strains: 2,000 "
                         "near-duplicate strain genomes (4 Gbp), 10M x 150 bp at 1%% error, E=7")
    ap.add_argument("--cpu-reads", type=int, default=-1,
                    help="reads in the oracle's timed sample (0 skips the CPU baseline; default: 1M for batched, "
                         "2000 for uneven, 0 for strains)")
    ap.add_argument("--no-timing", action="store_true", help="do not record per-stage HIP events")
    ap.add_argument("--genomes", type=int, default=200, help="genomes of 2.5 Mbp in the database")
    ap.add_argument("--autotune", type=int, default=-1,
                    help="1: time the filter variants on the batch (up to 2M reads) first and keep the fastest per "
                         "bucket (default: on for the uneven workload); 0: built-in defaults")
    ap.add_argument("--serving", type=int, default=1,
                    help="1: also measure the served workload (batched workload only); 0: skip it")
    ap.add_argument("--strands-bench", type=int, default=1,
                    help="also time both-strand classification of the batch with half its reads reversed")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="length of each served trace")
    ap.add_argument("--serve-streams", type=int, default=0, help="server worker streams (0: library default, 4)")
    ap.add_argument("--serve-threads", type=int, default=8, help="client threads submitting served requests")
    ap.add_argument("--serve-max-batch", type=int, default=0,
                    help="reads per served device batch (0: library default, 262,144)")
    ap.add_argument("--serve-only", action="store_true",
                    help="only the served workload (no batched timing, no sequential baselines)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 times), to scale HBM byte counters")
    args = ap.parse_args()
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

    import torch
    import paper_2311_02029_amd as mt
    import synth

    torch.cuda.set_device(0)
    t = time.time()
    if args.cpu_reads < 0:
        args.cpu_reads = {"batched": 1_000_000, "uneven": 2000, "strains": 0}[args.workload]
    e_mode, e_value = mt.MT_E_FIXED, args.E
    if args.workload == "strains":
        log("[bench] generating 400 roots x 5 strains x 2 Mbp and the reads ...")
        db = synth.workload_strains_db()
        reads = synth.workload_strain_reads(db, args.reads if args.reads != 1_000_000 else 10_000_000)
        workload = (f"strains: 2,000 genomes (400 roots x 5 strains, 1-5% divergence) = 4 Gbp, {reads.n} x 150 bp "
                    f"at 1% error, k=21 w=11, min_hits=3, top_n={args.top_n}, E={args.E}")
    elif args.workload == "uneven":
        log("[bench] generating the database and the uneven reads ...")
        db = synth.workload_batched_db(n_genomes=args.genomes)
        reads = synth.workload_uneven_reads(db, args.reads if args.reads != 1_000_000 else 2_000_000)
        e_mode, e_value = mt.MT_E_CEIL_PERMILLE, 50
        workload = (f"uneven: 500 Mbp / 200 genomes, {reads.n} reads (95% of 75-300 bp, 5% of 1-10 kbp), k=21 w=11, "
                    f"min_hits=3, top_n={args.top_n}, E=ceil(5% of length)")
    else:
        db = synth.workload_batched_db(n_genomes=args.genomes)
        reads = synth.workload_batched_reads(db, args.reads)
        workload = (f"500 Mbp / 200 genomes, {reads.n // 1000}k x 150 bp reads, k=21 w=11, min_hits=3, top_n={args.top_n}, "
                    f"E={args.E}")
    log(f"[bench] data generated in {time.time() - t:.1f}s: {db.n} genomes, {reads.n} reads, "
        f"{int(reads.offsets[-1])} bases")
    pool = None
    if args.serving and args.workload == "batched":
        t = time.time()
        pool = synth.served_read_pool(db)
        log(f"[bench] served read pool generated in {time.time() - t:.1f}s")
    ga = db.ascii()
    dgen = mt.to_device(ga)
    dreads = mt.to_device(reads)
    del db
    torch.cuda.synchronize()
    log(f"[bench] inputs on the device")
    mt.mt_set_timing(True)
    t = time.time()
    ix = mt.Index(dgen, 21, 11)
    torch.cuda.synchronize()
    index_s = time.time() - t
    log(f"[bench] index stages (ms): {mt.last_timings()}")
    mt.mt_set_timing(False)
    info = ix.info()
    log(f"[bench] index built in {index_s:.2f}s: {info['n_minimizers']} minimizers, {info['n_keys']} keys, "
        f"{info['device_bytes'] / 2**30:.2f} GiB")
    del dgen

    if args.serve_only:
        sv = serving_bench(mt, ix, pool, seconds=args.serve_seconds, n_streams=args.serve_streams,
                           max_batch_reads=args.serve_max_batch, baseline_s=0, threads=args.serve_threads)
        print(json.dumps({"metric": "served reads/s; p50/p99 request latency", "serving": sv}), flush=True)
        return 0

    mode = {"fused": mt.MT_MODE_FUSED, "graph": mt.MT_MODE_FUSED_GRAPH, "per_stage": mt.MT_MODE_PER_STAGE}[args.mode]
    q = dict(min_hits=3, top_n=args.top_n, e_mode=e_mode, e_value=e_value, mode=mode)

    tune = None
    if args.autotune < 0:
        args.autotune = 1 if args.workload == "uneven" else 0
    if args.autotune:
        t = time.time()
        sample = mt.to_device(reads.subset(np.arange(min(reads.n, 2_000_000))))
        info = ix.autotune(sample, reps=3, **{k: v for k, v in q.items() if k != "mode"})
        del sample
        tune = {b["name"]: b["current"] for b in info if b["pairs"]}
        log(f"[bench] autotuned in {time.time() - t:.1f}s: "
            + "; ".join(f"{b['name']} ({b['pairs']} pairs): " + ", ".join(f"{k} {v:.3f} ms" for k, v in b["ms"].items())
                        for b in info if b["pairs"]))

    n_cands = 0
    for i in range(args.warmup):
        t = time.time()
        r = ix.classify(dreads, **q)
        n_cands = r.n_cands
        r.free()
        log(f"[bench] warmup step {i}: {time.time() - t:.3f}s")
    log(f"[bench] warmup done ({args.warmup} steps), {n_cands} candidates per step")

    mt.mt_set_timing(not args.no_timing)
    stage_ms: dict[str, float] = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = ix.classify(dreads, **q)
        n_cands = r.n_cands
        r.free()
        if not args.no_timing:
            for name, ms in mt.last_timings():
                stage_ms[name] = stage_ms.get(name, 0.0) + ms
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mt.mt_set_timing(False)
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    pairs_s = n_cands / (ms_per_step / 1000.0)
    reads_s = reads.n / (ms_per_step / 1000.0)
    stages = {k: v / args.steps for k, v in stage_ms.items()}
    log(f"[bench] {ms_per_step:.3f} ms/step, {pairs_s:.3e} pairs/s, {reads_s:.3e} reads/s")
    log(f"[bench] stages (ms/step): {json.dumps({k: round(v, 4) for k, v in stages.items()})}")

    # Roofline of the dominant kernel from the live HIP-event timings.
    roofline = None
    stats = mt.last_stats() if hasattr(mt, "last_stats") else {}
    if stages:
        dom = max(stages, key=stages.get)
        dur_s = stages[dom] / 1000.0
        if dom == "lookup" and stats.get("n_minimizers"):
            alg = stats["n_minimizers"] * LOOKUP_BYTES_PER_MIN
        elif dom == "fused" and stats.get("n_minimizers"):
            alg = (stats["fused_bases"] + 16 * stats["fused_minimizers"] + 16 * stats["fused_window_blocks"]
                   + 19 * stats["fused_cands"] + 11 * stats["fused_reads"])
        else:
            alg = None
        if alg is not None and dur_s > 0:
            ach = alg / dur_s / 1e9
            roofline = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                        "traffic": measured_traffic(dom) if args.workload == "batched" else None,
                        "avg_ms": round(stages[dom], 4), "algorithmic_bytes": int(alg)}
            if roofline["traffic"]:
                # the same launch against its counter-measured HBM bytes
                roofline["traffic_gbs"] = round(roofline["traffic"] / dur_s / 1e9, 1)
                roofline["traffic_frac"] = round(roofline["traffic_gbs"] / HBM_PEAK_GBS, 4)
            vi = measured_valu(dom) if args.workload == "batched" and args.E == 7 else None
            if vi is not None:
                # counter-measured VALU issue against the integer VALU peak (same live duration)
                roofline["valu"] = {"wave_instructions": int(vi), "peak_lane_ops_per_s": VALU_WAVE_INSTR_PEAK * 64,
                                    "issue_frac": round(vi / (dur_s * VALU_WAVE_INSTR_PEAK), 4)}
            if dom == "fused":
                # the filter's useful integer work by the op model (one more, untimed classification)
                r = ix.classify(dreads, **q)
                useful = filter_useful_ops(r.to_host(), reads.lengths())
                r.free()
                roofline["filter_useful_ops"] = {
                    "lane_ops": int(useful),
                    "model": "per pair 6*(2E+1)*ceil(m/64) + 8*(2E+1)*(min(approx,E)+1) int32 ops",
                    "frac_of_peak_over_kernel_time": round(useful / (dur_s * VALU_WAVE_INSTR_PEAK * 64), 5)}
        else:
            roofline = {"kernel": dom, "bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": None, "traffic": None, "avg_ms": round(stages[dom], 4)}

    # Stage 1 (containment search) on the same resident index and batch.
    containment = None
    if args.workload == "batched" and hasattr(ix, "containment"):
        hits = ix.containment(dreads)  # warm
        torch.cuda.synchronize()
        reps = 5
        t = time.perf_counter()
        for _ in range(reps):
            hits = ix.containment(dreads)
            sel, mx = mt.select_genomes(hits, 1, 10_000)
        torch.cuda.synchronize()
        c_ms = (time.perf_counter() - t) * 1000.0 / reps
        total = int(hits.cpu().numpy().view(np.uint64).sum())
        containment = {"ms": round(c_ms, 3), "reads_per_s": round(reads.n / (c_ms / 1000.0), 1),
                       "seed_hits_per_s": round(total / (c_ms / 1000.0), 1), "seed_hits": total,
                       "genomes": int(hits.numel()), "kept_at_1e-4": int(sel.numel()), "max_hits": mx}
        log(f"[bench] containment: {json.dumps(containment)}")

    # Table 1's filter choice on the batch's own pair stream (its candidates).
    filters = None
    if args.workload == "batched" and hasattr(mt, "MT_FILTER_HAMMING"):
        r = ix.classify(dreads, **q)
        h = r.to_host()
        r.free()
        co = np.asarray(h["cand_offsets"], dtype=np.int64)
        pr = np.repeat(np.arange(len(co) - 1, dtype=np.int64), np.diff(co)).astype(np.int32)
        pe = np.asarray(h["read_E"], dtype=np.uint16)[pr]
        dev = [torch.from_numpy(x).cuda() for x in (pr, np.asarray(h["genome"]).view(np.int32),
                                                    np.asarray(h["diag"], dtype=np.int64), pe.view(np.int16))]
        filters = {}
        for name, kind in (("obstacle", mt.MT_FILTER_OBSTACLE), ("hamming", mt.MT_FILTER_HAMMING),
                           ("base_count", mt.MT_FILTER_BASE_COUNT), ("qgram", mt.MT_FILTER_QGRAM),
                           ("shd", mt.MT_FILTER_SHD)):
            ix.filter_pairs(dreads, *dev, kind=kind)  # warm
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(5):
                _, acc = ix.filter_pairs(dreads, *dev, kind=kind)
            torch.cuda.synchronize()
            f_ms = (time.perf_counter() - t) * 1000.0 / 5
            filters[name] = {"ms": round(f_ms, 3), "pairs_per_s": round(len(pr) / (f_ms / 1000.0), 1),
                             "accepted": round(float(acc.float().mean().item()), 4)}
        filters["pairs"] = int(len(pr))
        log(f"[bench] filters on the pair stream (mt_filter_pairs_kind, incl. read packing): {json.dumps(filters)}")

    # Stage 3b (relative abundance) on the batch's classification result.
    abundance = None
    if args.workload == "batched":
        r = ix.classify(dreads, **q)
        ix.abundance(r)  # warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(5):
            counts, ab, kept = ix.abundance(r)
        torch.cuda.synchronize()
        a_ms = (time.perf_counter() - t) * 1000.0 / 5
        abundance = {"ms": round(a_ms, 3), "reads_per_s": round(reads.n / (a_ms / 1000.0), 1), "kept_taxa": kept,
                     "max_abundance": round(float(ab.max().item()), 6)}
        r.free()
        log(f"[bench] abundance (mt_abundance on the classification result): {json.dumps(abundance)}")

    # Both strands: the batch with half its reads taken from the reverse strand.
    strands = None
    if args.workload == "batched" and args.strands_bench:
        flipped = synth.from_reverse_strand(np.random.default_rng(77), reads, 0.5)
        dflip = mt.to_device(flipped)
        one = ix.classify(dflip, **q).to_host()
        strands = {}
        for name, m in (("fused", q["mode"]), ("per_stage", mt.MT_MODE_PER_STAGE)):
            r = ix.classify(dflip, **dict(q, mode=m), strands=2)  # warm
            r.free()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(3):
                r = ix.classify(dflip, **dict(q, mode=m), strands=2)
                torch.cuda.synchronize()
                nc2 = r.n_cands
                r.free()
            s_ms = (time.perf_counter() - t) * 1000.0 / 3
            strands[name] = {"ms": round(s_ms, 3), "reads_per_s": round(flipped.n / (s_ms / 1000.0), 1),
                             "pairs_per_s": round(nc2 / (s_ms / 1000.0), 1)}
        r = ix.classify(dflip, **q, strands=2)
        two = r.to_host()
        r.free()
        strands.update({"pairs": int(len(two["genome"])),
                        "accepted_both": round(float(two["read_accepted"].mean()), 4),
                        "accepted_forward_only": round(float(one["read_accepted"].mean()), 4),
                        "reverse_cands": round(float(two["strand"].mean()), 4)})
        del dflip
        log(f"[bench] both strands (two-strand read set; fused kernel / per-stage chain): {json.dumps(strands)}")

    serving = None
    if pool is not None:
        serving = serving_bench(mt, ix, pool, seconds=args.serve_seconds, n_streams=args.serve_streams,
                                max_batch_reads=args.serve_max_batch, threads=args.serve_threads)

    cpu = None
    if args.cpu_reads > 0:
        import oracle
        t = time.time()
        oix = oracle.Index(ga, 21, 11)
        log(f"[bench] oracle index built in {time.time() - t:.1f}s (not timed)")
        sample = reads.subset(np.arange(min(args.cpu_reads, reads.n)))
        t = time.perf_counter()
        out = oix.classify(sample, 3, args.top_n, e_mode, e_value)
        dt = time.perf_counter() - t
        cpu = {"value": round(len(out["genome"]) / dt, 1), "unit": "pairs/s", "cores": 1, "kind": "oracle",
               "reads_per_s": round(sample.n / dt, 1),
               "sample": f"first {sample.n} reads of the batch, single-threaded C oracle, {dt:.1f}s"}
        log(f"[bench] oracle: {cpu['value']:.3e} pairs/s on {sample.n} reads in {dt:.1f}s")

    out = {
        "metric": METRIC, "value": round(pairs_s, 1), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": workload, "reads": reads.n, "bases": int(reads.offsets[-1]),
                   "pairs_per_step": int(n_cands), "mode": args.mode, "parallelism": "single GPU"},
        "reads_per_s": round(reads_s, 1),
        "index_build_s": round(index_s, 3),
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "roofline": roofline,
        "filter_tuning": tune,
        "cpu_baseline": cpu,
        "containment": containment,
        "filters": filters,
        "strands": strands,
        "abundance": abundance,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
