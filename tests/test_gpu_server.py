"""The serving loop (mt_server_*): every request's result, taken from a mix
of concurrent requests batched together on the GPU, is bit-identical to
classifying that request alone (mt_classify), per-request taxon counts
included; admission by memory, request splitting and error paths.
"""
import threading

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FIELDS = ("cand_offsets", "read_accepted", "read_E", "genome", "diag", "hits", "approx", "accept", "unique",
          "multi")


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_02029_amd as mt
    gen, _, p = synth.workload_small(0)
    ga = gen.ascii()
    taxon = np.arange(ga.n, dtype=np.uint32) // 2  # two genomes per taxon
    ix = mt.Index(ga, p["k"], p["w"], taxon=taxon, n_taxa=5)
    return dict(mt=mt, gen=gen, ga=ga, ix=ix, taxon=taxon, k=p["k"], w=p["w"])


def _requests(gen, seed, sizes):
    """Requests of uneven sizes and lengths, a few with N bases, some long reads."""
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        kind = rng.integers(0, 4)
        if kind == 0:
            lens = np.full(n, int(rng.integers(100, 251)))
        elif kind == 1:
            lens = rng.integers(75, 301, n)
        elif kind == 2:
            lens = np.where(rng.random(n) < 0.1, rng.integers(400, 2001, n), rng.integers(100, 251, n))
        else:
            lens = np.full(n, 150)
        reads, _ = synth.make_reads(rng, gen, lens, 0.005, 0.0005)
        if kind == 3:
            reads = synth.inject_n(rng, reads, 0.002)
        out.append(reads)
    return out


QUERIES = [dict(min_hits=3, top_n=3, e_mode=0, e_value=7),
           dict(min_hits=3, top_n=3, e_mode=1, e_value=50),
           dict(min_hits=2, top_n=0, e_mode=0, e_value=5),
           dict(min_hits=3, top_n=1, e_mode=2, e_value=60)]


def _alone(env, reads, q):
    mt = env["mt"]
    res = env["ix"].classify(mt.to_device(reads), mode=mt.MT_MODE_FUSED, **q)
    out = res.to_host()
    res.free()
    return out


def _same(got, ref, ctx):
    for f in FIELDS:
        a, b = np.asarray(got[f]), np.asarray(ref[f])
        assert a.shape == b.shape and np.array_equal(a, b), (ctx, f)
    assert got["unmapped"] == ref["unmapped"], ctx


def _serve(env, reqs, queries, threads=4, **server_args):
    mt = env["mt"]
    results = [None] * len(reqs)
    errors = []
    with mt.Server(env["ix"], **server_args) as sv:
        def client(tid):
            try:
                mine = list(range(tid, len(reqs), threads))
                ids = [sv.submit(reqs[i], **queries[i]) for i in mine]
                for i, rid in zip(mine, ids):
                    res = sv.wait(rid)
                    assert res.on_host
                    t0, t1 = res.times_ns()
                    assert 0 < t0 <= t1
                    results[i] = res.to_host()
                    res.free()
            except Exception as e:  # noqa: BLE001
                errors.append(e)
        ts = [threading.Thread(target=client, args=(t,)) for t in range(threads)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
    assert not errors, errors
    return results


def test_served_equals_alone_in_a_mix(env):
    sizes = [0, 1, 7, 100, 1000, 2600, 5000, 3, 40, 800, 1, 2000, 4000, 150, 9, 6000]
    reqs = _requests(env["gen"], 11, sizes)
    queries = [QUERIES[i % 2] for i in range(len(reqs))]
    # small batches: requests are split across batches and share them
    got = _serve(env, reqs, queries, threads=4, max_batch_reads=2500, n_streams=3)
    for i, (r, q) in enumerate(zip(reqs, queries)):
        _same(got[i], _alone(env, r, q), f"request {i} ({r.n} reads)")
    assert got[0]["cand_offsets"].tolist() == [0] and got[0]["unmapped"] == 0


def test_served_filter_kinds(env):
    """Requests with different filters of Table 1 are batched apart and each
    result equals the same request classified alone, and the oracle."""
    sizes = [200, 35, 900, 4, 300, 1500, 60, 700, 10, 250]
    reqs = _requests(env["gen"], 13, sizes)
    queries = [dict(QUERIES[0], filter_kind=i % 5) for i in range(len(reqs))]
    got = _serve(env, reqs, queries, threads=3, max_batch_reads=1200, n_streams=2)
    oix = oracle.Index(env["ga"], env["k"], env["w"], taxon=env["taxon"], n_taxa=5)
    for i, (r, q) in enumerate(zip(reqs, queries)):
        _same(got[i], _alone(env, r, q), f"request {i}")
        ref = oix.classify(r, q["min_hits"], q["top_n"], q["e_mode"], q["e_value"], filter_kind=q["filter_kind"])
        _same(got[i], ref, f"request {i} vs oracle")


def test_served_query_mix_and_oracle(env):
    sizes = [300, 50, 1200, 7, 600, 90, 2000, 15]
    reqs = _requests(env["gen"], 12, sizes)
    queries = [QUERIES[i % len(QUERIES)] for i in range(len(reqs))]
    got = _serve(env, reqs, queries, threads=3, max_batch_reads=1000, n_streams=2)
    oix = oracle.Index(env["ga"], env["k"], env["w"], taxon=env["taxon"], n_taxa=5)
    for i, (r, q) in enumerate(zip(reqs, queries)):
        _same(got[i], _alone(env, r, q), f"request {i}")
        ref = oix.classify(r, q["min_hits"], q["top_n"], q["e_mode"], q["e_value"])
        _same(got[i], ref, f"request {i} vs oracle")


def test_tight_memory_budget_still_exact(env):
    reqs = _requests(env["gen"], 13, [3000, 20, 1500, 1])
    queries = [QUERIES[0]] * len(reqs)
    # a budget of a few MB admits a few thousand reads per batch at most
    got = _serve(env, reqs, queries, threads=2, mem_budget_bytes=3 << 20, n_streams=2)
    for i, (r, q) in enumerate(zip(reqs, queries)):
        _same(got[i], _alone(env, r, q), f"request {i}")


def test_submit_errors_and_wait_semantics(env):
    mt = env["mt"]
    good = _requests(env["gen"], 14, [200])[0]
    with mt.Server(env["ix"], max_queued_requests=2, pinned_arena_bytes=1 << 20) as sv:
        bad = synth.SeqSet(seq=good.seq.copy(), offsets=good.offsets.copy())
        bad.seq[17] = ord("X")
        with pytest.raises(mt.MTError) as e:
            sv.submit(bad)
        assert e.value.status == mt._abi.MT_EINVAL
        too_long = synth.SeqSet.from_list(["A" * 65536])
        with pytest.raises(mt.MTError) as e:
            sv.submit(too_long)
        assert e.value.status == mt._abi.MT_EINVAL
        big = synth.SeqSet.from_list(["ACGT" * 1000] * 300)  # 1.2 MB > the 1 MiB arena
        with pytest.raises(mt.MTError) as e:
            sv.submit(big)
        assert e.value.status == mt._abi.MT_EINVAL
        with pytest.raises(mt.MTError) as e:
            sv.submit(good, e_mode=1, e_value=500_000)  # E above 65534
        assert e.value.status == mt._abi.MT_EINVAL
        a = sv.submit(good)
        b = sv.submit(good)
        with pytest.raises(mt.MTError) as e:  # two requests not yet waited for
            sv.submit(good)
        assert e.value.status == mt._abi.MT_EAGAIN
        with pytest.raises(mt.MTError) as e:
            sv.wait(a + b + 100)
        assert e.value.status == mt._abi.MT_EINVAL
        ra = sv.wait(a)
        rb = sv.wait(b, timeout_s=60)
        assert rb is not None
        _same(ra.to_host(), rb.to_host(), "same request twice")
        with pytest.raises(mt.MTError):  # handed over already
            sv.wait(a, timeout_s=0)
        c = sv.submit(good)  # room again
        r = sv.wait(c, timeout_s=0)
        if r is None:  # not finished yet: a timed-out wait can be repeated
            r = sv.wait(c)
        _same(r.to_host(), ra.to_host(), "after a timed-out wait")


def test_destroy_with_pending_requests(env):
    mt = env["mt"]
    reqs = _requests(env["gen"], 15, [3000, 3000, 3000, 10])
    sv = mt.Server(env["ix"], max_batch_reads=1000, n_streams=2)
    ids = [sv.submit(r) for r in reqs]
    first = sv.wait(ids[0])
    assert first.to_host()["read_E"].shape == (3000,)
    sv.close()  # finishes and releases the others
    with mt.Server(env["ix"]) as sv2:  # the index still serves afterwards
        r = sv2.wait(sv2.submit(reqs[3]))
        _same(r.to_host(), _alone(env, reqs[3], {}), "after destroy")


def test_served_trace_on_500mbp_index_matches_oracle(env, batched_db, batched_oracle):
    """The served workload on its own database: 160 requests of a Poisson trace
    (U{1..50,000} reads of one length in 100-250 bp at 0.5% error, E = ceil(5%
    of m)) submitted at their arrival times by 8 client threads to a server
    holding the 500 Mbp index, several requests in flight at once; every
    request's result, taken from the mix, equals the oracle's classification of
    that request's reads alone, per-request taxon counts included."""
    import time
    mt = env["mt"]
    ix = mt.Index(mt.to_device(batched_db["ga"]), 21, 11)
    pool = synth.served_read_pool(batched_db["db"])
    trace = synth.request_trace(3, 160, 3000.0, lengths=synth.SERVED_LENGTHS)
    reqs = [synth.request_reads(pool, n, m) for _, n, m in trace]
    q = dict(min_hits=3, top_n=3, e_mode=1, e_value=50)
    results = [None] * len(reqs)
    spans = [None] * len(reqs)
    errors = []
    threads = 8
    with mt.Server(ix, n_streams=4, max_batch_reads=1 << 18) as sv:
        t0 = time.monotonic()

        def client(tid):
            try:
                mine = list(range(tid, len(reqs), threads))
                ids = []
                for i in mine:
                    delay = t0 + trace[i][0] - time.monotonic()
                    if delay > 0:
                        time.sleep(delay)
                    ids.append(sv.submit(reqs[i], **q))
                for i, rid in zip(mine, ids):
                    res = sv.wait(rid)
                    spans[i] = res.times_ns()
                    results[i] = res.to_host()
                    res.free()
            except Exception as e:  # noqa: BLE001
                errors.append(e)
        ts = [threading.Thread(target=client, args=(t,)) for t in range(threads)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        st = sv.stats()
    assert not errors, errors
    # device spans of the batches' kernels: every batch timed; the time covered
    # plus the time with two or more batches running cannot exceed their sum
    assert st["timed_batches"] == st["batches"] > 0 and st["reads"] == sum(r.n for r in reqs)
    assert 0 < st["kernel_ms_union"] <= st["kernel_ms_sum"] + 1e-3
    assert st["kernel_ms_union"] + st["kernel_ms_overlap"] <= st["kernel_ms_sum"] + 1e-3
    for i, r in enumerate(reqs):
        ref = batched_oracle.classify(r, q["min_hits"], q["top_n"], q["e_mode"], q["e_value"])
        _same(results[i], ref, f"served request {i} ({r.n} reads of {trace[i][2]} bp) vs oracle")
    # requests overlapped: some request was submitted before an earlier one completed
    order = np.argsort([s for s, _ in spans])
    sub = np.array([spans[i][0] for i in order])
    done = np.array([spans[i][1] for i in order])
    assert (sub[1:] < np.maximum.accumulate(done)[:-1]).any()
    assert sum(r.n for r in reqs) > 1_000_000
