"""Parity at full size, read by read against the CPU oracle, in the launch
configuration the benchmark times:

  * batched: 200 genomes / 500 Mbp, all 1M reads of 150 bp, k=21, w=11, >= 3
    hits, top 3, at every E of the sweep {0, 3, 7, 15}, fused and per-stage
    (and the graph form at E = 7), every output field of every read against
    the oracle's classification of the same 1M reads;
  * uneven: 2M reads (95% of 75-300 bp, 5% of 1-10 kbp, E = ceil(5% of m)),
    every read across the three forms and against the oracle;
  * strains: 2,000 near-duplicate strain genomes (4 Gbp), 10M reads of
    150 bp, E=7: every read across the forms and against the oracle on the
    same 4 Gbp database (the oracle's index of it takes about 30 GB of host
    memory);
  * both strands (every read) and stage 1 (containment) on the batched
    workload;
  * properties that hold at any size: canonical candidate order, >= min_hits,
    accept == (approx <= E), approx <= E + 1, per-taxon conservation.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FIELDS = ("cand_offsets", "read_accepted", "read_E", "genome", "diag", "hits", "approx", "accept", "unique",
          "multi")
READ_FIELDS = ("cand_offsets", "read_accepted", "read_E", "genome", "diag", "hits", "approx", "accept")
E_SWEEP = (0, 3, 7, 15)


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _same(got, ref, ctx, fields=FIELDS, unmapped=True):
    for f in fields:
        a, b = np.asarray(got[f]), np.asarray(ref[f])
        assert a.shape == b.shape, (ctx, f, a.shape, b.shape)
        bad = np.flatnonzero(a.astype(b.dtype) != b)
        assert bad.size == 0, (ctx, f, bad[:8])
    if unmapped:
        assert got["unmapped"] == ref["unmapped"], ctx


def _run(ix, dr, **q):
    res = ix.classify(dr, **q)
    out = res.to_host()
    res.free()
    return out


@pytest.fixture(scope="module")
def full(gpu, batched_db, batched_oracle):
    import paper_2311_02029_amd as mt
    ga = batched_db["ga"]
    reads = synth.workload_batched_reads(batched_db["db"], 1_000_000)
    ix = mt.Index(mt.to_device(ga), 21, 11)
    dr = mt.to_device(reads)
    fused = _run(ix, dr, min_hits=3, top_n=3, e_value=7, mode=mt.MT_MODE_FUSED)
    return dict(ga=ga, reads=reads, fused=fused, oracle=batched_oracle, ix=ix, dr=dr)


@pytest.mark.parametrize("E", E_SWEEP)
def test_batched_every_read_matches_oracle(full, E):
    """Every output of every one of the 1M reads at this E equals the oracle's,
    fused and per-stage (and the graph form at E = 7): candidate lists, seed
    counts, approximate edit counts, accept bits, read flags and taxon counts."""
    import paper_2311_02029_amd as mt
    ref = full["oracle"].classify(full["reads"], 3, 3, 0, E)
    modes = [("fused", mt.MT_MODE_FUSED), ("per-stage", mt.MT_MODE_PER_STAGE)]
    if E == 7:
        modes.append(("graph", mt.MT_MODE_FUSED_GRAPH))
    for name, mode in modes:
        got = full["fused"] if (E == 7 and mode == mt.MT_MODE_FUSED) else \
            _run(full["ix"], full["dr"], min_hits=3, top_n=3, e_value=E, mode=mode)
        _same(got, ref, f"E={E} {name}")
    assert len(ref["genome"]) > full["reads"].n and ref["read_accepted"].mean() > (0.4 if E == 0 else 0.97)


def test_containment_full_size_against_oracle(full):
    """Stage 1 over the whole batch on the resident index: every genome's seed-hit
    count equals the oracle's, and so does the subset at the paper's cutoff."""
    import paper_2311_02029_amd as mt
    hits = full["ix"].containment(full["dr"])
    got = hits.cpu().numpy().view(np.uint64)
    want = full["oracle"].containment(full["reads"])
    assert np.array_equal(got, want), np.flatnonzero(got != want)[:10]
    sel, mx = mt.select_genomes(hits, 1, 10_000)
    osel, omx = oracle.select_genomes(want, 1, 10_000)
    assert mx == omx and np.array_equal(sel.cpu().numpy().astype(np.uint32), osel)
    assert want.min() > 0 and len(osel) == len(want)


def test_both_strands_full_size(full):
    """Both strands at full size (half the reads taken from the reverse strand):
    every read against the oracle, and the canonical order with the strand as
    the last key and accept == (approx <= E)."""
    import paper_2311_02029_amd as mt
    reads = synth.from_reverse_strand(np.random.default_rng(77), full["reads"], 0.5)
    got = _run(full["ix"], mt.to_device(reads), min_hits=3, top_n=3, e_value=7, mode=mt.MT_MODE_FUSED, strands=2)
    ref = full["oracle"].classify(reads, 3, 3, 0, 7, strands=2)
    _same(got, ref, "both strands", fields=FIELDS + ("strand",))
    co = got["cand_offsets"].astype(np.int64)
    nc = np.diff(co)
    same = np.repeat(np.arange(len(nc)), nc)
    nxt = np.flatnonzero(same[1:] == same[:-1])
    key = np.stack([-got["hits"].astype(np.int64), got["genome"].astype(np.int64), got["diag"],
                    got["strand"].astype(np.int64)], 1)
    a, b = key[nxt], key[nxt + 1]
    diff = a != b
    first = np.argmax(diff, 1)
    assert diff.any(1).all() and (a[np.arange(len(a)), first] < b[np.arange(len(b)), first]).all()
    E = np.repeat(got["read_E"], nc)
    assert np.array_equal(got["accept"], (got["approx"] <= E).astype(np.uint8))
    assert got["read_accepted"].mean() > 0.97 and 0.4 < got["strand"].mean() < 0.6


def test_properties_at_full_size(full):
    res = full["fused"]
    co = res["cand_offsets"].astype(np.int64)
    n = len(co) - 1
    nc = np.diff(co)
    assert nc.max() <= 3
    assert (res["hits"] >= 3).all()
    E = np.repeat(res["read_E"], nc)
    assert np.array_equal(res["accept"], (res["approx"] <= E).astype(np.uint8))
    assert (res["approx"] <= E + 1).all()
    # canonical order inside every read: hits desc, genome asc, diag asc
    same = np.repeat(np.arange(n), nc)
    nxt = np.flatnonzero(same[1:] == same[:-1])
    h, g, d = res["hits"].astype(np.int64), res["genome"].astype(np.int64), res["diag"]
    ok = (h[nxt] > h[nxt + 1]) | ((h[nxt] == h[nxt + 1]) & ((g[nxt] < g[nxt + 1]) |
                                                            ((g[nxt] == g[nxt + 1]) & (d[nxt] < d[nxt + 1]))))
    assert ok.all()
    # read flags and per-taxon conservation
    acc = np.zeros(n, np.uint8)
    np.maximum.at(acc, same, res["accept"])
    assert np.array_equal(res["read_accepted"], acc)
    n_acc = int(acc.sum())
    assert n_acc + res["unmapped"] == n
    n_unique = int(res["unique"].sum())
    assert n_unique <= n_acc and int(res["multi"].sum()) >= 2 * (n_acc - n_unique)
    assert n_acc > 0.99 * n


# ---------------------------------------------------------------- uneven --

@pytest.fixture(scope="module")
def uneven(full, batched_db):
    """The uneven workload at full size: 2M reads, 95% of 75-300 bp and 5% of
    1-10 kbp, E = ceil(5% of length), on the same 500 Mbp database."""
    import paper_2311_02029_amd as mt
    reads = synth.workload_uneven_reads(batched_db["db"], 2_000_000)
    dr = mt.to_device(reads)
    out = {}
    for name, mode in (("fused", mt.MT_MODE_FUSED), ("stage", mt.MT_MODE_PER_STAGE),
                       ("graph", mt.MT_MODE_FUSED_GRAPH)):
        out[name] = _run(full["ix"], dr, min_hits=3, top_n=3, e_mode=mt.MT_E_CEIL_PERMILLE, e_value=50, mode=mode)
    out["reads"] = reads
    out["dr"] = dr
    return out


def test_uneven_all_forms_agree_on_every_read(uneven):
    for other in ("stage", "graph"):
        _same(uneven[other], uneven["fused"], other)


def test_uneven_every_read_matches_oracle(full, uneven):
    """All 2M reads (1.9M of 75-300 bp, about 100,000 of 1-10 kbp with E up to
    500) against the oracle: every output field, taxon counts included."""
    reads = uneven["reads"]
    ref = full["oracle"].classify(reads, 3, 3, 1, 50)
    _same(uneven["fused"], ref, "uneven, every read")
    assert (ref["read_E"] >= 50).sum() >= 90_000


# --------------------------------------------------------------- strains --

def test_strains_full_size_against_oracle(gpu):
    """The dense-candidate workload at full size (2,000 strain genomes = 4 Gbp,
    10M reads, E=7): fused and per-stage agree on every read, the candidate
    lists are dense, every read equals the oracle's classification on the
    same 4 Gbp database, taxon counts included, and the relative abundances of
    the 2,000 strains equal the oracle's bit for bit (their total, in units of
    2^-32 read, needs more than 53 bits)."""
    import paper_2311_02029_amd as mt
    db = synth.workload_strains_db()
    reads = synth.workload_strain_reads(db, 10_000_000)
    ga = db.ascii()
    del db
    ix = mt.Index(mt.to_device(ga), 21, 11)
    dr = mt.to_device(reads)
    res = ix.classify(dr, mode=mt.MT_MODE_FUSED)
    fused = res.to_host()
    counts, ab, kept = ix.abundance(res)  # stage 3b over 10M reads: the kept total is far above 2^53 units
    counts, ab = counts.cpu().numpy().view(np.uint64), ab.cpu().numpy()
    res.free()
    stage = _run(ix, dr, mode=mt.MT_MODE_PER_STAGE)
    _same(stage, fused, "strains per-stage")
    del stage
    assert len(fused["genome"]) > 2.5 * reads.n
    oracle.set_threads(0)
    oix = oracle.Index(ga, 21, 11)
    del ga
    ref = oix.classify(reads, 3, 3, 0, 7)
    del oix
    _same(fused, ref, "strains, every read")
    assert int(ref["multi"].sum()) > 0
    oc, oa, okept = oracle.abundance(ref, np.arange(2000, dtype=np.uint32), 2000)
    assert np.array_equal(counts, oc) and kept == okept
    assert np.array_equal(ab, oa), np.flatnonzero(ab != oa)[:8]
    assert int(oc.sum()) > 2 ** 53
