"""Parity at the benchmark's full size: 200 genomes / 500 Mbp, 1M reads of
150 bp, k=21, w=11, >= 3 hits, top 3, E=7, in the launch configuration the
benchmark times (fused), against

  * the CPU oracle, read by read, on a seeded sample of the batch (the oracle
    finishes a sample in seconds; its index over 500 Mbp takes ~40 s);
  * the per-stage GPU form on every read (both GPU forms must agree bit for
    bit everywhere);
  * properties that hold at any size: canonical candidate order, >= min_hits,
    accept == (approx <= E), approx <= E + 1, per-taxon conservation.

The uneven workload (2M reads up to 10 kbp) and the strain workload (4 Gbp,
10M reads) are checked the same way: every read across the execution forms,
and seeded samples (or a reduced strain database) against the oracle.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FIELDS = ("cand_offsets", "read_accepted", "read_E", "genome", "diag", "hits", "approx", "accept", "unique",
          "multi")


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def full(gpu):
    import paper_2311_02029_amd as mt
    db = synth.workload_batched_db()
    reads = synth.workload_batched_reads(db, 1_000_000)
    ga = db.ascii()
    ix = mt.Index(mt.to_device(ga), 21, 11)
    dr = mt.to_device(reads)
    res = ix.classify(dr, min_hits=3, top_n=3, e_value=7, mode=mt.MT_MODE_FUSED)
    fused = res.to_host()
    res.free()
    res = ix.classify(dr, min_hits=3, top_n=3, e_value=7, mode=mt.MT_MODE_PER_STAGE)
    stage = res.to_host()
    res.free()
    res = ix.classify(dr, min_hits=3, top_n=3, e_value=7, mode=mt.MT_MODE_FUSED_GRAPH)
    graph = res.to_host()
    res.free()
    cache = {}

    def oracle_index():
        if "ix" not in cache:
            cache["ix"] = oracle.Index(ga, 21, 11)
        return cache["ix"]

    return dict(ga=ga, reads=reads, fused=fused, stage=stage, graph=graph, oracle=oracle_index, ix=ix, dr=dr)


def _slice(res, idx):
    co = res["cand_offsets"].astype(np.int64)
    out = {f: [] for f in ("genome", "diag", "hits", "approx", "accept")}
    offs = [0]
    for r in idx:
        for f in out:
            out[f].append(res[f][co[r]:co[r + 1]])
        offs.append(offs[-1] + co[r + 1] - co[r])
    out = {f: np.concatenate(v) if v else np.zeros(0) for f, v in out.items()}
    out["cand_offsets"] = np.array(offs, np.uint64)
    out["read_accepted"] = res["read_accepted"][idx]
    out["read_E"] = res["read_E"][idx]
    return out


def test_containment_full_size_against_oracle(full):
    """Stage 1 over the whole batch on the resident index: every genome's seed-hit
    count equals the oracle's, and so does the subset at the paper's cutoff."""
    import paper_2311_02029_amd as mt
    hits = full["ix"].containment(full["dr"])
    got = hits.cpu().numpy().view(np.uint64)
    want = full["oracle"]().containment(full["reads"])
    assert np.array_equal(got, want), np.flatnonzero(got != want)[:10]
    sel, mx = mt.select_genomes(hits, 1, 10_000)
    osel, omx = oracle.select_genomes(want, 1, 10_000)
    assert mx == omx and np.array_equal(sel.cpu().numpy().astype(np.uint32), osel)
    assert want.min() > 0 and len(osel) == len(want)


def test_fused_equals_per_stage_on_every_read(full):
    for other in ("stage", "graph"):
        for f in FIELDS:
            assert np.array_equal(full["fused"][f], full[other][f]), (other, f)
        assert full["fused"]["unmapped"] == full[other]["unmapped"], other


def test_sampled_reads_match_oracle(full):
    reads = full["reads"]
    idx = np.sort(np.random.default_rng(2024).choice(reads.n, 3000, replace=False))
    ref = full["oracle"]().classify(reads.subset(idx), 3, 3, 0, 7)
    got = _slice(full["fused"], idx)
    for f in ("cand_offsets", "read_accepted", "read_E", "genome", "diag", "hits", "approx", "accept"):
        a, b = np.asarray(got[f]), np.asarray(ref[f])
        assert a.shape == b.shape and np.array_equal(a.astype(b.dtype), b), f


def test_both_strands_full_size(full):
    """Both strands at full size (half the reads taken from the reverse strand),
    per-stage over the two-strand read set: a seeded sample against the oracle,
    and on every read the canonical order with the strand as the last key and
    accept == (approx <= E)."""
    import paper_2311_02029_amd as mt
    reads = synth.from_reverse_strand(np.random.default_rng(77), full["reads"], 0.5)
    res = full["ix"].classify(mt.to_device(reads), min_hits=3, top_n=3, e_value=7, strands=2)
    got = res.to_host()
    res.free()
    idx = np.sort(np.random.default_rng(2025).choice(reads.n, 2000, replace=False))
    ref = full["oracle"]().classify(reads.subset(idx), 3, 3, 0, 7, strands=2)
    co = got["cand_offsets"].astype(np.int64)
    sl = np.concatenate([np.arange(co[r], co[r + 1]) for r in idx])
    for f in ("genome", "diag", "hits", "approx", "accept", "strand"):
        assert np.array_equal(got[f][sl], ref[f]), f
    assert np.array_equal(np.diff(co)[idx], np.diff(ref["cand_offsets"].astype(np.int64)))
    assert np.array_equal(got["read_accepted"][idx], ref["read_accepted"])
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
def uneven(full):
    """The uneven workload at full size: 2M reads, 95% of 75-300 bp and 5% of
    1-10 kbp, E = ceil(5% of length), on the same 500 Mbp database."""
    import paper_2311_02029_amd as mt
    db = synth.workload_batched_db()
    reads = synth.workload_uneven_reads(db, 2_000_000)
    ix = mt.Index(mt.to_device(full["ga"]), 21, 11)
    dr = mt.to_device(reads)
    out = {}
    for name, mode in (("fused", mt.MT_MODE_FUSED), ("stage", mt.MT_MODE_PER_STAGE),
                       ("graph", mt.MT_MODE_FUSED_GRAPH)):
        res = ix.classify(dr, min_hits=3, top_n=3, e_mode=mt.MT_E_CEIL_PERMILLE, e_value=50, mode=mode)
        out[name] = res.to_host()
        res.free()
    out["reads"] = reads
    return out


def test_uneven_all_forms_agree_on_every_read(uneven):
    for other in ("stage", "graph"):
        for f in FIELDS:
            assert np.array_equal(uneven["fused"][f], uneven[other][f]), (other, f)
        assert uneven["fused"]["unmapped"] == uneven[other]["unmapped"], other


def test_uneven_sampled_reads_match_oracle(full, uneven):
    """A seeded sample of 2000 short and 60 long reads against the oracle."""
    reads = uneven["reads"]
    lens = reads.lengths()
    rng = np.random.default_rng(2025)
    idx = np.sort(np.concatenate([rng.choice(np.flatnonzero(lens <= 300), 2000, replace=False),
                                  rng.choice(np.flatnonzero(lens > 300), 60, replace=False)]))
    ref = full["oracle"]().classify(reads.subset(idx), 3, 3, 1, 50)
    got = _slice(uneven["fused"], idx)
    for f in ("cand_offsets", "read_accepted", "read_E", "genome", "diag", "hits", "approx", "accept"):
        a, b = np.asarray(got[f]), np.asarray(ref[f])
        assert a.shape == b.shape and np.array_equal(a.astype(b.dtype), b), f


# --------------------------------------------------------------- strains --

def test_strains_full_size_forms_agree(gpu):
    """The dense-candidate workload at full size (2,000 strain genomes = 4 Gbp,
    10M reads): fused and per-stage agree on every read, and the candidate
    lists are dense (several near-duplicate strains per read)."""
    import paper_2311_02029_amd as mt
    db = synth.workload_strains_db()
    reads = synth.workload_strain_reads(db, 10_000_000)
    ix = mt.Index(mt.to_device(db.ascii()), 21, 11)
    del db
    dr = mt.to_device(reads)
    res = ix.classify(dr, mode=mt.MT_MODE_FUSED)
    fused = res.to_host()
    res.free()
    res = ix.classify(dr, mode=mt.MT_MODE_PER_STAGE)
    stage = res.to_host()
    res.free()
    for f in FIELDS:
        assert np.array_equal(fused[f], stage[f]), f
    assert len(fused["genome"]) > 2.5 * reads.n


def test_strains_reduced_database_matches_oracle(gpu):
    """The strain structure on a database the oracle indexes in seconds (40
    roots x 5 strains x 2 Mbp = 400 Mbp): 2000 reads against the oracle."""
    import paper_2311_02029_amd as mt
    db = synth.workload_strains_db(n_roots=40)
    reads = synth.workload_strain_reads(db, 2000)
    ga = db.ascii()
    ix = mt.Index(mt.to_device(ga), 21, 11)
    res = ix.classify(mt.to_device(reads), mode=mt.MT_MODE_FUSED)
    got = res.to_host()
    res.free()
    ref = oracle.Index(ga, 21, 11).classify(reads, 3, 3, 0, 7)
    for f in ("cand_offsets", "read_accepted", "read_E", "genome", "diag", "hits", "approx", "accept", "unique",
              "multi"):
        assert np.array_equal(np.asarray(got[f]), np.asarray(ref[f]).astype(got[f].dtype)), f
    assert got["unmapped"] == ref["unmapped"]
    assert int(got["multi"].sum()) > 0
