"""Both strands (query strands = 2) on the GPU against the oracle, bit-exact:
candidate lists with their strands, filter values of every Table 1 filter on
the oriented read, read outcomes and per-taxon counts; in every execution form
(all of them run the per-stage chain over the two-strand read set), served,
and at the benchmark's full size on a seeded sample.
"""
import random

import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import _random_case

pytestmark = pytest.mark.gpu

FIELDS = ("cand_offsets", "read_accepted", "read_E", "genome", "diag", "hits", "approx", "accept", "strand",
          "unique", "multi")
MODES = [0, 1, 2]


@pytest.fixture(scope="module")
def mt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_02029_amd as mt_
    return mt_


def assert_same(gpu, ref, ctx=""):
    for f in FIELDS:
        a, b = np.asarray(gpu[f]), np.asarray(ref[f])
        assert a.shape == b.shape, (ctx, f, a.shape, b.shape)
        if not np.array_equal(a, b):
            bad = np.flatnonzero(a != b)[:10]
            raise AssertionError(f"{ctx} {f} differs at {bad.tolist()}: gpu {a[bad].tolist()} oracle {b[bad].tolist()}")
    assert gpu["unmapped"] == ref["unmapped"], ctx


def run_both(mt, genomes, reads, k, w, max_occ=0, taxon=None, n_taxa=None, mode=0, filter_kind=0, **q):
    ix = mt.Index(genomes, k, w, max_occ=max_occ, taxon=taxon, n_taxa=n_taxa)
    res = ix.classify(mt.to_device(reads), mode=mode, filter_kind=filter_kind, strands=2, **q)
    got = res.to_host()
    res.free()
    ref = oracle.Index(genomes, k, w, max_occ=max_occ, taxon=taxon, n_taxa=n_taxa).classify(
        reads, q.get("min_hits", 3), q.get("top_n", 3), q.get("e_mode", 0), q.get("e_value", 7),
        filter_kind=filter_kind, strands=2)
    return got, ref


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("top_n", [3, 0, 1])
def test_small_workload_both_strands(mt, top_n, mode):
    gen, reads, p = synth.workload_small(3000)
    reads = synth.from_reverse_strand(np.random.default_rng(1), reads, 0.5)
    got, ref = run_both(mt, gen.ascii(), reads, p["k"], p["w"], min_hits=3, top_n=top_n, e_value=7, mode=mode)
    assert_same(got, ref, f"small top_n={top_n} mode={mode}")
    st = ref["strand"].astype(bool)
    assert st.sum() > 1000 and (~st).sum() > 1000 and ref["read_accepted"].mean() > 0.95


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("seed", range(8))
def test_random_small_cases_both_strands(mt, seed, mode):
    """Repeats, N, lower case, empty and short reads, max_occ, every E mode."""
    rnd = random.Random(500 + seed)
    genomes, reads = _random_case(rnd)
    rs = synth.from_reverse_strand(np.random.default_rng(seed), synth.SeqSet.from_list(reads), 0.5)
    k, w = rnd.randint(3, 16), rnd.randint(1, 12)
    n_tax = max(1, len(genomes) // 2)
    taxon = np.array([rnd.randrange(n_tax) for _ in genomes], np.uint32)
    q = dict(min_hits=rnd.choice([1, 2, 3]), top_n=rnd.choice([0, 1, 3]), e_mode=rnd.choice([0, 1, 2]),
             e_value=rnd.choice([0, 2, 50, 120]))
    if q["e_mode"] == 0:
        q["e_value"] = rnd.randint(0, 9)
    got, ref = run_both(mt, synth.SeqSet.from_list(genomes), rs, k, w, max_occ=rnd.choice([0, 0, 4]), taxon=taxon,
                        n_taxa=n_tax, mode=mode, **q)
    assert_same(got, ref, f"seed {seed} mode {mode}")


@pytest.mark.parametrize("kind", [0, 1, 2, 3, 4])
def test_each_filter_both_strands(mt, kind):
    rnd = np.random.default_rng(60 + kind)
    gen = synth.make_genomes(rnd, 6, 40_000, (0.3, 0.7))
    reads, _ = synth.make_reads(rnd, gen, rnd.integers(60, 400, 1500), 0.02, 0.005)
    reads = synth.from_reverse_strand(rnd, synth.inject_n(rnd, reads, 0.001), 0.5)
    got, ref = run_both(mt, gen.ascii(), reads, 13, 7, min_hits=2, top_n=3, e_mode=1, e_value=60,
                        filter_kind=kind)
    assert_same(got, ref, f"kind {kind}")
    assert ref["strand"].sum() > 500


@pytest.mark.parametrize("mode", [0, 1])
def test_long_reads_both_strands(mt, mode):
    """Reads up to 6 kbp with large E: the long filter path on reverse complements."""
    rnd = np.random.default_rng(15)
    gen = synth.make_genomes(rnd, 3, 60_000, 0.5)
    lens = np.concatenate([rnd.integers(1000, 6000, 30), rnd.integers(75, 300, 150)])
    reads, _ = synth.make_reads(rnd, gen, lens, 0.02, 0.03)
    reads = synth.from_reverse_strand(rnd, reads, 0.5)
    got, ref = run_both(mt, gen.ascii(), reads, 15, 10, min_hits=3, top_n=3, e_mode=1, e_value=50, mode=mode)
    assert_same(got, ref, "long")
    assert ref["read_E"].max() >= 100


def test_many_hits_both_strands(mt):
    """A repetitive genome and its reverse: hundreds of locations per read on both strands."""
    rnd = random.Random(78)
    unit = "".join(rnd.choice("ACGT") for _ in range(40))
    genome = "".join(unit if rnd.random() < 0.9 else rnd.choice("ACGT") * 40 for _ in range(300))
    reads = [genome[i:i + 400] for i in range(0, 4000, 397)]
    rs = synth.from_reverse_strand(np.random.default_rng(2), synth.SeqSet.from_list(reads), 0.5)
    got, ref = run_both(mt, synth.SeqSet.from_list([genome, genome[::-1]]), rs, 8, 3, min_hits=2, top_n=0,
                        e_value=10)
    assert_same(got, ref, "large")
    assert np.diff(ref["cand_offsets"].astype(np.int64)).max() > 100 and ref["strand"].any()


def test_one_strand_result_has_no_strand_array(mt):
    gen, reads, p = synth.workload_small(200)
    ix = mt.Index(gen.ascii(), p["k"], p["w"])
    dr = mt.to_device(reads)
    one = ix.classify(dr, strands=1)
    assert one._strands() is None
    zero = ix.classify(dr, strands=0)          # 0 also means the forward strand alone
    a, b = one.to_host(), zero.to_host()
    for f in FIELDS:
        assert np.array_equal(a[f], b[f]), f
    assert not a["strand"].any()
    two = ix.classify(dr, strands=2).to_host()
    # forward reads: every forward candidate of the one-strand run survives when
    # nothing is cut (top_n 0)
    o = ix.classify(dr, top_n=0).to_host()
    t = ix.classify(dr, top_n=0, strands=2).to_host()
    fwd = t["strand"] == 0
    assert np.array_equal(t["genome"][fwd], o["genome"]) and np.array_equal(t["approx"][fwd], o["approx"])
    assert two["read_accepted"].sum() >= a["read_accepted"].sum()


@pytest.mark.parametrize("mode", MODES)
def test_empty_and_errors_both_strands(mt, mode):
    gen, _, p = synth.workload_small(10)
    got, ref = run_both(mt, gen.ascii(), synth.SeqSet.from_list([]), p["k"], p["w"], mode=mode)
    assert_same(got, ref, "empty set")
    got, ref = run_both(mt, gen.ascii(), synth.SeqSet.from_list(["", "A", ""]), p["k"], p["w"], mode=mode)
    assert_same(got, ref, "empty reads")
    ix = mt.Index(gen.ascii(), p["k"], p["w"])
    with pytest.raises(mt.MTError) as e:
        ix.classify(mt.to_device(synth.SeqSet.from_list(["ACGTACGTAC", "ACGT*ACG"])), mode=mode, strands=2)
    assert e.value.status == -1
    with pytest.raises(mt.MTError) as e:
        ix.classify(mt.to_device(synth.SeqSet.from_list(["ACGT" * 20000])), mode=mode, strands=2)
    assert e.value.status == -1
    with pytest.raises(mt.MTError) as e:
        ix.classify(mt.to_device(synth.SeqSet.from_list(["ACGTACGT"])), mode=mode, strands=3)
    assert e.value.status == -1


def test_bad_offsets_refused_before_any_byte_is_read(mt):
    import torch
    gen, _, p = synth.workload_small(10)
    ix = mt.Index(gen.ascii(), p["k"], p["w"])
    good = mt.to_device(synth.SeqSet.from_list(["ACGTACGTACGTACGTAC", "ACGTACGTACGT"]))
    # past the end, decreasing, not from 0, short of the end
    for offs in ([0, 31, 30], [0, 20, 10], [1, 18, 30], [0, 12, 29]):
        bad = mt.DeviceSeqs(good.seq, torch.tensor(offs, dtype=torch.int64, device="cuda"), 2, 30)
        with pytest.raises(mt.MTError) as e:
            ix.classify(bad, strands=2)
        assert e.value.status == -1 and "offsets" in str(e.value)


def test_served_both_strands(mt):
    gen, _, p = synth.workload_small(0)
    ga = gen.ascii()
    taxon = np.arange(ga.n, dtype=np.uint32) // 2
    ix = mt.Index(ga, p["k"], p["w"], taxon=taxon, n_taxa=5)
    oix = oracle.Index(ga, p["k"], p["w"], taxon=taxon, n_taxa=5)
    rng = np.random.default_rng(21)
    reqs = []
    for n in (300, 7, 1500, 0, 900, 40):
        r, _ = synth.make_reads(rng, gen, rng.integers(75, 301, n), 0.005, 0.0005)
        reqs.append(synth.from_reverse_strand(rng, r, 0.5))
    strands = [2, 1, 2, 2, 1, 2]
    with mt.Server(ix, max_batch_reads=1000, n_streams=2) as sv:
        ids = [sv.submit(r, min_hits=3, top_n=3, e_value=7, strands=s) for r, s in zip(reqs, strands)]
        got = []
        for rid in ids:
            res = sv.wait(rid)
            got.append(res.to_host())
            res.free()
    for i, (r, s) in enumerate(zip(reqs, strands)):
        ref = oix.classify(r, 3, 3, 0, 7, strands=s)
        assert_same(got[i], ref, f"request {i} strands {s}")
