"""GPU (HIP, gfx950) vs CPU oracle, element by element, bit-exact.

Candidate lists (genome, diagonal, seed hits, canonical order), approximate
edit counts, accept bits, read flags and per-taxon counts must be identical:
the whole path is integer work.
"""
import random

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FIELDS = ("cand_offsets", "read_accepted", "read_E", "genome", "diag", "hits", "approx", "accept", "unique",
          "multi")


@pytest.fixture(scope="module")
def mt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_02029_amd as mt_
    return mt_


def assert_same(gpu: dict, ref: dict, ctx=""):
    for f in FIELDS:
        a, b = np.asarray(gpu[f]), np.asarray(ref[f])
        assert a.shape == b.shape, (ctx, f, a.shape, b.shape)
        if not np.array_equal(a, b):
            bad = np.flatnonzero(a != b)[:10]
            raise AssertionError(f"{ctx} {f} differs at {bad.tolist()}: gpu {a[bad].tolist()} oracle {b[bad].tolist()}")
    assert gpu["unmapped"] == ref["unmapped"], ctx


def run_both(mt, genomes, reads, k, w, max_occ=0, taxon=None, n_taxa=None, mode=0, **q):
    ix = mt.Index(genomes, k, w, max_occ=max_occ, taxon=taxon, n_taxa=n_taxa)
    dr = mt.to_device(reads)
    res = ix.classify(dr, mode=mode, **q)
    got = res.to_host()
    res.free()
    ref = oracle.Index(genomes, k, w, max_occ=max_occ, taxon=taxon, n_taxa=n_taxa).classify(
        reads, q.get("min_hits", 3), q.get("top_n", 3), q.get("e_mode", 0), q.get("e_value", 7))
    return got, ref


MODES = [0, 1, 2]  # per-stage, fused, fused as one HIP graph


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("top_n", [3, 0, 1])
@pytest.mark.parametrize("E", [0, 3, 7, 15, 31])
def test_small_workload_bit_exact(mt, top_n, E, mode):
    gen, reads, p = synth.workload_small()
    got, ref = run_both(mt, gen.ascii(), reads, p["k"], p["w"], min_hits=3, top_n=top_n, e_value=E, mode=mode)
    assert_same(got, ref, f"small top_n={top_n} E={E} mode={mode}")
    assert len(ref["genome"]) > 9000


def _random_case(rnd):
    motif = "".join(rnd.choice("ACGT") for _ in range(rnd.randint(3, 9)))
    genomes = []
    for _ in range(rnd.randint(1, 5)):
        s = []
        L = rnd.randint(1, 700)
        while len(s) < L:
            u = rnd.random()
            s.extend(motif if u < 0.3 else rnd.choice(["A", "C", "G", "T", "N"] if u < 0.32 else "ACGT"))
        genomes.append("".join(s[:L]))
    reads = []
    for _ in range(rnd.randint(0, 60)):
        g = rnd.choice(genomes)
        m = rnd.choice([0, 1, 5, rnd.randint(10, 70), rnd.randint(60, 300)])
        st = rnd.randint(-5, max(0, len(g) - 1))
        r = list(g[max(st, 0):max(st, 0) + m])
        while len(r) < m:
            r.append(rnd.choice("ACGT"))
        for i in range(len(r)):
            u = rnd.random()
            if u < 0.03:
                r[i] = rnd.choice("ACGTN")
            elif u < 0.04:
                r[i] = r[i].lower()
        if rnd.random() < 0.1 and len(r) > 3:
            del r[rnd.randrange(len(r))]
        reads.append("".join(r))
    return genomes, reads


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("seed", range(12))
def test_random_small_cases_bit_exact(mt, seed, mode):
    rnd = random.Random(seed)
    genomes, reads = _random_case(rnd)
    k, w = rnd.randint(3, 16), rnd.randint(1, 12)
    n_tax = max(1, len(genomes) // 2)
    taxon = np.array([rnd.randrange(n_tax) for _ in genomes], np.uint32)
    q = dict(min_hits=rnd.choice([1, 2, 3]), top_n=rnd.choice([0, 1, 3]), e_mode=rnd.choice([0, 1, 2]),
             e_value=rnd.choice([0, 2, 50, 120]) if True else 0)
    if q["e_mode"] == 0:
        q["e_value"] = rnd.randint(0, 9)
    if mode == 1 and rnd.random() < 0.7:
        q["top_n"] = rnd.randint(1, 4)
    got, ref = run_both(mt, synth.SeqSet.from_list(genomes), synth.SeqSet.from_list(reads), k, w,
                        max_occ=rnd.choice([0, 0, 4]), taxon=taxon, n_taxa=n_tax, mode=mode, **q)
    assert_same(got, ref, f"seed {seed} mode {mode}")


@pytest.mark.parametrize("mode", MODES)
def test_many_hits_per_read_uses_large_path(mt, mode):
    """Reads with more seed hits than one block holds in LDS (repetitive reference)."""
    rnd = random.Random(77)
    unit = "".join(rnd.choice("ACGT") for _ in range(40))
    genome = "".join(unit if rnd.random() < 0.9 else rnd.choice("ACGT") * 40 for _ in range(300))
    reads = [genome[i:i + 400] for i in range(0, 4000, 397)]
    got, ref = run_both(mt, synth.SeqSet.from_list([genome, genome[::-1]]), synth.SeqSet.from_list(reads), 8, 3,
                        min_hits=2, top_n=0, e_value=10, mode=mode)
    assert_same(got, ref, "large")
    co = ref["cand_offsets"].astype(np.int64)
    assert np.diff(co).max() > 100


@pytest.mark.parametrize("seed", range(8))
def test_minimizer_counts_match_oracle(mt, seed):
    """Reference and read minimizers counted exactly: both tile sizes (reads
    averaging over 512 bases take the 1024-start tiles), windows of 1 to 20
    (unrolled and looped), N bases, repeats and sequences shorter than one
    window."""
    rnd = random.Random(500 + seed)
    k, w = rnd.choice([3, 5, 11, 15, 21, 31]), rnd.choice([1, 2, 10, 11, 12, 13, 20])
    motif = "".join(rnd.choice("ACGT") for _ in range(rnd.randint(3, 12)))

    def seq(L):
        s = []
        while len(s) < L:
            u = rnd.random()
            s.extend(motif if u < 0.2 else ("N" if u < 0.22 else rnd.choice("ACGT")))
        return "".join(s[:L])

    genomes = [seq(rnd.randint(1, 5000)) for _ in range(rnd.randint(1, 6))]
    long_reads = seed % 2 == 1
    reads = [seq(rnd.choice([0, 1, k - 1, k, k + w - 2, rnd.randint(20, 300)] +
                            ([rnd.randint(600, 4000)] * 4 if long_reads else []))) for _ in range(80)]
    ix = mt.Index(synth.SeqSet.from_list(genomes), k, w)
    gm = [oracle.minimizers(g.encode(), k, w) for g in genomes]
    info = ix.info()
    assert info["n_minimizers"] == sum(len(p) for p, _ in gm)
    assert info["n_keys"] == len({x for _, xs in gm for x in xs.tolist()})
    res = ix.classify(mt.to_device(synth.SeqSet.from_list(reads)), min_hits=1, top_n=0, mode=0)
    res.free()
    rm = [oracle.minimizers(r.encode(), k, w) for r in reads]
    assert mt.last_stats()["n_minimizers"] == sum(len(p) for p, _ in rm)
    assert (np.mean([len(r) for r in reads]) > 512) == long_reads


def _hits_per_read(genomes, reads, k, w):
    """Seed hits of every read: each read minimizer counts every occurrence
    of its k-mer value among the genomes' minimizers."""
    occ = {}
    for g in genomes:
        for x in oracle.minimizers(g.encode(), k, w)[1].tolist():
            occ[x] = occ.get(x, 0) + 1
    return np.array([sum(occ.get(x, 0) for x in oracle.minimizers(r.encode(), k, w)[1].tolist()) for r in reads])


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("top_n", [0, 3])
def test_hit_count_tiers(mt, mode, top_n):
    """Reads whose seed-hit totals fall in every counting tier of the
    per-stage kernels (one wavefront holding one or four hits per lane, one
    block counting in an LDS hash table, the global-memory sort), many with
    tied counts."""
    rnd = random.Random(91)
    unit = "".join(rnd.choice("ACGT") for _ in range(40))
    rand = "".join(rnd.choice("ACGT") for _ in range(12_000))
    rep = "".join(unit if rnd.random() < 0.8 else rnd.choice("ACGT") * 40 for _ in range(150))
    genomes = [rand[:6000] + rep[:3000], rand[6000:] + rep[3000:]]
    reads = []
    for L in (20, 40, 60, 100, 150, 250, 400, 700, 1000, 1500):
        for _ in range(3):
            g = genomes[rnd.randrange(2)]
            st = rnd.randrange(0, 6000 - L) if rnd.random() < 0.7 else rnd.randrange(5000, 9000 - L)
            reads.append(g[st:st + L])
    H = _hits_per_read(genomes, reads, 8, 3)
    assert (H <= 64).any() and ((H > 64) & (H <= 256)).any()
    assert ((H > 256) & (H <= 2048)).any() and (H > 2048).any()
    got, ref = run_both(mt, synth.SeqSet.from_list(genomes), synth.SeqSet.from_list(reads), 8, 3, min_hits=2,
                        top_n=top_n, e_value=5, mode=mode)
    assert_same(got, ref, f"tiers mode {mode} top_n {top_n}")


def test_fused_fallback_for_hit_overflow(mt):
    """Short reads with more seed hits than the fused kernel holds go to the
    per-stage kernels and still match the oracle."""
    rnd = random.Random(78)
    unit = "".join(rnd.choice("ACGT") for _ in range(30))
    genome = "".join(unit if rnd.random() < 0.95 else rnd.choice("ACGT") * 30 for _ in range(400))
    others = ["".join(rnd.choice("ACGT") for _ in range(5000)) for _ in range(3)]
    reads = [genome[i:i + 150] for i in range(0, 6000, 149)] + [o[i:i + 150] for o in others for i in (0, 999)]
    got, ref = run_both(mt, synth.SeqSet.from_list([genome] + others), synth.SeqSet.from_list(reads), 9, 3,
                        min_hits=2, top_n=4, e_value=7, mode=1)
    assert_same(got, ref, "fused overflow")


@pytest.mark.parametrize("mode", MODES)
def test_keep_all_candidates_short_reads(mt, mode):
    """top_n = 0 with short reads: near-identical genome families give reads
    with up to 8 candidates (fused staging) and with more (per-stage finish,
    placed after the compaction), in one call."""
    rnd = np.random.default_rng(41)
    base6 = synth.random_codes(rnd, 20_000)
    base12 = synth.random_codes(rnd, 20_000)
    fam = [synth.substitute(rnd, base6, 0.002) for _ in range(6)] + \
          [synth.substitute(rnd, base12, 0.002) for _ in range(12)]
    genomes = synth.SeqSet.from_list([synth.ACGT[f].tobytes() for f in fam])
    starts = rnd.integers(0, 19_800, 300)
    src = rnd.integers(0, len(fam), 300)
    reads = synth.SeqSet.from_list([synth.ACGT[fam[g][st:st + 150]].tobytes() for g, st in zip(src, starts)])
    got, ref = run_both(mt, genomes, reads, 15, 10, min_hits=2, top_n=0, e_value=7, mode=mode)
    assert_same(got, ref, "keep-all")
    nc = np.diff(ref["cand_offsets"].astype(np.int64))
    assert (nc > 8).any() and ((nc > 0) & (nc <= 8)).any()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n_taxa", [3, 5000])
def test_taxon_counts_few_and_many_taxa(mt, mode, n_taxa):
    """Per-taxon unique/multi/unmapped counts with several genomes per taxon
    and with more taxa than a block of the taxon step counts in LDS; genome
    families make reads map to several genomes at the same count."""
    rnd = np.random.default_rng(n_taxa)
    bases = [synth.random_codes(rnd, 15_000) for _ in range(3)]
    fam = [synth.substitute(rnd, b, 0.003) for b in bases for _ in range(4)] + [synth.random_codes(rnd, 15_000)]
    genomes = synth.SeqSet.from_list([synth.ACGT[f].tobytes() for f in fam])
    starts = rnd.integers(0, 14_800, 3000)
    src = rnd.integers(0, len(fam), 3000)
    reads = [synth.ACGT[fam[g][st:st + 150]].tobytes() for g, st in zip(src, starts)]
    reads += [synth.ACGT[synth.random_codes(rnd, 150)].tobytes() for _ in range(100)]  # unmapped
    taxon = rnd.integers(0, n_taxa, len(fam)).astype(np.uint32)
    got, ref = run_both(mt, genomes, synth.SeqSet.from_list(reads), 15, 10, taxon=taxon, n_taxa=n_taxa, min_hits=2,
                        top_n=0, e_value=7, mode=mode)
    assert_same(got, ref, f"taxa {n_taxa} mode {mode}")
    assert ref["multi"].sum() > 100 and ref["unique"].sum() > 100 and ref["unmapped"] >= 100


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("E", [0, 31, 32])
def test_fused_limit_boundaries(mt, mode, E):
    """Reads at the fused kernel's limits and just past them (256 / 257 bases,
    E 31 / 32) and at the 64-base word boundaries of its planes and band rows
    give the oracle's result in every form."""
    rnd = np.random.default_rng(17)
    gen = synth.make_genomes(rnd, 4, 30_000, 0.5)
    lens = np.array([1, 20, 63, 64, 65, 127, 128, 129, 191, 192, 193, 255, 256, 257, 300] * 12)
    reads, _ = synth.make_reads(rnd, gen, lens, 0.01, 0.002)
    got, ref = run_both(mt, gen.ascii(), reads, 15, 10, min_hits=2, top_n=3, e_value=E, mode=mode)
    assert_same(got, ref, f"E={E} mode {mode}")
    assert ref["read_accepted"].sum() > (10 if E == 0 else len(lens) // 2)


@pytest.mark.parametrize("mode", MODES)
def test_long_reads_large_E_bit_exact(mt, mode):
    rnd = np.random.default_rng(5)
    gen = synth.make_genomes(rnd, 3, 60_000, 0.5)
    lens = np.concatenate([rnd.integers(1000, 6000, 40), rnd.integers(75, 300, 200)])
    reads, _ = synth.make_reads(rnd, gen, lens, 0.02, 0.03)
    got, ref = run_both(mt, gen.ascii(), reads, 15, 10, min_hits=3, top_n=3, e_mode=1, e_value=50, mode=mode)
    assert_same(got, ref, "long")
    assert ref["read_E"].max() >= 100


@pytest.mark.parametrize("mode", MODES)
def test_empty_read_set(mt, mode):
    gen, _, p = synth.workload_small(10)
    got, ref = run_both(mt, gen.ascii(), synth.SeqSet.from_list([]), p["k"], p["w"], mode=mode)
    assert_same(got, ref, "empty")


@pytest.mark.parametrize("mode", MODES)
def test_invalid_byte_rejected(mt, mode):
    gen, _, p = synth.workload_small(10)
    ix = mt.Index(gen.ascii(), p["k"], p["w"])
    with pytest.raises(mt.MTError) as e:
        ix.classify(mt.to_device(synth.SeqSet.from_list(["ACGTACGTAC", "ACGT*ACG"])), mode=mode)
    assert e.value.status == -1
    with pytest.raises(mt.MTError) as e:
        ix.classify(mt.to_device(synth.SeqSet.from_list(["ACGT" * 20000])), mode=mode)
    assert e.value.status == -1
    with pytest.raises(mt.MTError):
        mt.Index(synth.SeqSet.from_list(["ACGTXACGT"]), 4, 2)


def test_filter_pairs_against_oracle(mt):
    import torch
    rnd = np.random.default_rng(11)
    gen = synth.make_genomes(rnd, 4, 20_000, (0.3, 0.7))
    lens = np.concatenate([rnd.integers(0, 300, 300), rnd.integers(300, 1500, 20)])
    reads, origin = synth.make_reads(rnd, gen, lens, 0.01, 0.01)
    reads = synth.inject_n(rnd, reads, 0.002)
    n = 4000
    pr = rnd.integers(0, reads.n, n).astype(np.uint32)
    pg = np.where(rnd.random(n) < 0.7, origin[pr, 0], rnd.integers(0, 4, n)).astype(np.uint32)
    pdg = (origin[pr, 1] + rnd.integers(-20, 21, n)).astype(np.int64)
    pdg[:50] = rnd.integers(-400, 0, 50)
    pdg[50:100] = 20_000 + rnd.integers(-300, 50, 50)
    pe = rnd.integers(0, 40, n).astype(np.uint16)
    ga = gen.ascii()
    ix = mt.Index(ga, 15, 10)
    dev = lambda a, t: torch.from_numpy(a.view(t) if a.dtype.itemsize == np.dtype(t).itemsize else a).cuda()
    ap, ac = ix.filter_pairs(mt.to_device(reads), torch.from_numpy(pr.view(np.int32)).cuda(),
                             torch.from_numpy(pg.view(np.int32)).cuda(), torch.from_numpy(pdg).cuda(),
                             torch.from_numpy(pe.view(np.int16)).cuda())
    ap = ap.cpu().numpy().view(np.uint16)
    ac = ac.cpu().numpy()
    oap, oac = oracle.Index(ga, 15, 10).filter_pairs(reads, pr, pg, pdg, pe)
    assert np.array_equal(ap, oap), np.flatnonzero(ap != oap)[:10]
    assert np.array_equal(ac, oac)
    assert (oap <= pe).mean() > 0.3 and (oap > pe).mean() > 0.05


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("kind", [1, 2, 3, 4])
def test_classify_with_each_filter(mt, mode, kind):
    """Classification with another filter of Table 1 (it runs per stage in
    every mode): candidates as with the obstacle walk, values of that filter."""
    rnd = np.random.default_rng(60 + kind)
    gen = synth.make_genomes(rnd, 5, 30_000, (0.3, 0.7))
    lens = np.concatenate([rnd.integers(60, 300, 600), rnd.integers(800, 3000, 10)])
    reads, _ = synth.make_reads(rnd, gen, lens, 0.02, 0.01)
    reads = synth.inject_n(rnd, reads, 0.002)
    ga = gen.ascii()
    ix = mt.Index(ga, 13, 7)
    res = ix.classify(mt.to_device(reads), min_hits=2, top_n=3, e_mode=1, e_value=40, mode=mode, filter_kind=kind)
    got = res.to_host()
    res.free()
    ref = oracle.Index(ga, 13, 7).classify(reads, 2, 3, 1, 40, filter_kind=kind)
    assert_same(got, ref, f"filter {kind} mode {mode}")
    assert 0 < ref["accept"].mean() < 1 or kind in (2, 3)


@pytest.mark.parametrize("kind", [1, 2, 3, 4])
def test_filter_kinds_against_oracle(mt, kind):
    """The Hamming, base-counting, q-gram and shifted-Hamming filters on one
    pair stream: reads of 0 to 3,000 bases with N, genomes with N, windows past
    either genome end."""
    import torch
    rnd = np.random.default_rng(31 + kind)
    gen = synth.make_genomes(rnd, 4, 20_000, (0.3, 0.7))
    lens = np.concatenate([rnd.integers(0, 300, 400), rnd.integers(300, 3000, 40), [64, 128, 192, 256, 65]])
    reads, origin = synth.make_reads(rnd, gen, lens, 0.01, 0.005)
    reads = synth.inject_n(rnd, reads, 0.003)
    ga = gen.ascii()
    seq = ga.seq.copy()
    seq[rnd.random(len(seq)) < 0.0005] = ord("N")
    ga = synth.SeqSet(seq=seq, offsets=ga.offsets)
    n = 5000
    pr = rnd.integers(0, reads.n, n).astype(np.uint32)
    pg = np.where(rnd.random(n) < 0.8, origin[pr, 0], rnd.integers(0, 4, n)).astype(np.uint32)
    pdg = (origin[pr, 1] + rnd.integers(-3, 4, n)).astype(np.int64)
    pdg[:100] = rnd.integers(-400, 20, 100)
    pdg[100:200] = 20_000 - lens[pr[100:200]] + rnd.integers(-20, 400, 100)
    pe = rnd.choice([0, 1, 3, 7, 15, 40, 300], n).astype(np.uint16)
    ix = mt.Index(ga, 15, 10)
    ap, ac = ix.filter_pairs(mt.to_device(reads), torch.from_numpy(pr.view(np.int32)).cuda(),
                             torch.from_numpy(pg.view(np.int32)).cuda(), torch.from_numpy(pdg).cuda(),
                             torch.from_numpy(pe.view(np.int16)).cuda(), kind=kind)
    ap = ap.cpu().numpy().view(np.uint16)
    oap, oac = oracle.Index(ga, 15, 10).filter_pairs(reads, pr, pg, pdg, pe, kind=kind)
    assert np.array_equal(ap, oap), np.flatnonzero(ap != oap)[:10]
    assert np.array_equal(ac.cpu().numpy(), oac)
    assert (oap <= pe).mean() > 0.2 and (oap > pe).mean() > 0.05


def test_filter_long_pairs_at_edges_and_n(mt):
    """Long-read pairs (E > 31, LDS kernel) whose window runs past either end
    of the genome, lies in a genome with N bases, or lies inside a genome
    without N (the kernel drops the window's N plane only there)."""
    import torch
    rnd = np.random.default_rng(23)
    gen = synth.make_genomes(rnd, 3, 40_000, 0.5)
    lens = rnd.integers(800, 4000, 60)
    reads, origin = synth.make_reads(rnd, gen, lens, 0.02, 0.02)
    reads = synth.inject_n(rnd, reads, 0.001)
    ga = gen.ascii()
    seq = ga.seq.copy()  # genome 2 gets N bases
    g2 = slice(int(ga.offsets[2]), int(ga.offsets[3]))
    hit = rnd.random(g2.stop - g2.start) < 0.002
    seq[g2][hit] = ord("N")
    ga = synth.SeqSet(seq=seq, offsets=ga.offsets)
    n = 900
    pr = rnd.integers(0, reads.n, n).astype(np.uint32)
    pg = origin[pr, 0].astype(np.uint32)
    pdg = (origin[pr, 1] + rnd.integers(-30, 31, n)).astype(np.int64)
    pdg[:100] = rnd.integers(-600, 40, 100)  # window before the genome start
    pdg[100:200] = 40_000 - lens[pr[100:200]] + rnd.integers(-40, 600, 100)  # past the end
    pe = rnd.integers(32, 260, n).astype(np.uint16)
    ix = mt.Index(ga, 15, 10)
    ap, ac = ix.filter_pairs(mt.to_device(reads), torch.from_numpy(pr.view(np.int32)).cuda(),
                             torch.from_numpy(pg.view(np.int32)).cuda(), torch.from_numpy(pdg).cuda(),
                             torch.from_numpy(pe.view(np.int16)).cuda())
    ap = ap.cpu().numpy().view(np.uint16)
    oap, oac = oracle.Index(ga, 15, 10).filter_pairs(reads, pr, pg, pdg, pe)
    assert np.array_equal(ap, oap), np.flatnonzero(ap != oap)[:10]
    assert np.array_equal(ac.cpu().numpy(), oac)
    inside = (pdg - pe >= 0) & (pdg + lens[pr] + pe <= 40_000) & (pg != 2)
    assert inside.sum() > 100 and (~inside).sum() > 100 and (oap <= pe).mean() > 0.2


def test_filter_long_pairs_very_large_E(mt):
    """E of 1,000-1,600 (over 32 band rows per lane: a lane's rows take two
    chunks, the second only partly filled), on long reads near and far from
    their true diagonal."""
    import torch
    rnd = np.random.default_rng(29)
    gen = synth.make_genomes(rnd, 2, 30_000, 0.5)
    lens = rnd.integers(5000, 8000, 40)
    reads, origin = synth.make_reads(rnd, gen, lens, 0.05, 0.05)
    n = 48
    pr = rnd.integers(0, reads.n, n).astype(np.uint32)
    pg = origin[pr, 0].astype(np.uint32)
    pdg = (origin[pr, 1] + rnd.integers(-900, 900, n)).astype(np.int64)
    pdg[::2] = rnd.integers(-2000, 25_000, n // 2)  # unrelated windows: rejected
    pe = rnd.integers(1000, 1600, n).astype(np.uint16)
    ga = gen.ascii()
    ix = mt.Index(ga, 15, 10)
    ap, ac = ix.filter_pairs(mt.to_device(reads), torch.from_numpy(pr.view(np.int32)).cuda(),
                             torch.from_numpy(pg.view(np.int32)).cuda(), torch.from_numpy(pdg).cuda(),
                             torch.from_numpy(pe.view(np.int16)).cuda())
    ap = ap.cpu().numpy().view(np.uint16)
    oap, oac = oracle.Index(ga, 15, 10).filter_pairs(reads, pr, pg, pdg, pe)
    assert np.array_equal(ap, oap), np.flatnonzero(ap != oap)[:10]
    assert np.array_equal(ac.cpu().numpy(), oac)
    assert (2 * pe.astype(int) + 1 > 64 * 32).sum() > 10 and 0 < oac.sum() < n


def test_repeat_calls_and_modes_identical(mt):
    gen, reads, p = synth.workload_small(3000)
    ix = mt.Index(gen.ascii(), p["k"], p["w"])
    dr = mt.to_device(reads)
    a = ix.classify(dr).to_host()
    b = ix.classify(dr).to_host()
    c = ix.classify(dr, mode=1).to_host()
    d = ix.classify(dr, mode=1).to_host()
    assert_same(a, b, "repeat")
    assert_same(a, c, "per-stage vs fused")
    assert_same(c, d, "fused repeat")


def test_graph_replays_between_eager_calls(mt):
    """The graph form, replayed (updated in place) many times with eager calls
    of other sizes and shapes in between, equals the eager result every time."""
    gen, reads, p = synth.workload_small(4000)
    ix = mt.Index(gen.ascii(), p["k"], p["w"])
    sizes = [4000, 1, 257, 4000, 3999, 64, 4000]
    sets = {m: mt.to_device(reads.subset(np.arange(m))) for m in set(sizes)}
    eager = {m: ix.classify(sets[m], mode=1).to_host() for m in sets}
    for i, m in enumerate(sizes):
        got = ix.classify(sets[m], mode=2).to_host()
        assert_same(got, eager[m], f"graph replay {i} ({m} reads)")
        other = sizes[(i + 3) % len(sizes)]
        assert_same(ix.classify(sets[other], mode=0).to_host(), eager[other], f"eager between replays {i}")


def test_filter_buckets_long_reads_against_oracle(mt):
    """Pairs in every filter bucket: E <= 7, <= 15, <= 31, the LDS long-read
    kernel (E > 31) and pairs too large for its LDS budget (30 kbp, E = 1500)."""
    import torch
    rnd = np.random.default_rng(21)
    gen = synth.make_genomes(rnd, 2, 120_000, 0.5)
    lens = np.array([150, 150, 280, 900, 2500, 6000, 10_000, 30_000, 30_000, 75])
    reads, origin = synth.make_reads(rnd, gen, lens, 0.02, 0.02)
    pr, pg, pd, pe = [], [], [], []
    for i in range(reads.n):
        for E in (0, 5, 12, 25, 40, 130, 500, 1500):
            for shift in (0, -3, 17):
                pr.append(i)
                pg.append(origin[i, 0])
                pd.append(origin[i, 1] + shift)
                pe.append(E)
    pr = np.array(pr, np.uint32)
    pg = np.array(pg, np.uint32)
    pd = np.array(pd, np.int64)
    pe = np.array(pe, np.uint16)
    ga = gen.ascii()
    ix = mt.Index(ga, 15, 10)
    ap, ac = ix.filter_pairs(mt.to_device(reads), torch.from_numpy(pr.view(np.int32)).cuda(),
                             torch.from_numpy(pg.view(np.int32)).cuda(), torch.from_numpy(pd).cuda(),
                             torch.from_numpy(pe.view(np.int16)).cuda())
    ap = ap.cpu().numpy().view(np.uint16)
    oap, oac = oracle.Index(ga, 15, 10).filter_pairs(reads, pr, pg, pd, pe)
    assert np.array_equal(ap, oap), np.flatnonzero(ap != oap)[:10]
    assert np.array_equal(ac.cpu().numpy(), oac)
    assert ((oap <= pe) & (pe >= 130)).any() and (oap == pe + 1).any()
