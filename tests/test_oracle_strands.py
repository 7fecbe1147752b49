"""Pins of the oracle's both-strand classification (reads come from either
strand of a genome; the reverse strand is met by the read's reverse
complement against the forward genome).

* brute force: every seed match of the read and of its reverse complement
  (written here with str.translate, independently of the oracle) against every
  reference minimizer occurrence, counted per (genome, diag, strand), ordered
  and cut as the classification orders and cuts;
* reads cut from the reverse strand without errors are found at their true
  position on strand 1 with value 0 under every filter;
* the filter of a strand-1 candidate equals the pair filter on the reverse
  complement;
* symmetry: classifying the reverse complements swaps the strands and keeps
  every count;
* a reverse-complement palindrome has each location twice, forward first;
* the step-3a counts follow the brute-force rule over both strands.
"""
import random
from collections import Counter

import numpy as np
import pytest

import oracle
import synth
from test_oracle_pins import _brute_taxa, _minimizers_second_form, _repetitive_case

_COMP = str.maketrans("ACGTNacgtn", "TGCANtgcan")


def rc(s):
    return s.translate(_COMP)[::-1]


def _brute_both(genomes, reads, k, w, min_hits, top_n, max_occ=0):
    occ = {}
    for g, gs in enumerate(genomes):
        for q, x in zip(*_minimizers_second_form(gs, k, w)):
            occ.setdefault(x, []).append((g, q))
    out = []
    for rs in reads:
        cnt = Counter()
        for strand, oriented in enumerate((rs, rc(rs))):
            for p, x in zip(*_minimizers_second_form(oriented, k, w)):
                lst = occ.get(x, [])
                if max_occ and len(lst) > max_occ:
                    continue
                for g, q in lst:
                    cnt[(g, q - p, strand)] += 1
        cands = sorted(((h, g, d, s) for (g, d, s), h in cnt.items() if h >= min_hits),
                       key=lambda t: (-t[0], t[1], t[2], t[3]))
        out.append(cands[:top_n] if top_n else cands)
    return out


def _cands(res, n):
    co = res["cand_offsets"].astype(np.int64)
    return [[(int(res["hits"][c]), int(res["genome"][c]), int(res["diag"][c]), int(res["strand"][c]))
             for c in range(co[r], co[r + 1])] for r in range(n)]


def _mixed_strand_case(rnd):
    genomes, reads = _repetitive_case(rnd, rnd.randint(1, 4), rnd.randint(20, 120), 40, rnd.randint(3, 7))
    reads = [rc(r) if rnd.random() < 0.5 else r for r in reads]
    return genomes, reads


@pytest.mark.parametrize("seed", range(8))
def test_both_strand_candidates_match_brute_force(seed):
    rnd = random.Random(300 + seed)
    genomes, reads = _mixed_strand_case(rnd)
    k, w = rnd.randint(2, 6), rnd.randint(1, 5)
    min_hits = rnd.choice([1, 2, 3])
    top_n = rnd.choice([0, 1, 3])
    max_occ = rnd.choice([0, 0, 3])
    ix = oracle.Index(synth.SeqSet.from_list(genomes), k, w, max_occ=max_occ)
    res = ix.classify(synth.SeqSet.from_list(reads), min_hits, top_n, 0, 2, strands=2)
    assert _cands(res, len(reads)) == _brute_both(genomes, reads, k, w, min_hits, top_n, max_occ)


def test_one_strand_has_only_forward_candidates():
    rnd = random.Random(390)
    genomes, reads = _mixed_strand_case(rnd)
    ix = oracle.Index(synth.SeqSet.from_list(genomes), 4, 3)
    res = ix.classify(synth.SeqSet.from_list(reads), 1, 0, 0, 2)
    assert not res["strand"].any()
    both = _brute_both(genomes, reads, 4, 3, 1, 0)
    assert _cands(res, len(reads)) == [[c for c in b if c[3] == 0] for b in both]


@pytest.mark.parametrize("kind", [0, 1, 2, 3, 4])
def test_reverse_strand_reads_found_exactly(kind):
    rnd = np.random.default_rng(40 + kind)
    gen = synth.make_genomes(rnd, 3, 8000, 0.5)
    gs = [bytes(gen.ascii().seq[gen.offsets[g]:gen.offsets[g + 1]]).decode() for g in range(3)]
    truth, reads = [], []
    for _ in range(60):
        g = int(rnd.integers(3))
        m = int(rnd.integers(40, 200))
        p = int(rnd.integers(0, len(gs[g]) - m))
        truth.append((g, p))
        reads.append(rc(gs[g][p:p + m]))
    ix = oracle.Index(gen.ascii(), 11, 5)
    rs = synth.SeqSet.from_list(reads)
    res = ix.classify(rs, 2, 0, 0, 3, filter_kind=kind, strands=2)
    co = res["cand_offsets"].astype(np.int64)
    for r, (g, p) in enumerate(truth):
        hit = [c for c in range(co[r], co[r + 1])
               if (res["genome"][c], res["diag"][c], res["strand"][c]) == (g, p, 1)]
        assert len(hit) == 1 and res["approx"][hit[0]] == 0, r
    assert res["read_accepted"].all()
    fwd = ix.classify(rs, 2, 0, 0, 3, filter_kind=kind)
    assert fwd["read_accepted"].sum() < 5   # the forward strand alone misses them


@pytest.mark.parametrize("kind", [0, 1, 2, 3, 4])
def test_strand1_values_are_the_pair_filter_on_the_reverse_complement(kind):
    rnd = np.random.default_rng(70 + kind)
    gen = synth.make_genomes(rnd, 4, 20_000, 0.5)
    reads, _ = synth.make_reads(rnd, gen, rnd.integers(60, 250, 200), 0.03, 0.01)
    strs = [bytes(reads.seq[reads.offsets[i]:reads.offsets[i + 1]]).decode() for i in range(reads.n)]
    strs = [rc(s) if i % 2 else s for i, s in enumerate(strs)]
    rs = synth.SeqSet.from_list(strs)
    ix = oracle.Index(gen.ascii(), 13, 7)
    res = ix.classify(rs, 2, 3, 1, 50, filter_kind=kind, strands=2)
    co = res["cand_offsets"].astype(np.int64)
    pr = np.repeat(np.arange(rs.n), np.diff(co)).astype(np.uint32)
    st = res["strand"].astype(bool)
    assert st.sum() > 100 and (~st).sum() > 100
    rcs = synth.SeqSet.from_list([rc(s) for s in strs])
    e = res["read_E"][pr]
    a0, _ = ix.filter_pairs(rs, pr[~st], res["genome"][~st], res["diag"][~st], e[~st], kind=kind)
    a1, _ = ix.filter_pairs(rcs, pr[st], res["genome"][st], res["diag"][st], e[st], kind=kind)
    assert np.array_equal(res["approx"][~st], a0) and np.array_equal(res["approx"][st], a1)
    if kind == 0:
        for c in np.flatnonzero(st)[:50]:
            g = int(res["genome"][c])
            ref = bytes(gen.ascii().seq[gen.offsets[g]:gen.offsets[g + 1]]).decode()
            assert res["approx"][c] == oracle.approx(rc(strs[pr[c]]), ref, int(res["diag"][c]), int(e[c]))


def test_strand_symmetry():
    """Classifying the reverse complements swaps the strands of every location
    and keeps the read outcomes and the per-taxon counts."""
    rnd = np.random.default_rng(5)
    gen = synth.make_genomes(rnd, 6, 10_000, 0.5)
    reads, _ = synth.make_reads(rnd, gen, rnd.integers(50, 300, 300), 0.03, 0.01)
    strs = [bytes(reads.seq[reads.offsets[i]:reads.offsets[i + 1]]).decode() for i in range(reads.n)]
    strs = [rc(s) if i % 3 == 0 else s for i, s in enumerate(strs)]
    taxon = np.array([0, 1, 1, 2, 3, 3], np.uint32)
    ix = oracle.Index(gen.ascii(), 12, 6, taxon=taxon, n_taxa=4)
    a = ix.classify(synth.SeqSet.from_list(strs), 2, 0, 1, 60, strands=2)
    b = ix.classify(synth.SeqSet.from_list([rc(s) for s in strs]), 2, 0, 1, 60, strands=2)
    for f in ("cand_offsets", "read_accepted", "read_E", "unique", "multi"):
        assert np.array_equal(a[f], b[f]), f
    assert a["unmapped"] == b["unmapped"]
    ca, cb = _cands(a, len(strs)), _cands(b, len(strs))
    co = a["cand_offsets"].astype(np.int64)
    for r in range(len(strs)):
        va = sorted((h, g, d, s, int(a["approx"][co[r] + i])) for i, (h, g, d, s) in enumerate(ca[r]))
        vb = sorted((h, g, d, 1 - s, int(b["approx"][co[r] + i])) for i, (h, g, d, s) in enumerate(cb[r]))
        assert va == vb, r
    assert a["read_accepted"].sum() > 250


def test_palindromic_read_twice_forward_first():
    unit = "ACGCGT"  # its own reverse complement
    assert rc(unit) == unit
    rnd = random.Random(11)
    flank = "".join(rnd.choice("ACGT") for _ in range(40))
    genome = flank + unit * 5 + rc(flank)
    read = genome[10:len(genome) - 10]
    assert rc(read) == read
    ix = oracle.Index(synth.SeqSet.from_list([genome]), 5, 2)
    res = ix.classify(synth.SeqSet.from_list([read]), 1, 0, 0, 2, strands=2)
    c = _cands(res, 1)[0]
    assert c and len(c) % 2 == 0
    for i in range(0, len(c), 2):
        assert c[i][:3] == c[i + 1][:3] and (c[i][3], c[i + 1][3]) == (0, 1)
    assert res["approx"][0] == 0 and res["approx"][1] == 0 and c[0][2] == 10


def test_both_strand_taxa_brute_force():
    rnd = random.Random(7100)
    root = "".join(rnd.choice("ACGT") for _ in range(3000))
    genomes = []
    for _ in range(5):
        s = list(root)
        for i in rnd.sample(range(len(s)), 30):
            s[i] = rnd.choice("ACGT")
        genomes.append("".join(s))
    taxon = np.array([0, 1, 1, 2, 3], np.uint32)
    reads = []
    for _ in range(200):
        g = rnd.choice(genomes)
        st = rnd.randint(0, len(g) - 100)
        r = list(g[st:st + 100])
        for i in rnd.sample(range(100), rnd.randint(0, 6)):
            r[i] = rnd.choice("ACGT")
        r = "".join(r)
        reads.append(rc(r) if rnd.random() < 0.5 else r)
    ix = oracle.Index(synth.SeqSet.from_list(genomes), 9, 5, taxon=taxon, n_taxa=4)
    rs = synth.SeqSet.from_list(reads)
    for top_n, e in ((3, 3), (0, 5)):
        res = ix.classify(rs, 2, top_n, 0, e, strands=2)
        acc, uni, mul, unm = _brute_taxa(res, taxon, 4, len(reads))
        assert np.array_equal(res["read_accepted"], acc)
        assert np.array_equal(res["unique"], uni) and np.array_equal(res["multi"], mul)
        assert res["unmapped"] == unm
        assert acc.sum() > 150


def test_invalid_strand_count_rejected():
    ix = oracle.Index(synth.SeqSet.from_list(["ACGTACGTAC"]), 3, 2)
    rs = synth.SeqSet.from_list(["ACGTA"])
    for bad in (0, 3):
        with pytest.raises(ValueError):
            ix.classify(rs, strands=bad)
