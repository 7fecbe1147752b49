"""Pins of the oracle's alternative filters on one pair stream (Table 1's
Hamming-distance filter, the base-counting comparison, the q-gram filter and
the shifted Hamming distance).

* brute force from the definitions, on strings, with N and windows that run
  past either end of the genome;
* order: obstacle count <= Hamming distance and base count <= Hamming distance
  (each saturated at E + 1): the greedy walk may use any row of the band, the
  Hamming distance only row 0, and one mismatching column changes the base
  counts by at most two;
* special cases: Hamming 0 iff the read occurs exactly at the diagonal; base
  count 0 for a window that is a rearrangement of the read;
* the q-gram lemma: the q-gram value never exceeds the semi-global banded edit
  distance (an independent DP) nor the Hamming distance;
* shifted Hamming distance: brute force with the masks written as strings and
  the short-match amendment as a regular expression; 0 whenever the read
  occurs exactly on any diagonal of the band.
"""
import random
import re
from collections import Counter

import numpy as np
import pytest

import oracle
import synth
from test_oracle_pins import semi_global_banded

Q = 5


def _ref_at(ref, p):
    return ref[p] if 0 <= p < len(ref) else None


def _hamming(q, ref, diag, E):
    c = sum(1 for j, b in enumerate(q) if b == "N" or _ref_at(ref, diag + j) in (None, "N")
            or _ref_at(ref, diag + j) != b)
    return min(c, E + 1)


def _base_count(q, ref, diag, E):
    nq = Counter(b for b in q if b != "N")
    nw = Counter(x for x in (_ref_at(ref, diag + j) for j in range(len(q))) if x not in (None, "N"))
    l1 = sum(abs(nq[c] - nw[c]) for c in "ACGT")
    return min((l1 + 1) // 2, E + 1)


def _qgram(q, ref, diag, E):
    m = len(q)
    if m < Q:
        return 0
    win = [_ref_at(ref, p) for p in range(diag - E, diag + m + E)]
    cw = Counter("".join(win[i:i + Q]) for i in range(len(win) - Q + 1)
                 if all(x not in (None, "N") for x in win[i:i + Q]))
    cq = Counter(q[j:j + Q] for j in range(m - Q + 1) if "N" not in q[j:j + Q])
    shared = sum(min(c, cw[g]) for g, c in cq.items())
    missing = (m - Q + 1) - shared
    return min(-(-missing // Q), E + 1)


def _shd(q, ref, diag, E):
    m = len(q)
    if m == 0:
        return 0
    final = [1] * m
    for d in range(-E, E + 1):
        mask = "".join("1" if (b == "N" or _ref_at(ref, diag + d + j) in (None, "N")
                               or _ref_at(ref, diag + d + j) != b) else "0" for j, b in enumerate(q))
        # one or two zeros between two ones become ones (lookarounds keep the flanking ones)
        amended = re.sub(r"(?<=1)0{1,2}(?=1)", lambda mo: "1" * len(mo.group(0)), mask)
        final = [f & int(c) for f, c in zip(final, amended)]
    return min(sum(final), E + 1)


def _pairs(rnd, n):
    genomes = ["".join(rnd.choice("ACGTN" if rnd.random() < 0.05 else "ACGT") for _ in range(rnd.randint(1, 300)))
               for _ in range(3)]
    reads, pr, pg, pd, pe = [], [], [], [], []
    for i in range(n):
        g = rnd.randrange(3)
        m = rnd.randint(0, 120)
        d = rnd.randint(-40, len(genomes[g]) + 10)
        src = genomes[g][max(d, 0):max(d, 0) + m]
        r = [c if rnd.random() > 0.08 else rnd.choice("ACGTN") for c in src] + \
            [rnd.choice("ACGT") for _ in range(m - len(src))]
        if rnd.random() < 0.3:
            rnd.shuffle(r)
        reads.append("".join(r))
        pr.append(i)
        pg.append(g)
        pd.append(d)
        pe.append(rnd.choice([0, 1, 3, 7, 20, 200]))
    return genomes, reads, np.array(pr, np.uint32), np.array(pg, np.uint32), np.array(pd, np.int64), \
        np.array(pe, np.uint16)


@pytest.mark.parametrize("seed", range(6))
def test_hamming_and_base_count_match_brute_force(seed):
    rnd = random.Random(seed)
    genomes, reads, pr, pg, pd, pe = _pairs(rnd, 300)
    ix = oracle.Index(synth.SeqSet.from_list(genomes), 5, 3)
    rs = synth.SeqSet.from_list(reads)
    hd, hacc = ix.filter_pairs(rs, pr, pg, pd, pe, kind=1)
    bc, bacc = ix.filter_pairs(rs, pr, pg, pd, pe, kind=2)
    qg, _ = ix.filter_pairs(rs, pr, pg, pd, pe, kind=3)
    small = pe <= 20  # the brute-force SHD is quadratic in E
    sh, _ = ix.filter_pairs(rs, pr[small], pg[small], pd[small], pe[small], kind=4)
    for i in range(len(pr)):
        q, ref, d, E = reads[i], genomes[pg[i]], int(pd[i]), int(pe[i])
        assert hd[i] == _hamming(q, ref, d, E), i
        assert bc[i] == _base_count(q, ref, d, E), i
        assert qg[i] == _qgram(q, ref, d, E), i
    for s_i, i in enumerate(np.flatnonzero(small)):
        assert sh[s_i] == _shd(reads[i], genomes[pg[i]], int(pd[i]), int(pe[i])), i
    assert np.array_equal(hacc, (hd <= pe).astype(np.uint8)) and np.array_equal(bacc, (bc <= pe).astype(np.uint8))


@pytest.mark.parametrize("seed", range(4))
def test_filter_order_obstacles_below_hamming_base_count_below_hamming(seed):
    rnd = random.Random(50 + seed)
    genomes, reads, pr, pg, pd, pe = _pairs(rnd, 400)
    ix = oracle.Index(synth.SeqSet.from_list(genomes), 5, 3)
    rs = synth.SeqSet.from_list(reads)
    ob, _ = ix.filter_pairs(rs, pr, pg, pd, pe, kind=0)
    hd, _ = ix.filter_pairs(rs, pr, pg, pd, pe, kind=1)
    bc, _ = ix.filter_pairs(rs, pr, pg, pd, pe, kind=2)
    assert (ob <= hd).all() and (bc <= hd).all()
    assert (ob < hd).any() and (bc < hd).any()  # the bounds are not all tight


@pytest.mark.parametrize("seed", range(4))
def test_qgram_lemma(seed):
    rnd = random.Random(80 + seed)
    genomes, reads, pr, pg, pd, pe = _pairs(rnd, 250)
    pe = np.array([rnd.choice([1, 2, 4, 8]) for _ in pe], np.uint16)  # small bands keep the DP fast
    ix = oracle.Index(synth.SeqSet.from_list(genomes), 5, 3)
    rs = synth.SeqSet.from_list(reads)
    qg, _ = ix.filter_pairs(rs, pr, pg, pd, pe, kind=3)
    hd, _ = ix.filter_pairs(rs, pr, pg, pd, pe, kind=1)
    tight = 0
    for i in range(len(pr)):
        E = int(pe[i])
        sg = semi_global_banded(reads[i], genomes[pg[i]], int(pd[i]), E)
        assert qg[i] <= min(sg, E + 1), i
        tight += qg[i] == min(sg, E + 1) and sg > 0
    assert (qg <= hd).all() and tight > 5


def test_special_cases():
    g = "ACGTTGCAAGGCTTACCGATGCAGTAAC"
    ix = oracle.Index(synth.SeqSet.from_list([g]), 5, 3)
    exact, shuffled = g[4:20], "".join(sorted(g[4:20]))
    rs = synth.SeqSet.from_list([exact, shuffled, "ACGNACGT"])
    pr = np.array([0, 1, 2, 0], np.uint32)
    pg = np.zeros(4, np.uint32)
    pd = np.array([4, 4, 0, 5], np.int64)
    pe = np.full(4, 30, np.uint16)
    hd, _ = ix.filter_pairs(rs, pr, pg, pd, pe, kind=1)
    bc, _ = ix.filter_pairs(rs, pr, pg, pd, pe, kind=2)
    assert hd[0] == 0 and bc[0] == 0          # exact occurrence
    assert hd[1] > 0 and bc[1] == 0           # a rearrangement of the window
    assert hd[2] >= 1                         # N never matches
    assert hd[3] > 0                          # shifted by one
    qg, _ = ix.filter_pairs(rs, pr, pg, pd, pe, kind=3)
    assert qg[0] == 0 and qg[3] == 0          # shifted by one: inside the band, every q-gram is shared
    sh, _ = ix.filter_pairs(rs, pr, pg, pd, np.full(4, 3, np.uint16), kind=4)
    assert sh[0] == 0 and sh[3] == 0          # exact on the diagonal, and one row off it
    assert sh[2] >= 1                         # the N column is a one in every mask
    short = synth.SeqSet.from_list(["ACG"])
    assert ix.filter_pairs(short, [0], [0], [0], [0], kind=3)[0][0] == 0  # fewer than q bases
    with pytest.raises(ValueError):
        ix.filter_pairs(rs, pr, pg, pd, pe, kind=5)


@pytest.mark.parametrize("kind", [0, 1, 2, 3, 4])
def test_classification_uses_the_chosen_filter(kind):
    """Classification with a filter kind: the candidates are those of the
    obstacle run, and each one's value is that filter's value on the pair."""
    rnd = np.random.default_rng(kind)
    gen = synth.make_genomes(rnd, 4, 20_000, 0.5)
    reads, _ = synth.make_reads(rnd, gen, rnd.integers(60, 250, 300), 0.02, 0.01)
    ix = oracle.Index(gen.ascii(), 13, 7)
    base = ix.classify(reads, 2, 3, 0, 6, filter_kind=0)
    res = ix.classify(reads, 2, 3, 0, 6, filter_kind=kind)
    for f in ("cand_offsets", "genome", "diag", "hits", "read_E"):
        assert np.array_equal(res[f], base[f]), f
    co = res["cand_offsets"].astype(np.int64)
    pr = np.repeat(np.arange(reads.n), np.diff(co)).astype(np.uint32)
    ap, ac = ix.filter_pairs(reads, pr, res["genome"], res["diag"], res["read_E"][pr], kind=kind)
    assert np.array_equal(ap, res["approx"]) and np.array_equal(ac, res["accept"])
    assert len(ap) > 200
