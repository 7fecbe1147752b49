"""Pins of the oracle's containment search (stage 1) and subset selection.

* brute force: every read minimizer against every reference minimizer
  occurrence, from the second (per-position) minimizer formulation, counted per
  genome;
* conservation: a genome's seed-hit count equals the sum of the stage-2 hit
  counts of its locations over all reads (min_hits 1, every location kept);
* selection at the exact boundary of the normalised cutoff (strictly above),
  with 64-bit counts whose products need more than 64 bits, and with no hits.
"""
import random
from collections import Counter

import numpy as np
import pytest

import oracle
import synth
from test_oracle_pins import _minimizers_second_form, _repetitive_case


def _brute_containment(genomes, reads, k, w, max_occ=0):
    occ = {}
    for g, gs in enumerate(genomes):
        for x in _minimizers_second_form(gs, k, w)[1]:
            occ.setdefault(x, []).append(g)
    hits = Counter()
    for rs in reads:
        for x in _minimizers_second_form(rs, k, w)[1]:
            lst = occ.get(x, [])
            if max_occ and len(lst) > max_occ:
                continue
            for g in lst:
                hits[g] += 1
    return [hits[g] for g in range(len(genomes))]


@pytest.mark.parametrize("seed", range(10))
def test_containment_matches_brute_force(seed):
    rnd = random.Random(300 + seed)
    genomes, reads = _repetitive_case(rnd, rnd.randint(1, 5), rnd.randint(20, 150), 50, rnd.randint(3, 7))
    k, w = rnd.randint(2, 6), rnd.randint(1, 5)
    max_occ = rnd.choice([0, 0, 3])
    ix = oracle.Index(synth.SeqSet.from_list(genomes), k, w, max_occ=max_occ)
    got = ix.containment(synth.SeqSet.from_list(reads)).tolist()
    assert got == _brute_containment(genomes, reads, k, w, max_occ)


@pytest.mark.parametrize("seed", range(3))
def test_containment_conserves_stage2_hits(seed):
    rnd = np.random.default_rng(seed)
    gen = synth.make_genomes(rnd, 6, 20_000, (0.3, 0.7))
    reads, _ = synth.make_reads(rnd, gen, rnd.integers(20, 300, 800), 0.01, 0.002)
    reads = synth.inject_n(rnd, reads, 0.002)
    ix = oracle.Index(gen.ascii(), 13, 7, max_occ=0 if seed else 2)
    hits = ix.containment(reads)
    res = ix.classify(reads, min_hits=1, top_n=0, e_mode=0, e_value=0)
    per_genome = np.bincount(res["genome"].astype(np.int64), weights=res["hits"].astype(np.float64),
                             minlength=gen.n)
    assert hits.tolist() == per_genome.astype(np.int64).tolist()
    assert hits.sum() > 0


def test_containment_counts_every_read_and_skips_bad_input():
    genome = "ACGTTGCAAGGCTTACCGATGCAGT" * 4
    ix = oracle.Index(synth.SeqSet.from_list([genome, "TTTTTTTTTT"]), 5, 3)
    one = ix.containment(synth.SeqSet.from_list([genome[10:60]]))
    two = ix.containment(synth.SeqSet.from_list([genome[10:60], genome[10:60]]))
    assert one[0] > 0 and one[1] == 0 and (two == 2 * one).all()
    assert ix.containment(synth.SeqSet.from_list([])).tolist() == [0, 0]
    assert ix.containment(synth.SeqSet.from_list(["NNNNNNNN", "AC"])).tolist() == [0, 0]
    with pytest.raises(ValueError):
        ix.containment(synth.SeqSet.from_list(["ACGTX"]))


def test_selection_is_strictly_above_the_normalised_cutoff():
    sel, mx = oracle.select_genomes([10_000, 1, 2, 0, 9_999], 1, 10_000)
    assert mx == 10_000 and sel.tolist() == [0, 2, 4]  # 1/10000 is not above 1/10000
    sel, mx = oracle.select_genomes([5, 5, 4], 1, 1)  # cutoff 1: nothing is above the maximum
    assert sel.tolist() == [] and mx == 5
    sel, _ = oracle.select_genomes([5, 5, 4], 0, 1)  # cutoff 0: every genome with a hit
    assert sel.tolist() == [0, 1, 2]
    assert oracle.select_genomes([0, 0, 0])[0].tolist() == []
    assert oracle.select_genomes([])[0].tolist() == []
    with pytest.raises(ValueError):
        oracle.select_genomes([1], 1, 0)


def test_selection_products_beyond_64_bits():
    big = (1 << 63) + 12_345
    thr = big // 10_000  # thr * 10000 <= big < (thr + 1) * 10000
    sel, mx = oracle.select_genomes([big, thr, thr + 1, 1 << 62], 1, 10_000)
    assert mx == big and sel.tolist() == [0, 2, 3]
    rnd = random.Random(7)
    for _ in range(200):
        h = [rnd.getrandbits(rnd.choice([8, 40, 64])) for _ in range(rnd.randint(1, 12))]
        num, den = rnd.randint(0, 50), rnd.randint(1, 10 ** rnd.randint(1, 6))
        m = max(h)
        want = [g for g, v in enumerate(h) if v * den > m * num]  # Python integers are exact
        assert oracle.select_genomes(h, num, den)[0].tolist() == want
