"""Pins of the oracle's relative-abundance step (stage 3b).  The paper takes
the apportionment of multi-mapped reads from Metalign and does not state it,
so the rule itself is parity unpinned; what is pinned here is what the
reading fixes by arithmetic:

* closed forms: a set of unique reads gives counts 2^32 * u_t and abundances
  u_t / sum(u); a read on two taxa with unique counts 3 : 1 splits 3/4 : 1/4
  exactly; with no unique evidence a read splits into equal floors;
* only accepted candidates at the read's best value count, unmapped reads
  count nothing, and no read at all gives zeros;
* the cutoff at its exact boundary (a taxon at 1/10^4 of the total is kept,
  one unit below is dropped) and the renormalisation over kept taxa;
* invariants on real classifications with multi-mapped reads: each taxon's
  count lies between its unique reads and its unique plus multi-mapped reads,
  the total loses at most one unit per (multi-mapped read, taxon) to the
  floors, kept abundances sum to one, and relabelling taxa permutes the
  outputs.
"""
import numpy as np
import pytest

import oracle
import synth

ONE = 1 << 32


def _res(reads):
    """Result dict from per-read candidate lists [(genome, approx, accept), ...]."""
    co, g, ap, ac = [0], [], [], []
    for cands in reads:
        for genome, approx, acc in cands:
            g.append(genome)
            ap.append(approx)
            ac.append(acc)
        co.append(len(g))
    return dict(cand_offsets=np.array(co, np.uint64), genome=np.array(g, np.uint32),
                approx=np.array(ap, np.uint16), accept=np.array(ac, np.uint8))


def test_unique_reads_closed_form():
    reads = [[(0, 0, 1)]] * 5 + [[(1, 2, 1)]] * 3 + [[(2, 1, 1), (2, 3, 1)]] * 2
    c, a, kept = oracle.abundance(_res(reads), np.arange(3), 3)
    assert c.tolist() == [5 * ONE, 3 * ONE, 2 * ONE] and kept == 3
    assert a.tolist() == [0.5, 0.3, 0.2]


def test_proportional_split_three_to_one():
    reads = [[(0, 0, 1)]] * 3 + [[(1, 0, 1)]] + [[(0, 1, 1), (1, 1, 1)]]
    c, a, _ = oracle.abundance(_res(reads), np.arange(2), 2)
    assert c.tolist() == [3 * ONE + 3 * ONE // 4, ONE + ONE // 4]
    assert a.tolist() == [0.75, 0.25]


def test_equal_floors_without_unique_evidence():
    reads = [[(0, 1, 1), (1, 1, 1), (2, 1, 1)]]
    c, a, kept = oracle.abundance(_res(reads), np.arange(3), 3)
    assert c.tolist() == [ONE // 3] * 3 and kept == 3
    assert a.tolist() == [1 / 3] * 3


def test_only_accepted_candidates_at_the_best_value_count():
    reads = [[(0, 0, 1)],                          # unique to taxon 0
             [(1, 2, 1), (0, 1, 1)],               # best value 1: taxon 0 alone -> unique
             [(1, 0, 0), (0, 4, 1)],               # rejected candidate ignored -> unique 0
             [(1, 9, 0)],                          # unmapped
             [],                                   # no candidates
             [(0, 3, 1), (2, 3, 1), (1, 5, 1)]]    # multi over taxa 0 and 2 (u = 3 and 0)
    c, a, _ = oracle.abundance(_res(reads), np.arange(3), 3)
    assert c.tolist() == [3 * ONE + ONE, 0, 0]
    assert a.tolist() == [1.0, 0.0, 0.0]
    # genomes of one taxon are one taxon: the multi read becomes unique
    c, _, _ = oracle.abundance(_res(reads), np.array([0, 1, 0]), 2)
    assert c.tolist() == [4 * ONE, 0]
    c, a, kept = oracle.abundance(_res([[(0, 5, 0)], []]), np.arange(1), 1)
    assert c.tolist() == [0] and a.tolist() == [0.0] and kept == 0


def test_cutoff_boundary_and_renormalisation():
    at = [[(0, 0, 1)]] * 9999 + [[(1, 0, 1)]]       # taxon 1 at exactly 1/10^4 of the total
    c, a, kept = oracle.abundance(_res(at), np.arange(2), 2)
    assert kept == 2 and a[1] == 1 / 10_000
    below = [[(0, 0, 1)]] * 10_000 + [[(1, 0, 1)]]  # below 1/10^4
    c, a, kept = oracle.abundance(_res(below), np.arange(2), 2)
    assert kept == 1 and a.tolist() == [1.0, 0.0] and c[1] == ONE
    c, a, kept = oracle.abundance(_res(below), np.arange(2), 2, num=0, den=1)  # cutoff 0 keeps all
    assert kept == 2 and a[0] == 10_000 / 10_001
    with pytest.raises(ValueError):
        oracle.abundance(_res(below), np.arange(2), 2, num=1, den=0)


@pytest.mark.parametrize("seed", range(3))
def test_invariants_on_classifications_with_multi_mapped_reads(seed):
    rng = np.random.default_rng(seed)
    gen = synth.make_strain_genomes(rng, 3, 20_000, 4, (0.001, 0.004))
    taxon = (np.arange(gen.n) // 2).astype(np.uint32)     # two strains per taxon
    n_taxa = int(taxon.max()) + 1
    reads, _ = synth.make_reads(rng, gen, rng.integers(100, 300, 600), 0.01, 0.001)
    ix = oracle.Index(gen.ascii(), 15, 8, taxon=taxon, n_taxa=n_taxa)
    res = ix.classify(reads, 2, 0, 1, 50)
    c, a, kept = oracle.abundance(res, taxon, n_taxa)
    u, m = res["unique"].astype(object), res["multi"].astype(object)
    n_multi = int(res["read_accepted"].sum()) - int(res["unique"].sum())
    assert n_multi > 50 and (res["multi"] > 0).sum() >= 2
    cc = c.astype(object)
    assert all(u[t] * ONE <= cc[t] <= (u[t] + m[t]) * ONE for t in range(n_taxa))
    total = sum(cc)
    full = int(res["read_accepted"].sum()) * ONE
    assert full - int(res["multi"].sum()) <= total <= full
    keep = [cc[t] * 10_000 >= total for t in range(n_taxa)]
    assert kept == sum(keep) and all((a[t] > 0) == keep[t] for t in range(n_taxa) if cc[t])
    assert abs(a.sum() - 1.0) < 1e-12
    perm = rng.permutation(n_taxa).astype(np.uint32)
    c2, a2, _ = oracle.abundance(res, perm[taxon], n_taxa)
    assert np.array_equal(c2[perm], c) and np.array_equal(a2[perm], a)


def _big_mixture(seed, n_reads=3_000_000, n_taxa=40):
    """A result of n_reads mapped reads in arrays: a third unique to one taxon,
    the rest on two or three taxa at the best value (so the counts carry
    fractional shares), which puts the kept total above 2^53 units."""
    rng = np.random.default_rng(seed)
    k = rng.choice([1, 1, 2, 3], n_reads)
    co = np.zeros(n_reads + 1, np.uint64)
    np.cumsum(k, out=co[1:])
    weights = rng.random(n_taxa) ** 3 + 0.01
    g = rng.choice(n_taxa, int(co[-1]), p=weights / weights.sum()).astype(np.uint32)
    return dict(cand_offsets=co, genome=g, approx=np.zeros(len(g), np.uint16), accept=np.ones(len(g), np.uint8))


def test_abundance_is_the_nearest_double_of_the_exact_ratio():
    """count_t / K is rounded once, to the nearest double, even when K needs
    more than 53 bits: against Python's exact rationals (Fraction to float
    rounds correctly), on a mixture whose kept total is above 2^53 and where
    converting count and K to double before dividing would differ."""
    from fractions import Fraction
    n_taxa = 40
    res = _big_mixture(5, n_taxa=n_taxa)
    c, a, kept = oracle.abundance(res, np.arange(n_taxa), n_taxa)
    total = sum(int(x) for x in c)
    K = sum(int(x) for x in c if int(x) * 10_000 >= total)
    assert K > 2 ** 53 and kept > 0
    want = [float(Fraction(int(x), K)) if int(x) * 10_000 >= total else 0.0 for x in c]
    assert a.tolist() == want
    naive = [float(int(x)) / float(K) if int(x) * 10_000 >= total else 0.0 for x in c]
    assert naive != want  # the double rounding the nearest-double rule avoids happens here
