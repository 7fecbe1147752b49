"""The oracle's parallel loops change nothing: its index holds exactly the
minimizers of every genome, in (k-mer value, genome, position) order, and
every result is the same on one thread and on all of them.

The index order is checked against Python's own sort of the minimizers that
the one-sequence minimizer function gives per genome (itself pinned by the
second minimizer formulation in test_oracle_pins.py), for k-mers whose values
span many of the bucket pass's top-bit buckets and for a k small enough that
every value is its own bucket.
"""
import numpy as np
import pytest

import oracle
import synth


def _genomes(seed, n, length, gc=(0.3, 0.7)):
    rng = np.random.default_rng(seed)
    g = synth.make_genomes(rng, n, length, gc)
    return g, g.ascii()


@pytest.mark.parametrize("k,w", [(15, 10), (21, 11), (4, 3), (31, 5)])
def test_index_holds_every_minimizer_in_order(k, w):
    _, ga = _genomes(11, 12, 20_000)
    ga = synth.inject_n(np.random.default_rng(5), ga, 0.001)
    ix = oracle.Index(ga, k, w)
    x, g, p = ix.occurrences()
    want = []
    for gi in range(ga.n):
        pos, xs = oracle.minimizers(ga.get(gi), k, w)
        want.extend(zip(xs.tolist(), [gi] * len(pos), pos.tolist()))
    want.sort()
    got = list(zip(x.tolist(), g.tolist(), p.tolist()))
    assert got == want


def _same(a, b):
    assert a.keys() == b.keys()
    for f in a:
        assert np.array_equal(np.asarray(a[f]), np.asarray(b[f])), f


def test_results_do_not_depend_on_thread_count():
    gen, ga = _genomes(3, 6, 50_000)
    rng = np.random.default_rng(9)
    lens = rng.integers(60, 400, 3000)
    reads, _ = synth.make_reads(rng, gen, lens, 0.01, 0.002)
    reads = synth.from_reverse_strand(rng, reads, 0.3)
    reads = synth.inject_n(rng, reads, 0.0005)
    outs = []
    for t in (1, 0, 3):
        oracle.set_threads(t)
        ix = oracle.Index(ga, 15, 10)
        res = {}
        for kind in range(5):
            res[kind] = ix.classify(reads, 2, 0, 1, 50, filter_kind=kind)
        res["both"] = ix.classify(reads, 3, 3, 0, 9, strands=2)
        co = res[0]["cand_offsets"].astype(np.int64)
        pr = np.repeat(np.arange(reads.n), np.diff(co))
        pe = np.asarray(res[0]["read_E"])[pr]
        res["pairs"] = dict(zip(("approx", "accept"),
                                ix.filter_pairs(reads, pr, res[0]["genome"], res[0]["diag"], pe, kind=0)))
        res["contain"] = {"hits": ix.containment(reads)}
        outs.append(res)
    oracle.set_threads(0)
    for other in outs[1:]:
        for key in outs[0]:
            _same(outs[0][key], other[key])
    assert len(outs[0][0]["genome"]) > reads.n // 2 and len(outs[0]["both"]["genome"]) > reads.n


def test_errors_still_reported_with_threads():
    _, ga = _genomes(4, 2, 5_000)
    ix = oracle.Index(ga, 15, 10)
    oracle.set_threads(0)
    bad = synth.SeqSet.from_list(["ACGT" * 40] * 200 + ["ACGTX" * 30] + ["ACGT" * 40] * 200)
    with pytest.raises(ValueError):
        ix.classify(bad)
    with pytest.raises(ValueError):
        ix.containment(bad)
    with pytest.raises(ValueError):
        ix.filter_pairs(bad, [200], [0], [10], [7])
