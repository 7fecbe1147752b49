"""Relative abundance (mt_abundance) on the GPU against the oracle, bit for
bit: fixed-point counts, kept taxa and the double abundances, on results of
strain mixtures with many multi-mapped reads, in both LDS and global counter
paths, on both-strand and served results, and at the cutoff's edges.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_02029_amd as mt_
    return mt_


def _strains(seed, n_reads=3000):
    rng = np.random.default_rng(seed)
    gen = synth.make_strain_genomes(rng, 4, 30_000, 4, (0.001, 0.004))
    reads, _ = synth.make_reads(rng, gen, rng.integers(100, 300, n_reads), 0.01, 0.001)
    return gen, reads


def _check(mt, ix, res, ref_res, taxon, n_taxa, num=1, den=10_000):
    c, a, kept = ix.abundance(res, num, den)
    oc, oa, okept = oracle.abundance(ref_res, taxon, n_taxa, num, den)
    gc = c.cpu().numpy().view(np.uint64)
    ga = a.cpu().numpy()
    assert np.array_equal(gc, oc), np.flatnonzero(gc != oc)[:10]
    assert np.array_equal(ga.view(np.uint64), oa.view(np.uint64)), np.flatnonzero(ga != oa)[:10]
    assert kept == okept
    return oc, oa, okept


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("cut", [(1, 10_000), (0, 1), "median", (1, 1)])
def test_strain_mixture_matches_oracle(mt, mode, cut):
    gen, reads = _strains(1)
    taxon = (np.arange(gen.n) // 2).astype(np.uint32)
    n_taxa = int(taxon.max()) + 1
    ga = gen.ascii()
    ix = mt.Index(ga, 15, 8, taxon=taxon, n_taxa=n_taxa)
    res = ix.classify(mt.to_device(reads), min_hits=2, top_n=0 if mode == 0 else 4, e_mode=1, e_value=50,
                      mode=mode)
    ref = oracle.Index(ga, 15, 8, taxon=taxon, n_taxa=n_taxa).classify(reads, 2, 0 if mode == 0 else 4, 1, 50)
    if cut == "median":   # a cutoff at the median taxon's share keeps about half the taxa
        oc, _, _ = oracle.abundance(ref, taxon, n_taxa, 0, 1)
        cut = (int(np.median(oc)), int(oc.sum()))
    oc, oa, kept = _check(mt, ix, res, ref, taxon, n_taxa, *cut)
    assert int(ref["multi"].sum()) > 500
    if cut[0] > 1:
        assert 0 < kept < n_taxa


def test_many_taxa_global_counters(mt):
    gen, reads = _strains(2, 2000)
    rng = np.random.default_rng(3)
    n_taxa = 6000                          # above the per-block LDS counters
    taxon = rng.choice(n_taxa, gen.n, replace=False).astype(np.uint32)
    taxon[1] = taxon[0]                    # two strains share a taxon
    ga = gen.ascii()
    ix = mt.Index(ga, 15, 8, taxon=taxon, n_taxa=n_taxa)
    res = ix.classify(mt.to_device(reads), min_hits=2, top_n=3, e_mode=1, e_value=50, mode=1)
    ref = oracle.Index(ga, 15, 8, taxon=taxon, n_taxa=n_taxa).classify(reads, 2, 3, 1, 50)
    _check(mt, ix, res, ref, taxon, n_taxa)


def test_both_strands_and_served_results(mt):
    gen, reads = _strains(4, 1500)
    reads = synth.from_reverse_strand(np.random.default_rng(5), reads, 0.5)
    taxon = (np.arange(gen.n) // 4).astype(np.uint32)
    n_taxa = int(taxon.max()) + 1
    ga = gen.ascii()
    ix = mt.Index(ga, 15, 8, taxon=taxon, n_taxa=n_taxa)
    oix = oracle.Index(ga, 15, 8, taxon=taxon, n_taxa=n_taxa)
    res = ix.classify(mt.to_device(reads), min_hits=2, top_n=3, e_mode=1, e_value=50, mode=1, strands=2)
    _check(mt, ix, res, oix.classify(reads, 2, 3, 1, 50, strands=2), taxon, n_taxa)
    with mt.Server(ix) as sv:
        rid = sv.submit(reads, min_hits=2, top_n=3, e_mode=1, e_value=50)
        served = sv.wait(rid)
    assert served.on_host
    _check(mt, ix, served, oix.classify(reads, 2, 3, 1, 50), taxon, n_taxa)


def test_empty_and_errors(mt):
    gen, _, p = synth.workload_small(0)
    ga = gen.ascii()
    ix = mt.Index(ga, p["k"], p["w"])
    res = ix.classify(mt.to_device(synth.SeqSet.from_list([])))
    c, a, kept = ix.abundance(res)
    assert kept == 0 and not c.cpu().numpy().any() and not a.cpu().numpy().any()
    res = ix.classify(mt.to_device(synth.SeqSet.from_list(["ACGT" * 30])))   # unmapped
    c, a, kept = ix.abundance(res)
    assert kept == 0 and not a.cpu().numpy().any()
    with pytest.raises(mt.MTError):
        ix.abundance(res, 1, 0)
    other = mt.Index(ga, p["k"], p["w"], taxon=np.zeros(ga.n, np.uint32), n_taxa=1)
    with pytest.raises(mt.MTError):
        other.abundance(res)
