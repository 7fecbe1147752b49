"""Repetitive databases (near-identical strains), where most k-mers occur in
several genomes: the fused kernel's instance for such an index counts the
seed hits of reads whose probes return several occurrences in registers
(when a read has at most 64 hits and no k-mer occurs more than 15 times) and
falls back to the per-read LDS table otherwise.  Every read against the
oracle, in the three forms, at every filter group size (E up to 7, 15, 31)
and with E proportional to the read length.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FIELDS = ("cand_offsets", "read_accepted", "read_E", "genome", "diag", "hits", "approx", "accept", "unique",
          "multi")
MODES = [0, 1, 2]


@pytest.fixture(scope="module")
def mt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_02029_amd as mt_
    return mt_


def _db(strains, seed):
    rng = np.random.default_rng(seed)
    return synth.make_strain_genomes(rng, n_roots=12, root_len=60_000, strains=strains)


@pytest.fixture(scope="module")
def five(mt):
    """12 roots x 5 strains (1-5% divergence) x 60 kbp; 20,000 reads: half of
    150 bp, half of 75-300 bp, at 1% error, a few with N."""
    gen = _db(5, 41)
    rng = np.random.default_rng(42)
    lens = np.where(rng.random(20_000) < 0.5, 150, rng.integers(75, 301, 20_000))
    reads, _ = synth.make_reads(rng, gen, lens, 0.009, 0.001)
    reads = synth.inject_n(rng, reads, 0.0005)
    ga = gen.ascii()
    return dict(ga=ga, reads=reads, ix=mt.Index(ga, 21, 11), oix=oracle.Index(ga, 21, 11))


@pytest.fixture(scope="module")
def many(mt):
    """12 roots x 24 strains at 0.2-1% divergence: k-mers in up to 24 genomes
    and reads with more than 64 hits (the table path of the same instance)."""
    rng = np.random.default_rng(43)
    gen = synth.make_strain_genomes(rng, n_roots=12, root_len=30_000, strains=24, p_div=(0.002, 0.01))
    reads, _ = synth.make_reads(rng, gen, np.full(6_000, 150), 0.009, 0.001)
    ga = gen.ascii()
    return dict(ga=ga, reads=reads, ix=mt.Index(ga, 21, 11), oix=oracle.Index(ga, 21, 11))


def _same(got, ref, ctx):
    for f in FIELDS:
        a, b = np.asarray(got[f]), np.asarray(ref[f])
        assert a.shape == b.shape, (ctx, f, a.shape, b.shape)
        bad = np.flatnonzero(a.astype(b.dtype) != b)
        assert bad.size == 0, (ctx, f, bad[:8])
    assert got["unmapped"] == ref["unmapped"], ctx


def _check(mt, d, mode, **q):
    res = d["ix"].classify(mt.to_device(d["reads"]), mode=mode, **q)
    got = res.to_host()
    res.free()
    ref = d["oix"].classify(d["reads"], q.get("min_hits", 3), q.get("top_n", 3), q.get("e_mode", 0),
                            q.get("e_value", 7))
    _same(got, ref, f"mode {mode} {q}")
    return ref


def test_indexes_are_repetitive(five, many):
    """At least one occurrence in eight belongs to a repeated k-mer: the launch
    takes the kernel instance for repetitive indexes."""
    for d in (five, many):
        info = d["ix"].info()
        assert info["n_multi_occ"] * 8 >= info["n_minimizers"] > 0, info
    x, _, _ = many["oix"].occurrences()
    assert np.unique(x, return_counts=True)[1].max() > 15  # some k-mer occurs in more than 15 genomes


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("E", [0, 7, 15, 31])
def test_strains_every_read_fixed_E(mt, five, mode, E):
    ref = _check(mt, five, mode, min_hits=3, top_n=3, e_value=E)
    assert len(ref["genome"]) > 2 * five["reads"].n


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("top_n", [0, 1])
def test_strains_every_read_proportional_E(mt, five, mode, top_n):
    _check(mt, five, mode, min_hits=3, top_n=top_n, e_mode=1, e_value=50)


@pytest.mark.parametrize("mode", MODES)
def test_many_strains_every_read(mt, many, mode):
    ref = _check(mt, many, mode, min_hits=3, top_n=3, e_value=7)
    hits = np.diff(ref["cand_offsets"].astype(np.int64))
    assert hits.max() == 3 and int(ref["multi"].sum()) > 0


@pytest.mark.parametrize("copies", [15, 16])
@pytest.mark.parametrize("mode", MODES)
def test_occurrence_count_boundary(mt, copies, mode):
    """Identical copies of one genome, so every k-mer occurs exactly `copies`
    times: at 15 a short read's hits (a few probes x 15 <= 64) are counted in
    registers, at 16 every read goes to the per-read table; reads of 30-90 bp
    give hit totals on both sides of 64.  Every read against the oracle."""
    rng = np.random.default_rng(44)
    one = synth.make_genomes(rng, 1, 20_000)
    gen = synth.Genomes(codes=np.tile(one.codes, copies),
                        offsets=np.arange(copies + 1, dtype=np.uint64) * np.uint64(20_000),
                        taxon=np.arange(copies, dtype=np.uint32) % 4, n_taxa=4)
    reads, _ = synth.make_reads(rng, gen, rng.integers(30, 91, 3000), 0.005, 0.0005)
    ga = gen.ascii()
    d = dict(reads=reads, ix=mt.Index(ga, 21, 11, taxon=gen.taxon, n_taxa=gen.n_taxa),
             oix=oracle.Index(ga, 21, 11, taxon=gen.taxon, n_taxa=gen.n_taxa))
    info = d["ix"].info()
    assert info["n_multi_occ"] == info["n_minimizers"] > 0  # every k-mer repeated
    for top_n in (3, 0):
        ref = _check(mt, d, mode, min_hits=2, top_n=top_n, e_value=3)
        assert ref["read_accepted"].mean() > 0.8
