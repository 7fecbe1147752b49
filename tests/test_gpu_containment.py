"""Containment search (stage 1) and subset selection on the GPU against the
CPU oracle, exactly: per-genome 64-bit seed-hit counts and the kept genomes."""
import random

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


def _case(rnd, n_gen, glen, n_reads, long_reads):
    motif = "".join(rnd.choice("ACGT") for _ in range(rnd.randint(3, 12)))

    def seq(L):
        s = []
        while len(s) < L:
            u = rnd.random()
            s.extend(motif if u < 0.15 else ("N" if u < 0.16 else rnd.choice("ACGT")))
        return "".join(s[:L])

    genomes = [seq(rnd.randint(1, glen)) for _ in range(n_gen)]
    reads = []
    for _ in range(n_reads):
        g = rnd.choice(genomes)
        m = rnd.choice([0, 5, 30, 150, 300] + ([2000, 5000] if long_reads else []))
        st = rnd.randint(0, max(0, len(g) - 1))
        r = list(g[st:st + m])
        for i in range(len(r)):
            if rnd.random() < 0.02:
                r[i] = rnd.choice("ACGTN")
        reads.append("".join(r))
    return genomes, reads


def _both(mt, genomes, reads, k, w, max_occ=0):
    gs, rs = synth.SeqSet.from_list(genomes), synth.SeqSet.from_list(reads)
    ix = mt.Index(gs, k, w, max_occ=max_occ)
    got = ix.containment(mt.to_device(rs)).cpu().numpy().view(np.uint64)
    want = oracle.Index(gs, k, w, max_occ=max_occ).containment(rs)
    return got, want


@pytest.mark.parametrize("seed", range(10))
def test_containment_random_cases(mt, seed):
    """Repeats, N bases, max_occ caps, empty and sub-k reads, both minimizer
    tile sizes (long-read batches average over 512 bases)."""
    rnd = random.Random(700 + seed)
    genomes, reads = _case(rnd, rnd.randint(1, 12), 8000, rnd.randint(0, 300), seed % 2 == 1)
    k, w = rnd.choice([5, 11, 15, 21]), rnd.choice([1, 5, 10, 11, 20])
    got, want = _both(mt, genomes, reads, k, w, max_occ=rnd.choice([0, 0, 3]))
    assert np.array_equal(got, want), (seed, np.flatnonzero(got != want)[:10])


def test_containment_many_genomes_global_counters(mt):
    """More genomes than one block counts in LDS: the counts go to memory
    directly."""
    rnd = np.random.default_rng(5)
    gen = synth.make_genomes(rnd, 5000, 400, 0.5)
    reads, _ = synth.make_reads(rnd, gen, np.full(20_000, 100), 0.01, 0.001)
    ga = gen.ascii()
    genomes = [ga.get(i).decode() for i in range(gen.n)]
    got, want = _both(mt, genomes, [reads.get(i).decode() for i in range(reads.n)], 15, 10)
    assert np.array_equal(got, want)
    assert (want > 0).sum() > 3000


def test_containment_strain_families(mt):
    """Near-identical genomes: most seeds have several occurrences."""
    rnd = np.random.default_rng(8)
    base = synth.random_codes(rnd, 30_000)
    fam = [synth.substitute(rnd, base, 0.01) for _ in range(5)] + [synth.random_codes(rnd, 30_000)]
    genomes = [synth.ACGT[f].tobytes().decode() for f in fam]
    starts = rnd.integers(0, 29_800, 4000)
    src = rnd.integers(0, len(fam), 4000)
    reads = [genomes[g][s:s + 150] for g, s in zip(src, starts)]
    got, want = _both(mt, genomes, reads, 21, 11)
    assert np.array_equal(got, want)
    assert want.min() > 0


def test_select_genomes_exact(mt):
    import torch
    big = (1 << 63) + 12_345
    thr = big // 10_000
    cases = [([10_000, 1, 2, 0, 9_999], 1, 10_000), ([5, 5, 4], 1, 1), ([5, 5, 4], 0, 1), ([0, 0, 0], 1, 10_000),
             ([big, thr, thr + 1, 1 << 62], 1, 10_000), ([7], 1, 10_000)]
    rnd = random.Random(9)
    for _ in range(30):
        n = rnd.randint(1, 3000)
        cases.append(([rnd.getrandbits(rnd.choice([8, 40, 63])) for _ in range(n)], rnd.randint(0, 50),
                      rnd.randint(1, 10 ** rnd.randint(1, 6))))
    for h, num, den in cases:
        arr = np.array(h, dtype=np.uint64)
        sel, mx = mt.select_genomes(torch.from_numpy(arr.view(np.int64)).cuda(), num, den)
        osel, omx = oracle.select_genomes(arr, num, den)
        assert mx == omx and np.array_equal(sel.cpu().numpy().astype(np.uint32), osel), (h[:5], num, den)


def test_containment_invalid_byte_fails_and_index_still_serves(mt):
    """A read with a byte outside ACGTN (among short, long and empty reads) makes
    the call fail with MT_EINVAL; the same index then counts a clean batch
    exactly like the oracle."""
    rnd = random.Random(5)
    genomes, reads = _case(rnd, 4, 3000, 400, 20)
    ix = mt.Index(synth.SeqSet.from_list(genomes), 15, 10)
    bad = list(reads)
    i = next(i for i in range(137, len(reads)) if 30 <= len(reads[i]) <= 256)  # a read the fused kernel takes
    bad[i] = bad[i][:20] + "*" + bad[i][21:]
    with pytest.raises(mt.MTError) as e:
        ix.containment(mt.to_device(synth.SeqSet.from_list(bad)))
    assert e.value.status == -1
    got = ix.containment(mt.to_device(synth.SeqSet.from_list(reads))).cpu().numpy().view(np.uint64)
    want = oracle.Index(synth.SeqSet.from_list(genomes), 15, 10).containment(synth.SeqSet.from_list(reads))
    assert np.array_equal(got, want)
