"""The seeded input generators: reads taken from the reverse strand are the
reverse complements of forward reads (case kept, N and other bytes kept),
the chosen fraction is flipped, and flipping every read twice gives the input
back."""
import numpy as np

import synth


def _strs(s):
    return [bytes(s.seq[s.offsets[i]:s.offsets[i + 1]]).decode() for i in range(s.n)]


def test_reverse_strand_known_strings():
    s = synth.SeqSet.from_list(["ACGTN", "", "AAC", "gatc", "ACGTX", "aCgT"])
    t = synth.from_reverse_strand(np.random.default_rng(0), s, 1.0)
    assert _strs(t) == ["NACGT", "", "GTT", "gatc", "XACGT", "AcGt"]
    assert np.array_equal(t.offsets, s.offsets)
    assert _strs(synth.from_reverse_strand(np.random.default_rng(0), s, 0.0)) == _strs(s)


def test_reverse_strand_fraction_and_involution():
    rng = np.random.default_rng(3)
    gen = synth.make_genomes(rng, 2, 5000, 0.5)
    reads, _ = synth.make_reads(rng, gen, rng.integers(0, 200, 2000), 0.01, 0.001)
    t = synth.from_reverse_strand(np.random.default_rng(1), reads, 0.5)
    changed = sum(a != b for a, b in zip(_strs(t), _strs(reads)))
    assert 800 < changed < 1200
    twice = synth.from_reverse_strand(np.random.default_rng(1), t, 0.5)  # same reads flipped again
    assert np.array_equal(twice.seq, reads.seq)
