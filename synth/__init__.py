"""Seeded synthetic genomes, reads and request traces.

Input generation only: this module holds none of the classifier's arithmetic
(no encoding, hashing, minimizer, seed, candidate or filter logic).  Both the
CPU oracle's tests and the GPU path's tests and benchmarks draw their inputs
from here, so the two sides see byte-identical ASCII sequences.

The shapes follow the paper's workloads: short fixed-length Illumina-like
reads (150 bp CAMI sets, 100 bp TARA; Evaluation Methodology of the containment
search and read-mapping sections) against a bacterial-genome-sized database.
None of those datasets is reproduced; every base is drawn from numpy's PCG64
generator with a fixed seed.

Error model of a read (all events are per emitted read base):
  insertion   p_indel/2  a uniform random base is emitted, reference not advanced
  deletion    p_indel/2  one reference base is skipped, nothing emitted
  substitution p_sub     one of the three other bases is emitted
  otherwise              the reference base is copied
The read's start is uniform over the positions where the consumed reference
span fits inside the genome.  Forward strand only.
"""
from __future__ import annotations

import dataclasses
import numpy as np

ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)


@dataclasses.dataclass
class SeqSet:
    """Concatenated ASCII sequences with CSR offsets (offsets[n] == len(seq))."""
    seq: np.ndarray       # uint8 ASCII
    offsets: np.ndarray   # uint64, n+1

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets.astype(np.int64))

    def get(self, i: int) -> bytes:
        return self.seq[int(self.offsets[i]):int(self.offsets[i + 1])].tobytes()

    def subset(self, idx) -> "SeqSet":
        idx = np.asarray(idx, dtype=np.int64)
        lens = self.lengths()[idx]
        offs = np.zeros(len(idx) + 1, dtype=np.uint64)
        np.cumsum(lens, out=offs[1:])
        parts = [self.seq[int(self.offsets[i]):int(self.offsets[i + 1])] for i in idx]
        seq = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
        return SeqSet(seq=np.ascontiguousarray(seq, dtype=np.uint8), offsets=offs)

    @staticmethod
    def from_list(items) -> "SeqSet":
        bs = [s.encode() if isinstance(s, str) else bytes(s) for s in items]
        offs = np.zeros(len(bs) + 1, dtype=np.uint64)
        np.cumsum([len(b) for b in bs], out=offs[1:])
        seq = np.frombuffer(b"".join(bs), dtype=np.uint8).copy()
        return SeqSet(seq=seq, offsets=offs)

    @staticmethod
    def concat(sets) -> "SeqSet":
        seq = np.concatenate([s.seq for s in sets])
        lens = np.concatenate([s.lengths() for s in sets])
        offs = np.zeros(len(lens) + 1, dtype=np.uint64)
        np.cumsum(lens, out=offs[1:])
        return SeqSet(seq=seq, offsets=offs)


def random_codes(rng: np.random.Generator, length: int, gc: float = 0.5) -> np.ndarray:
    """i.i.d. bases as codes 0..3 (A,C,G,T) with P(C)=P(G)=gc/2, P(A)=P(T)=(1-gc)/2."""
    out = np.empty(length, dtype=np.uint8)
    a = (1.0 - gc) / 2.0
    t1, t2, t3 = a, a + gc / 2.0, a + gc
    chunk = 1 << 24
    for s in range(0, length, chunk):
        u = rng.random(min(chunk, length - s), dtype=np.float32)
        out[s:s + len(u)] = (u >= t1).astype(np.uint8) + (u >= t2) + (u >= t3)
    return out


def substitute(rng: np.random.Generator, codes: np.ndarray, p: float) -> np.ndarray:
    """Copy of `codes` with each base replaced, with probability p, by one of the other three."""
    out = codes.copy()
    hit = np.flatnonzero(rng.random(len(codes), dtype=np.float32) < p)
    out[hit] = (out[hit] + rng.integers(1, 4, size=len(hit), dtype=np.uint8)) % 4
    return out


@dataclasses.dataclass
class Genomes:
    codes: np.ndarray        # uint8 codes 0..3 of all genomes, concatenated
    offsets: np.ndarray      # uint64, n+1
    taxon: np.ndarray        # uint32 taxon of each genome
    n_taxa: int

    def ascii(self) -> SeqSet:
        return SeqSet(seq=ACGT[self.codes], offsets=self.offsets.copy())

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)


def make_genomes(rng, n: int, length: int, gc=0.5) -> Genomes:
    """n genomes of `length` bases.  gc: a float, or a (lo, hi) range drawn per genome."""
    parts = []
    for _ in range(n):
        g = rng.uniform(gc[0], gc[1]) if isinstance(gc, tuple) else gc
        parts.append(random_codes(rng, length, g))
    offs = np.arange(n + 1, dtype=np.uint64) * np.uint64(length)
    return Genomes(codes=np.concatenate(parts), offsets=offs,
                   taxon=np.arange(n, dtype=np.uint32), n_taxa=n)


def make_strain_genomes(rng, n_roots: int, root_len: int, strains: int,
                        p_div=(0.01, 0.05), gc=0.5) -> Genomes:
    """n_roots random roots, each with `strains` substitution-only strains
    (divergence p drawn per strain from U(p_div)).  Taxon = strain."""
    parts = []
    for _ in range(n_roots):
        root = random_codes(rng, root_len, gc)
        for _ in range(strains):
            parts.append(substitute(rng, root, rng.uniform(*p_div)))
    n = n_roots * strains
    offs = np.arange(n + 1, dtype=np.uint64) * np.uint64(root_len)
    return Genomes(codes=np.concatenate(parts), offsets=offs,
                   taxon=np.arange(n, dtype=np.uint32), n_taxa=n)


def _reads_one_length(rng, genomes: Genomes, n: int, m: int, p_sub, p_indel, pad: int):
    """n reads of exactly m bases.  p_sub / p_indel: per-read arrays."""
    p_ins = p_indel / 2.0
    p_del = p_indel / 2.0
    gl = np.diff(genomes.offsets.astype(np.int64))
    goff = genomes.offsets[:-1].astype(np.int64)
    out = np.empty((n, m), dtype=np.uint8)
    origin = np.empty((n, 2), dtype=np.int64)
    if m == 0:
        origin[:, 0] = rng.integers(0, genomes.n, size=n)
        origin[:, 1] = 0
        return out, origin
    done = np.zeros(n, dtype=bool)
    while not done.all():
        rows = np.flatnonzero(~done)
        S = m + pad
        u = rng.random((len(rows), S))
        pi = p_ins[rows, None]
        pd = pi + p_del[rows, None]
        ps = pd + p_sub[rows, None]
        ins = u < pi
        dele = (u >= pi) & (u < pd)
        sub = (u >= pd) & (u < ps)
        emits = ~dele
        cum = np.cumsum(emits, axis=1)
        ok = cum[:, -1] >= m
        last = np.argmax(cum >= m, axis=1)
        refadv = ~ins
        refoff = np.cumsum(refadv, axis=1) - refadv
        consumed = refoff[np.arange(len(rows)), last] + refadv[np.arange(len(rows)), last]
        g = rng.integers(0, genomes.n, size=len(rows))
        room = gl[g] - consumed
        ok &= room >= 0
        start = np.floor(rng.random(len(rows)) * (np.maximum(room, 0) + 1)).astype(np.int64)
        cols = np.arange(S)[None, :]
        keep = emits & (cols <= last[:, None])
        pos = np.clip(goff[g][:, None] + start[:, None] + refoff, 0, len(genomes.codes) - 1)
        base = genomes.codes[pos]
        base = np.where(sub, (base + rng.integers(1, 4, size=base.shape, dtype=np.uint8)) % 4, base)
        base = np.where(ins, rng.integers(0, 4, size=base.shape, dtype=np.uint8), base).astype(np.uint8)
        okr = rows[ok]
        out[okr] = base[ok][keep[ok]].reshape(-1, m)
        origin[okr, 0] = g[ok]
        origin[okr, 1] = start[ok]
        done[okr] = True
    return out, origin


def make_reads(rng, genomes: Genomes, lengths: np.ndarray, p_sub, p_indel,
               chunk: int = 65536):
    """Reads of the given lengths.  p_sub / p_indel: scalars or per-read arrays.
    Returns (SeqSet, origin[n,2] = (genome, start)) — the origin is for sanity
    statistics only."""
    lengths = np.asarray(lengths, dtype=np.int64)
    n = len(lengths)
    p_sub = np.broadcast_to(np.asarray(p_sub, dtype=np.float64), (n,)).copy()
    p_indel = np.broadcast_to(np.asarray(p_indel, dtype=np.float64), (n,)).copy()
    offs = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lengths, out=offs[1:])
    seq = np.empty(int(offs[-1]), dtype=np.uint8)
    origin = np.empty((n, 2), dtype=np.int64)
    for m in np.unique(lengths):
        idx = np.flatnonzero(lengths == m)
        pad = int(8 + m * (4 * float(p_indel[idx].max()) + 0.02))
        step = max(1, min(chunk, (1 << 24) // max(1, int(m) + pad)))
        for s in range(0, len(idx), step):
            sel = idx[s:s + step]
            codes, org = _reads_one_length(rng, genomes, len(sel), int(m),
                                           p_sub[sel], p_indel[sel], pad)
            if np.all(np.diff(sel) == 1):
                seq[int(offs[sel[0]]):int(offs[sel[-1] + 1])] = ACGT[codes].reshape(-1)
            else:
                for j, r in enumerate(sel):
                    seq[int(offs[r]):int(offs[r + 1])] = ACGT[codes[j]]
            origin[sel] = org
    return SeqSet(seq=seq, offsets=offs), origin


def inject_n(rng, s: SeqSet, p: float) -> SeqSet:
    """Copy of s with each base turned into 'N' with probability p."""
    seq = s.seq.copy()
    seq[rng.random(len(seq)) < p] = ord("N")
    return SeqSet(seq=seq, offsets=s.offsets.copy())


def from_reverse_strand(rng, s: SeqSet, frac: float = 0.5) -> SeqSet:
    """Copy of s in which a random `frac` of the reads are replaced by their
    reverse complement, as if sequenced from the other strand of the genome
    (vectorised over the whole set: one gather of the reversed positions and a
    byte lookup for the complement)."""
    flip = rng.random(s.n) < frac
    lens = np.diff(s.offsets.astype(np.int64))
    start = s.offsets[:-1].astype(np.int64)
    idx = np.arange(len(s.seq), dtype=np.int64)
    read_of = np.repeat(np.arange(s.n), lens)
    flipped = flip[read_of] if s.n else np.zeros(0, bool)
    src = idx.copy()
    src[flipped] = (2 * start[read_of[flipped]] + lens[read_of[flipped]] - 1) - idx[flipped]
    table = np.arange(256, dtype=np.uint8)
    for a, b in (b"AT", b"TA", b"CG", b"GC", b"at", b"ta", b"cg", b"gc"):
        table[a] = b
    seq = s.seq[src].copy()
    seq[flipped] = table[seq[flipped]]
    return SeqSet(seq=seq, offsets=s.offsets.copy())


# ---------------------------------------------------------------------------
# The paper-shaped workloads.  Each returns (genomes, reads, params dict).
# ---------------------------------------------------------------------------

def workload_small(n_reads: int = 10_000):
    """10 genomes x 100 kbp (GC 0.5, seed 0); 150 bp reads, 0.5% substitutions,
    0.05% 1-bp indels; k=15, w=10, >=3 seed hits, top 3, E=7."""
    rng = np.random.default_rng(0)
    gen = make_genomes(rng, 10, 100_000, 0.5)
    reads, _ = make_reads(rng, gen, np.full(n_reads, 150), 0.005, 0.0005)
    return gen, reads, dict(k=15, w=10, min_hits=3, top_n=3, E=7)


def workload_batched_db(seed: int = 1, n_genomes: int = 200, length: int = 2_500_000):
    """200 genomes x 2.5 Mbp (500 Mbp), per-genome GC ~ U(0.30, 0.70)."""
    rng = np.random.default_rng(seed)
    return make_genomes(rng, n_genomes, length, (0.30, 0.70))


def workload_batched_reads(gen: Genomes, n_reads: int = 1_000_000, seed: int = 101):
    """150 bp reads, per-read substitution rate ~ U(0.1%, 1%), indel rate ~ U(0.01%, 0.1%)."""
    rng = np.random.default_rng(seed)
    p_sub = rng.uniform(0.001, 0.01, n_reads)
    p_indel = rng.uniform(0.0001, 0.001, n_reads)
    reads, _ = make_reads(rng, gen, np.full(n_reads, 150), p_sub, p_indel)
    return reads


def workload_uneven_reads(gen: Genomes, n_reads: int = 2_000_000, seed: int = 102,
                          long_frac: float = 0.05):
    """95% reads of length U{75..300} with the batched error model, 5% reads of
    length U{1000..10000} at 5% indel-rich error (2% substitutions, 3% indels)."""
    rng = np.random.default_rng(seed)
    is_long = rng.random(n_reads) < long_frac
    lens = np.where(is_long, rng.integers(1000, 10001, n_reads), rng.integers(75, 301, n_reads))
    p_sub = np.where(is_long, 0.02, rng.uniform(0.001, 0.01, n_reads))
    p_indel = np.where(is_long, 0.03, rng.uniform(0.0001, 0.001, n_reads))
    reads, _ = make_reads(rng, gen, lens, p_sub, p_indel)
    return reads


def workload_strains_db(seed: int = 4, n_roots: int = 400, root_len: int = 2_000_000, strains: int = 5):
    """400 random roots x 2 Mbp, 5 substitution-only strains each (1-5% divergence): 4 Gbp."""
    rng = np.random.default_rng(seed)
    return make_strain_genomes(rng, n_roots, root_len, strains)


def workload_strain_reads(gen: Genomes, n_reads: int = 10_000_000, seed: int = 104):
    """150 bp reads at 1% error (0.9% substitutions, 0.1% indels) from the strain database."""
    rng = np.random.default_rng(seed)
    reads, _ = make_reads(rng, gen, np.full(n_reads, 150), 0.009, 0.001)
    return reads


def request_trace(seed: int, n_requests: int, qps: float, max_reads: int = 50_000,
                  len_range=(100, 250), lengths=None):
    """Poisson arrivals at `qps`; each request has U{1..max_reads} reads of one
    length drawn from U{len_range} (or uniformly from `lengths` when given).
    Returns a list of (arrival_s, n_reads, length)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, n_requests)
    t = np.cumsum(gaps)
    nr = rng.integers(1, max_reads + 1, n_requests)
    if lengths is None:
        ln = rng.integers(len_range[0], len_range[1] + 1, n_requests)
    else:
        ln = rng.choice(np.asarray(lengths, dtype=np.int64), n_requests)
    return [(float(a), int(b), int(c)) for a, b, c in zip(t, nr, ln)]


SERVED_LENGTHS = tuple(int(v) for v in np.linspace(100, 250, 16).round())


def served_read_pool(gen: Genomes, n_per_length: int = 50_000, lengths=SERVED_LENGTHS, seed: int = 3,
                     p_sub: float = 0.0045, p_indel: float = 0.0005) -> dict:
    """Per read length, n_per_length reads at 0.5% error (0.45% substitutions,
    0.05% indels).  A served request of n reads of length m takes the first n
    reads of pool[m] (request_reads), so a long trace needs no more generation."""
    rng = np.random.default_rng(seed)
    return {m: make_reads(rng, gen, np.full(n_per_length, m), p_sub, p_indel)[0] for m in lengths}


def request_reads(pool: dict, n: int, m: int) -> SeqSet:
    """The first n reads of pool[m] (views, no copy)."""
    s = pool[m]
    return SeqSet(seq=s.seq[:n * m], offsets=s.offsets[:n + 1])
