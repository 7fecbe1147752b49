"""CPU oracle for the seed-count + approximate-edit-distance classifier.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product path (the HIP library and
its Python binding) never imports, links or runs anything from here, and this
package imports nothing from the product.

The arithmetic lives in plain C (`oracle.c`, compiled with gcc); this module
only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(out: str = _SO, extra_flags=()) -> str:
    """Compiles oracle.c with gcc into a shared library."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", *extra_flags, "-o", out, _SRC, "-lm"]
    subprocess.check_call(cmd)
    return out


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def _declare(lib):
    u8p, u16p, u32p, u64p, i64p = (C.POINTER(C.c_uint8), C.POINTER(C.c_uint16), C.POINTER(C.c_uint32),
                                   C.POINTER(C.c_uint64), C.POINTER(C.c_int64))
    lib.or_mix64.restype = C.c_uint64
    lib.or_mix64.argtypes = [C.c_uint64]
    lib.or_minimizers.restype = C.c_int64
    lib.or_minimizers.argtypes = [u8p, C.c_int64, C.c_int, C.c_int, i64p, u64p]
    lib.or_index_build.restype = C.c_void_p
    lib.or_index_build.argtypes = [u8p, u64p, C.c_uint64, C.c_int, C.c_int, C.c_uint32, u32p, C.c_uint32]
    lib.or_index_free.restype = None
    lib.or_index_free.argtypes = [C.c_void_p]
    lib.or_index_n_occ.restype = C.c_int64
    lib.or_index_n_occ.argtypes = [C.c_void_p]
    lib.or_index_copy_occ.restype = None
    lib.or_index_copy_occ.argtypes = [C.c_void_p, u64p, u32p, u32p]
    lib.or_set_threads.restype = C.c_int
    lib.or_set_threads.argtypes = [C.c_int]
    lib.or_approx.restype = C.c_int
    lib.or_approx.argtypes = [u8p, C.c_int64, u8p, C.c_int64, C.c_int64, C.c_int]
    lib.or_read_E.restype = C.c_int
    lib.or_read_E.argtypes = [C.c_int64, C.c_uint32, C.c_uint32]
    lib.or_classify_kind.restype = C.c_void_p
    lib.or_classify_kind.argtypes = [C.c_void_p, u8p, u64p, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                     C.c_uint32, C.c_uint32]
    lib.or_classify_strands.restype = C.c_void_p
    lib.or_classify_strands.argtypes = [C.c_void_p, u8p, u64p, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                        C.c_uint32, C.c_uint32, C.c_uint32]
    lib.or_result_strand.restype = None
    lib.or_result_strand.argtypes = [C.c_void_p, u8p]
    lib.or_classify.restype = C.c_void_p
    lib.or_classify.argtypes = [C.c_void_p, u8p, u64p, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                C.c_uint32]
    lib.or_result_n_cands.restype = C.c_uint64
    lib.or_result_n_cands.argtypes = [C.c_void_p]
    lib.or_result_copy.restype = None
    lib.or_result_copy.argtypes = [C.c_void_p, u64p, u8p, u16p, u32p, i64p, u32p, u16p, u8p, u64p, u64p, u64p]
    lib.or_result_free.restype = None
    lib.or_result_free.argtypes = [C.c_void_p]
    lib.or_filter_pairs.restype = C.c_int
    lib.or_filter_pairs.argtypes = [C.c_void_p, u8p, u64p, C.c_uint64, u32p, u32p, i64p, u16p, C.c_uint64,
                                    u16p, u8p]
    lib.or_filter_pairs_kind.restype = C.c_int
    lib.or_filter_pairs_kind.argtypes = [C.c_void_p, u8p, u64p, C.c_uint64, u32p, u32p, i64p, u16p, C.c_uint64,
                                         C.c_uint32, u16p, u8p]
    lib.or_containment.restype = C.c_int
    lib.or_containment.argtypes = [C.c_void_p, u8p, u64p, C.c_uint64, u64p]
    lib.or_abundance.restype = C.c_int64
    lib.or_abundance.argtypes = [C.c_uint64, u64p, u32p, u16p, u8p, u32p, C.c_uint32, C.c_uint64, C.c_uint64,
                                 u64p, C.POINTER(C.c_double)]
    lib.or_select_genomes.restype = C.c_int64
    lib.or_select_genomes.argtypes = [u64p, C.c_uint64, C.c_uint64, C.c_uint64, u32p, u64p]
    return lib


def load(path: str | None = None):
    """Loads the compiled oracle (building it first if it is not there).

    ORACLE_LIB in the environment names another build of oracle.c to load
    instead: the mutation tests point it at copies with a planted mistake."""
    global _lib
    if path is not None:
        return _declare(C.CDLL(path))
    if _lib is None and os.environ.get("ORACLE_LIB"):
        _lib = _declare(C.CDLL(os.environ["ORACLE_LIB"]))
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        _lib = _declare(C.CDLL(_SO))
    return _lib


def _u8(b) -> np.ndarray:
    if isinstance(b, str):
        b = b.encode()
    if isinstance(b, (bytes, bytearray)):
        return np.frombuffer(bytes(b) + b"\0", dtype=np.uint8)[:len(b)].copy()
    return np.ascontiguousarray(b, dtype=np.uint8)


def mix64(x: int, lib=None) -> int:
    return int((lib or load()).or_mix64(C.c_uint64(x & (2**64 - 1))))


def minimizers(seq, k: int, w: int, lib=None):
    """Selected minimizer positions and their k-mer values (None on a bad byte)."""
    lib = lib or load()
    s = _u8(seq)
    n = max(len(s) - k + 1, 1)
    pos = np.zeros(n, np.int64)
    x = np.zeros(n, np.uint64)
    c = lib.or_minimizers(_p(s, C.c_uint8), len(s), k, w, _p(pos, C.c_int64), _p(x, C.c_uint64))
    if c < 0:
        return None
    return pos[:c].copy(), x[:c].copy()


def approx(q, ref, diag: int, E: int, lib=None) -> int:
    """The filter on one pair: read q against reference ref at diagonal diag."""
    lib = lib or load()
    qa, ra = _u8(q), _u8(ref)
    return int(lib.or_approx(_p(qa, C.c_uint8), len(qa), _p(ra, C.c_uint8), len(ra), int(diag), int(E)))


def set_threads(n: int = 0, lib=None) -> int:
    """Threads the oracle's parallel loops use from now on (0: the default,
    OMP_NUM_THREADS if set, else every processor).  Returns the number in use.
    Results do not depend on it."""
    return int((lib or load()).or_set_threads(int(n)))


def read_E(m: int, e_mode: int, e_value: int, lib=None) -> int:
    return int((lib or load()).or_read_E(m, e_mode, e_value))


class Index:
    """Sorted-array seed index over genomes (ASCII SeqSet-like: .seq, .offsets)."""

    def __init__(self, genomes, k: int, w: int, max_occ: int = 0, taxon=None, n_taxa=None, lib=None):
        self.lib = lib or load()
        self.seq = np.ascontiguousarray(genomes.seq, dtype=np.uint8)
        self.offsets = np.ascontiguousarray(genomes.offsets, dtype=np.uint64)
        n = len(self.offsets) - 1
        self.n_genomes = n
        if taxon is None:
            taxon = np.arange(n, dtype=np.uint32)
        self.taxon = np.ascontiguousarray(taxon, dtype=np.uint32)
        self.n_taxa = int(n_taxa if n_taxa is not None else (int(self.taxon.max()) + 1 if n else 0))
        self.k, self.w, self.max_occ = k, w, max_occ
        h = self.lib.or_index_build(_p(self.seq, C.c_uint8), _p(self.offsets, C.c_uint64), n, k, w, max_occ,
                                    _p(self.taxon, C.c_uint32), self.n_taxa)
        if not h:
            raise ValueError("oracle index build rejected its input")
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.or_index_free(self.h)
            self.h = None

    @property
    def n_occ(self) -> int:
        return int(self.lib.or_index_n_occ(self.h))

    def occurrences(self):
        """The index's occurrence array as (x, genome, pos), in its stored order."""
        n = self.n_occ
        x, g, p = np.zeros(n, np.uint64), np.zeros(n, np.uint32), np.zeros(n, np.uint32)
        self.lib.or_index_copy_occ(self.h, _p(x, C.c_uint64), _p(g, C.c_uint32), _p(p, C.c_uint32))
        return x, g, p

    def classify(self, reads, min_hits=3, top_n=3, e_mode=0, e_value=7, filter_kind=0, strands=1) -> dict:
        """Stage 2 and the step-3a counts; filter_kind 0 is the obstacle walk, 1-4 the
        Hamming, base-counting, q-gram and shifted-Hamming filters; strands 2 adds the
        reverse strand (the result's "strand" holds each candidate's)."""
        seq = np.ascontiguousarray(reads.seq, dtype=np.uint8)
        offs = np.ascontiguousarray(reads.offsets, dtype=np.uint64)
        n = len(offs) - 1
        if strands == 1:
            r = self.lib.or_classify_kind(self.h, _p(seq, C.c_uint8), _p(offs, C.c_uint64), n, min_hits, top_n,
                                          e_mode, e_value, filter_kind)
        else:
            r = self.lib.or_classify_strands(self.h, _p(seq, C.c_uint8), _p(offs, C.c_uint64), n, min_hits,
                                             top_n, e_mode, e_value, filter_kind, strands)
        if not r:
            raise ValueError("oracle classify rejected its input")
        nc = int(self.lib.or_result_n_cands(r))
        out = dict(
            cand_offsets=np.zeros(n + 1, np.uint64), read_accepted=np.zeros(n, np.uint8),
            read_E=np.zeros(n, np.uint16), genome=np.zeros(nc, np.uint32), diag=np.zeros(nc, np.int64),
            hits=np.zeros(nc, np.uint32), approx=np.zeros(nc, np.uint16), accept=np.zeros(nc, np.uint8),
            unique=np.zeros(self.n_taxa, np.uint64), multi=np.zeros(self.n_taxa, np.uint64))
        unm = np.zeros(1, np.uint64)
        self.lib.or_result_copy(r, _p(out["cand_offsets"], C.c_uint64), _p(out["read_accepted"], C.c_uint8),
                                _p(out["read_E"], C.c_uint16), _p(out["genome"], C.c_uint32),
                                _p(out["diag"], C.c_int64), _p(out["hits"], C.c_uint32),
                                _p(out["approx"], C.c_uint16), _p(out["accept"], C.c_uint8),
                                _p(out["unique"], C.c_uint64), _p(out["multi"], C.c_uint64), _p(unm, C.c_uint64))
        out["strand"] = np.zeros(nc, np.uint8)
        self.lib.or_result_strand(r, _p(out["strand"], C.c_uint8))
        self.lib.or_result_free(r)
        out["unmapped"] = int(unm[0])
        return out

    def filter_pairs(self, reads, pair_read, pair_genome, pair_diag, pair_E, kind: int = 0):
        """Filter of kind 0 (obstacle walk), 1 (Hamming) or 2 (base counting) over pairs."""
        seq = np.ascontiguousarray(reads.seq, dtype=np.uint8)
        offs = np.ascontiguousarray(reads.offsets, dtype=np.uint64)
        pr = np.ascontiguousarray(pair_read, dtype=np.uint32)
        pg = np.ascontiguousarray(pair_genome, dtype=np.uint32)
        pd = np.ascontiguousarray(pair_diag, dtype=np.int64)
        pe = np.ascontiguousarray(pair_E, dtype=np.uint16)
        n = len(pr)
        ap = np.zeros(n, np.uint16)
        ac = np.zeros(n, np.uint8)
        rc = self.lib.or_filter_pairs_kind(self.h, _p(seq, C.c_uint8), _p(offs, C.c_uint64), len(offs) - 1,
                                           _p(pr, C.c_uint32), _p(pg, C.c_uint32), _p(pd, C.c_int64),
                                           _p(pe, C.c_uint16), n, kind, _p(ap, C.c_uint16), _p(ac, C.c_uint8))
        if rc != 0:
            raise ValueError("oracle filter_pairs rejected its input")
        return ap, ac

    def containment(self, reads) -> np.ndarray:
        """Stage 1: seed hits of every genome over the read set (uint64 per genome)."""
        seq = np.ascontiguousarray(reads.seq, dtype=np.uint8)
        offs = np.ascontiguousarray(reads.offsets, dtype=np.uint64)
        hits = np.zeros(max(self.n_genomes, 1), np.uint64)
        rc = self.lib.or_containment(self.h, _p(seq, C.c_uint8), _p(offs, C.c_uint64), len(offs) - 1,
                                     _p(hits, C.c_uint64))
        if rc != 0:
            raise ValueError("oracle containment rejected its input")
        return hits[:self.n_genomes]


def select_genomes(hits, num: int = 1, den: int = 10_000, lib=None):
    """Subset database: (kept genome indices ascending, largest seed-hit count)."""
    lib = lib or load()
    h = np.ascontiguousarray(hits, dtype=np.uint64)
    sel = np.zeros(max(len(h), 1), np.uint32)
    mx = np.zeros(1, np.uint64)
    c = lib.or_select_genomes(_p(h, C.c_uint64), len(h), num, den, _p(sel, C.c_uint32), _p(mx, C.c_uint64))
    if c < 0:
        raise ValueError("cutoff denominator must be nonzero")
    return sel[:c].copy(), int(mx[0])


def abundance(res: dict, taxon, n_taxa: int, num: int = 1, den: int = 10_000, lib=None):
    """Stage 3b (reading O16, parity unpinned): per-taxon counts in units of
    2^-32 read, relative abundances and the number of taxa kept at the cutoff,
    from a classification result dict (cand_offsets, genome, approx, accept)."""
    lib = lib or load()
    co = np.ascontiguousarray(res["cand_offsets"], dtype=np.uint64)
    g = np.ascontiguousarray(res["genome"], dtype=np.uint32)
    ap = np.ascontiguousarray(res["approx"], dtype=np.uint16)
    ac = np.ascontiguousarray(res["accept"], dtype=np.uint8)
    tx = np.ascontiguousarray(taxon, dtype=np.uint32)
    counts = np.zeros(max(n_taxa, 1), np.uint64)
    ab = np.zeros(max(n_taxa, 1), np.float64)
    kept = lib.or_abundance(len(co) - 1, _p(co, C.c_uint64), _p(g, C.c_uint32), _p(ap, C.c_uint16),
                            _p(ac, C.c_uint8), _p(tx, C.c_uint32), n_taxa, num, den, _p(counts, C.c_uint64),
                            ab.ctypes.data_as(C.POINTER(C.c_double)))
    if kept < 0:
        raise ValueError("cutoff denominator must be nonzero")
    return counts[:n_taxa], ab[:n_taxa], int(kept)
