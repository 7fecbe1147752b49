"""MI355X (gfx950) seed-count + approximate-edit-distance read classifier.

Python binding of the C ABI (include/metatrinity.h).  The functions here only
marshal arguments: torch provides device memory and streams, and every step of
the classifier runs in the HIP kernels of libmetatrinity.so.  There is no CPU
fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _abi
from ._abi import (MT_E_CEIL_PERMILLE, MT_E_FIXED, MT_E_FLOOR_PERMILLE, MT_FILTER_BASE_COUNT,  # noqa: F401
                   MT_FILTER_HAMMING, MT_FILTER_OBSTACLE, MT_FILTER_QGRAM, MT_FILTER_SHD, MT_MODE_FUSED, MT_MODE_FUSED_GRAPH,
                   MT_MODE_PER_STAGE, MT_OK)

__all__ = ["MTError", "DeviceSeqs", "Index", "Result", "Server", "to_device", "mt_set_timing", "last_timings",
           "memory_stats", "use_torch_allocator",
           "tune_info", "tune_set", "tune_reset", "tune_save", "tune_load", "select_genomes"]


class MTError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


def _check(rc: int, lib) -> None:
    if rc != MT_OK:
        raise MTError(rc, lib.mt_last_error().decode())


def _torch():
    import torch
    return torch


def _stream_ptr(stream) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


@dataclass
class DeviceSeqs:
    """A sequence set in device memory: ASCII bytes + n+1 offsets (torch tensors)."""
    seq: object       # torch.uint8 cuda tensor
    offsets: object   # torch.int64 cuda tensor (bit-identical to uint64 offsets)
    n: int
    total: int

    def abi(self) -> _abi.mt_seqs:
        return _abi.mt_seqs(self.seq.data_ptr(), self.offsets.data_ptr(), self.n, self.total)


def to_device(seqset, device="cuda") -> DeviceSeqs:
    """Copies a host sequence set (.seq uint8 ASCII, .offsets n+1) to the GPU."""
    torch = _torch()
    seq = np.ascontiguousarray(seqset.seq, dtype=np.uint8)
    offs = np.ascontiguousarray(seqset.offsets, dtype=np.uint64).view(np.int64)
    ts = torch.from_numpy(seq if len(seq) else np.zeros(1, np.uint8)).to(device)
    to = torch.from_numpy(offs).to(device)
    return DeviceSeqs(ts, to, int(len(offs) - 1), int(offs[-1]) if len(offs) else 0)


def _host_array(ptr: int, n: int, dtype) -> np.ndarray:
    """Copy of n elements at a host pointer owned by the library."""
    out = np.empty(n, dtype=dtype)
    if n:
        C.memmove(out.ctypes.data, ptr, out.nbytes)
    return out


_graph_streams = {}


def _graph_stream():
    """A torch stream per device for the graph form when the caller is on the null stream."""
    torch = _torch()
    dev = torch.cuda.current_device()
    if dev not in _graph_streams:
        _graph_streams[dev] = torch.cuda.Stream(device=dev)
    return _graph_streams[dev]


def _copy_to_host(ptr: int, n: int, dtype) -> np.ndarray:
    """Device -> host copy of n elements at a device pointer (HIP runtime memcpy)."""
    out = np.empty(n, dtype=dtype)
    if n:
        _check_hip(_hip().hipMemcpy(out.ctypes.data_as(C.c_void_p), C.c_void_p(ptr), C.c_size_t(out.nbytes), 2))
    return out


_hiprt = None


def _hip():
    global _hiprt
    if _hiprt is None:
        _hiprt = C.CDLL("libamdhip64.so")
        _hiprt.hipMemcpy.restype = C.c_int
        _hiprt.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    return _hiprt


def _check_hip(rc: int) -> None:
    if rc != 0:
        raise MTError(_abi.MT_EDEVICE, f"hipMemcpy failed with {rc}")


def mt_set_timing(enabled: bool) -> None:
    lib = _abi.load()
    _check(lib.mt_set_timing(1 if enabled else 0), lib)


def memory_stats() -> dict:
    """The library's allocation counters (mt_memory_stats): hipMalloc calls of its
    own pool, allocations through the installed hook (torch's allocator by
    default), live and cached device bytes, and whether a hook is installed."""
    lib = _abi.load()
    st = _abi.mt_mem_stats()
    _check(lib.mt_memory_stats(C.byref(st)), lib)
    return {f: getattr(st, f) for f, _ in st._fields_ if f != "reserved"}


def use_torch_allocator(on: bool = True) -> bool:
    """Device memory of the library from torch's caching allocator (on, the
    default) or from the library's own pool (off)."""
    _abi.load()
    return _abi.use_torch_allocator(on)


def last_stats() -> dict:
    """Work counts of the last classification on this thread."""
    lib = _abi.load()
    st = _abi.mt_stats()
    _check(lib.mt_last_stats(C.byref(st)), lib)
    return {f: getattr(st, f) for f, _ in st._fields_}


def last_timings() -> list[tuple[str, float]]:
    """(stage, ms) of the last classification on this thread (timing enabled)."""
    lib = _abi.load()
    cap = 64
    names = (C.c_char_p * cap)()
    ms = (C.c_float * cap)()
    n = C.c_uint32()
    _check(lib.mt_last_timings(names, ms, cap, C.byref(n)), lib)
    return [(names[i].decode(), float(ms[i])) for i in range(n.value)]


def select_genomes(hits, cutoff_num: int = 1, cutoff_den: int = 10_000, stream=None):
    """Subset database (mt_select_genomes): the genomes whose seed-hit count over
    the largest exceeds cutoff_num / cutoff_den.  hits: device int64 tensor of
    uint64 counts.  Returns (kept genome indices as a device int32 tensor,
    ascending; the largest count)."""
    torch = _torch()
    lib = _abi.load()
    n = int(hits.numel())
    sel = torch.empty(max(n, 1), dtype=torch.int32, device=hits.device if n else "cuda")
    ns, mx = C.c_uint64(), C.c_uint64()
    _check(lib.mt_select_genomes(hits.data_ptr() if n else None, n, cutoff_num, cutoff_den, sel.data_ptr(),
                                 C.byref(ns), C.byref(mx), _stream_ptr(stream)), lib)
    return sel[:ns.value], int(mx.value)


def tune_info() -> list[dict]:
    """State of every filter bucket: name, variants, the one in use, last autotune times."""
    lib = _abi.load()
    n = C.c_uint32()
    _check(lib.mt_tune_buckets(C.byref(n)), lib)
    out = []
    for b in range(n.value):
        tb = _abi.mt_tune_bucket()
        _check(lib.mt_tune_info(b, C.byref(tb)), lib)
        names = [tb.variant_names[v].decode() for v in range(tb.n_variants)]
        out.append(dict(bucket=b, name=tb.name.decode(), variants=names, current=names[tb.current],
                        ms={names[v]: float(tb.ms[v]) for v in range(tb.n_variants) if tb.ms[v] > 0},
                        pairs=int(tb.pairs)))
    return out


def tune_set(bucket: int, variant: int) -> None:
    lib = _abi.load()
    _check(lib.mt_tune_set(bucket, variant), lib)


def tune_reset() -> None:
    lib = _abi.load()
    _check(lib.mt_tune_reset(), lib)


def tune_save(path: str) -> None:
    lib = _abi.load()
    _check(lib.mt_tune_save(path.encode()), lib)


def tune_load(path: str) -> None:
    lib = _abi.load()
    _check(lib.mt_tune_load(path.encode()), lib)


class Result:
    """Owns an mt_result; arrays are device pointers until to_host()."""

    def __init__(self, handle: int, lib):
        self.h = handle
        self.lib = lib

    def _reads(self):
        n = C.c_uint64()
        co, ra, re = C.c_void_p(), C.c_void_p(), C.c_void_p()
        _check(self.lib.mt_result_reads(self.h, C.byref(n), C.byref(co), C.byref(ra), C.byref(re)), self.lib)
        return n.value, co.value, ra.value, re.value

    def _cands(self):
        n = C.c_uint64()
        ps = [C.c_void_p() for _ in range(5)]
        _check(self.lib.mt_result_cands(self.h, C.byref(n), *[C.byref(p) for p in ps]), self.lib)
        return n.value, [p.value for p in ps]

    def _taxa(self):
        n = C.c_uint32()
        ps = [C.c_void_p() for _ in range(3)]
        _check(self.lib.mt_result_taxa(self.h, C.byref(n), *[C.byref(p) for p in ps]), self.lib)
        return n.value, [p.value for p in ps]

    @property
    def n_cands(self) -> int:
        return self._cands()[0]

    @property
    def on_host(self) -> bool:
        return bool(self.lib.mt_result_on_host(self.h))

    def times_ns(self) -> tuple[int, int]:
        """(submit, done) steady-clock times of a served request."""
        a, b = C.c_uint64(), C.c_uint64()
        _check(self.lib.mt_result_times(self.h, C.byref(a), C.byref(b)), self.lib)
        return a.value, b.value

    def _strands(self):
        p = C.c_void_p()
        _check(self.lib.mt_result_strands(self.h, C.byref(p)), self.lib)
        return p.value

    def to_host(self) -> dict:
        """Host copies of every output; "strand" is all zeros for a one-strand query."""
        nr, co, ra, re = self._reads()
        nc, (g, d, h, a, ac) = self._cands()
        nt, (u, mu, un) = self._taxa()
        st = self._strands()
        cp = _host_array if self.on_host else _copy_to_host
        return dict(
            cand_offsets=cp(co, nr + 1, np.uint64), read_accepted=cp(ra, nr, np.uint8),
            read_E=cp(re, nr, np.uint16), genome=cp(g, nc, np.uint32), diag=cp(d, nc, np.int64),
            hits=cp(h, nc, np.uint32), approx=cp(a, nc, np.uint16), accept=cp(ac, nc, np.uint8),
            strand=cp(st, nc, np.uint8) if st else np.zeros(nc, np.uint8),
            unique=cp(u, nt, np.uint64), multi=cp(mu, nt, np.uint64), unmapped=int(cp(un, 1, np.uint64)[0]))

    def free(self) -> None:
        if self.h:
            self.lib.mt_result_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Index:
    """Device-resident seed index (mt_index_build)."""

    def __init__(self, genomes, k: int, w: int, max_occ: int = 0, taxon=None, n_taxa=None, stream=None):
        self.lib = _abi.load()
        dg = genomes if isinstance(genomes, DeviceSeqs) else to_device(genomes)
        n = dg.n
        if taxon is None:
            taxon = np.arange(n, dtype=np.uint32)
        self.taxon = np.ascontiguousarray(taxon, dtype=np.uint32)
        n_taxa = int(n_taxa if n_taxa is not None else (int(self.taxon.max()) + 1 if n else 0))
        p = _abi.mt_index_params(k, w, max_occ, 0)
        h = C.c_void_p()
        rc = self.lib.mt_index_build(C.byref(p), C.byref(dg.abi()), self.taxon.ctypes.data_as(C.c_void_p),
                                     n_taxa, _stream_ptr(stream), C.byref(h))
        _check(rc, self.lib)
        self.h = h.value
        self.n_taxa = n_taxa

    def info(self) -> dict:
        inf = _abi.mt_index_info()
        _check(self.lib.mt_index_get_info(self.h, C.byref(inf)), self.lib)
        return {f: getattr(inf, f) for f, _ in inf._fields_}

    def containment(self, reads: DeviceSeqs, stream=None):
        """Stage 1: seed hits of every genome over the read set (mt_containment);
        a device int64 tensor holding the uint64 counts."""
        torch = _torch()
        n = int(self.info()["n_genomes"])
        hits = torch.empty(max(n, 1), dtype=torch.int64, device="cuda")
        _check(self.lib.mt_containment(self.h, C.byref(reads.abi()), hits.data_ptr(), _stream_ptr(stream)),
               self.lib)
        return hits[:n]

    def abundance(self, result: "Result", num: int = 1, den: int = 10_000, stream=None):
        """Stage 3b (mt_abundance): (counts in units of 2^-32 read as a device int64
        tensor holding uint64, abundances as a device float64 tensor, kept taxa)."""
        torch = _torch()
        n = self.n_taxa
        counts = torch.empty(max(n, 1), dtype=torch.int64, device="cuda")
        ab = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
        kept = C.c_uint64()
        _check(self.lib.mt_abundance(self.h, result.h, num, den, counts.data_ptr(), ab.data_ptr(),
                                     C.byref(kept), _stream_ptr(stream)), self.lib)
        return counts[:n], ab[:n], kept.value

    def classify(self, reads: DeviceSeqs, min_hits=3, top_n=3, e_mode=MT_E_FIXED, e_value=7,
                 mode=MT_MODE_PER_STAGE, stream=None, filter_kind=MT_FILTER_OBSTACLE, strands=1) -> Result:
        """mt_classify; strands=2 adds the reverse strand of every genome."""
        q = _abi.mt_query_params(min_hits, top_n, e_mode, e_value, mode, filter_kind, strands)
        h = C.c_void_p()
        sp = _stream_ptr(stream)
        if mode == MT_MODE_FUSED_GRAPH and sp == 0:
            # a graph is captured on a stream of its own, ordered after and before the null stream's work
            torch = _torch()
            cur = torch.cuda.current_stream()
            own = _graph_stream()
            own.wait_stream(cur)
            rc = self.lib.mt_classify(self.h, C.byref(q), C.byref(reads.abi()), int(own.cuda_stream), C.byref(h))
            cur.wait_stream(own)
        else:
            rc = self.lib.mt_classify(self.h, C.byref(q), C.byref(reads.abi()), sp, C.byref(h))
        _check(rc, self.lib)
        return Result(h.value, self.lib)

    def autotune(self, reads: DeviceSeqs, min_hits=3, top_n=3, e_mode=MT_E_FIXED, e_value=7, reps=3,
                 stream=None) -> list[dict]:
        """Times the filter variants of every bucket on these reads' pairs and keeps the fastest."""
        q = _abi.mt_query_params(min_hits, top_n, e_mode, e_value, MT_MODE_PER_STAGE)
        _check(self.lib.mt_autotune(self.h, C.byref(q), C.byref(reads.abi()), reps, _stream_ptr(stream)), self.lib)
        return tune_info()

    def filter_pairs(self, reads: DeviceSeqs, pair_read, pair_genome, pair_diag, pair_E, stream=None,
                     kind: int = 0):
        """Device tensors in (uint32/int32 read and genome, int64 diag, int16/uint16 E); returns
        device tensors (approx int16 holding uint16 bits, accept uint8).  kind: MT_FILTER_OBSTACLE
        (the band walk), MT_FILTER_HAMMING, MT_FILTER_BASE_COUNT, MT_FILTER_QGRAM or MT_FILTER_SHD."""
        torch = _torch()
        n = int(pair_read.numel())
        approx = torch.empty(max(n, 1), dtype=torch.int16, device=pair_read.device)
        accept = torch.empty(max(n, 1), dtype=torch.uint8, device=pair_read.device)
        rc = self.lib.mt_filter_pairs_kind(self.h, C.byref(reads.abi()), pair_read.data_ptr(),
                                           pair_genome.data_ptr(), pair_diag.data_ptr(), pair_E.data_ptr(), n, kind,
                                           approx.data_ptr(), accept.data_ptr(), _stream_ptr(stream))
        _check(rc, self.lib)
        return approx[:n], accept[:n]

    def free(self) -> None:
        if getattr(self, "h", None):
            self.lib.mt_index_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """Continuous-batching request server over an Index (mt_server_*).

    submit() takes HOST reads (a sequence set with .seq / .offsets) and
    returns a request id; wait() returns that request's Result (host arrays),
    or None if it is not finished within the timeout.  Both release the GIL
    inside the library, so several Python threads can submit and wait.
    """

    def __init__(self, index: Index, mem_budget_bytes=0, max_batch_reads=0, n_streams=0, max_queued_requests=0,
                 pinned_arena_bytes=0):
        self.lib = index.lib
        self.index = index  # the index must outlive the server
        p = _abi.mt_server_params(mem_budget_bytes, max_batch_reads, n_streams, max_queued_requests,
                                  pinned_arena_bytes)
        h = C.c_void_p()
        _check(self.lib.mt_server_create(index.h, C.byref(p), C.byref(h)), self.lib)
        self.h = h.value

    def submit(self, seqset, min_hits=3, top_n=3, e_mode=MT_E_FIXED, e_value=7,
               filter_kind=MT_FILTER_OBSTACLE, strands=1) -> int:
        seq = np.ascontiguousarray(seqset.seq, dtype=np.uint8)
        offs = np.ascontiguousarray(seqset.offsets, dtype=np.uint64)
        q = _abi.mt_query_params(min_hits, top_n, e_mode, e_value, MT_MODE_FUSED, filter_kind, strands)
        rid = C.c_uint64()
        rc = self.lib.mt_server_submit(self.h, C.byref(q), seq.ctypes.data if len(seq) else None,
                                       offs.ctypes.data, len(offs) - 1, C.byref(rid))
        _check(rc, self.lib)
        return rid.value

    def wait(self, request_id: int, timeout_s: float | None = None):
        t = -1 if timeout_s is None else int(timeout_s * 1e6)
        h = C.c_void_p()
        rc = self.lib.mt_server_wait(self.h, request_id, t, C.byref(h))
        if rc == _abi.MT_ETIMEDOUT:
            return None
        _check(rc, self.lib)
        return Result(h.value, self.lib)

    def stats(self) -> dict:
        """mt_server_stats: batches, reads, budget-limited admissions, peaks."""
        st = _abi.mt_server_counters()
        _check(self.lib.mt_server_stats(self.h, C.byref(st)), self.lib)
        return {f: getattr(st, f) for f, _ in st._fields_ if f != "reserved"}

    def close(self) -> None:
        if getattr(self, "h", None):
            self.lib.mt_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
