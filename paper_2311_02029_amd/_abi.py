"""ctypes declarations of the C ABI in include/metatrinity.h (same names).

Argument marshalling only: every step of the classifier runs in the HIP
library.  Loading fails loudly when libmetatrinity.so has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmetatrinity.so")
TORCH_ALLOC_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmt_torch_alloc.so")

MT_OK, MT_EINVAL, MT_ENOMEM, MT_EDEVICE, MT_EAGAIN, MT_ETIMEDOUT, MT_ECANCELED, MT_EINTERNAL = 0, -1, -2, -3, -4, -5, -6, -7
MT_E_FIXED, MT_E_CEIL_PERMILLE, MT_E_FLOOR_PERMILLE = 0, 1, 2
MT_MODE_PER_STAGE, MT_MODE_FUSED, MT_MODE_FUSED_GRAPH = 0, 1, 2
MT_FILTER_OBSTACLE, MT_FILTER_HAMMING, MT_FILTER_BASE_COUNT, MT_FILTER_QGRAM, MT_FILTER_SHD = 0, 1, 2, 3, 4

# Every function the header declares; a test checks the library exports them.
ABI_FUNCTIONS = (
    "mt_index_build", "mt_index_free", "mt_index_get_info", "mt_classify", "mt_result_reads",
    "mt_result_cands", "mt_result_taxa", "mt_result_strands", "mt_result_free", "mt_last_timings", "mt_set_timing",
    "mt_filter_pairs", "mt_trim", "mt_last_error", "mt_abi_version", "mt_last_stats", "mt_server_create",
    "mt_server_submit", "mt_server_wait", "mt_server_destroy", "mt_result_on_host", "mt_result_times",
    "mt_tune_buckets", "mt_tune_info", "mt_tune_set", "mt_tune_reset", "mt_autotune", "mt_tune_save",
    "mt_tune_load", "mt_containment", "mt_select_genomes", "mt_filter_pairs_kind", "mt_abundance",
    "mt_set_allocator", "mt_memory_stats", "mt_server_stats", "mt_select_genomes_noalloc",
)


class mt_seqs(C.Structure):
    _fields_ = [("seq", C.c_void_p), ("offsets", C.c_void_p), ("n", C.c_uint64), ("total", C.c_uint64)]


class mt_index_params(C.Structure):
    _fields_ = [("k", C.c_uint32), ("w", C.c_uint32), ("max_occ", C.c_uint32), ("reserved", C.c_uint32)]


class mt_query_params(C.Structure):
    _fields_ = [("min_hits", C.c_uint32), ("top_n", C.c_uint32), ("e_mode", C.c_uint32), ("e_value", C.c_uint32),
                ("mode", C.c_uint32), ("filter", C.c_uint32), ("strands", C.c_uint32), ("reserved", C.c_uint32)]


class mt_index_info(C.Structure):
    _fields_ = [("n_genomes", C.c_uint64), ("total_bases", C.c_uint64), ("n_minimizers", C.c_uint64),
                ("n_keys", C.c_uint64), ("n_slots", C.c_uint64), ("n_multi_occ", C.c_uint64),
                ("device_bytes", C.c_uint64), ("k", C.c_uint32), ("w", C.c_uint32), ("max_occ", C.c_uint32),
                ("n_taxa", C.c_uint32)]


class mt_stats(C.Structure):
    _fields_ = [(f, C.c_uint64) for f in ("n_reads", "n_minimizers", "n_hits", "n_cands", "fused_reads",
                                          "fused_bases", "fused_minimizers", "fused_window_blocks", "fused_cands",
                                          "fused_occ")]


class mt_mem_stats(C.Structure):
    _fields_ = [("device_mallocs", C.c_uint64), ("hook_allocs", C.c_uint64), ("live_bytes", C.c_uint64),
                ("cached_bytes", C.c_uint64), ("hooked", C.c_uint32), ("reserved", C.c_uint32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class mt_server_params(C.Structure):
    _fields_ = [("mem_budget_bytes", C.c_uint64), ("max_batch_reads", C.c_uint64), ("n_streams", C.c_uint32),
                ("max_queued_requests", C.c_uint32), ("pinned_arena_bytes", C.c_uint64),
                ("reserved", C.c_uint32 * 4)]


class mt_server_counters(C.Structure):
    _fields_ = [("batches", C.c_uint64), ("reads", C.c_uint64), ("budget_limited", C.c_uint64),
                ("peak_inflight_bytes", C.c_uint64), ("mem_budget_bytes", C.c_uint64),
                ("max_batch_reads", C.c_uint64), ("peak_batches", C.c_uint32), ("reserved", C.c_uint32),
                ("timed_batches", C.c_uint64), ("kernel_ms_sum", C.c_double), ("kernel_ms_union", C.c_double),
                ("kernel_ms_overlap", C.c_double)]


class mt_tune_bucket(C.Structure):
    _fields_ = [("name", C.c_char_p), ("n_variants", C.c_uint32), ("current", C.c_uint32),
                ("variant_names", C.c_char_p * 6), ("ms", C.c_float * 6), ("pairs", C.c_uint64)]


_lib = None


def load(path: str = LIB_PATH):
    """Loads the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(the classifier has no CPU fallback)")
    # torch first: the library must bind to the HIP runtime torch loads, or the
    # process ends up with two runtimes and the second sees no device
    import torch  # noqa: F401
    lib = C.CDLL(path)
    vp, u64, u32, i32 = C.c_void_p, C.c_uint64, C.c_uint32, C.c_int
    pp = C.POINTER(C.c_void_p)
    sig = {
        "mt_index_build": (i32, [C.POINTER(mt_index_params), C.POINTER(mt_seqs), vp, u32, vp, pp]),
        "mt_index_free": (i32, [vp]),
        "mt_index_get_info": (i32, [vp, C.POINTER(mt_index_info)]),
        "mt_classify": (i32, [vp, C.POINTER(mt_query_params), C.POINTER(mt_seqs), vp, pp]),
        "mt_result_reads": (i32, [vp, C.POINTER(u64), pp, pp, pp]),
        "mt_result_cands": (i32, [vp, C.POINTER(u64), pp, pp, pp, pp, pp]),
        "mt_result_strands": (i32, [vp, pp]),
        "mt_abundance": (i32, [vp, vp, u64, u64, vp, vp, C.POINTER(u64), vp]),
        "mt_result_taxa": (i32, [vp, C.POINTER(u32), pp, pp, pp]),
        "mt_result_free": (i32, [vp]),
        "mt_last_timings": (i32, [C.POINTER(C.c_char_p), C.POINTER(C.c_float), u32, C.POINTER(u32)]),
        "mt_set_timing": (i32, [i32]),
        "mt_filter_pairs": (i32, [vp, C.POINTER(mt_seqs), vp, vp, vp, vp, u64, vp, vp, vp]),
        "mt_trim": (i32, []),
        "mt_last_error": (C.c_char_p, []),
        "mt_abi_version": (i32, []),
        "mt_last_stats": (i32, [C.POINTER(mt_stats)]),
        "mt_server_create": (i32, [vp, C.POINTER(mt_server_params), pp]),
        "mt_server_submit": (i32, [vp, C.POINTER(mt_query_params), vp, vp, u64, C.POINTER(u64)]),
        "mt_server_wait": (i32, [vp, u64, C.c_int64, pp]),
        "mt_server_destroy": (i32, [vp]),
        "mt_result_on_host": (i32, [vp]),
        "mt_result_times": (i32, [vp, C.POINTER(u64), C.POINTER(u64)]),
        "mt_tune_buckets": (i32, [C.POINTER(u32)]),
        "mt_tune_info": (i32, [u32, C.POINTER(mt_tune_bucket)]),
        "mt_tune_set": (i32, [u32, u32]),
        "mt_tune_reset": (i32, []),
        "mt_autotune": (i32, [vp, C.POINTER(mt_query_params), C.POINTER(mt_seqs), u32, vp]),
        "mt_tune_save": (i32, [C.c_char_p]),
        "mt_tune_load": (i32, [C.c_char_p]),
        "mt_containment": (i32, [vp, C.POINTER(mt_seqs), vp, vp]),
        "mt_filter_pairs_kind": (i32, [vp, C.POINTER(mt_seqs), vp, vp, vp, vp, u64, u32, vp, vp, vp]),
        "mt_select_genomes": (i32, [vp, u64, u64, u64, vp, C.POINTER(u64), C.POINTER(u64), vp]),
        "mt_select_genomes_noalloc": (i32, [vp, u64, u64, u64, vp, C.POINTER(u64), C.POINTER(u64), vp]),
        "mt_set_allocator": (i32, [vp, vp, vp]),
        "mt_memory_stats": (i32, [C.POINTER(mt_mem_stats)]),
        "mt_server_stats": (i32, [vp, C.POINTER(mt_server_counters)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path == LIB_PATH:
        _lib = lib
        if os.environ.get("MT_TORCH_ALLOCATOR", "1") != "0":
            use_torch_allocator(True)
    return lib


_shim = None


def use_torch_allocator(on: bool = True) -> bool:
    """Installs PyTorch's caching allocator as the library's device allocator
    (mt_set_allocator with the shim's two functions), or with on=False goes
    back to the library's own pool.  Needs a GPU (torch's allocator is set up
    by its CUDA initialisation); without one nothing is installed.  Returns
    whether torch's allocator is now in use.  Loading the library installs it
    unless MT_TORCH_ALLOCATOR=0 is set."""
    global _shim
    import torch
    lib = _lib
    if lib is None:
        raise RuntimeError("load() the library first")
    if not on:
        rc = lib.mt_set_allocator(None, None, None)
        if rc != MT_OK:
            raise RuntimeError(lib.mt_last_error().decode())
        return False
    if not torch.cuda.is_available():
        return False
    if not os.path.exists(TORCH_ALLOC_PATH):
        raise RuntimeError(f"{TORCH_ALLOC_PATH} is missing: build it with __graft_entry__.build()")
    torch.cuda.init()
    if _shim is None:
        _shim = C.CDLL(TORCH_ALLOC_PATH)
    alloc = C.cast(_shim.mt_torch_alloc, C.c_void_p)
    free = C.cast(_shim.mt_torch_free, C.c_void_p)
    rc = lib.mt_set_allocator(alloc, free, None)
    if rc != MT_OK:
        raise RuntimeError(lib.mt_last_error().decode())
    return True
