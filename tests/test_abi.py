"""The C-ABI library loads and exports every function include/*.h declares,
and the binding's struct layouts match the header's (CPU only: no compute)."""
import ctypes as C
import glob
import os
import re
import subprocess

import pytest

from paper_2311_02029_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(mt_[a-z_0-9]+)\s*\(", src))
    return names


def test_library_exports_every_declared_function():
    lib = C.CDLL(_abi.LIB_PATH)
    declared = _declared_functions()
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(_abi.ABI_FUNCTIONS)
    assert _abi.load().mt_abi_version() == 1


def test_struct_layouts_match_header(tmp_path):
    prog = tmp_path / "sizes.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "metatrinity.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(mt_seqs), sizeof(mt_index_params),
         sizeof(mt_query_params), sizeof(mt_index_info), offsetof(mt_query_params, mode),
         offsetof(mt_index_info, k), sizeof(mt_server_params), offsetof(mt_server_params, pinned_arena_bytes),
         sizeof(mt_stats));
  printf("%zu %zu %zu\n", sizeof(mt_tune_bucket), offsetof(mt_tune_bucket, ms), offsetof(mt_tune_bucket, pairs));
  printf("%zu %zu %zu %zu %zu\n", sizeof(mt_mem_stats), offsetof(mt_mem_stats, hooked), sizeof(mt_server_counters),
         offsetof(mt_server_counters, timed_batches), offsetof(mt_server_counters, kernel_ms_overlap));
  return 0;
}''')
    exe = tmp_path / "sizes"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [C.sizeof(_abi.mt_seqs), C.sizeof(_abi.mt_index_params), C.sizeof(_abi.mt_query_params),
            C.sizeof(_abi.mt_index_info), _abi.mt_query_params.mode.offset, _abi.mt_index_info.k.offset,
            C.sizeof(_abi.mt_server_params), _abi.mt_server_params.pinned_arena_bytes.offset,
            C.sizeof(_abi.mt_stats), C.sizeof(_abi.mt_tune_bucket), _abi.mt_tune_bucket.ms.offset,
            _abi.mt_tune_bucket.pairs.offset, C.sizeof(_abi.mt_mem_stats), _abi.mt_mem_stats.hooked.offset,
            C.sizeof(_abi.mt_server_counters), _abi.mt_server_counters.timed_batches.offset,
            _abi.mt_server_counters.kernel_ms_overlap.offset]
    assert got == want


def test_null_arguments_are_errors_not_crashes():
    lib = _abi.load()
    h = C.c_void_p()
    assert lib.mt_index_build(None, None, None, 0, None, C.byref(h)) == _abi.MT_EINVAL
    assert b"null" in lib.mt_last_error()
    assert lib.mt_classify(None, None, None, None, C.byref(h)) == _abi.MT_EINVAL
    assert lib.mt_result_reads(None, None, None, None, None) == _abi.MT_EINVAL
    assert lib.mt_server_create(None, None, C.byref(h)) == _abi.MT_EINVAL
    rid = C.c_uint64()
    assert lib.mt_server_submit(None, None, None, None, 0, C.byref(rid)) == _abi.MT_EINVAL
    assert lib.mt_server_wait(None, 1, 0, C.byref(h)) == _abi.MT_EINVAL
    assert lib.mt_server_destroy(None) == _abi.MT_OK
    assert lib.mt_result_on_host(None) == 0
    assert lib.mt_result_times(None, None, None) == _abi.MT_EINVAL
    n = C.c_uint32()
    assert lib.mt_tune_buckets(C.byref(n)) == _abi.MT_OK and n.value == 8
    tb = _abi.mt_tune_bucket()
    assert lib.mt_tune_info(0, C.byref(tb)) == _abi.MT_OK and tb.name == b"E<=7" and tb.n_variants == 3
    assert lib.mt_tune_info(8, C.byref(tb)) == _abi.MT_EINVAL
    assert lib.mt_tune_set(0, 3) == _abi.MT_EINVAL
    assert lib.mt_tune_set(6, 3) == _abi.MT_EINVAL  # 8 wavefronts x 768 blocks of LDS exceed a workgroup
    assert lib.mt_autotune(None, None, None, 1, None) == _abi.MT_EINVAL
    assert lib.mt_tune_load(None) == _abi.MT_EINVAL
    assert lib.mt_containment(None, None, None, None) == _abi.MT_EINVAL
    ns, mx = C.c_uint64(7), C.c_uint64(7)
    assert lib.mt_select_genomes(None, 0, 1, 0, None, C.byref(ns), C.byref(mx), None) == _abi.MT_EINVAL
    assert b"denominator" in lib.mt_last_error()
    assert lib.mt_select_genomes(None, 5, 1, 10_000, None, C.byref(ns), C.byref(mx), None) == _abi.MT_EINVAL
    # no genomes: nothing to launch, nothing kept
    assert lib.mt_select_genomes(None, 0, 1, 10_000, None, C.byref(ns), C.byref(mx), None) == _abi.MT_OK
    assert ns.value == 0 and mx.value == 0
    assert lib.mt_filter_pairs_kind(None, None, None, None, None, None, 0, 0, None, None, None) == _abi.MT_EINVAL
    st = C.c_void_p()
    assert lib.mt_result_strands(None, C.byref(st)) == _abi.MT_EINVAL
    kept = C.c_uint64()
    assert lib.mt_abundance(None, None, 1, 10_000, None, None, C.byref(kept), None) == _abi.MT_EINVAL
    assert b"null" in lib.mt_last_error()


def test_query_struct_strands_field():
    """strands sits where the first reserved word was: callers that zeroed the
    reserved words ask for the forward strand alone (0 reads as 1)."""
    q = _abi.mt_query_params(3, 3, 0, 7, 0, 0)
    assert q.strands == 0 and q.reserved == 0
    assert _abi.mt_query_params.strands.offset == 24 and C.sizeof(_abi.mt_query_params) == 32
