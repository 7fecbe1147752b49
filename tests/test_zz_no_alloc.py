"""mt_select_genomes_noalloc (the allocation-free entry point) through the C
ABI: two calls in a row, the second with fewer genomes, each equal to
mt_select_genomes on the same counts and to the oracle's selection, and no
device allocation by the library during either call (its allocation counters,
which count every block with PyTorch's allocator installed, do not move)."""
import ctypes as C

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _select(lib, fn, hits_dev, n, num, den):
    import torch
    sel = torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda")
    ns, mx = C.c_uint64(), C.c_uint64()
    rc = getattr(lib, fn)(C.c_void_p(hits_dev.data_ptr()), n, num, den, C.c_void_p(sel.data_ptr()), C.byref(ns),
                          C.byref(mx), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, lib.mt_last_error()
    return sel[:ns.value].cpu().numpy().astype(np.uint32), mx.value


def test_noalloc_selection_matches_and_allocates_nothing():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_02029_amd as mt
    from paper_2311_02029_amd import _abi
    lib = _abi.load()
    rng = np.random.default_rng(31)
    # counts spanning the scan's multi-block path (1M genomes) and a small second call;
    # heavy-tailed so that the cutoff splits them, with the maximum near 2^62
    big = (rng.pareto(1.2, 1_000_000) * 1e6).astype(np.uint64)
    big[123_457] = np.uint64(1) << np.uint64(62)
    small = (rng.pareto(1.2, 5_000) * 1e3).astype(np.uint64)
    for counts, num, den in ((big, 1, 10_000), (small, 3, 1_000)):
        n = len(counts)
        dev = torch.from_numpy(counts.view(np.int64)).cuda()
        want, want_mx = _select(lib, "mt_select_genomes", dev, n, num, den)
        torch.cuda.synchronize()
        before = mt.memory_stats()
        got, got_mx = _select(lib, "mt_select_genomes_noalloc", dev, n, num, den)
        after = mt.memory_stats()
        assert after["device_mallocs"] == before["device_mallocs"]
        assert after["hook_allocs"] == before["hook_allocs"]
        assert after["live_bytes"] == before["live_bytes"]
        assert got_mx == want_mx and np.array_equal(got, want)
        osel, omx = oracle.select_genomes(counts, num, den)
        assert omx == got_mx and np.array_equal(got, osel)
        assert 0 < len(got) < n


def test_noalloc_selection_limits():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_02029_amd import _abi
    lib = _abi.load()
    dev = torch.zeros(4, dtype=torch.int64, device="cuda")
    ns, mx = C.c_uint64(), C.c_uint64()
    sel = torch.zeros(4, dtype=torch.int32, device="cuda")
    # more genomes than the scratch holds: refused before any device work
    rc = lib.mt_select_genomes_noalloc(C.c_void_p(dev.data_ptr()), (1 << 20) + 1, 1, 10_000,
                                       C.c_void_p(sel.data_ptr()), C.byref(ns), C.byref(mx), None)
    assert rc == _abi.MT_EINVAL
    rc = lib.mt_select_genomes_noalloc(C.c_void_p(dev.data_ptr()), 4, 1, 0, C.c_void_p(sel.data_ptr()),
                                       C.byref(ns), C.byref(mx), None)
    assert rc == _abi.MT_EINVAL
    # no genomes: nothing selected
    rc = lib.mt_select_genomes_noalloc(None, 0, 1, 10_000, None, C.byref(ns), C.byref(mx), None)
    assert rc == 0 and ns.value == 0 and mx.value == 0
    # all zero counts: the maximum is 0 and nothing is kept
    rc = lib.mt_select_genomes_noalloc(C.c_void_p(dev.data_ptr()), 4, 1, 10_000, C.c_void_p(sel.data_ptr()),
                                       C.byref(ns), C.byref(mx), None)
    assert rc == 0 and ns.value == 0 and mx.value == 0
