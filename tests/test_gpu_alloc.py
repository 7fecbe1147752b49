"""Device memory through the caller's allocator (mt_set_allocator).

With PyTorch's caching allocator installed (the binding's default), an index
build, classifications in every form, a containment search and a served
batch make no hipMalloc of the library's own; torch.cuda.memory_allocated()
covers the index; everything is released back to torch; results equal the
oracle's.  A hook written here in Python sees every allocation with the
stream of the call that makes it.  Switching back to the library's own pool
gives the same results.
"""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FIELDS = ("cand_offsets", "read_accepted", "read_E", "genome", "diag", "hits", "approx", "accept", "unique",
          "multi")


@pytest.fixture(scope="module")
def small():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gen, reads, p = synth.workload_small(3000)
    ga = gen.ascii()
    ref = oracle.Index(ga, p["k"], p["w"]).classify(reads, p["min_hits"], p["top_n"], 0, p["E"])
    return dict(ga=ga, reads=reads, p=p, ref=ref)


def _check(got, ref, ctx):
    for f in FIELDS:
        assert np.array_equal(np.asarray(got[f]), np.asarray(ref[f]).astype(np.asarray(got[f]).dtype)), (ctx, f)
    assert got["unmapped"] == ref["unmapped"], ctx


def _exercise(mt, small):
    """Index build, three forms, containment and a served batch; returns the
    index's device bytes and the growth of torch's allocated memory by the
    index build."""
    import torch
    p = small["p"]
    dg = mt.to_device(small["ga"])
    dr = mt.to_device(small["reads"])
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    ix = mt.Index(dg, p["k"], p["w"])
    torch.cuda.synchronize()
    grown = torch.cuda.memory_allocated() - before
    dev_bytes = ix.info()["device_bytes"]
    for mode in (mt.MT_MODE_PER_STAGE, mt.MT_MODE_FUSED, mt.MT_MODE_FUSED_GRAPH):
        res = ix.classify(dr, min_hits=p["min_hits"], top_n=p["top_n"], e_value=p["E"], mode=mode)
        _check(res.to_host(), small["ref"], f"mode {mode}")
        res.free()
    hits = ix.containment(dr)
    assert int(hits.sum().item()) > 0
    with mt.Server(ix, n_streams=2, max_batch_reads=1000) as sv:
        rid = sv.submit(small["reads"], min_hits=p["min_hits"], top_n=p["top_n"], e_value=p["E"])
        r = sv.wait(rid)
        _check(r.to_host(), small["ref"], "served")
        r.free()
    ix.free()
    return dev_bytes, grown


def test_torch_allocator_owns_library_memory(small):
    import torch
    import paper_2311_02029_amd as mt
    assert mt.use_torch_allocator(True)
    st0 = mt.memory_stats()
    assert st0["hooked"] == 1 and st0["cached_bytes"] == 0
    dev_bytes, grown = _exercise(mt, small)
    st1 = mt.memory_stats()
    assert st1["device_mallocs"] == st0["device_mallocs"], "the library called hipMalloc itself"
    assert st1["hook_allocs"] > st0["hook_allocs"]
    assert grown >= dev_bytes > 0, (grown, dev_bytes)
    assert st1["live_bytes"] == st0["live_bytes"], "blocks not handed back to torch"
    torch.cuda.synchronize()


def test_own_pool_gives_the_same_results(small):
    import paper_2311_02029_amd as mt
    try:
        assert not mt.use_torch_allocator(False)
        st0 = mt.memory_stats()
        assert st0["hooked"] == 0
        _exercise(mt, small)
        st1 = mt.memory_stats()
        assert st1["hook_allocs"] == st0["hook_allocs"]
        assert st1["cached_bytes"] > 0  # the pool keeps released blocks
        mt._abi.load().mt_trim()
        assert mt.memory_stats()["cached_bytes"] == 0
    finally:
        assert mt.use_torch_allocator(True)


def test_python_hook_sees_the_call_stream(small):
    """A hook made of two Python callbacks: every allocation of a classification
    on a side stream names that stream, every block comes back, and the
    result is the oracle's."""
    import torch
    import paper_2311_02029_amd as mt
    from paper_2311_02029_amd import _abi
    lib = _abi.load()
    held, seen = {}, []

    @_abi.ALLOC_FN
    def alloc(nbytes, stream, ctx):
        t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        held[t.data_ptr()] = t
        seen.append(stream or 0)
        return t.data_ptr()

    @_abi.FREE_FN
    def free(ptr, ctx):
        held.pop(ptr)

    p = small["p"]
    side = torch.cuda.Stream()
    try:
        assert lib.mt_set_allocator(C.cast(alloc, C.c_void_p), C.cast(free, C.c_void_p), None) == 0
        ix = mt.Index(mt.to_device(small["ga"]), p["k"], p["w"])
        dr = mt.to_device(small["reads"])
        torch.cuda.synchronize()
        seen.clear()
        res = ix.classify(dr, min_hits=p["min_hits"], top_n=p["top_n"], e_value=p["E"], mode=mt.MT_MODE_FUSED,
                          stream=side)
        assert seen and set(seen) == {side.cuda_stream}, set(seen)
        _check(res.to_host(), small["ref"], "python hook")
        res.free()
        ix.free()
        assert not held, f"{len(held)} blocks never freed"
    finally:
        assert mt.use_torch_allocator(True)
    # a half-set hook is refused
    assert lib.mt_set_allocator(C.cast(alloc, C.c_void_p), None, None) == _abi.MT_EINVAL
