// PyTorch's caching allocator as the library's device allocator: the two
// functions below have the signatures mt_set_allocator takes, and the Python
// binding installs them, so that one allocator owns the GPU's memory and
// torch.cuda.memory_allocated() covers the index, results and scratch of
// libmetatrinity.so.  Host code only (no kernels); built against the torch
// headers and libraries of the running PyTorch.
#include <cstddef>

#include <c10/hip/HIPCachingAllocator.h>

extern "C" void *mt_torch_alloc(size_t bytes, void *stream, void *) {
    try {
        // stream-ordered: the block may still have queued work of its last
        // user on this stream, which the library's own work follows
        return c10::hip::HIPCachingAllocator::raw_alloc_with_stream(bytes, (hipStream_t)stream);
    } catch (...) {
        return nullptr;  // out of memory: the library call fails with MT_ENOMEM
    }
}

extern "C" void mt_torch_free(void *ptr, void *) {
    try {
        c10::hip::HIPCachingAllocator::raw_delete(ptr);
    } catch (...) {
    }
}
