// Host runtime of the library: status/error plumbing, the caching device
// allocator, scans, and per-launch event timing.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/metatrinity.h"
#include "device.hpp"

namespace mt {

// An error that maps to an mt_status at the ABI boundary.
struct Error : std::runtime_error {
    int status;
    Error(int s, const std::string &msg) : std::runtime_error(msg), status(s) {}
};

void set_last_error(const std::string &msg);

#define MT_HIP(call)                                                                                     \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess)                                                                            \
            throw ::mt::Error(e_ == hipErrorOutOfMemory ? MT_ENOMEM : MT_EDEVICE,                        \
                              std::string(#call) + ": " + hipGetErrorString(e_));                         \
    } while (0)

#define MT_REQUIRE(cond, msg)                                                                            \
    do {                                                                                                 \
        if (!(cond)) throw ::mt::Error(MT_EINVAL, (msg));                                                \
    } while (0)

// Device allocator.  By default a caching pool: blocks are rounded up (power
// of two below 1 MiB, 2 MiB multiples above) and kept on free lists after
// release, so the per-call scratch of a classification costs no hipMalloc
// after warm-up.  With an allocator hook installed (mt_set_allocator) every
// allocation goes to the hook, with the stream its memory is first used on,
// and every release back to it; the pool then holds nothing.  Every library
// call synchronizes its stream before releasing scratch, so a released block
// is idle when it is handed out again.
void *pool_alloc(size_t bytes);                      // stream: the open CallScope's, else the null stream
void *pool_alloc_on(size_t bytes, hipStream_t stream);
void pool_free(void *p);
void pool_trim();
void set_allocator(void *(*alloc)(size_t, void *, void *), void (*free_)(void *, void *), void *ctx);
mt_mem_stats memory_stats();

// Scope of one ABI call on one stream.  Blocks released while a scope is open
// on the calling thread are parked until the scope ends; the scope then
// synchronizes its stream and only after that returns them to the pool, so
// no other thread can be handed a block that queued kernels still touch.
struct CallScope {
    hipStream_t stream;
    std::vector<void *> deferred;
    CallScope *prev;
    explicit CallScope(hipStream_t s);
    ~CallScope();
    CallScope(const CallScope &) = delete;
    CallScope &operator=(const CallScope &) = delete;
};

// RAII device buffer from the pool.
template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    void alloc(size_t count) {
        release();
        n = count;
        p = static_cast<T *>(pool_alloc((count ? count : 1) * sizeof(T)));
    }
    void release() {
        if (p) pool_free(p);
        p = nullptr;
        n = 0;
    }
    T *release_ownership() {
        T *q = p;
        p = nullptr;
        n = 0;
        return q;
    }
    ~DBuf() { release(); }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), n(o.n) {
        o.p = nullptr;
        o.n = 0;
    }
    DBuf &operator=(DBuf &&o) noexcept {
        release();
        p = o.p;
        n = o.n;
        o.p = nullptr;
        o.n = 0;
        return *this;
    }
};

// Exclusive scan of n u64 (or u32 widened) values into out[0..n], with
// out[n] = total.  in and out may not alias.
void scan_u64(const u64 *in, u64 *out, u64 n, hipStream_t s);
void scan_u32(const u32 *in, u64 *out, u64 n, hipStream_t s);
// The same scan with the caller's workspace instead of the allocator: ws
// holds scan_ws_words(n) words (n up to 2048 * 2048).
u64 scan_ws_words(u64 n);
void scan_u32_ws(const u32 *in, u64 *out, u64 n, u64 *ws, u64 ws_words, hipStream_t s);

// Writes map[b] = s for every block b < cap of segment s given the segment
// offsets off[0..n] (exclusive scan of the segment sizes).
void segment_map(const u64 *off, u64 n, u32 *map, u64 cap, hipStream_t s);

// Grid size for a 1-D launch of `items` work items at `per_block` per block.
inline unsigned grid_for(u64 items, u64 per_block) {
    u64 g = (items + per_block - 1) / per_block;
    if (g == 0) g = 1;
    if (g > 0x7fffffffull) throw Error(MT_EINVAL, "launch too large");
    return (unsigned)g;
}

// HIP-event timing of named launches on one stream (enabled by mt_set_timing).
struct Timer {
    hipStream_t stream = nullptr;
    bool on = false;
    std::vector<std::pair<const char *, hipEvent_t>> marks;
    void begin(hipStream_t s);
    void mark(const char *name);  // ends the stage that began at the previous mark
    void finish();                // synchronizes and publishes the timings
    ~Timer();
};

bool timing_enabled();

// Work counts of the last classification on this thread (mt_last_stats).
mt_stats &last_stats();

// Validation flags the kernels raise, decoded into an error.
void check_flags(u32 flags);

// Runs f as the body of an ABI call: maps exceptions to an mt_status and
// records the message for mt_last_error.
template <class F>
int guarded(const char *what, F &&f) {
    try {
        f();
        set_last_error("");
        return MT_OK;
    } catch (const Error &e) {
        set_last_error(std::string(what) + ": " + e.what());
        return e.status;
    } catch (const std::bad_alloc &) {
        set_last_error(std::string(what) + ": host allocation failed");
        return MT_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(std::string(what) + ": " + e.what());
        return MT_EINTERNAL;
    }
}

}  // namespace mt
