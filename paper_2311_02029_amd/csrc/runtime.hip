// Host runtime: errors, caching allocator, scans, segment maps, timing.
#include "runtime.hpp"

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>

namespace mt {

// ------------------------------------------------------------------ errors --

static thread_local std::string g_last_error;

void set_last_error(const std::string &msg) { g_last_error = msg; }

void check_flags(u32 f) {
    if (!f) return;
    if (f & ERR_INTERNAL) throw Error(MT_EINTERNAL, "internal invariant failed on the device");
    if (f & ERR_BAD_BYTE) throw Error(MT_EINVAL, "sequence byte outside A, C, G, T, N (either case)");
    if (f & ERR_READ_TOO_LONG) throw Error(MT_EINVAL, "read longer than 65535 bases");
    if (f & ERR_E_TOO_LARGE) throw Error(MT_EINVAL, "edit threshold E above 65534");
    if (f & ERR_PAIR_RANGE) throw Error(MT_EINVAL, "pair read or genome index out of range");
    if (f & ERR_KEY_OVERFLOW) throw Error(MT_EINVAL, "a k-mer occurs more than 2^23-1 times; set max_occ");
    if (f & ERR_OFFSETS) throw Error(MT_EINVAL, "offsets must start at 0, never decrease and end at total");
    throw Error(MT_EINTERNAL, "unknown device flag");
}

// --------------------------------------------------------------- allocator --

namespace {
// A device allocation hook (mt_set_allocator); alloc == nullptr means the
// built-in caching pool.
struct Hook {
    void *(*alloc)(size_t, void *, void *) = nullptr;
    void (*free_)(void *, void *) = nullptr;
    void *ctx = nullptr;
};
struct Block {
    size_t size;
    Hook hook;  // the allocator that made the block (hook.alloc null: the pool)
};
struct Pool {
    std::mutex mu;
    std::multimap<size_t, void *> free_blocks;
    std::unordered_map<void *, Block> live;
    Hook hook;
    size_t cached_bytes = 0;
    mt_mem_stats stats{};
};
Pool &pool() {
    static Pool *p = new Pool();  // never destroyed: outlives static handles at exit
    return *p;
}
size_t round_size(size_t b) {
    if (b < (1u << 20)) {
        size_t r = 512;
        while (r < b) r <<= 1;
        return r;
    }
    size_t u = 2u << 20;
    return (b + u - 1) / u * u;
}
}  // namespace

static thread_local CallScope *g_scope = nullptr;

void *pool_alloc(size_t bytes) { return pool_alloc_on(bytes, g_scope ? g_scope->stream : nullptr); }

void *pool_alloc_on(size_t bytes, hipStream_t stream) {
    Pool &P = pool();
    Hook h;
    {
        std::lock_guard<std::mutex> g(P.mu);
        h = P.hook;
    }
    if (h.alloc) {
        // the caller's allocator: no cache here (it keeps its own)
        const size_t sz = bytes ? bytes : 1;
        void *p = h.alloc(sz, (void *)stream, h.ctx);
        if (!p) throw Error(MT_ENOMEM, "device allocation of " + std::to_string(sz) + " bytes failed (allocator hook)");
        std::lock_guard<std::mutex> g(P.mu);
        P.live[p] = Block{sz, h};
        P.stats.hook_allocs++;
        P.stats.live_bytes += sz;
        return p;
    }
    size_t sz = round_size(bytes);
    {
        std::lock_guard<std::mutex> g(P.mu);
        auto it = P.free_blocks.find(sz);
        if (it != P.free_blocks.end()) {
            void *p = it->second;
            P.free_blocks.erase(it);
            P.cached_bytes -= sz;
            P.live[p] = Block{sz, Hook{}};
            P.stats.live_bytes += sz;
            return p;
        }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, sz);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        pool_trim();
        e = hipMalloc(&p, sz);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(e == hipErrorOutOfMemory ? MT_ENOMEM : MT_EDEVICE,
                    "device allocation of " + std::to_string(sz) + " bytes failed: " + hipGetErrorString(e));
    }
    std::lock_guard<std::mutex> g(P.mu);
    P.live[p] = Block{sz, Hook{}};
    P.stats.device_mallocs++;
    P.stats.live_bytes += sz;
    return p;
}

CallScope::CallScope(hipStream_t s) : stream(s), prev(g_scope) { g_scope = this; }

CallScope::~CallScope() {
    g_scope = prev;
    (void)hipStreamSynchronize(stream);
    for (void *p : deferred) pool_free(p);
}

void pool_free(void *p) {
    if (!p) return;
    if (g_scope) {
        g_scope->deferred.push_back(p);
        return;
    }
    Pool &P = pool();
    Block b;
    {
        std::lock_guard<std::mutex> g(P.mu);
        auto it = P.live.find(p);
        if (it == P.live.end()) return;
        b = it->second;
        P.live.erase(it);
        P.stats.live_bytes -= b.size;
        if (!b.hook.alloc) {
            P.free_blocks.emplace(b.size, p);
            P.cached_bytes += b.size;
            return;
        }
    }
    b.hook.free_(p, b.hook.ctx);  // outside the lock: the hook may allocate or free itself
}

void pool_trim() {
    Pool &P = pool();
    std::lock_guard<std::mutex> g(P.mu);
    for (auto &kv : P.free_blocks) (void)hipFree(kv.second);
    P.free_blocks.clear();
    P.cached_bytes = 0;
}

void set_allocator(void *(*alloc)(size_t, void *, void *), void (*free_)(void *, void *), void *ctx) {
    MT_REQUIRE((alloc == nullptr) == (free_ == nullptr), "alloc and free must both be set or both be NULL");
    pool_trim();  // the library keeps no idle device memory of its own behind a hook
    Pool &P = pool();
    std::lock_guard<std::mutex> g(P.mu);
    P.hook.alloc = alloc;
    P.hook.free_ = free_;
    P.hook.ctx = ctx;
}

mt_mem_stats memory_stats() {
    Pool &P = pool();
    std::lock_guard<std::mutex> g(P.mu);
    mt_mem_stats s = P.stats;
    s.cached_bytes = P.cached_bytes;
    s.hooked = P.hook.alloc != nullptr;
    return s;
}

// ------------------------------------------------------------------- scans --

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// Exclusive scan of the 256 thread totals of a block; returns this thread's
// prefix and the block total through *total.
__device__ inline u64 block_exclusive(u64 v, u64 *total) {
    __shared__ u64 wave_tot[SCAN_THREADS / 64];
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    u64 x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        u64 y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wave_tot[wid] = x;
    __syncthreads();
    u64 before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < SCAN_THREADS / 64; i++) {
        if (i < wid) before += wave_tot[i];
        all += wave_tot[i];
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

template <class T>
__global__ void k_scan_sums(const T *__restrict__ in, u64 n, u64 *__restrict__ sums) {
    u64 base = (u64)blockIdx.x * SCAN_TILE + (u64)threadIdx.x * SCAN_ITEMS;
    u64 s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++)
        if (base + i < n) s += (u64)in[base + i];
    u64 tot;
    block_exclusive(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <class T>
__global__ void k_scan_final(const T *__restrict__ in, u64 n, u64 *__restrict__ out,
                             const u64 *__restrict__ block_off) {
    u64 base = (u64)blockIdx.x * SCAN_TILE + (u64)threadIdx.x * SCAN_ITEMS;
    u64 v[SCAN_ITEMS];
    u64 s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        v[i] = base + i < n ? (u64)in[base + i] : 0;
        s += v[i];
    }
    u64 tot;
    u64 run = block_exclusive(s, &tot) + (block_off ? block_off[blockIdx.x] : 0);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_THREADS - 1) out[n] = run;
}

template <class T>
static void scan_impl(const T *in, u64 *out, u64 n, hipStream_t s) {
    u64 nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb <= 1) {
        k_scan_final<T><<<1, SCAN_THREADS, 0, s>>>(in, n, out, nullptr);
        MT_HIP(hipGetLastError());
        return;
    }
    DBuf<u64> sums(nb), sums_scan(nb + 1);
    k_scan_sums<T><<<grid_for(n, SCAN_TILE), SCAN_THREADS, 0, s>>>(in, n, sums.p);
    MT_HIP(hipGetLastError());
    scan_impl<u64>(sums.p, sums_scan.p, nb, s);
    k_scan_final<T><<<grid_for(n, SCAN_TILE), SCAN_THREADS, 0, s>>>(in, n, out, sums_scan.p);
    MT_HIP(hipGetLastError());
}

void scan_u64(const u64 *in, u64 *out, u64 n, hipStream_t s) { scan_impl<u64>(in, out, n, s); }
void scan_u32(const u32 *in, u64 *out, u64 n, hipStream_t s) { scan_impl<u32>(in, out, n, s); }

u64 scan_ws_words(u64 n) {
    const u64 nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    return nb <= 1 ? 0 : 2 * nb + 1;
}

void scan_u32_ws(const u32 *in, u64 *out, u64 n, u64 *ws, u64 ws_words, hipStream_t s) {
    const u64 nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb <= 1) {
        k_scan_final<u32><<<1, SCAN_THREADS, 0, s>>>(in, n, out, nullptr);
        MT_HIP(hipGetLastError());
        return;
    }
    if (nb > (u64)SCAN_TILE || ws_words < 2 * nb + 1) throw Error(MT_EINTERNAL, "scan workspace too small");
    u64 *sums = ws, *sums_scan = ws + nb;  // nb block sums, then their nb + 1 offsets
    k_scan_sums<u32><<<grid_for(n, SCAN_TILE), SCAN_THREADS, 0, s>>>(in, n, sums);
    MT_HIP(hipGetLastError());
    k_scan_final<u64><<<1, SCAN_THREADS, 0, s>>>(sums, nb, sums_scan, nullptr);
    MT_HIP(hipGetLastError());
    k_scan_final<u32><<<grid_for(n, SCAN_TILE), SCAN_THREADS, 0, s>>>(in, n, out, sums_scan);
    MT_HIP(hipGetLastError());
}

__global__ void k_segment_map(const u64 *__restrict__ off, u64 n, u32 *__restrict__ map, u64 cap) {
    u64 sidx = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (sidx >= n) return;
    u64 e = off[sidx + 1] < cap ? off[sidx + 1] : cap;
    for (u64 b = off[sidx]; b < e; b++) map[b] = (u32)sidx;
}

void segment_map(const u64 *off, u64 n, u32 *map, u64 cap, hipStream_t s) {
    if (n == 0) return;
    k_segment_map<<<grid_for(n, 256), 256, 0, s>>>(off, n, map, cap);
    MT_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ timing --

static bool g_timing = false;
static thread_local std::vector<std::pair<std::string, float>> g_timings;

bool timing_enabled() { return g_timing; }

static thread_local mt_stats g_stats;
mt_stats &last_stats() { return g_stats; }

// MT_TRACE=1 in the environment: every stage mark waits for its stream and
// logs the stage to stderr (locates a slow or stuck stage).
static bool trace_on() {
    static int t = -1;
    if (t < 0) {
        const char *e = getenv("MT_TRACE");
        t = e && *e && *e != '0';
    }
    return t != 0;
}

void Timer::begin(hipStream_t s) {
    stream = s;
    on = g_timing;
    marks.clear();
    if (on) mark("begin");
    if (trace_on()) fprintf(stderr, "[mt] begin\n");
}

void Timer::mark(const char *name) {
    if (trace_on()) {
        auto t0 = std::chrono::steady_clock::now();
        hipError_t e = hipStreamSynchronize(stream);
        double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        fprintf(stderr, "[mt] %s done (wait %.3f ms, %s)\n", name, ms, hipGetErrorString(e));
        fflush(stderr);
    }
    if (!on) return;
    hipEvent_t e;
    MT_HIP(hipEventCreate(&e));
    MT_HIP(hipEventRecord(e, stream));
    marks.emplace_back(name, e);
}

void Timer::finish() {
    if (!on) return;
    MT_HIP(hipStreamSynchronize(stream));
    g_timings.clear();
    for (size_t i = 1; i < marks.size(); i++) {
        float ms = 0;
        MT_HIP(hipEventElapsedTime(&ms, marks[i - 1].second, marks[i].second));
        g_timings.emplace_back(marks[i].first, ms);
    }
}

Timer::~Timer() {
    for (auto &m : marks) (void)hipEventDestroy(m.second);
}

}  // namespace mt

// ------------------------------------------------------------ ABI helpers --

extern "C" const char *mt_last_error(void) { return mt::g_last_error.c_str(); }

extern "C" int mt_abi_version(void) { return MT_ABI_VERSION; }

extern "C" int mt_trim(void) {
    mt::pool_trim();
    return MT_OK;
}

extern "C" int mt_set_allocator(void *(*alloc)(size_t, void *, void *), void (*free_)(void *, void *), void *ctx) {
    return mt::guarded("mt_set_allocator", [&] { mt::set_allocator(alloc, free_, ctx); });
}

extern "C" int mt_memory_stats(mt_mem_stats *out) {
    if (!out) {
        mt::set_last_error("mt_memory_stats: null argument");
        return MT_EINVAL;
    }
    *out = mt::memory_stats();
    return MT_OK;
}

extern "C" int mt_set_timing(int enabled) {
    mt::g_timing = enabled != 0;
    return MT_OK;
}

extern "C" int mt_last_stats(mt_stats *out) {
    if (!out) {
        mt::set_last_error("mt_last_stats: null argument");
        return MT_EINVAL;
    }
    *out = mt::g_stats;
    return MT_OK;
}

extern "C" int mt_last_timings(const char **names, float *ms, uint32_t cap, uint32_t *n) {
    if (!n || (cap && (!names || !ms))) {
        mt::set_last_error("mt_last_timings: null argument");
        return MT_EINVAL;
    }
    uint32_t k = 0;
    for (auto &t : mt::g_timings) {
        if (k >= cap) break;
        names[k] = t.first.c_str();
        ms[k] = t.second;
        k++;
    }
    *n = k;
    return MT_OK;
}
