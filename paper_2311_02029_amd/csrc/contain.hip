// Containment search (Fig. 1 steps 1a-1d; "Containment Search"): the seed-hit
// count of every reference genome over a whole read set, on the index that
// stage 2 uses, and the subset-database selection by the normalised cutoff.
//
// Reads of up to 256 bases run in one fused kernel (fused.hip).  Longer reads
// take the per-stage chain here: bases packed to bit planes, minimizer tiles,
// then one kernel that probes the table for every read minimizer and adds one
// hit to the genome of each occurrence.  Integer atomics on per-block LDS
// counters take the place of the paper's mutex-guarded per-thread seed maps.
#include <mutex>

#include "classify.hpp"
#include "seq.hpp"

namespace mt {

constexpr int CT_TPB = 256;
constexpr u64 CT_LDS_GENOMES = 4096;  // genomes counted per block in LDS (64-bit counters, 32 KB)

// Grid-stride over the read minimizers.  With at most CT_LDS_GENOMES genomes a
// block counts in LDS and adds its nonzero counters to `hits` at the end (one
// atomic per genome and block instead of one per seed hit); with more it adds
// to `hits` directly.
__global__ __launch_bounds__(CT_TPB) void k_contain(const u64 *__restrict__ min_x, u64 n_min,
                                                    const u64x2 *__restrict__ table, u64 nbuckets,
                                                    const u64 *__restrict__ occ, u64 n_genomes,
                                                    unsigned long long *__restrict__ hits) {
    __shared__ unsigned long long cnt[CT_LDS_GENOMES];
    const bool in_lds = n_genomes <= CT_LDS_GENOMES;  // uniform over the grid
    unsigned long long *dst = in_lds ? cnt : hits;
    if (in_lds) {
        for (u64 g = threadIdx.x; g < n_genomes; g += CT_TPB) cnt[g] = 0;
        __syncthreads();
    }
    const u64 stride = (u64)gridDim.x * CT_TPB;
    for (u64 i = (u64)blockIdx.x * CT_TPB + threadIdx.x; i < n_min; i += stride) {
        const u64 v = table_lookup(table, nbuckets, min_x[i]);
        if (v == SLOT_NONE) continue;
        if (!(v & SLOT_MULTI)) {
            atomicAdd(&dst[v >> 32], 1ull);
            continue;
        }
        const u32 c = slot_count(v);  // 0 for a k-mer above max_occ
        const u64 st = slot_start(v);
        for (u32 u = 0; u < c; u++) atomicAdd(&dst[occ[st + u] >> 32], 1ull);
    }
    if (in_lds) {
        __syncthreads();
        for (u64 g = threadIdx.x; g < n_genomes; g += CT_TPB)
            if (cnt[g]) atomicAdd(&hits[g], cnt[g]);
    }
}

// Largest count.
__global__ void k_max_hits(const u64 *__restrict__ hits, u64 n, unsigned long long *__restrict__ mx) {
    u64 local = 0;
    for (u64 g = (u64)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (u64)gridDim.x * blockDim.x)
        local = hits[g] > local ? hits[g] : local;
    atomicMax(mx, (unsigned long long)local);
}

// keep[g] = hits[g] / max > num / den, decided as hits[g] * den > max * num on
// 128-bit products (high and low halves compared in turn).
__global__ void k_keep(const u64 *__restrict__ hits, u64 n, const unsigned long long *__restrict__ mx, u64 num,
                       u64 den, u32 *__restrict__ keep) {
    const u64 g = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const u64 a = hits[g], m = *mx;
    const u64 lh = __umul64hi(a, den), ll = a * den;
    const u64 rh = __umul64hi(m, num), rl = m * num;
    keep[g] = lh > rh || (lh == rh && ll > rl);
}

__global__ void k_place(const u32 *__restrict__ keep, const u64 *__restrict__ at, u64 n, u32 *__restrict__ out) {
    const u64 g = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n && keep[g]) out[at[g]] = (u32)g;
}

__global__ void k_zero_u64(unsigned long long *__restrict__ p) {
    if (threadIdx.x == 0) *p = 0;
}

// The selection's launches on caller-provided buffers: mx (one word), keep (n),
// at (n + 1) and the scan workspace; `ws == nullptr` lets the scan allocate.
static void select_into(const u64 *hits, u64 n, u64 num, u64 den, u32 *selected, unsigned long long *mx, u32 *keep,
                        u64 *at, u64 *ws, u64 ws_words, hipStream_t s) {
    k_zero_u64<<<1, 64, 0, s>>>(mx);  // a kernel rather than a memset node: callers may capture this
    MT_HIP(hipGetLastError());
    k_max_hits<<<(unsigned)std::min<u64>(grid_for(n, 256), 1024), 256, 0, s>>>(hits, n, mx);
    MT_HIP(hipGetLastError());
    k_keep<<<grid_for(n, 256), 256, 0, s>>>(hits, n, mx, num, den, keep);
    MT_HIP(hipGetLastError());
    if (ws)
        scan_u32_ws(keep, at, n, ws, ws_words, s);
    else
        scan_u32(keep, at, n, s);
    k_place<<<grid_for(n, 256), 256, 0, s>>>(keep, at, n, selected);
    MT_HIP(hipGetLastError());
}

// ---------------------------------------------- the allocation-free variant --
//
// mt_select_genomes_noalloc keeps its scratch in one static device array of
// fixed size (each GPU holds its own copy until the process ends).  Host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device, taken once per device.  Layout: the maximum (one word, its
// own 256-byte line), keep flags (u32 per genome), offsets (u64 per genome +
// 1), the scan workspace.
constexpr u64 SEL_NOALLOC_MAX = 1ull << 20;  // genomes
constexpr u64 SEL_KEEP_OFF = 256;
constexpr u64 SEL_AT_OFF = SEL_KEEP_OFF + ((SEL_NOALLOC_MAX * 4 + 255) / 256) * 256;
constexpr u64 SEL_WS_OFF = SEL_AT_OFF + (((SEL_NOALLOC_MAX + 1) * 8 + 255) / 256) * 256;
constexpr u64 SEL_WS_WORDS = 2 * ((SEL_NOALLOC_MAX + 2047) / 2048) + 1;
constexpr u64 SEL_SCRATCH_BYTES = SEL_WS_OFF + SEL_WS_WORDS * 8;

static __device__ __align__(256) unsigned char scratch[SEL_SCRATCH_BYTES];

constexpr int SEL_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static unsigned char *g_scratch_ptr[SEL_MAX_DEVICES];

// The current device's copy of `scratch` (its address looked up on the first
// call on that device).
static unsigned char *scratch_on_device() {
    int dev = 0;
    MT_HIP(hipGetDevice(&dev));
    MT_REQUIRE(dev >= 0 && dev < SEL_MAX_DEVICES, "device index beyond the scratch table");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        MT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        MT_REQUIRE(p != nullptr, "no device address for the selection scratch");
        g_scratch_ptr[dev] = (unsigned char *)p;
    }
    return g_scratch_ptr[dev];
}

static unsigned contain_blocks(u64 n_min) {
    int dev = 0, cus = 0;
    MT_HIP(hipGetDevice(&dev));
    MT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    return (unsigned)std::max<u64>(1, std::min<u64>(grid_for(n_min, CT_TPB), (u64)std::max(cus, 1) * 8));
}

void containment_per_stage(const mt_index &ix, const mt_seqs &reads, u64 *hits, hipStream_t s) {
    if (reads.n == 0 || ix.n_genomes == 0) return;
    ReadBatch rb;
    rb.prepare(reads, MT_E_FIXED, 0, s);  // validates lengths and bytes; E is unused here
    MinimizerPlan mp;
    const int tile = reads.total / reads.n > 512 ? 1024 : 256;
    minimizer_plan(reads, rb.planes, ix.k, ix.w, tile, mp, s);
    u32 f = 0;
    u64 n_min = 0;
    MT_HIP(hipMemcpyAsync(&f, rb.flags.p, sizeof f, hipMemcpyDeviceToHost, s));
    read_back(s, mp.min_off.p + mp.tiles_cap, &n_min, sizeof n_min);
    check_flags(f);
    if (n_min == 0) return;
    DBuf<u64> min_x(n_min);
    minimizer_emit(reads, rb.planes, ix.k, ix.w, mp, min_x.p, nullptr, nullptr, s);
    k_contain<<<contain_blocks(n_min), CT_TPB, 0, s>>>(min_x.p, n_min, ix.table.p, ix.nbuckets, ix.occ.p,
                                                        ix.n_genomes, (unsigned long long *)hits);
    MT_HIP(hipGetLastError());
}

}  // namespace mt

using namespace mt;

extern "C" int mt_containment(const mt_index *index, const mt_seqs *reads, uint64_t *hits, void *stream) {
    if (!index || !reads || (!hits && index->n_genomes)) {
        set_last_error("mt_containment: null argument");
        return MT_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    return guarded("mt_containment", [&] {
        MT_REQUIRE(reads->n == 0 || (reads->seq && reads->offsets), "null read arrays");
        CallScope scope(s);
        if (index->n_genomes) MT_HIP(hipMemsetAsync(hits, 0, index->n_genomes * sizeof(uint64_t), s));
        containment(*index, *reads, hits, s);
    });
}

extern "C" int mt_select_genomes(const uint64_t *hits, uint64_t n_genomes, uint64_t cutoff_num, uint64_t cutoff_den,
                                 uint32_t *selected, uint64_t *n_selected, uint64_t *max_hits, void *stream) {
    if ((!hits || !selected) && n_genomes) {
        set_last_error("mt_select_genomes: null argument");
        return MT_EINVAL;
    }
    if (!n_selected || !max_hits) {
        set_last_error("mt_select_genomes: null argument");
        return MT_EINVAL;
    }
    if (cutoff_den == 0) {
        set_last_error("mt_select_genomes: cutoff denominator must be nonzero");
        return MT_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    return guarded("mt_select_genomes", [&] {
        *n_selected = 0;
        *max_hits = 0;
        if (n_genomes == 0) return;
        CallScope scope(s);
        DBuf<unsigned long long> mx(1);
        DBuf<u32> keep(n_genomes);
        DBuf<u64> at(n_genomes + 1);
        select_into(hits, n_genomes, cutoff_num, cutoff_den, selected, mx.p, keep.p, at.p, nullptr, 0, s);
        u64 out[2];
        MT_HIP(hipMemcpyAsync(&out[0], at.p + n_genomes, sizeof(u64), hipMemcpyDeviceToHost, s));
        MT_HIP(hipMemcpyAsync(&out[1], mx.p, sizeof(u64), hipMemcpyDeviceToHost, s));
        MT_HIP(hipStreamSynchronize(s));
        *n_selected = out[0];
        *max_hits = out[1];
    });
}

extern "C" int mt_select_genomes_noalloc(const uint64_t *hits, uint64_t n_genomes, uint64_t cutoff_num,
                                         uint64_t cutoff_den, uint32_t *selected, uint64_t *n_selected,
                                         uint64_t *max_hits, void *stream) {
    if ((!hits || !selected) && n_genomes) {
        set_last_error("mt_select_genomes_noalloc: null argument");
        return MT_EINVAL;
    }
    if (!n_selected || !max_hits) {
        set_last_error("mt_select_genomes_noalloc: null argument");
        return MT_EINVAL;
    }
    if (cutoff_den == 0) {
        set_last_error("mt_select_genomes_noalloc: cutoff denominator must be nonzero");
        return MT_EINVAL;
    }
    if (n_genomes > SEL_NOALLOC_MAX) {
        set_last_error("mt_select_genomes_noalloc: more than 1,048,576 genomes (use mt_select_genomes)");
        return MT_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    return guarded("mt_select_genomes_noalloc", [&] {
        *n_selected = 0;
        *max_hits = 0;
        if (n_genomes == 0) return;
        unsigned char *base = scratch_on_device();
        auto *mx = (unsigned long long *)base;
        auto *keep = (u32 *)(base + SEL_KEEP_OFF);
        auto *at = (u64 *)(base + SEL_AT_OFF);
        auto *ws = (u64 *)(base + SEL_WS_OFF);
        select_into(hits, n_genomes, cutoff_num, cutoff_den, selected, mx, keep, at, ws, SEL_WS_WORDS, s);
        u64 out[2];
        MT_HIP(hipMemcpyAsync(&out[0], at + n_genomes, sizeof(u64), hipMemcpyDeviceToHost, s));
        MT_HIP(hipMemcpyAsync(&out[1], mx, sizeof(u64), hipMemcpyDeviceToHost, s));
        MT_HIP(hipStreamSynchronize(s));
        *n_selected = out[0];
        *max_hits = out[1];
    });
}
