// Read classification, one kernel launch per step of the path (Fig. 1 steps
// 2b-2d, 3a):
//   setup     read lengths and thresholds E
//   pack      ASCII -> bit planes
//   seed      minimizers of every read (count pass, then emit)
//   lookup    one hash-table probe per minimizer -> occurrence count
//   gather    every (minimizer, occurrence) pair -> location key (genome, diag)
//   count     per read: sort keys, count hits per location, keep >= min_hits,
//             order by (hits desc, genome, diag), keep top_n
//   compact   CSR of candidates
//   filter    obstacle count per (read, location) pair, accept if <= E
//   reduce    read accepted flag, per-taxon unique / multi / unmapped counts
#include <algorithm>
#include <cstring>

#include "classify.hpp"

namespace mt {

// ------------------------------------------------------------------ setup --

__global__ void k_read_setup(const u64 *__restrict__ off, u64 n, u32 e_mode, u32 e_value, u16 *__restrict__ read_E,
                             u32 *__restrict__ flags, u32 *__restrict__ max_E) {
    u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    u64 m = off[r + 1] - off[r];
    u64 E = e_mode == MT_E_FIXED ? e_value
            : e_mode == MT_E_CEIL_PERMILLE ? (m * e_value + 999) / 1000
                                           : (m * e_value) / 1000;
    u32 f = 0;
    if (m > 65535) f |= ERR_READ_TOO_LONG;
    if (E > 65534) f |= ERR_E_TOO_LARGE;
    if (f) atomicOr(flags, f);
    u32 e = E > 65535 ? 65535u : (u32)E;
    read_E[r] = (u16)e;
    atomicMax(max_E, e);
}

// ----------------------------------------------------------------- lookup --

__global__ void k_lookup(const u64 *__restrict__ min_x, u64 n_min, const u64x2 *__restrict__ table, u64 nbuckets,
                         u64 *__restrict__ min_val, u32 *__restrict__ min_nocc) {
    u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_min) return;
    u64 x = min_x[i];
    u64 v = table_lookup(table, nbuckets, x);
    min_val[i] = v;
    min_nocc[i] = v == SLOT_NONE ? 0u : slot_count(v);
}

__global__ void k_gather(const u32 *__restrict__ min_pos, const u64 *__restrict__ min_val,
                         const u64 *__restrict__ hit_off, u64 n_min, const u64 *__restrict__ occ,
                         u64 *__restrict__ hit_key) {
    u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_min) return;
    u64 v = min_val[i];
    u64 o = hit_off[i], e = hit_off[i + 1];
    if (o == e) return;
    i64 p = (i64)min_pos[i];
    if (!(v & SLOT_MULTI)) {
        hit_key[o] = cand_key((u32)(v >> 32), (i64)(u32)v - p);
        return;
    }
    u64 st = slot_start(v);
    for (u64 t = 0; o + t < e; t++) {
        u64 gp = occ[st + t];
        hit_key[o + t] = cand_key((u32)(gp >> 32), (i64)(u32)gp - p);
    }
}

// First hit of every read (n + 1 entries): through the read's first tile and
// that tile's first minimizer.
__global__ void k_read_hits(const u64 *__restrict__ tile_off, const u64 *__restrict__ min_off,
                            const u64 *__restrict__ hit_off, u64 n, u64 *__restrict__ read_hs) {
    u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > n) return;
    read_hs[r] = hit_off[min_off[tile_off[r]]];
}

// ------------------------------------------------------------------ count --

// Pair index t of a bitonic sub-step -> the two positions compared (i < l).
// Every comparison puts the smaller element first ("all ascending" form),
// so positions past the segment act as +infinity and are never touched.
__device__ inline void bitonic_pair(u64 t, u64 k, u64 j, bool mirror, u64 &i, u64 &l) {
    if (mirror) {
        u64 half = k >> 1, blk = t / half, off = t % half;
        i = blk * k + off;
        l = blk * k + k - 1 - off;
    } else {
        i = (t / j) * 2 * j + (t % j);
        l = i + j;
    }
}

__device__ inline bool cand_before(u32 ha, u64 ka, u32 hb, u64 kb) { return ha > hb || (ha == hb && ka < kb); }

constexpr int COUNT_TPB = 256;
constexpr int COUNT_CAP = 2048;
constexpr int WAVE_CAP = 256;  // most hits one wavefront counts in registers
constexpr int CW_WPB = 4;      // reads (wavefronts) per block of k_count_wave

__device__ inline u64 wave_readlane64(u64 v, int l) {
    const u32 lo = __builtin_amdgcn_readlane((u32)v, l), hi = __builtin_amdgcn_readlane((u32)(v >> 32), l);
    return ((u64)hi << 32) | lo;
}

// Hit counting of one read by one wavefront, the read's H <= 64 * S hits held
// S to a lane (hit i in lane i % 64, slot i / 64).  Each distinct key is
// counted with one ballot per slot and its count kept by the lane of its first
// hit; the candidates (count >= T) are then ranked in registers in the
// canonical order and the first top_n (all if 0) are written to the read's
// staging area.  Returns the number of candidates before the top-N cut.
template <int S>
__device__ inline u32 count_in_wave(const u64 *__restrict__ hit_key, u64 hs, u32 H, u32 lane, u32 T, u32 top_n,
                                    u64 *__restrict__ stage_key, u32 *__restrict__ stage_hits) {
    u64 key[S], pend[S];
    u32 cnt[S];
#pragma unroll
    for (int s = 0; s < S; s++) {
        const u32 i = lane + 64 * s;
        key[s] = i < H ? hit_key[hs + i] : 0;
        pend[s] = __ballot(i < H);
        cnt[s] = 0;
    }
#pragma unroll
    for (int s0 = 0; s0 < S; s0++) {
        while (pend[s0]) {
            const int ld = __builtin_ctzll(pend[s0]);
            const u64 k = wave_readlane64(key[s0], ld);
            u32 c = 0;
#pragma unroll
            for (int s = s0; s < S; s++) {
                const u64 eq = __ballot(((pend[s] >> lane) & 1) && key[s] == k);
                c += (u32)__popcll(eq);
                pend[s] &= ~eq;
            }
            if (lane == (u32)ld) cnt[s0] = c;
        }
    }
    u32 C = 0, rank[S];
    u64 cm[S];
#pragma unroll
    for (int s = 0; s < S; s++) {
        cm[s] = __ballot(cnt[s] >= T);
        C += (u32)__popcll(cm[s]);
        rank[s] = 0;
    }
#pragma unroll
    for (int sb = 0; sb < S; sb++) {
        u64 it = cm[sb];
        while (it) {
            const int b = __builtin_ctzll(it);
            it &= it - 1;
            const u64 kb = wave_readlane64(key[sb], b);
            const u32 hb = __builtin_amdgcn_readlane(cnt[sb], b);
#pragma unroll
            for (int s = 0; s < S; s++) rank[s] += cand_before(hb, kb, cnt[s], key[s]);
        }
    }
#pragma unroll
    for (int s = 0; s < S; s++)
        if (cnt[s] >= T && (top_n == 0 || rank[s] < top_n)) {
            stage_key[hs + rank[s]] = key[s];
            stage_hits[hs + rank[s]] = cnt[s];
        }
    return C;
}

// One wavefront per read with at most WAVE_CAP hits; larger reads are queued
// for k_count_block.
__global__ __launch_bounds__(64 * CW_WPB) void k_count_wave(const u64 *__restrict__ hit_key,
                                                            const u64 *__restrict__ read_hs, u64 n, u32 min_hits,
                                                            u32 top_n, u64 *__restrict__ stage_key,
                                                            u32 *__restrict__ stage_hits, u32 *__restrict__ ncand,
                                                            u32 *__restrict__ mid_list, u32 *__restrict__ n_mid) {
    const u32 lane = threadIdx.x & 63;
    const u64 r = (u64)blockIdx.x * CW_WPB + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (r >= n) return;
    const u64 hs = read_hs[r], H = read_hs[r + 1] - hs;
    const u32 T = min_hits ? min_hits : 1;
    u32 C;
    if (H <= 64) {
        C = count_in_wave<1>(hit_key, hs, (u32)H, lane, T, top_n, stage_key, stage_hits);
    } else if (H <= WAVE_CAP) {
        C = count_in_wave<4>(hit_key, hs, (u32)H, lane, T, top_n, stage_key, stage_hits);
    } else {
        if (lane == 0) mid_list[atomicAdd(n_mid, 1u)] = (u32)r;
        return;
    }
    if (lane == 0) ncand[r] = top_n && C > top_n ? top_n : C;
}

// Blocks of k_count_block: a few per CU, each looping over the queue (its
// length is known only on the device).
static unsigned count_blocks() {
    int dev = 0, cus = 0;
    MT_HIP(hipGetDevice(&dev));
    MT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    return (unsigned)std::max(cus, 1) * 4;
}

constexpr u32 COUNT_SLOTS = 2 * COUNT_CAP;  // LDS hash table of a read's locations

// Slot of a location key in a table of `slots` (a power of two) slots.
__device__ inline u32 count_slot(u64 key, u32 slots) {
    const u32 x = (u32)key ^ (u32)(key >> 29);
    return (x * 0x9E3779B1u) >> (32 - __builtin_ctz(slots));
}

// One block per queued read whose hits fit in LDS: its hits are counted in an
// LDS hash table of locations (CAS on the key, atomic add on the count; ~0 is
// never a key, since genomes number fewer than 2^31), the locations with at
// least min_hits hits are compacted in place and ranked in the canonical
// order.  Reads with more hits are queued again for k_count_large.
__global__ __launch_bounds__(COUNT_TPB) void k_count_block(const u64 *__restrict__ hit_key,
                                                           const u64 *__restrict__ read_hs, u32 min_hits, u32 top_n,
                                                           u64 *__restrict__ stage_key, u32 *__restrict__ stage_hits,
                                                           u32 *__restrict__ ncand, const u32 *__restrict__ mid_list,
                                                           const u32 *__restrict__ n_mid, u32 *__restrict__ large_list,
                                                           u32 *__restrict__ n_large) {
    __shared__ u64 tkey[COUNT_SLOTS];
    __shared__ u32 tcnt[COUNT_SLOTS];
    const u32 nm = *n_mid;
    const u32 T = min_hits ? min_hits : 1;
    for (u32 li = blockIdx.x; li < nm; li += gridDim.x) {
        __syncthreads();  // the previous read is done with the LDS arrays
        const u64 r = mid_list[li];
        const u64 hs = read_hs[r], H = read_hs[r + 1] - hs;
        if (H > COUNT_CAP) {
            if (threadIdx.x == 0) large_list[atomicAdd(n_large, 1u)] = (u32)r;
            continue;
        }
        u32 slots = COUNT_TPB;  // a power of two >= 2H: load at most one half
        while (slots < 2 * H) slots <<= 1;
        for (u32 i = threadIdx.x; i < slots; i += COUNT_TPB) {
            tkey[i] = ~0ull;
            tcnt[i] = 0;
        }
        __syncthreads();
        for (u64 i = threadIdx.x; i < H; i += COUNT_TPB) {
            const u64 key = hit_key[hs + i];
            for (u32 sl = count_slot(key, slots);; sl = (sl + 1) & (slots - 1)) {
                u64 cur = tkey[sl];
                if (cur == ~0ull) {
                    cur = atomicCAS((unsigned long long *)&tkey[sl], ~0ull, (unsigned long long)key);
                    if (cur == ~0ull) cur = key;
                }
                if (cur == key) {
                    atomicAdd(&tcnt[sl], 1u);
                    break;
                }
            }
        }
        __syncthreads();
        // candidates to the front of the table, in slot order: a candidate
        // moves to index <= its slot, and every slot of a round is read
        // before the round's barrier, every move made after it
        u32 C = 0;
        for (u32 base = 0; base < slots; base += COUNT_TPB) {
            const u32 t = base + threadIdx.x;
            const u64 key = tkey[t];
            const u32 c = tcnt[t];
            const u32 is_c = key != ~0ull && c >= T;
            u32 tot;
            const u32 pre = block_exclusive_sum<COUNT_TPB, u32>(is_c, &tot);
            if (is_c) {
                tkey[C + pre] = key;
                tcnt[C + pre] = c;
            }
            C += tot;
        }
        __syncthreads();
        for (u32 a = threadIdx.x; a < C; a += COUNT_TPB) {
            const u64 ka = tkey[a];
            const u32 ha = tcnt[a];
            u32 rank = 0;
            for (u32 b = 0; b < C; b++) rank += cand_before(tcnt[b], tkey[b], ha, ka);
            if (top_n == 0 || rank < top_n) {
                stage_key[hs + rank] = ka;
                stage_hits[hs + rank] = ha;
            }
        }
        if (threadIdx.x == 0) ncand[r] = top_n && C > top_n ? top_n : C;
    }
}

// Reads with more hits than fit in LDS: sort in global memory, one block per
// read (rare: long reads against repetitive references).
__global__ __launch_bounds__(COUNT_TPB) void k_count_large(u64 *__restrict__ hit_key, const u64 *__restrict__ read_hs,
                                                           u32 min_hits, u32 top_n, u64 *__restrict__ stage_key,
                                                           u32 *__restrict__ stage_hits, u32 *__restrict__ ncand,
                                                           const u32 *__restrict__ large_list,
                                                           const u32 *__restrict__ n_large) {
    u32 nl = *n_large;
    for (u32 li = blockIdx.x; li < nl; li += gridDim.x) {
        u64 r = large_list[li];
        u64 hs = read_hs[r], H = read_hs[r + 1] - hs;
        u64 *key = hit_key + hs;
        u64 P = 1;
        while (P < H) P <<= 1;
        for (u64 k = 2; k <= P; k <<= 1)
            for (u64 j = k >> 1; j > 0; j >>= 1) {
                bool mirror = j == (k >> 1);
                for (u64 t = threadIdx.x; t < P / 2; t += COUNT_TPB) {
                    u64 i, l;
                    bitonic_pair(t, k, j, mirror, i, l);
                    if (l < H && key[i] > key[l]) {
                        u64 tmp = key[i];
                        key[i] = key[l];
                        key[l] = tmp;
                    }
                }
                __syncthreads();
            }
        u32 T = min_hits ? min_hits : 1;
        u64 C = 0;
        for (u64 c0 = 0; c0 < H; c0 += COUNT_TPB) {
            u64 i = c0 + threadIdx.x;
            u32 is_c = 0, c = 0;
            if (i < H && (i == 0 || key[i] != key[i - 1])) {
                u64 j = i + 1;
                while (j < H && key[j] == key[i]) j++;
                c = (u32)(j - i);
                is_c = c >= T;
            }
            u32 tot;
            u32 pre = block_exclusive_sum<COUNT_TPB, u32>(is_c, &tot);
            if (is_c) {
                stage_key[hs + C + pre] = key[i];
                stage_hits[hs + C + pre] = c;
            }
            C += tot;
        }
        __syncthreads();
        u64 *sk = stage_key + hs;
        u32 *sh = stage_hits + hs;
        P = 1;
        while (P < C) P <<= 1;
        for (u64 k = 2; k <= P; k <<= 1)
            for (u64 j = k >> 1; j > 0; j >>= 1) {
                bool mirror = j == (k >> 1);
                for (u64 t = threadIdx.x; t < P / 2; t += COUNT_TPB) {
                    u64 i, l;
                    bitonic_pair(t, k, j, mirror, i, l);
                    if (l < C && cand_before(sh[l], sk[l], sh[i], sk[i])) {
                        u64 tk = sk[i];
                        sk[i] = sk[l];
                        sk[l] = tk;
                        u32 th = sh[i];
                        sh[i] = sh[l];
                        sh[l] = th;
                    }
                }
                __syncthreads();
            }
        if (threadIdx.x == 0) ncand[r] = (u32)(top_n && C > top_n ? top_n : C);
        __syncthreads();
    }
}

__global__ void k_compact(const u64 *__restrict__ read_hs, const u32 *__restrict__ ncand,
                          const u64 *__restrict__ cand_off, u64 n, const u64 *__restrict__ stage_key,
                          const u32 *__restrict__ stage_hits, u32 *__restrict__ genome, i64 *__restrict__ diag,
                          u32 *__restrict__ hits, u32 *__restrict__ pair_read) {
    u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    u64 hs = read_hs[r], o = cand_off[r];
    for (u32 i = 0; i < ncand[r]; i++) {
        u64 key = stage_key[hs + i];
        genome[o + i] = key_genome(key);
        diag[o + i] = key_diag(key);
        hits[o + i] = stage_hits[hs + i];
        pair_read[o + i] = (u32)r;
    }
}

// ----------------------------------------------------------------- reduce --

// Where a read's taxon counts go: global 64-bit counters, or a block's LDS
// counters {unique[n_taxa], multi[n_taxa], unmapped} added to the global ones
// when the block ends.
struct GlobalCounts {
    unsigned long long *uniq, *multi, *unmapped;
    __device__ void unique_read(u32 t) const { atomicAdd(&uniq[t], 1ull); }
    __device__ void multi_read(u32 t) const { atomicAdd(&multi[t], 1ull); }
    __device__ void unmapped_read() const { atomicAdd(unmapped, 1ull); }
};

struct LdsCounts {
    u32 *c;
    u32 n_taxa;
    __device__ void unique_read(u32 t) const { atomicAdd(&c[t], 1u); }
    __device__ void multi_read(u32 t) const { atomicAdd(&c[n_taxa + t], 1u); }
    __device__ void unmapped_read() const { atomicAdd(&c[2 * n_taxa], 1u); }
};

// One read of the taxon step (Fig. 1 step 3a): its mapped taxa are the taxa of
// its accepted candidates at the smallest count; one taxon counts as unique,
// several as multi-mapped for each, none as unmapped.  Returns whether the
// read has an accepted candidate.
template <class Counts>
__device__ inline bool reduce_read(u64 cs, u64 ce, u32 E, const u32 *__restrict__ genome,
                                   const u16 *__restrict__ approx, const u32 *__restrict__ taxon,
                                   const Counts &out) {
    u32 best = 0xFFFFFFFFu;
    for (u64 c = cs; c < ce; c++)
        if (approx[c] <= E && approx[c] < best) best = approx[c];
    if (best == 0xFFFFFFFFu) {
        out.unmapped_read();
        return false;
    }
    // Distinct taxa of the accepted candidates at the best count.
    u32 ntax = 0, first = 0;
    for (u64 c = cs; c < ce; c++) {
        if (approx[c] != best) continue;
        u32 t = taxon[genome[c]];
        bool seen = false;
        for (u64 d = cs; d < c; d++)
            if (approx[d] == best && taxon[genome[d]] == t) seen = true;
        if (seen) continue;
        if (ntax == 0) first = t;
        ntax++;
    }
    if (ntax == 1) {
        out.unique_read(first);
        return true;
    }
    for (u64 c = cs; c < ce; c++) {
        if (approx[c] != best) continue;
        u32 t = taxon[genome[c]];
        bool seen = false;
        for (u64 d = cs; d < c; d++)
            if (approx[d] == best && taxon[genome[d]] == t) seen = true;
        if (!seen) out.multi_read(t);
    }
    return true;
}

constexpr int RED_TPB = 256;
constexpr u32 RED_LDS_TAXA = 2048;  // taxa counted per block in LDS

// Grid-stride over the reads.  Up to RED_LDS_TAXA taxa each block counts in
// LDS and adds its nonzero counters to the global ones at the end (one atomic
// per counter and block instead of one per read); more taxa count globally.
__global__ __launch_bounds__(RED_TPB) void k_reduce(const u64 *__restrict__ cand_off, u64 n,
                                                    const u32 *__restrict__ genome, const u16 *__restrict__ approx,
                                                    const u16 *__restrict__ read_E, const u32 *__restrict__ taxon,
                                                    u32 n_taxa, u8 *__restrict__ read_accepted,
                                                    unsigned long long *__restrict__ uniq,
                                                    unsigned long long *__restrict__ multi,
                                                    unsigned long long *__restrict__ unmapped) {
    __shared__ u32 cnt[2 * RED_LDS_TAXA + 1];
    const u64 stride = (u64)gridDim.x * RED_TPB;
    if (n_taxa > RED_LDS_TAXA) {
        const GlobalCounts out{uniq, multi, unmapped};
        for (u64 r = (u64)blockIdx.x * RED_TPB + threadIdx.x; r < n; r += stride)
            read_accepted[r] = reduce_read(cand_off[r], cand_off[r + 1], read_E[r], genome, approx, taxon, out);
        return;
    }
    const u32 nc = 2 * n_taxa + 1;
    for (u32 i = threadIdx.x; i < nc; i += RED_TPB) cnt[i] = 0;
    __syncthreads();
    const LdsCounts out{cnt, n_taxa};
    for (u64 r = (u64)blockIdx.x * RED_TPB + threadIdx.x; r < n; r += stride)
        read_accepted[r] = reduce_read(cand_off[r], cand_off[r + 1], read_E[r], genome, approx, taxon, out);
    __syncthreads();
    for (u32 i = threadIdx.x; i < nc; i += RED_TPB) {
        const u32 v = cnt[i];
        if (!v) continue;
        unsigned long long *dst = i < n_taxa ? &uniq[i] : i < 2 * n_taxa ? &multi[i - n_taxa] : unmapped;
        atomicAdd(dst, (unsigned long long)v);
    }
}

// The taxon step per request slot of a served batch: reads [slot_off[s],
// slot_off[s + 1]) count into counts[s] = {unique[n_taxa], multi[n_taxa],
// unmapped}.
__global__ void k_reduce_slots(const u64 *__restrict__ cand_off, u64 n, const u32 *__restrict__ genome,
                               const u16 *__restrict__ approx, const u16 *__restrict__ read_E,
                               const u32 *__restrict__ taxon, const u64 *__restrict__ slot_off, u32 n_slots,
                               unsigned long long *const *__restrict__ counts, u32 n_taxa) {
    u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    u32 lo = 0, hi = n_slots;  // last slot with slot_off[s] <= r
    while (hi - lo > 1) {
        u32 mid = (lo + hi) >> 1;
        if (slot_off[mid] <= r) lo = mid; else hi = mid;
    }
    unsigned long long *c = counts[lo];
    const GlobalCounts out{c, c + n_taxa, c + 2 * (u64)n_taxa};
    reduce_read(cand_off[r], cand_off[r + 1], read_E[r], genome, approx, taxon, out);
}

void launch_reduce_slots(const mt_result &res, const mt_index &ix, const u64 *slot_off, u32 n_slots,
                         unsigned long long *const *counts, hipStream_t s) {
    if (res.n_reads == 0 || n_slots == 0) return;
    k_reduce_slots<<<grid_for(res.n_reads, 256), 256, 0, s>>>(res.cand_off.p, res.n_reads, res.genome.p,
                                                              res.approx.p, res.read_E.p, ix.taxon.p, slot_off,
                                                              n_slots, counts, ix.n_taxa);
    MT_HIP(hipGetLastError());
}

// ----------------------------------------------------------------- driver --

void ReadBatch::prepare(const mt_seqs &reads, u32 e_mode, u32 e_value, hipStream_t s) {
    n = reads.n;
    flags.alloc(1);
    maxE.alloc(1);
    MT_HIP(hipMemsetAsync(flags.p, 0, sizeof(u32), s));
    MT_HIP(hipMemsetAsync(maxE.p, 0, sizeof(u32), s));
    read_E.alloc(n);
    if (n) {
        k_read_setup<<<grid_for(n, 256), 256, 0, s>>>(reads.offsets, n, e_mode, e_value, read_E.p, flags.p,
                                                      maxE.p);
        MT_HIP(hipGetLastError());
    }
    pack_sequences(reads, 65535, ERR_READ_TOO_LONG, "read longer than 65535 bases", planes, flags.p, nullptr, s);
}

void validate_query(const mt_query_params &q) {
    MT_REQUIRE(q.e_mode <= MT_E_FLOOR_PERMILLE, "unknown e_mode");
    MT_REQUIRE(q.e_mode != MT_E_FIXED || q.e_value <= 65534, "E must be at most 65534");
    MT_REQUIRE(q.mode <= MT_MODE_FUSED_GRAPH, "unknown mode");
    MT_REQUIRE(q.filter <= MT_FILTER_SHD, "unknown filter");
    MT_REQUIRE(q.strands <= 2, "strands must be 0, 1 or 2");
    MT_REQUIRE(q.reserved == 0, "reserved fields must be 0");
}

// Seeds, lookup, gather, count and select of the per-stage form: for every
// read its ncand[r] candidates at stage_key / stage_hits[read_hs[r] ...], in
// the canonical order with min_hits and top_n applied.
struct StagedCands {
    DBuf<u64> stage_key, read_hs;
    DBuf<u32> stage_hits, ncand;
    u64 H = 0;      // seed hits (bounds every candidate count)
    u32 max_E = 0;  // largest E of the reads
};

static void stage_seed_count(const mt_index &ix, const mt_query_params &q, const mt_seqs &reads, ReadBatch &rb,
                             StagedCands &sc, Timer &tm, hipStream_t s) {
    u64 n = reads.n;
    // seeds
    MinimizerPlan mp;
    // tiles of 256 k-mer starts fit short reads; long reads amortize the
    // window halo and the block over tiles of 1024
    const int tile = reads.n && reads.total / reads.n > 512 ? 1024 : 256;
    minimizer_plan(reads, rb.planes, ix.k, ix.w, tile, mp, s);
    tm.mark("seed_count");
    u32 hf[2];
    u64 n_min = 0;
    MT_HIP(hipMemcpyAsync(&hf[0], rb.flags.p, sizeof(u32), hipMemcpyDeviceToHost, s));
    MT_HIP(hipMemcpyAsync(&hf[1], rb.maxE.p, sizeof(u32), hipMemcpyDeviceToHost, s));
    read_back(s, mp.min_off.p + mp.tiles_cap, &n_min, sizeof(u64));
    check_flags(hf[0]);
    sc.max_E = hf[1];
    DBuf<u64> min_x(n_min), min_val(n_min);
    DBuf<u32> min_seq(n_min), min_pos(n_min), min_nocc(n_min);
    minimizer_emit(reads, rb.planes, ix.k, ix.w, mp, min_x.p, min_seq.p, min_pos.p, s);
    tm.mark("seed_emit");
    // lookup + gather
    if (n_min) {
        k_lookup<<<grid_for(n_min, 256), 256, 0, s>>>(min_x.p, n_min, ix.table.p, ix.nbuckets, min_val.p,
                                                      min_nocc.p);
        MT_HIP(hipGetLastError());
    }
    tm.mark("lookup");
    DBuf<u64> hit_off(n_min + 1);
    scan_u32(min_nocc.p, hit_off.p, n_min, s);
    u64 H = 0;
    read_back(s, hit_off.p + n_min, &H, sizeof(u64));
    sc.H = H;
    DBuf<u64> hit_key(H);
    sc.read_hs.alloc(n + 1);
    if (n_min) {
        k_gather<<<grid_for(n_min, 256), 256, 0, s>>>(min_pos.p, min_val.p, hit_off.p, n_min, ix.occ.p, hit_key.p);
        MT_HIP(hipGetLastError());
    }
    k_read_hits<<<grid_for(n + 1, 256), 256, 0, s>>>(mp.tile_off.p, mp.min_off.p, hit_off.p, n, sc.read_hs.p);
    MT_HIP(hipGetLastError());
    tm.mark("gather");
    // count + select
    sc.stage_key.alloc(H);
    sc.stage_hits.alloc(H);
    sc.ncand.alloc(n);
    DBuf<u32> mid_list(n), large_list(n), lists(2);
    u32 *n_mid = lists.p, *n_large = lists.p + 1;
    MT_HIP(hipMemsetAsync(lists.p, 0, 2 * sizeof(u32), s));
    last_stats().n_minimizers += n_min;
    last_stats().n_hits += H;
    if (n) {
        k_count_wave<<<grid_for(n, CW_WPB), 64 * CW_WPB, 0, s>>>(hit_key.p, sc.read_hs.p, n, q.min_hits, q.top_n,
                                                                  sc.stage_key.p, sc.stage_hits.p, sc.ncand.p,
                                                                  mid_list.p, n_mid);
        MT_HIP(hipGetLastError());
        k_count_block<<<count_blocks(), COUNT_TPB, 0, s>>>(hit_key.p, sc.read_hs.p, q.min_hits, q.top_n,
                                                           sc.stage_key.p, sc.stage_hits.p, sc.ncand.p, mid_list.p,
                                                           n_mid, large_list.p, n_large);
        MT_HIP(hipGetLastError());
        k_count_large<<<256, COUNT_TPB, 0, s>>>(hit_key.p, sc.read_hs.p, q.min_hits, q.top_n, sc.stage_key.p,
                                                sc.stage_hits.p, sc.ncand.p, large_list.p, n_large);
        MT_HIP(hipGetLastError());
    }
    tm.mark("count_select");
}

// Filter the candidates of res (pair_read indexes `reads`, whose planes are
// in rb) and reduce them per result read with read_E.
static void stage_filter_reduce(const mt_index &ix, const mt_query_params &q, const mt_seqs &reads,
                                const ReadBatch &rb, const u32 *pair_read, u64 cap, u32 max_E, const u16 *read_E,
                                mt_result &res, Timer &tm, hipStream_t s) {
    const u64 n = res.n_reads;
    FilterArgs fa{};
    fa.pair_read = pair_read;
    fa.pair_genome = res.genome.p;
    fa.pair_diag = res.diag.p;
    fa.pair_E = nullptr;
    fa.read_E = rb.read_E.p;
    fa.n_dev = res.cand_off.p + n;
    fa.n_host = cap;
    fa.n_reads = reads.n;
    fa.read_off = reads.offsets;
    fa.read_blk = rb.planes.blk_off.p;
    fa.read_lohi = rb.planes.lohi.p;
    fa.read_nb = rb.planes.nb.p;
    fa.n_genomes = ix.n_genomes;
    fa.meta = ix.meta.p;
    fa.ref_lohi = ix.ref.lohi.p;
    fa.ref_nb = ix.ref.nb.p;
    fa.approx = res.approx.p;
    fa.accept = res.accept.p;
    fa.flags = rb.flags.p;
    if (q.filter == MT_FILTER_OBSTACLE) {
        launch_filter(fa, cap, max_E, s, &tm);
    } else {
        launch_filter_simple(fa, cap, q.filter, s);
        tm.mark("filter");
    }
    // reduce
    if (n) {
        const unsigned blocks = std::min<u64>(grid_for(n, RED_TPB), (u64)count_blocks() / 2);
        k_reduce<<<blocks, RED_TPB, 0, s>>>(res.cand_off.p, n, res.genome.p, res.approx.p, read_E, ix.taxon.p,
                                            ix.n_taxa, res.read_accepted.p, (unsigned long long *)res.uniq.p,
                                            (unsigned long long *)res.multi.p,
                                            (unsigned long long *)res.unmapped.p);
        MT_HIP(hipGetLastError());
    }
    tm.mark("reduce");
}

void classify_per_stage(const mt_index &ix, const mt_query_params &q, const mt_seqs &reads, ReadBatch &rb,
                        mt_result &res, Timer &tm, hipStream_t s) {
    const u64 n = reads.n;
    StagedCands sc;
    stage_seed_count(ix, q, reads, rb, sc, tm, s);
    // candidates
    u64 cap = q.top_n ? std::min<u64>(sc.H, n * (u64)q.top_n) : sc.H;
    res.alloc_cands(cap);
    scan_u32(sc.ncand.p, res.cand_off.p, n, s);
    DBuf<u32> pair_read(cap);
    if (n) {
        k_compact<<<grid_for(n, 256), 256, 0, s>>>(sc.read_hs.p, sc.ncand.p, res.cand_off.p, n, sc.stage_key.p,
                                                   sc.stage_hits.p, res.genome.p, res.diag.p, res.hits.p,
                                                   pair_read.p);
        MT_HIP(hipGetLastError());
    }
    tm.mark("compact");
    stage_filter_reduce(ix, q, reads, rb, pair_read.p, cap, sc.max_E, rb.read_E.p, res, tm, s);
}

// ------------------------------------------------------------ both strands --

// Complement of an ASCII base (either case); N and any other byte unchanged,
// so that invalid bytes are still refused by the packing step.
__device__ inline u8 complement_base(u8 c) {
    switch (c) {
    case 'A': return 'T';
    case 'C': return 'G';
    case 'G': return 'C';
    case 'T': return 'A';
    case 'a': return 't';
    case 'c': return 'g';
    case 'g': return 'c';
    case 't': return 'a';
    default: return c;
    }
}

// Offsets of the two-strand read set: sequence r is read r and sequence
// n + r its reverse complement, the reverse complements stored after all the
// reads (at total + off[r]).  Checks the caller's offsets as the packing step
// does.
__global__ void k_strand_offsets(const u64 *__restrict__ off, u64 n, u64 total, u64 *__restrict__ off2,
                                 u32 *__restrict__ flags) {
    const u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > n) return;
    if (r == n) {
        off2[2 * n] = 2 * total;
        return;
    }
    const u64 a = off[r], b = off[r + 1];
    if (b < a || b > total || (r == 0 && a != 0) || (r == n - 1 && b != total)) atomicOr(flags, ERR_OFFSETS);
    off2[r] = a;
    off2[n + r] = total + a;
}

constexpr int SR_WPB = 4;  // reads (one wavefront each) per block

// One wavefront per read: its reverse complement at rev + off[r] (the reads
// themselves are one device copy).  Runs only after the offsets passed
// k_strand_offsets.
__global__ __launch_bounds__(64 * SR_WPB) void k_strand_revcomp(const u8 *__restrict__ seq,
                                                                const u64 *__restrict__ off, u64 n,
                                                                u8 *__restrict__ rev) {
    const u64 lane = threadIdx.x & 63;
    const u64 stride = (u64)gridDim.x * SR_WPB;
    for (u64 r = (u64)blockIdx.x * SR_WPB + (threadIdx.x >> 6); r < n; r += stride) {
        const u64 a = off[r], m = off[r + 1] - a;
        const u8 *src = seq + a;
        u8 *dst = rev + a;
        for (u64 j = lane; j < m; j += 64) dst[m - 1 - j] = complement_base(src[j]);
    }
}

// Candidates kept per read over both strands: the union, cut at top_n.
__global__ void k_strand_count(const u32 *__restrict__ ncand, u64 n, u32 top_n, u32 *__restrict__ nmerged) {
    const u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const u32 c = ncand[r] + ncand[n + r];
    nmerged[r] = top_n && c > top_n ? top_n : c;
}

// Merges the two sorted candidate lists of read r (forward: sequence r,
// reverse: n + r) in the order (hits desc, genome, diag, strand), keeping the
// first nmerged; pair_read names the oriented sequence the filter reads.
__global__ void k_strand_merge(const u64 *__restrict__ read_hs, const u32 *__restrict__ ncand,
                               const u64 *__restrict__ cand_off, u64 n, const u64 *__restrict__ stage_key,
                               const u32 *__restrict__ stage_hits, const u16 *__restrict__ read_E2,
                               u32 *__restrict__ genome, i64 *__restrict__ diag, u32 *__restrict__ hits,
                               u8 *__restrict__ strand, u32 *__restrict__ pair_read, u16 *__restrict__ read_E) {
    const u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const u64 h0 = read_hs[r], h1 = read_hs[n + r];
    const u32 n0 = ncand[r], n1 = ncand[n + r];
    const u64 o = cand_off[r], cnt = cand_off[r + 1] - o;
    u32 i = 0, j = 0;
    for (u64 t = 0; t < cnt; t++) {
        bool take_fwd;
        if (i == n0) take_fwd = false;
        else if (j == n1) take_fwd = true;
        else {
            const u32 a = stage_hits[h0 + i], b = stage_hits[h1 + j];
            // the key orders (genome, diag); the forward strand wins a full tie
            take_fwd = a > b || (a == b && stage_key[h0 + i] <= stage_key[h1 + j]);
        }
        const u64 src = take_fwd ? h0 + i : h1 + j;
        const u64 key = stage_key[src];
        genome[o + t] = key_genome(key);
        diag[o + t] = key_diag(key);
        hits[o + t] = stage_hits[src];
        strand[o + t] = take_fwd ? 0 : 1;
        pair_read[o + t] = (u32)(take_fwd ? r : n + r);
        if (take_fwd) i++;
        else j++;
    }
    read_E[r] = read_E2[r];
}

// Candidates kept per read from a finished two-strand result (its sequence
// r is read r, n + r the reverse complement): the union, cut at top_n.
__global__ void k_strand_count_done(const u64 *__restrict__ cand_off2, u64 n, u32 top_n,
                                    u32 *__restrict__ nmerged) {
    const u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const u64 c = (cand_off2[r + 1] - cand_off2[r]) + (cand_off2[n + r + 1] - cand_off2[n + r]);
    nmerged[r] = top_n && c > top_n ? top_n : (u32)c;
}

// k_strand_merge over filtered lists: the filter values travel with their
// candidates (a candidate's value does not depend on the others).
__global__ void k_strand_merge_done(const u64 *__restrict__ cand_off2, u64 n, const u32 *__restrict__ genome2,
                                    const i64 *__restrict__ diag2, const u32 *__restrict__ hits2,
                                    const u16 *__restrict__ approx2, const u8 *__restrict__ accept2,
                                    const u16 *__restrict__ read_E2, const u64 *__restrict__ cand_off,
                                    u32 *__restrict__ genome, i64 *__restrict__ diag, u32 *__restrict__ hits,
                                    u16 *__restrict__ approx, u8 *__restrict__ accept, u8 *__restrict__ strand,
                                    u16 *__restrict__ read_E) {
    const u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    u64 i = cand_off2[r], j = cand_off2[n + r];
    const u64 e0 = cand_off2[r + 1], e1 = cand_off2[n + r + 1];
    const u64 o = cand_off[r], cnt = cand_off[r + 1] - o;
    for (u64 t = 0; t < cnt; t++) {
        bool take_fwd;
        if (i == e0) take_fwd = false;
        else if (j == e1) take_fwd = true;
        else {
            const u32 a = hits2[i], b = hits2[j];
            const u32 ga = genome2[i], gb = genome2[j];
            take_fwd = a > b || (a == b && (ga < gb || (ga == gb && diag2[i] <= diag2[j])));
        }
        const u64 src = take_fwd ? i : j;
        genome[o + t] = genome2[src];
        diag[o + t] = diag2[src];
        hits[o + t] = hits2[src];
        approx[o + t] = approx2[src];
        accept[o + t] = accept2[src];
        strand[o + t] = take_fwd ? 0 : 1;
        if (take_fwd) i++;
        else j++;
    }
    read_E[r] = read_E2[r];
}

// Both strands with the obstacle walk in a fused mode: the fused kernel over
// the two-strand read set (each orientation keeps its own top_n and is
// filtered), then one merge per read and the reduce per read.
static void both_strands_fused(const mt_index &ix, const mt_query_params &q, const mt_seqs &two, ReadBatch &rb,
                               mt_result &res, Timer &tm, hipStream_t s) {
    const u64 n = res.n_reads;
    mt_query_params q1 = q;
    q1.strands = 1;
    mt_result r2;
    mt_result_init(r2, two.n, ix.n_taxa, s);
    classify_fused(ix, q1, two, rb, r2, tm, s, q.mode == MT_MODE_FUSED_GRAPH);
    DBuf<u32> nmerged(n);
    if (n) {
        k_strand_count_done<<<grid_for(n, 256), 256, 0, s>>>(r2.cand_off.p, n, q.top_n, nmerged.p);
        MT_HIP(hipGetLastError());
    }
    scan_u32(nmerged.p, res.cand_off.p, n, s);
    u64 total = 0;
    read_back(s, res.cand_off.p + n, &total, sizeof total);
    res.alloc_cands(total);
    res.strand.alloc(total);
    if (n) {
        k_strand_merge_done<<<grid_for(n, 256), 256, 0, s>>>(
            r2.cand_off.p, n, r2.genome.p, r2.diag.p, r2.hits.p, r2.approx.p, r2.accept.p, r2.read_E.p,
            res.cand_off.p, res.genome.p, res.diag.p, res.hits.p, res.approx.p, res.accept.p, res.strand.p,
            res.read_E.p);
        MT_HIP(hipGetLastError());
        tm.mark("merge");
        const unsigned blocks = std::min<u64>(grid_for(n, RED_TPB), (u64)count_blocks() / 2);
        k_reduce<<<blocks, RED_TPB, 0, s>>>(res.cand_off.p, n, res.genome.p, res.approx.p, res.read_E.p,
                                            ix.taxon.p, ix.n_taxa, res.read_accepted.p,
                                            (unsigned long long *)res.uniq.p, (unsigned long long *)res.multi.p,
                                            (unsigned long long *)res.unmapped.p);
        MT_HIP(hipGetLastError());
        tm.mark("reduce");
    }
    res.n_cands = total;
}

// Both strands: reads and their reverse complements as one read set.  The
// obstacle walk in a fused mode goes through the fused kernel; otherwise the
// per-stage seeding and counting over the two-strand set, one merge per read,
// then the filter on the oriented sequences and the reduce per read.
static void classify_both_strands(const mt_index &ix, const mt_query_params &q, const mt_seqs &reads,
                                  ReadBatch &rb, mt_result &res, Timer &tm, hipStream_t s) {
    const u64 n = reads.n;
    MT_REQUIRE(n < (1ull << 31), "at most 2^31 - 1 reads per call on both strands");
    DBuf<u64> off2(2 * n + 1);
    DBuf<u8> seq2(2 * reads.total);
    {
        DBuf<u32> f(1);
        MT_HIP(hipMemsetAsync(f.p, 0, sizeof(u32), s));
        k_strand_offsets<<<grid_for(n + 1, 256), 256, 0, s>>>(reads.offsets, n, reads.total, off2.p, f.p);
        MT_HIP(hipGetLastError());
        u32 fh = 0;
        read_back(s, f.p, &fh, sizeof fh);  // the offsets decide every address below
        check_flags(fh);
    }
    if (n && reads.total)
        MT_HIP(hipMemcpyAsync(seq2.p, reads.seq, reads.total, hipMemcpyDeviceToDevice, s));
    if (n) {
        const unsigned blocks = (unsigned)std::min<u64>(grid_for(n, SR_WPB), 1u << 20);
        k_strand_revcomp<<<blocks, 64 * SR_WPB, 0, s>>>((const u8 *)reads.seq, reads.offsets, n,
                                                        seq2.p + reads.total);
        MT_HIP(hipGetLastError());
    }
    const mt_seqs two{(const char *)seq2.p, off2.p, 2 * n, 2 * reads.total};
    if (q.mode != MT_MODE_PER_STAGE && q.filter == MT_FILTER_OBSTACLE) {
        tm.mark("pack");
        both_strands_fused(ix, q, two, rb, res, tm, s);
        return;
    }
    rb.prepare(two, q.e_mode, q.e_value, s);
    tm.mark("pack");
    StagedCands sc;
    stage_seed_count(ix, q, two, rb, sc, tm, s);
    // merge the strands of each read
    DBuf<u32> nmerged(n);
    if (n) {
        k_strand_count<<<grid_for(n, 256), 256, 0, s>>>(sc.ncand.p, n, q.top_n, nmerged.p);
        MT_HIP(hipGetLastError());
    }
    const u64 cap = q.top_n ? std::min<u64>(sc.H, n * (u64)q.top_n) : sc.H;
    res.alloc_cands(cap);
    res.strand.alloc(cap);
    scan_u32(nmerged.p, res.cand_off.p, n, s);
    DBuf<u32> pair_read(cap);
    if (n) {
        k_strand_merge<<<grid_for(n, 256), 256, 0, s>>>(sc.read_hs.p, sc.ncand.p, res.cand_off.p, n, sc.stage_key.p,
                                                        sc.stage_hits.p, rb.read_E.p, res.genome.p, res.diag.p,
                                                        res.hits.p, res.strand.p, pair_read.p, res.read_E.p);
        MT_HIP(hipGetLastError());
    }
    tm.mark("compact");
    stage_filter_reduce(ix, q, two, rb, pair_read.p, cap, sc.max_E, res.read_E.p, res, tm, s);
    u32 f = 0;
    read_back(s, rb.flags.p, &f, sizeof f);
    check_flags(f);
    read_back(s, res.cand_off.p + n, &res.n_cands, sizeof(u64));
}

void mt_result_init(mt_result &res, u64 n, u32 n_taxa, hipStream_t s) {
    res.n_reads = n;
    res.n_taxa = n_taxa;
    res.cand_off.alloc(n + 1);
    res.read_accepted.alloc(n);
    res.read_E.alloc(n);
    res.uniq.alloc(n_taxa);
    res.multi.alloc(n_taxa);
    res.unmapped.alloc(1);
    MT_HIP(hipMemsetAsync(res.uniq.p, 0, (n_taxa ? n_taxa : 1) * sizeof(u64), s));
    MT_HIP(hipMemsetAsync(res.multi.p, 0, (n_taxa ? n_taxa : 1) * sizeof(u64), s));
    MT_HIP(hipMemsetAsync(res.unmapped.p, 0, sizeof(u64), s));
    if (n == 0) MT_HIP(hipMemsetAsync(res.cand_off.p, 0, sizeof(u64), s));
}

}  // namespace mt

void mt_result::alloc_cands(mt::u64 c) {
    cap = c;
    genome.alloc(c);
    diag.alloc(c);
    hits.alloc(c);
    approx.alloc(c);
    accept.alloc(c);
}

// ---------------------------------------------------------------------- ABI --

using mt::Error;

using mt::guarded;

namespace mt {

void classify_staged(const mt_index &ix, const mt_query_params &q, const mt_seqs &reads, ReadBatch &rb,
                     mt_result &res, Timer &tm, hipStream_t s) {
    if (q.strands == 2) {
        classify_both_strands(ix, q, reads, rb, res, tm, s);
        return;
    }
    rb.prepare(reads, q.e_mode, q.e_value, s);
    MT_HIP(hipMemcpyAsync(res.read_E.p, rb.read_E.p, (reads.n ? reads.n : 1) * sizeof(u16), hipMemcpyDeviceToDevice,
                          s));
    tm.mark("pack");
    classify_per_stage(ix, q, reads, rb, res, tm, s);
    u32 f = 0;
    read_back(s, rb.flags.p, &f, sizeof f);
    check_flags(f);
    read_back(s, res.cand_off.p + reads.n, &res.n_cands, sizeof(u64));
}

}  // namespace mt

extern "C" int mt_classify(const mt_index *index, const mt_query_params *params, const mt_seqs *reads,
                           void *stream, mt_result **out) {
    if (!index || !params || !reads || !out) {
        mt::set_last_error("mt_classify: null argument");
        return MT_EINVAL;
    }
    *out = nullptr;
    mt_result *res = new (std::nothrow) mt_result();
    if (!res) return MT_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    int rc = guarded("mt_classify", [&] {
        mt::validate_query(*params);
        MT_REQUIRE(reads->n == 0 || (reads->seq && reads->offsets), "null read arrays");
        mt::Timer tm;
        mt::last_stats() = mt_stats{};
        mt::last_stats().n_reads = reads->n;
        {
            mt::CallScope scope(s);
            tm.begin(s);
            mt::mt_result_init(*res, reads->n, index->n_taxa, s);
            mt::ReadBatch rb;
            if (params->mode != MT_MODE_PER_STAGE)
                mt::classify_fused(*index, *params, *reads, rb, *res, tm, s, params->mode == MT_MODE_FUSED_GRAPH);
            else
                mt::classify_staged(*index, *params, *reads, rb, *res, tm, s);
            mt::last_stats().n_cands = res->n_cands;
        }
        tm.finish();
    });
    if (rc != MT_OK) {
        delete res;
        return rc;
    }
    *out = res;
    return MT_OK;
}

extern "C" int mt_result_reads(const mt_result *res, uint64_t *n_reads, const uint64_t **cand_offsets,
                               const uint8_t **read_accepted, const uint16_t **read_E) {
    if (!res) {
        mt::set_last_error("mt_result_reads: null result");
        return MT_EINVAL;
    }
    if (n_reads) *n_reads = res->n_reads;
    if (cand_offsets) *cand_offsets = res->on_host ? res->h.cand_off.data() : res->cand_off.p;
    if (read_accepted) *read_accepted = res->on_host ? res->h.read_accepted.data() : res->read_accepted.p;
    if (read_E) *read_E = res->on_host ? res->h.read_E.data() : res->read_E.p;
    return MT_OK;
}

extern "C" int mt_result_cands(const mt_result *res, uint64_t *n_cands, const uint32_t **genome,
                               const int64_t **diag, const uint32_t **hits, const uint16_t **approx,
                               const uint8_t **accept) {
    if (!res) {
        mt::set_last_error("mt_result_cands: null result");
        return MT_EINVAL;
    }
    if (n_cands) *n_cands = res->n_cands;
    const bool h = res->on_host;
    if (genome) *genome = h ? res->h.genome.data() : res->genome.p;
    if (diag) *diag = h ? res->h.diag.data() : res->diag.p;
    if (hits) *hits = h ? res->h.hits.data() : res->hits.p;
    if (approx) *approx = h ? res->h.approx.data() : res->approx.p;
    if (accept) *accept = h ? res->h.accept.data() : res->accept.p;
    return MT_OK;
}

extern "C" int mt_result_taxa(const mt_result *res, uint32_t *n_taxa, const uint64_t **unique_reads,
                              const uint64_t **multi_reads, const uint64_t **unmapped) {
    if (!res) {
        mt::set_last_error("mt_result_taxa: null result");
        return MT_EINVAL;
    }
    if (n_taxa) *n_taxa = res->n_taxa;
    if (res->on_host) {
        const mt::u64 *c = res->h.counts.data();
        if (unique_reads) *unique_reads = c;
        if (multi_reads) *multi_reads = c + res->n_taxa;
        if (unmapped) *unmapped = c + 2 * (mt::u64)res->n_taxa;
        return MT_OK;
    }
    if (unique_reads) *unique_reads = res->uniq.p;
    if (multi_reads) *multi_reads = res->multi.p;
    if (unmapped) *unmapped = res->unmapped.p;
    return MT_OK;
}

extern "C" int mt_result_strands(const mt_result *res, const uint8_t **strand) {
    if (!res || !strand) {
        mt::set_last_error("mt_result_strands: null argument");
        return MT_EINVAL;
    }
    if (res->on_host)
        *strand = res->h.strand.empty() ? nullptr : res->h.strand.data();
    else
        *strand = res->strand.p;
    return MT_OK;
}

extern "C" int mt_result_on_host(const mt_result *res) { return res && res->on_host ? 1 : 0; }

extern "C" int mt_result_times(const mt_result *res, uint64_t *submit_ns, uint64_t *done_ns) {
    if (!res) {
        mt::set_last_error("mt_result_times: null result");
        return MT_EINVAL;
    }
    if (submit_ns) *submit_ns = res->submit_ns;
    if (done_ns) *done_ns = res->done_ns;
    return MT_OK;
}

extern "C" int mt_result_free(mt_result *res) {
    delete res;
    return MT_OK;
}

extern "C" int mt_filter_pairs_kind(const mt_index *index, const mt_seqs *reads, const uint32_t *pair_read,
                                    const uint32_t *pair_genome, const int64_t *pair_diag, const uint16_t *pair_E,
                                    uint64_t n_pairs, uint32_t kind, uint16_t *approx_out, uint8_t *accept_out,
                                    void *stream) {
    if (!index || !reads) {
        mt::set_last_error("mt_filter_pairs: null argument");
        return MT_EINVAL;
    }
    if (n_pairs && (!pair_read || !pair_genome || !pair_diag || !pair_E || !approx_out || !accept_out)) {
        mt::set_last_error("mt_filter_pairs: null pair array");
        return MT_EINVAL;
    }
    if (kind > MT_FILTER_SHD) {
        mt::set_last_error("mt_filter_pairs: unknown filter kind");
        return MT_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    return guarded("mt_filter_pairs", [&] {
        MT_REQUIRE(reads->n == 0 || (reads->seq && reads->offsets), "null read arrays");
        mt::CallScope scope(s);
        mt::ReadBatch rb;
        rb.prepare(*reads, MT_E_FIXED, 0, s);
        mt::FilterArgs fa{};
        fa.pair_read = pair_read;
        fa.pair_genome = pair_genome;
        fa.pair_diag = pair_diag;
        fa.pair_E = pair_E;
        fa.read_E = rb.read_E.p;
        fa.n_dev = nullptr;
        fa.n_host = n_pairs;
        fa.n_reads = reads->n;
        fa.read_off = reads->offsets;
        fa.read_blk = rb.planes.blk_off.p;
        fa.read_lohi = rb.planes.lohi.p;
        fa.read_nb = rb.planes.nb.p;
        fa.n_genomes = index->n_genomes;
        fa.meta = index->meta.p;
        fa.ref_lohi = index->ref.lohi.p;
        fa.ref_nb = index->ref.nb.p;
        fa.approx = approx_out;
        fa.accept = accept_out;
        fa.flags = rb.flags.p;
        if (kind == MT_FILTER_OBSTACLE)
            mt::launch_filter(fa, n_pairs, 0, s);
        else
            mt::launch_filter_simple(fa, n_pairs, kind, s);
        mt::u32 f = 0;
        mt::read_back(s, rb.flags.p, &f, sizeof f);
        mt::check_flags(f);
    });
}

extern "C" int mt_filter_pairs(const mt_index *index, const mt_seqs *reads, const uint32_t *pair_read,
                               const uint32_t *pair_genome, const int64_t *pair_diag, const uint16_t *pair_E,
                               uint64_t n_pairs, uint16_t *approx_out, uint8_t *accept_out, void *stream) {
    return mt_filter_pairs_kind(index, reads, pair_read, pair_genome, pair_diag, pair_E, n_pairs, MT_FILTER_OBSTACLE,
                                approx_out, accept_out, stream);
}
