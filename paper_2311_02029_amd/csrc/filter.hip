// The obstacle-count filter over explicit pair lists (Fig. 1 step 2d), used by
// the per-stage form, by the fused form's fallback and by mt_filter_pairs.
//
// Pairs are bucketed by their threshold E so that each bucket gets the
// kernel shaped for it (uneven batching):
//   E <= 7   groups of 16 lanes, 4 pairs per wavefront, one band row per lane
//   E <= 15  groups of 32 lanes, 2 pairs per wavefront
//   E <= 31  one pair per wavefront
//   E > 31   long reads: one pair per wavefront with the read and its
//            reference window staged in LDS; each lane owns a contiguous
//            strip of the 2E+1 rows, so one 128-base reference fetch per step
//            serves its whole strip (k_filter_long); pairs too large for its
//            LDS budget use the 64-lane kernel that fetches from global memory.
#include "classify.hpp"

namespace mt {

constexpr int N_CLASSES = 5;
constexpr int LONG_WPB = 4;
constexpr int LONG_BLOCKS = 640;  // 64-base blocks of read + window staged per wavefront

__device__ inline void pair_fields(const FilterArgs &a, u64 p, u32 &r, u32 &g, int &E, bool &ok, u32 &err) {
    r = a.pair_read[p];
    g = a.pair_genome[p];
    ok = true;
    err = 0;
    if (r >= a.n_reads || g >= a.n_genomes) {
        ok = false;
        err = ERR_PAIR_RANGE;
        E = 0;
        return;
    }
    E = a.pair_E ? a.pair_E[p] : a.read_E[r];
    if (E > 65534) {
        ok = false;
        err = ERR_E_TOO_LARGE;
    }
}

__device__ inline int read_len(const FilterArgs &a, u32 r) { return (int)(a.read_off[r + 1] - a.read_off[r]); }

// Blocks the long kernel stages for a pair: the read's (with its padding
// block) and the reference window from diag - E, long enough for a 128-base
// fetch at any column < m of any row.
__device__ inline void long_blocks(int m, int E, int &nrb, int &nwb) {
    nrb = (m + 63) / 64 + 1;
    nwb = ((m + 2 * E + 190) >> 6) + 2;
}

// Class of pair p (0..3: the bucket kernels; 4: the general kernel).
__device__ inline u8 pair_class(const FilterArgs &a, u64 p) {
    u32 r, g, err;
    int E;
    bool ok;
    pair_fields(a, p, r, g, E, ok, err);
    if (!ok) return 4;  // the general kernel reports the error
    if (E <= 7) return 0;
    if (E <= 15) return 1;
    if (E <= 31) return 2;
    int nrb, nwb;
    long_blocks(read_len(a, r), E, nrb, nwb);
    return nrb + nwb <= LONG_BLOCKS ? 3 : 4;
}

// Counting and placing pairs use one atomic per wavefront and class: the
// lanes of a class are ranked by ballot, and their lowest lane adds them all.
__global__ void k_pair_class(FilterArgs a, u64 n_cap, u32 *__restrict__ count, u8 *__restrict__ cls) {
    const u64 p = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    const u64 np = a.n_dev ? *a.n_dev : a.n_host;
    const bool active = p < np && p < n_cap;
    const int lane = threadIdx.x & 63;
    u8 c = 0xFF;
    if (active) {
        c = pair_class(a, p);
        cls[p] = c;
    }
    for (int k = 0; k < N_CLASSES; k++) {
        const u64 m = __ballot(c == k);
        if (m && lane == __builtin_ctzll(m)) atomicAdd(&count[k], (u32)__builtin_popcountll(m));
    }
}

__global__ void k_pair_scatter(FilterArgs a, u64 n_cap, const u8 *__restrict__ cls, const u32 *__restrict__ base,
                               u32 *__restrict__ cursor, u32 *__restrict__ idx) {
    const u64 p = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    const u64 np = a.n_dev ? *a.n_dev : a.n_host;
    const bool active = p < np && p < n_cap;
    const int lane = threadIdx.x & 63;
    const u8 c = active ? cls[p] : (u8)0xFF;
    for (int k = 0; k < N_CLASSES; k++) {
        const u64 m = __ballot(c == k);
        if (!m) continue;
        const int leader = __builtin_ctzll(m);
        u32 first = 0;
        if (lane == leader) first = atomicAdd(&cursor[k], (u32)__builtin_popcountll(m));
        first = __shfl(first, leader, 64);
        if (c == k) idx[base[k] + first + __builtin_popcountll(m & ((1ull << lane) - 1))] = (u32)p;
    }
}

// G lanes per pair over the bucket idx[0, n).
template <int G>
__global__ __launch_bounds__(256) void k_filter(FilterArgs a, const u32 *__restrict__ idx, u64 n) {
    u64 tid = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    u64 t = tid / G;
    int lane = (int)(tid % G);
    if (t >= n) return;
    u64 p = idx[t];
    u32 r, g, err;
    int E;
    bool ok;
    pair_fields(a, p, r, g, E, ok, err);
    if (!ok) {
        if (lane == 0) {
            atomicOr(a.flags, err);
            a.approx[p] = 0xFFFF;
            a.accept[p] = 0;
        }
        return;
    }
    PairView v;
    v.qlohi = a.read_lohi + a.read_blk[r];
    v.qnb = a.read_nb + a.read_blk[r];
    v.m = read_len(a, r);
    GenomeMeta gm = a.meta[g];
    v.rlohi = a.ref_lohi + gm.blk;
    v.rnb = a.ref_nb + gm.blk;
    v.L = (i64)gm.len;
    v.has_n = meta_has_n(gm);
    v.diag = a.pair_diag[p];
    int approx = obstacle_walk<G>(v, E, lane);
    if (lane == 0) {
        a.approx[p] = (u16)approx;
        a.accept[p] = approx <= E;
    }
}

__device__ inline void lds_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 64 bases from position p of planes staged in LDS (p >= 0, block p/64 + 1 staged).
__device__ inline Bits64 lds_bits(const u64x2 *lohi, const u64 *nb, i64 p) {
    u64 b = (u64)p >> 6;
    u32 s = (u32)p & 63u;
    u64x2 x0 = lohi[b], x1 = lohi[b + 1];
    Bits64 r;
    r.lo = funnel(x0.lo, x1.lo, s);
    r.hi = funnel(x0.hi, x1.hi, s);
    r.nb = funnel(nb[b], nb[b + 1], s);
    return r;
}

// Long reads / large E: one wavefront per pair, planes in LDS.
__global__ __launch_bounds__(64 * LONG_WPB) void k_filter_long(FilterArgs a, const u32 *__restrict__ idx, u64 n) {
    __shared__ u64x2 s_lohi[LONG_WPB][LONG_BLOCKS];
    __shared__ u64 s_nb[LONG_WPB][LONG_BLOCKS];
    const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    u64x2 *L = s_lohi[wid];
    u64 *NB = s_nb[wid];
    for (u64 t = (u64)blockIdx.x * LONG_WPB + wid; t < n; t += (u64)gridDim.x * LONG_WPB) {
        const u64 p = idx[t];
        u32 r, g, err;
        int E;
        bool ok;
        pair_fields(a, p, r, g, E, ok, err);  // bucketed pairs are valid
        const int m = read_len(a, r);
        const i64 diag = a.pair_diag[p];
        const GenomeMeta gm = a.meta[g];
        int nrb, nwb;
        long_blocks(m, E, nrb, nwb);
        const i64 b0 = (diag - E) >> 6;  // first window block (floor)
        const i64 gblocks = ((i64)gm.len + 63) / 64 + 1;
        const u64 rb = a.read_blk[r];
        for (int b = lane; b < nrb; b += 64) {
            L[b] = a.read_lohi[rb + b];
            NB[b] = a.read_nb[rb + b];
        }
        for (int b = lane; b < nwb; b += 64) {
            const i64 gb = b0 + b;
            u64x2 v{0ull, 0ull};
            u64 nbv = ~0ull;
            if (gb >= 0 && gb < gblocks) {
                v = a.ref_lohi[gm.blk + (u64)gb];
                nbv = a.ref_nb[gm.blk + (u64)gb];
            }
            L[nrb + b] = v;
            NB[nrb + b] = nbv;
        }
        lds_wave_sync();
        const u64x2 *WL = L + nrb;
        const u64 *WN = NB + nrb;
        const i64 wbase = diag - 64 * b0;  // window offset of (row 0, column 0)
        // lane owns the contiguous rows [r0, r1): one 128-base reference fetch
        // per step serves all of them through funnel shifts
        const int rows = 2 * E + 1;
        const int S = (rows + 63) / 64;
        const int r0 = min(lane * S, rows), r1 = min(r0 + S, rows);
        int j = 0, c = 0;
        for (;;) {
            const Bits64 q0 = lds_bits(L, NB, j);
            int best = 0;
            for (int s0 = r0; s0 < r1; s0 += 64) {  // chunks of <= 64 rows (funnel shifts < 64)
                const i64 pos = wbase + (s0 - E) + j;  // window offset of (row s0, column j)
                const Bits64 wa = lds_bits(WL, WN, pos), wb = lds_bits(WL, WN, pos + 64);
                const int cnt = min(64, r1 - s0);
                for (int i = 0; i < cnt; i++) {
                    Bits64 w;
                    w.lo = funnel(wa.lo, wb.lo, (u32)i);
                    w.hi = funnel(wa.hi, wb.hi, (u32)i);
                    w.nb = funnel(wa.nb, wb.nb, (u32)i);
                    u64 mm = mismatch(q0, w);
                    int run;
                    if (mm) {
                        run = (int)__builtin_ctzll(mm);
                    } else {  // 64 matching columns: continue word by word
                        run = 64;
                        while (j + run < m) {
                            mm = mismatch(lds_bits(L, NB, j + run), lds_bits(WL, WN, pos + i + run));
                            if (mm) {
                                run += (int)__builtin_ctzll(mm);
                                break;
                            }
                            run += 64;
                        }
                    }
                    best = max(best, min(run, m - j));
                }
            }
            best = group_max<64>(best);
            j += best;
            if (j >= m) break;
            c += 1;
            if (c > E) break;
            j += 1;
        }
        const int ap = c < E + 1 ? c : E + 1;
        if (lane == 0) {
            a.approx[p] = (u16)ap;
            a.accept[p] = ap <= E;
        }
        lds_wave_sync();
    }
}

void launch_filter(const FilterArgs &a, u64 n_cap, u32 /*max_E*/, hipStream_t s) {
    if (n_cap == 0) return;
    DBuf<u32> count(N_CLASSES), cursor(N_CLASSES), base(N_CLASSES), idx(n_cap);
    DBuf<u8> cls(n_cap);
    MT_HIP(hipMemsetAsync(count.p, 0, N_CLASSES * sizeof(u32), s));
    MT_HIP(hipMemsetAsync(cursor.p, 0, N_CLASSES * sizeof(u32), s));
    k_pair_class<<<grid_for(n_cap, 256), 256, 0, s>>>(a, n_cap, count.p, cls.p);
    MT_HIP(hipGetLastError());
    u32 hc[N_CLASSES];
    read_back(s, count.p, hc, sizeof hc);
    u32 hb[N_CLASSES];
    u32 acc = 0;
    for (int c = 0; c < N_CLASSES; c++) {
        hb[c] = acc;
        acc += hc[c];
    }
    if (acc == 0) return;
    MT_HIP(hipMemcpyAsync(base.p, hb, sizeof hb, hipMemcpyHostToDevice, s));
    k_pair_scatter<<<grid_for(n_cap, 256), 256, 0, s>>>(a, n_cap, cls.p, base.p, cursor.p, idx.p);
    MT_HIP(hipGetLastError());
    if (hc[0]) k_filter<16><<<grid_for((u64)hc[0] * 16, 256), 256, 0, s>>>(a, idx.p + hb[0], hc[0]);
    if (hc[1]) k_filter<32><<<grid_for((u64)hc[1] * 32, 256), 256, 0, s>>>(a, idx.p + hb[1], hc[1]);
    if (hc[2]) k_filter<64><<<grid_for((u64)hc[2] * 64, 256), 256, 0, s>>>(a, idx.p + hb[2], hc[2]);
    if (hc[3]) {
        u64 blocks = ((u64)hc[3] + LONG_WPB - 1) / LONG_WPB;
        if (blocks > 4096) blocks = 4096;
        k_filter_long<<<(unsigned)blocks, 64 * LONG_WPB, 0, s>>>(a, idx.p + hb[3], hc[3]);
    }
    if (hc[4]) k_filter<64><<<grid_for((u64)hc[4] * 64, 256), 256, 0, s>>>(a, idx.p + hb[4], hc[4]);
    MT_HIP(hipGetLastError());
}

}  // namespace mt
