// The obstacle-count filter over explicit pair lists (Fig. 1 step 2d), used by
// the per-stage form, by the fused form's fallback and by mt_filter_pairs.
//
// Pairs are bucketed by their threshold E, and long pairs by the LDS they
// need, so that each bucket gets the kernel shaped for it (uneven batching):
//   E <= 7   groups of G lanes per pair, one band row per lane (G = 16, 32 or 64)
//   E <= 15  G = 32 or 64
//   E <= 31  G = 64: one pair per wavefront
//   E > 31   long reads, four bins by the 64-base blocks of read plus
//            reference window they stage in LDS (<= 96, 192, 384, 768): one
//            pair per wavefront, each lane owning a contiguous strip of the
//            2E+1 rows, compared 32 columns at a time from three window
//            dwords per chunk of 32 rows, with the bin's LDS tile and W
//            wavefronts per block;
//            or the rows-in-lanes kernel reading the window from global memory
//   larger   the rows-in-lanes kernel.
// The variant of each bucket (G, W, layout) is chosen by the autotuner
// (mt_autotune) or set by mt_tune_set; every variant gives the same result.
#include <mutex>
#include <string>

#include "classify.hpp"

namespace mt {

constexpr int N_CLASSES = 8;  // E<=7, E<=15, E<=31, four long bins, general
constexpr int CLS_LONG = 3, LONG_BINS = 4, CLS_GENERAL = 7;
constexpr int LONG_CAP[LONG_BINS] = {96, 192, 384, 768};  // 64-base blocks staged per wavefront
constexpr int LDS_BLOCK_BYTES = 24;                        // {lo, hi} + nb of one 64-base block
constexpr int LONG_LDS_MAX = 64 * 1024;                    // per workgroup

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
    if (!ok) return CLS_GENERAL;  // the general kernel reports the error
    if (E <= 7) return 0;
    if (E <= 15) return 1;
    if (E <= 31) return 2;
    int nrb, nwb;
    long_blocks(read_len(a, r), E, nrb, nwb);
    for (int b = 0; b < LONG_BINS; b++)
        if (nrb + nwb <= LONG_CAP[b]) return (u8)(CLS_LONG + b);
    return CLS_GENERAL;
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

// The obstacle walk of one pair by a group of G lanes with one band row per
// lane (2E + 1 <= G) for a read of at most 64 NW bases: lane l builds row
// d = l - E in NW registers (rows past 2E + 1 read as all obstacles and never
// lead), then every step is a run length per lane from its registers and a
// maximum over the group.  Returns min(count, E + 1).
template <int G, int NW>
__device__ inline int walk_in_registers(const PairView &v, int E, int lane) {
    const int nwr = (v.m + 63) / 64 + 1;  // the read's blocks, its padding block included
    u64 row[NW];
    if (lane < 2 * E + 1) {
        auto qword = [&](int w) {
            Bits64 q;
            if (w < nwr) {
                const u64x2 x = v.qlohi[w];
                q.lo = x.lo;
                q.hi = x.hi;
                q.nb = v.qnb[w];
            } else {
                q.lo = q.hi = 0;
                q.nb = ~0ull;
            }
            return q;
        };
        band_row<NW>(qword, v.rlohi, v.rnb, v.L, v.has_n, v.diag + (lane - E), row);
    } else {
#pragma unroll
        for (int w = 0; w < NW; w++) row[w] = ~0ull;
    }
    int j = 0, c = 0;
    for (;;) {
        j += group_max<G>(reg_run<NW>(row, j));
        if (j >= v.m) break;
        c += 1;
        if (c > E) break;
        j += 1;
    }
    return c < E + 1 ? c : E + 1;
}

// G lanes per pair over the bucket idx[0, n).// G lanes per pair over the bucket idx[0, n).
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
    const int rows = 2 * E + 1;
    int approx;
    // One band row per lane and reads of up to 256 bases (the E <= 7 / 15 / 31
    // buckets but their reads of 257+ bases): the row's mismatch words are
    // built once, from one fetch of each reference block it spans, and the
    // walk runs on registers.  The branch is uniform over the group.  (A
    // five-word path for reads up to 320 bases took the kernel from 69 to 81
    // registers and 7 to 5 wavefronts per SIMD.)
    if (rows <= G && v.m <= 256)
        approx = walk_in_registers<G, 4>(v, E, lane);
    else
        approx = obstacle_walk<G>(v, E, lane);
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

// 64 bases from position p of planes staged in LDS (p >= 0, block p/64 + 1
// staged); kWithN = false reads the N plane as zero.
template <bool kWithN = true>
__device__ inline Bits64 lds_bits(const u64x2 *lohi, const u64 *nb, i64 p) {
    u64 b = (u64)p >> 6;
    u32 s = (u32)p & 63u;
    u64x2 x0 = lohi[b], x1 = lohi[b + 1];
    Bits64 r;
    r.lo = funnel(x0.lo, x1.lo, s);
    r.hi = funnel(x0.hi, x1.hi, s);
    r.nb = kWithN ? funnel(nb[b], nb[b + 1], s) : 0ull;
    return r;
}

// Dword k (bases 32k .. 32k+31) of the lo (pl = 0) or hi (pl = 1) plane of
// {lo, hi} blocks staged in LDS, and of the nb plane.
__device__ inline u32 plane_dw(const u64x2 *lohi, int pl, u32 k) {
    return reinterpret_cast<const u32 *>(lohi)[(k >> 1) * 4 + pl * 2 + (k & 1)];
}
__device__ inline u32 nb_dw(const u64 *nb, u32 k) { return reinterpret_cast<const u32 *>(nb)[k]; }

// One chunk of a lane's rows in the long walk, without branches (a divergent
// branch costs scalar exec-mask instructions): row i's 32 window bases are
// bits [i, i + 32) of (x1:x0) per plane.  The trip count is the wave's rows
// per chunk (uniform); with kTail, rows past the lane's cnt repeat its last
// row, which leaves the maximum unchanged.  bmax gets the largest run (all
// ones for a row whose 32 columns match: the find-first-one value for 0), and
// full the rows whose 32 columns all match, to be continued by the caller.
template <bool kWithN, bool kTail>
__device__ inline void chunk_rows(u32 xl0, u32 xl1, u32 xh0, u32 xh1, u32 xn0, u32 xn1, u32 ql, u32 qh, u32 qn,
                                  int SC, int cnt, u32 &full, u32 &bmax) {
#pragma unroll 4
    for (int i = 0; i < SC; i++) {
        const u32 ie = kTail ? (u32)min(i, cnt - 1) : (u32)i;
        const u32 wl = __builtin_amdgcn_alignbit(xl1, xl0, ie);
        const u32 wh = __builtin_amdgcn_alignbit(xh1, xh0, ie);
        const u32 wn = kWithN ? __builtin_amdgcn_alignbit(xn1, xn0, ie) : 0u;
        // (ql ^ wl) | (qh ^ wh) | qn | wn in two (three with the window's N
        // plane) 3-input bit operations: truth table 0xde takes (x, z, y) to
        // (x ^ y) | z
        const u32 t = __builtin_amdgcn_bitop3_b32(ql, kWithN ? (qn | wn) : qn, wl, 0xde);
        const u32 mm = __builtin_amdgcn_bitop3_b32(qh, t, wh, 0xde);
        const u32 run = mm ? (u32)__builtin_ctz(mm) : ~0u;
        full |= (run >> 31) << i;
        bmax = max(bmax, run);
    }
    if (kTail) full &= cnt >= 32 ? ~0u : (1u << cnt) - 1u;  // the repeated rows are not continued
}

// The obstacle walk of one pair over planes staged in LDS (read at L / NB,
// window at WL / WN, row 0 and column 0 at window offset wbase), rows in
// contiguous strips per lane; returns the obstacle count.  kWithN = false
// leaves the window's N plane out: only for pairs whose compared window lies
// inside a genome without N, where that plane is zero.
template <bool kWithN>
__device__ inline int long_walk(const u64x2 *L, const u64 *NB, const u64x2 *WL, const u64 *WN, i64 wbase, int m,
                                int E, int lane) {
    // lane owns the contiguous rows [r0, r1); per step each chunk of 32 of
    // them is compared over 32 columns from three window dwords per plane
    // (one alignbit per plane and row), and only a row with no obstacle
    // in those columns continues 64 columns at a time
    const int rows = 2 * E + 1;
    const int S = (rows + 63) / 64;
    // every lane takes S rows; the last lanes repeat the band's last rows,
    // which leaves the maximum unchanged
    const int r0 = min(lane * S, rows - S), r1 = r0 + S;
    const int SC = min(32, S);
    int j = 0, c = 0;
    for (;;) {
        // 32 read bases from j (one alignbit per plane)
        const u32 kq = (u32)j >> 5, sq = (u32)j & 31u;
        const u32 ql = __builtin_amdgcn_alignbit(plane_dw(L, 0, kq + 1), plane_dw(L, 0, kq), sq);
        const u32 qh = __builtin_amdgcn_alignbit(plane_dw(L, 1, kq + 1), plane_dw(L, 1, kq), sq);
        const u32 qn = __builtin_amdgcn_alignbit(nb_dw(NB, kq + 1), nb_dw(NB, kq), sq);
        const int left = m - j;
        int best = 0;
        for (int s0 = r0; s0 < r1; s0 += 32) {  // chunks of <= 32 rows
            // window bases of rows s0.. at column j start at p0; three
            // dwords per plane cover every row of the chunk
            const i64 p0 = wbase + (s0 - E) + j;
            const u32 k0 = (u32)((u64)p0 >> 5), sh0 = (u32)p0 & 31u;
            const u32 l0 = plane_dw(WL, 0, k0), l1 = plane_dw(WL, 0, k0 + 1), l2 = plane_dw(WL, 0, k0 + 2);
            const u32 h0 = plane_dw(WL, 1, k0), h1 = plane_dw(WL, 1, k0 + 1), h2 = plane_dw(WL, 1, k0 + 2);
            u32 n0 = 0, n1 = 0, n2 = 0;
            if constexpr (kWithN) {
                n0 = nb_dw(WN, k0);
                n1 = nb_dw(WN, k0 + 1);
                n2 = nb_dw(WN, k0 + 2);
            }
            const int cnt = min(32, r1 - s0);
            // Bits [sh0, sh0 + 64) of the three dwords: row i's 32 window
            // bases are bits [i, i + 32) of them, one alignbit per plane.
            const u32 xl0 = __builtin_amdgcn_alignbit(l1, l0, sh0), xl1 = __builtin_amdgcn_alignbit(l2, l1, sh0);
            const u32 xh0 = __builtin_amdgcn_alignbit(h1, h0, sh0), xh1 = __builtin_amdgcn_alignbit(h2, h1, sh0);
            u32 xn0 = 0, xn1 = 0;
            if constexpr (kWithN) {
                xn0 = __builtin_amdgcn_alignbit(n1, n0, sh0);
                xn1 = __builtin_amdgcn_alignbit(n2, n1, sh0);
            }
            u32 full = 0, bmax = 0;
            if (S <= 32)  // every chunk row is the lane's own: no tail to mask
                chunk_rows<kWithN, false>(xl0, xl1, xh0, xh1, xn0, xn1, ql, qh, qn, SC, cnt, full, bmax);
            else
                chunk_rows<kWithN, true>(xl0, xl1, xh0, xh1, xn0, xn1, ql, qh, qn, SC, cnt, full, bmax);
            best = max(best, min((int)min(bmax, 32u), left));
            // 32 matching columns: continue 64 at a time
            while (full) {
                const int i = (int)__builtin_ctz(full);
                full &= full - 1;
                int run = 32;
                const i64 pos = p0 + i;
                while (j + run < m) {
                    const u64 m2 = mismatch(lds_bits(L, NB, j + run), lds_bits<kWithN>(WL, WN, pos + run));
                    if (m2) {
                        run += (int)__builtin_ctzll(m2);
                        break;
                    }
                    run += 64;
                }
                best = max(best, min(run, left));
            }
        }
        best = group_max<64>(best);
        j += best;
        if (j >= m) break;
        c += 1;
        if (c > E) break;
        j += 1;
    }
    return c;
}

// Long reads / large E: one wavefront per pair, planes in LDS (`tile` blocks
// per wavefront, at least the pairs' nrb + nwb; blockDim.x / 64 wavefronts).
__global__ __launch_bounds__(512) void k_filter_long(FilterArgs a, const u32 *__restrict__ idx, u64 n, int tile) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int wpb = blockDim.x >> 6;
    const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    u64x2 *L = (u64x2 *)(lds + (size_t)wid * tile * LDS_BLOCK_BYTES);
    u64 *NB = (u64 *)(lds + (size_t)wid * tile * LDS_BLOCK_BYTES + (size_t)tile * 16);
    for (u64 t = (u64)blockIdx.x * wpb + wid; t < n; t += (u64)gridDim.x * wpb) {
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
        const bool with_n = meta_has_n(gm) || diag - E < 0 || diag + m + E > (i64)gm.len;
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
                nbv = with_n ? a.ref_nb[gm.blk + (u64)gb] : 0ull;
            }
            L[nrb + b] = v;
            NB[nrb + b] = nbv;
        }
        lds_wave_sync();
        const u64x2 *WL = L + nrb;
        const u64 *WN = NB + nrb;
        const i64 wbase = diag - 64 * b0;  // window offset of (row 0, column 0)
        // every compared window position inside a genome without N: no N plane
        const int c = with_n ? long_walk<true>(L, NB, WL, WN, wbase, m, E, lane)
                             : long_walk<false>(L, NB, WL, WN, wbase, m, E, lane);
        const int ap = c < E + 1 ? c : E + 1;
        if (lane == 0) {
            a.approx[p] = (u16)ap;
            a.accept[p] = ap <= E;
        }
        lds_wave_sync();
    }
}

// ------------------------------------------------------------- variants --

namespace {

struct BucketDesc {
    const char *name;
    int n_variants;
    const char *variants[6];
};

// Variant v of a long bin: v < 4 -> strips in LDS with 1 << v wavefronts per
// block (if its LDS fits a workgroup), v == 4 -> rows in lanes from global memory.
const BucketDesc BUCKETS[N_CLASSES] = {
    {"E<=7", 3, {"g16", "g32", "g64"}},
    {"E<=15", 2, {"g32", "g64"}},
    {"E<=31", 1, {"g64"}},
    {"long<=96", 5, {"lds_w1", "lds_w2", "lds_w4", "lds_w8", "global"}},
    {"long<=192", 5, {"lds_w1", "lds_w2", "lds_w4", "lds_w8", "global"}},
    {"long<=384", 5, {"lds_w1", "lds_w2", "lds_w4", "lds_w8", "global"}},
    {"long<=768", 5, {"lds_w1", "lds_w2", "lds_w4", "lds_w8", "global"}},
    {"general", 1, {"global"}},
};

// Defaults: the narrowest groups for short E, the most wavefronts per block
// whose LDS fits 64 KB for the long bins.
const int DEFAULT_VARIANT[N_CLASSES] = {0, 0, 0, 3, 3, 2, 1, 0};

std::mutex g_tune_mu;
int g_variant[N_CLASSES] = {0, 0, 0, 3, 3, 2, 1, 0};
float g_tune_ms[N_CLASSES][6];
u64 g_tune_pairs[N_CLASSES];

bool variant_ok(int bucket, int v) {
    if (v < 0 || v >= BUCKETS[bucket].n_variants) return false;
    if (bucket >= CLS_LONG && bucket < CLS_LONG + LONG_BINS && v < 4)
        return (1 << v) * LONG_CAP[bucket - CLS_LONG] * LDS_BLOCK_BYTES <= LONG_LDS_MAX;
    return true;
}

int current_variant(int bucket) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    return g_variant[bucket];
}

}  // namespace

// Launches the pairs idx[0, cnt) of one bucket with one of its variants.
static void launch_bucket(const FilterArgs &a, const u32 *idx, u64 cnt, int bucket, int v, hipStream_t s) {
    if (cnt == 0) return;
    if (bucket == 0 || bucket == 1) {
        const int g = std::string(BUCKETS[bucket].variants[v]) == "g16" ? 16
                      : std::string(BUCKETS[bucket].variants[v]) == "g32" ? 32 : 64;
        if (g == 16) k_filter<16><<<grid_for(cnt * 16, 256), 256, 0, s>>>(a, idx, cnt);
        else if (g == 32) k_filter<32><<<grid_for(cnt * 32, 256), 256, 0, s>>>(a, idx, cnt);
        else k_filter<64><<<grid_for(cnt * 64, 256), 256, 0, s>>>(a, idx, cnt);
    } else if (bucket >= CLS_LONG && bucket < CLS_LONG + LONG_BINS && v < 4) {
        const int tile = LONG_CAP[bucket - CLS_LONG], wpb = 1 << v;
        u64 blocks = (cnt + wpb - 1) / wpb;
        if (blocks > 16384) blocks = 16384;
        k_filter_long<<<(unsigned)blocks, 64 * wpb, (size_t)wpb * tile * LDS_BLOCK_BYTES, s>>>(a, idx, cnt, tile);
    } else {
        k_filter<64><<<grid_for(cnt * 64, 256), 256, 0, s>>>(a, idx, cnt);
    }
    MT_HIP(hipGetLastError());
}

// Buckets the pairs (one synchronization for the bucket sizes); idx / counts
// receive the bucketed pair indices and the per-bucket counts and offsets.
static void bucket_pairs(const FilterArgs &a, u64 n_cap, DBuf<u32> &idx, u32 hc[N_CLASSES], u32 hb[N_CLASSES],
                         hipStream_t s) {
    DBuf<u32> count(N_CLASSES), cursor(N_CLASSES), base(N_CLASSES);
    DBuf<u8> cls(n_cap);
    idx.alloc(n_cap);
    MT_HIP(hipMemsetAsync(count.p, 0, N_CLASSES * sizeof(u32), s));
    MT_HIP(hipMemsetAsync(cursor.p, 0, N_CLASSES * sizeof(u32), s));
    k_pair_class<<<grid_for(n_cap, 256), 256, 0, s>>>(a, n_cap, count.p, cls.p);
    MT_HIP(hipGetLastError());
    read_back(s, count.p, hc, N_CLASSES * sizeof(u32));
    u32 acc = 0;
    for (int c = 0; c < N_CLASSES; c++) {
        hb[c] = acc;
        acc += hc[c];
    }
    if (acc == 0) return;
    MT_HIP(hipMemcpyAsync(base.p, hb, N_CLASSES * sizeof(u32), hipMemcpyHostToDevice, s));
    k_pair_scatter<<<grid_for(n_cap, 256), 256, 0, s>>>(a, n_cap, cls.p, base.p, cursor.p, idx.p);
    MT_HIP(hipGetLastError());
    MT_HIP(hipStreamSynchronize(s));  // hb lives on this host stack frame
}

// Pairs to filter: the device count when there is one (bounded by the
// launch's capacity), else the host count.
__device__ inline u64 pair_count(const FilterArgs &a, u64 n_cap) {
    const u64 n = a.n_dev ? *a.n_dev : a.n_host;
    return n < n_cap ? n : n_cap;
}

// Table 1's single-row and base-frequency filters on explicit pairs, one
// thread per pair over the read's 64-base words.  Kind 1 (Hamming distance)
// counts the mismatch bits of row 0 of the band, the diagonal alone; kind 2
// (base counting) compares the counts of A, C, G and T in the read and in the
// reference window [diag, diag + m) (N and positions outside the genome are no
// base) and reports ceil(L1 / 2).  Both saturate at E + 1.
template <int KIND>
__global__ void k_filter_simple(FilterArgs a, u64 n_cap) {
    const u64 p = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= pair_count(a, n_cap)) return;
    u32 r, g, err;
    int E;
    bool ok;
    pair_fields(a, p, r, g, E, ok, err);
    if (!ok) {
        atomicOr(a.flags, err);
        a.approx[p] = 0xFFFF;
        a.accept[p] = 0;
        return;
    }
    const int m = read_len(a, r);
    const u64 rb = a.read_blk[r];
    const GenomeMeta gm = a.meta[g];
    const u64x2 *rl = a.ref_lohi + gm.blk;
    const u64 *rn = a.ref_nb + gm.blk;
    const i64 L = (i64)gm.len;
    const bool hn = meta_has_n(gm);
    const i64 diag = a.pair_diag[p];
    int c = 0;
    int dA = 0, dC = 0, dG = 0, dT = 0;  // read count minus window count per base
    for (int w0 = 0; w0 < m; w0 += 64) {
        const u64x2 q = a.read_lohi[rb + (u64)(w0 >> 6)];
        const u64 qn = a.read_nb[rb + (u64)(w0 >> 6)];
        const int left = m - w0;
        const u64 vm = left >= 64 ? ~0ull : (1ull << left) - 1;
        const Bits64 wb = fetch_ref(rl, rn, L, hn, diag + w0);
        if constexpr (KIND == 1) {
            c += __popcll(((q.lo ^ wb.lo) | (q.hi ^ wb.hi) | qn | wb.nb) & vm);
            if (c > E) break;
        } else {
            const u64 qv = ~qn & vm, wv = ~wb.nb & vm;
            dA += __popcll(~q.lo & ~q.hi & qv) - __popcll(~wb.lo & ~wb.hi & wv);
            dC += __popcll(q.lo & ~q.hi & qv) - __popcll(wb.lo & ~wb.hi & wv);
            dG += __popcll(~q.lo & q.hi & qv) - __popcll(~wb.lo & wb.hi & wv);
            dT += __popcll(q.lo & q.hi & qv) - __popcll(wb.lo & wb.hi & wv);
        }
    }
    if constexpr (KIND == 2) c = (abs(dA) + abs(dC) + abs(dG) + abs(dT) + 1) / 2;
    const int v = c < E + 1 ? c : E + 1;
    a.approx[p] = (u16)v;
    a.accept[p] = v <= E;
}

// Table 1's q-gram filter (q = QG_Q), one wavefront per pair: the q-grams of
// the reference window [diag - E, diag + m + E) free of N and of positions
// outside the genome are counted in a per-wavefront LDS table of 4^q
// counters; each of the read's q-grams then takes one count (an atomic
// decrement that found it positive), so the number taken is the size of the
// multiset intersection.  Value: ceil((m - q + 1 - shared) / q), 0 for m < q,
// saturated at E + 1.
constexpr int QG_Q = 5;
constexpr int QG_WPB = 4;

__global__ __launch_bounds__(64 * QG_WPB) void k_filter_qgram(FilterArgs a, u64 n_cap) {
    const u64 n = pair_count(a, n_cap);
    __shared__ int cnt_all[QG_WPB][1 << (2 * QG_Q)];
    const int lane = threadIdx.x & 63;
    const u32 wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int *cnt = cnt_all[wid];
    constexpr u64 QMASK = (1ull << QG_Q) - 1;
    for (u64 p = (u64)blockIdx.x * QG_WPB + wid; p < n; p += (u64)gridDim.x * QG_WPB) {
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
            continue;
        }
        const int m = read_len(a, r);
        if (m < QG_Q) {
            if (lane == 0) {
                a.approx[p] = 0;
                a.accept[p] = 1;
            }
            continue;
        }
        for (int i = lane; i < (1 << (2 * QG_Q)); i += 64) cnt[i] = 0;
        lds_wave_sync();
        const GenomeMeta gm = a.meta[g];
        const u64x2 *rl = a.ref_lohi + gm.blk;
        const u64 *rn = a.ref_nb + gm.blk;
        const i64 L = (i64)gm.len;
        const bool hn = meta_has_n(gm);
        const i64 w0 = a.pair_diag[p] - E;
        const i64 nwq = (i64)m + 2 * (i64)E - QG_Q + 1;
        for (i64 t = lane; t < nwq; t += 64) {
            const Bits64 b = fetch_ref(rl, rn, L, hn, w0 + t);
            if ((b.nb & QMASK) == 0) atomicAdd(&cnt[kmer_value(b.lo, b.hi, QG_Q)], 1);
        }
        lds_wave_sync();
        const u64 rb = a.read_blk[r];
        int shared = 0;
        for (int j0 = 0; j0 <= m - QG_Q; j0 += 64) {
            const int j = j0 + lane;
            bool took = false;
            if (j <= m - QG_Q) {
                const Bits64 b = fetch_planes(a.read_lohi + rb, a.read_nb + rb, j);
                if ((b.nb & QMASK) == 0) took = atomicSub(&cnt[kmer_value(b.lo, b.hi, QG_Q)], 1) > 0;
            }
            shared += __popcll(__ballot(took));
        }
        const int missing = m - QG_Q + 1 - shared;
        const int v = min((missing + QG_Q - 1) / QG_Q, E + 1);
        if (lane == 0) {
            a.approx[p] = (u16)v;
            a.accept[p] = v <= E;
        }
        lds_wave_sync();  // the next pair clears the counters
    }
}

// Shifted Hamming distance (Table 1's SHD), one thread per pair.  Row d's
// mismatch word w covers columns 64w .. 64w+63 (zero at columns >= m); in
// each row, a run of one or two zeros with a one on both sides (inside the
// read) becomes ones; the value is the number of columns where every amended
// row is one, saturated at E + 1.
__device__ inline u64 shd_word(const FilterArgs &a, u64 rb, int m, const u64x2 *rl, const u64 *rn, i64 L, bool hn,
                               i64 diag, int d, int w) {
    if (w < 0 || 64 * w >= m) return 0;
    const u64x2 q = a.read_lohi[rb + (u64)w];
    const u64 qn = a.read_nb[rb + (u64)w];
    const Bits64 r = fetch_ref(rl, rn, L, hn, diag + d + 64 * (i64)w);
    const int left = m - 64 * w;
    const u64 vm = left >= 64 ? ~0ull : (1ull << left) - 1;
    return ((q.lo ^ r.lo) | (q.hi ^ r.hi) | qn | r.nb) & vm;
}

// Word x of a row with its neighbours xp (columns before) and xn (after),
// short zero runs between ones set.
__device__ inline u64 shd_amend(u64 xp, u64 x, u64 xn) {
    const u64 l1 = (x << 1) | (xp >> 63), l2 = (x << 2) | (xp >> 62);  // bit i: x[i - 1], x[i - 2]
    const u64 r1 = (x >> 1) | (xn << 63), r2 = (x >> 2) | (xn << 62);  // bit i: x[i + 1], x[i + 2]
    const u64 one = ~x & l1 & r1;            // 1 0 1
    const u64 first = ~x & ~r1 & l1 & r2;    // 1 [0] 0 1
    const u64 second = ~x & ~l1 & l2 & r1;   // 1 0 [0] 1
    return x | one | first | second;
}

__global__ void k_filter_shd(FilterArgs a, u64 n_cap) {
    const u64 p = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= pair_count(a, n_cap)) return;
    u32 r, g, err;
    int E;
    bool ok;
    pair_fields(a, p, r, g, E, ok, err);
    if (!ok) {
        atomicOr(a.flags, err);
        a.approx[p] = 0xFFFF;
        a.accept[p] = 0;
        return;
    }
    const int m = read_len(a, r);
    const u64 rb = a.read_blk[r];
    const GenomeMeta gm = a.meta[g];
    const u64x2 *rl = a.ref_lohi + gm.blk;
    const u64 *rn = a.ref_nb + gm.blk;
    const i64 L = (i64)gm.len;
    const bool hn = meta_has_n(gm);
    const i64 diag = a.pair_diag[p];
    int c = 0;
    if (m <= 256) {  // the whole read in four words: rows outer, four accumulators
        u64 acc[4];
#pragma unroll
        for (int w = 0; w < 4; w++) {
            const int left = m - 64 * w;
            acc[w] = left >= 64 ? ~0ull : left > 0 ? (1ull << left) - 1 : 0ull;
        }
        for (int d = -E; d <= E && (acc[0] | acc[1] | acc[2] | acc[3]); d++) {
            u64 x[4];
#pragma unroll
            for (int w = 0; w < 4; w++) x[w] = shd_word(a, rb, m, rl, rn, L, hn, diag, d, w);
#pragma unroll
            for (int w = 0; w < 4; w++) acc[w] &= shd_amend(w ? x[w - 1] : 0ull, x[w], w < 3 ? x[w + 1] : 0ull);
        }
        c = __popcll(acc[0]) + __popcll(acc[1]) + __popcll(acc[2]) + __popcll(acc[3]);
    } else {  // longer reads: words outer, each row word with its neighbours
        const int nw = (m + 63) / 64;
        for (int w = 0; w < nw && c <= E; w++) {
            const int left = m - 64 * w;
            u64 acc = left >= 64 ? ~0ull : (1ull << left) - 1;
            for (int d = -E; d <= E && acc; d++)
                acc &= shd_amend(shd_word(a, rb, m, rl, rn, L, hn, diag, d, w - 1),
                                 shd_word(a, rb, m, rl, rn, L, hn, diag, d, w),
                                 shd_word(a, rb, m, rl, rn, L, hn, diag, d, w + 1));
            c += __popcll(acc);
        }
    }
    const int v = c < E + 1 ? c : E + 1;
    a.approx[p] = (u16)v;
    a.accept[p] = v <= E;
}

void launch_filter_simple(const FilterArgs &a, u64 n, u32 kind, hipStream_t s) {
    if (n == 0) return;  // n: the capacity; the kernels read the count itself
    if (kind == MT_FILTER_HAMMING)
        k_filter_simple<1><<<grid_for(n, 256), 256, 0, s>>>(a, n);
    else if (kind == MT_FILTER_BASE_COUNT)
        k_filter_simple<2><<<grid_for(n, 256), 256, 0, s>>>(a, n);
    else if (kind == MT_FILTER_SHD)
        k_filter_shd<<<grid_for(n, 256), 256, 0, s>>>(a, n);
    else if (kind == MT_FILTER_QGRAM)
        k_filter_qgram<<<(unsigned)std::min<u64>(grid_for(n, QG_WPB), 65536), 64 * QG_WPB, 0, s>>>(a, n);
    else
        throw Error(MT_EINVAL, "unknown filter kind");
    MT_HIP(hipGetLastError());
}

// Stage names of the per-bucket timing marks.
static const char *const BUCKET_MARKS[N_CLASSES] = {"filter E<=7",     "filter E<=15",    "filter E<=31",
                                                    "filter long<=96", "filter long<=192", "filter long<=384",
                                                    "filter long<=768", "filter general"};

void launch_filter(const FilterArgs &a, u64 n_cap, u32 /*max_E*/, hipStream_t s, Timer *tm) {
    if (n_cap == 0) return;
    DBuf<u32> idx;
    u32 hc[N_CLASSES], hb[N_CLASSES];
    bucket_pairs(a, n_cap, idx, hc, hb, s);
    if (tm) tm->mark("filter buckets");
    for (int c = 0; c < N_CLASSES; c++) {
        if (hc[c] == 0) continue;
        launch_bucket(a, idx.p + hb[c], hc[c], c, current_variant(c), s);
        if (tm) tm->mark(BUCKET_MARKS[c]);
    }
}

// Times every variant of every bucket that holds pairs (best of `reps`
// launches each, after one untimed launch) and keeps the fastest.
void autotune_filter(const FilterArgs &a, u64 n_pairs, u32 reps, hipStream_t s) {
    if (n_pairs == 0) return;
    DBuf<u32> idx;
    u32 hc[N_CLASSES], hb[N_CLASSES];
    bucket_pairs(a, n_pairs, idx, hc, hb, s);
    hipEvent_t e0, e1;
    MT_HIP(hipEventCreate(&e0));
    MT_HIP(hipEventCreate(&e1));
    try {
        for (int c = 0; c < N_CLASSES; c++) {
            if (hc[c] == 0) continue;
            float best_ms = 0;
            int best = -1;
            float ms_v[6] = {0, 0, 0, 0, 0, 0};
            for (int v = 0; v < BUCKETS[c].n_variants; v++) {
                if (!variant_ok(c, v)) continue;
                launch_bucket(a, idx.p + hb[c], hc[c], c, v, s);
                float mn = 0;
                for (u32 r = 0; r < (reps ? reps : 1); r++) {
                    MT_HIP(hipEventRecord(e0, s));
                    launch_bucket(a, idx.p + hb[c], hc[c], c, v, s);
                    MT_HIP(hipEventRecord(e1, s));
                    MT_HIP(hipEventSynchronize(e1));
                    float ms = 0;
                    MT_HIP(hipEventElapsedTime(&ms, e0, e1));
                    if (r == 0 || ms < mn) mn = ms;
                }
                ms_v[v] = mn;
                if (best < 0 || mn < best_ms) {
                    best_ms = mn;
                    best = v;
                }
            }
            std::lock_guard<std::mutex> g(g_tune_mu);
            if (best >= 0) g_variant[c] = best;
            for (int v = 0; v < 6; v++) g_tune_ms[c][v] = ms_v[v];
            g_tune_pairs[c] = hc[c];
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

int tune_buckets() { return N_CLASSES; }

void tune_info(int bucket, mt_tune_bucket &out) {
    MT_REQUIRE(bucket >= 0 && bucket < N_CLASSES, "no such filter bucket");
    std::lock_guard<std::mutex> g(g_tune_mu);
    const BucketDesc &d = BUCKETS[bucket];
    out.name = d.name;
    out.n_variants = (u32)d.n_variants;
    out.current = (u32)g_variant[bucket];
    for (int v = 0; v < 6; v++) {
        out.variant_names[v] = v < d.n_variants ? d.variants[v] : nullptr;
        out.ms[v] = g_tune_ms[bucket][v];
    }
    out.pairs = g_tune_pairs[bucket];
}

void tune_set(int bucket, int variant) {
    MT_REQUIRE(bucket >= 0 && bucket < N_CLASSES, "no such filter bucket");
    MT_REQUIRE(variant_ok(bucket, variant), "variant not available for this bucket");
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_variant[bucket] = variant;
}

void tune_reset() {
    std::lock_guard<std::mutex> g(g_tune_mu);
    for (int c = 0; c < N_CLASSES; c++) {
        g_variant[c] = DEFAULT_VARIANT[c];
        for (int v = 0; v < 6; v++) g_tune_ms[c][v] = 0;
        g_tune_pairs[c] = 0;
    }
}

}  // namespace mt
