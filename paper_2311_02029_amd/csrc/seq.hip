// Packing sequences into bit planes and tiled minimizer extraction
// (seeding, Fig. 1 steps 2a and 2b).
#include "seq.hpp"

namespace mt {

void read_back(hipStream_t s, const void *dev, void *host, size_t bytes) {
    MT_HIP(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s));
    MT_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------ packing --

// Blocks per sequence: ceil(len / 64) + 1 (the last one is padding).  Also
// checks the offsets: 0 first, never decreasing, `total` last.
__global__ void k_seq_blocks(const u64 *__restrict__ off, u64 n, u64 total, u64 len_limit, u32 len_flag,
                             u64 *__restrict__ nblk, u32 *__restrict__ flags) {
    u64 s = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    u64 a = off[s], b = off[s + 1];
    u32 f = 0;
    if (b < a || b > total || (s == 0 && a != 0) || (s == n - 1 && b != total)) f |= ERR_OFFSETS;
    u64 len = b >= a ? b - a : 0;
    if (len > len_limit) f |= len_flag;
    if (f) {
        atomicOr(flags, f);
        len = 0;
    }
    nblk[s] = (len + 63) / 64 + 1;
}

// One thread per 64-base block: reads the block's bytes with aligned 32-bit
// loads (an aligned word holding a valid byte never crosses a page) and
// builds the lo / hi / nb words.
__global__ void k_pack(const u8 *__restrict__ seq, const u64 *__restrict__ off, const u64 *__restrict__ blk_off,
                       u64 n, u64 cap, const u32 *__restrict__ map, u64x2 *__restrict__ lohi, u64 *__restrict__ nbp,
                       u32 *__restrict__ flags, u32 *__restrict__ has_n) {
    u64 b = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= blk_off[n] || b >= cap) return;
    u32 s = map[b];
    u64 lb = b - blk_off[s];
    u64 beg = off[s] + 64 * lb, end = off[s + 1];
    if (end > beg + 64) end = beg + 64;
    u64 lo = 0, hi = 0, nb = ~0ull;
    if (beg < end) {
        u64 cnt = end - beg;
        nb = cnt < 64 ? (~0ull << cnt) : 0ull;
        bool bad = false, anyn = false;
        uintptr_t p0 = (uintptr_t)(seq + beg), p1 = (uintptr_t)(seq + end);
        for (uintptr_t a = p0 & ~(uintptr_t)3; a < p1; a += 4) {
            u32 v = *(const u32 *)a;
#pragma unroll
            for (int t = 0; t < 4; t++) {
                uintptr_t q = a + t;
                if (q < p0 || q >= p1) continue;
                u32 i = (u32)(q - p0);
                u32 c = base_code((v >> (8 * t)) & 0xFFu);
                if (c == 5) bad = true;
                if (c >= 4) {
                    nb |= 1ull << i;
                    anyn |= c == 4;
                } else {
                    lo |= (u64)(c & 1u) << i;
                    hi |= (u64)(c >> 1) << i;
                }
            }
        }
        if (bad) atomicOr(flags, ERR_BAD_BYTE);
        if (anyn && has_n) has_n[s] = 1;
    }
    lohi[b] = u64x2{lo, hi};
    nbp[b] = nb;
}

void pack_sequences(const mt_seqs &in, u64 len_limit, u32 len_flag, const char *len_message, PackedSeqs &out,
                    u32 *d_flags, u32 *has_n, hipStream_t s) {
    out.n = in.n;
    out.blk_off.alloc(in.n + 1);
    out.blocks_cap = in.total / 64 + 2 * in.n + 1;
    out.lohi.alloc(out.blocks_cap);
    out.nb.alloc(out.blocks_cap);
    if (in.n == 0) {
        MT_HIP(hipMemsetAsync(out.blk_off.p, 0, sizeof(u64), s));
        return;
    }
    DBuf<u64> nblk(in.n);
    k_seq_blocks<<<grid_for(in.n, 256), 256, 0, s>>>(in.offsets, in.n, in.total, len_limit, len_flag, nblk.p,
                                                      d_flags);
    MT_HIP(hipGetLastError());
    // The offsets decide every later address: refuse bad ones before any
    // kernel reads sequence bytes through them.
    u32 f = 0;
    read_back(s, d_flags, &f, sizeof f);
    if (f & len_flag) throw Error(MT_EINVAL, len_message);
    check_flags(f);
    scan_u64(nblk.p, out.blk_off.p, in.n, s);
    DBuf<u32> map(out.blocks_cap);
    segment_map(out.blk_off.p, in.n, map.p, out.blocks_cap, s);
    k_pack<<<grid_for(out.blocks_cap, 256), 256, 0, s>>>((const u8 *)in.seq, in.offsets, out.blk_off.p, in.n,
                                                          out.blocks_cap, map.p, out.lohi.p, out.nb.p, d_flags, has_n);
    MT_HIP(hipGetLastError());
}

// --------------------------------------------------------------- minimizers --

constexpr int MAX_HALO = 254;  // w - 1 for w <= 255

// Tiles per sequence: ceil(nk / tile) with nk = len - k + 1 k-mer starts.
__global__ void k_seq_tiles(const u64 *__restrict__ off, u64 n, u32 k, u64 tile, u64 *__restrict__ ntile) {
    u64 s = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    i64 len = (i64)(off[s + 1] - off[s]);
    i64 nk = len - (i64)k + 1;
    ntile[s] = nk > 0 ? ((u64)nk + tile - 1) / tile : 0;
}

// Leftmost smallest of the W hashes sh[i..i + W) (an invalid k-mer reads as
// ~0, which no valid k-mer hashes to: the hash is a bijection and the preimage
// of ~0 is above every 62-bit k-mer value); -1 when the window has no valid
// k-mer.  All W hashes are read before the compare chain.
template <int W>
__device__ inline int lds_window_argmin(const u64 *sh, int i) {
    u64 v[W];
#pragma unroll
    for (int t = 0; t < W; t++) v[t] = sh[i + t];
    u64 bh = ~0ull;
    int bt = -1;
#pragma unroll
    for (int t = 0; t < W; t++)
        if (v[t] < bh) {
            bh = v[t];
            bt = t;
        }
    return bt < 0 ? -1 : i + bt;
}

__device__ inline int lds_window_argmin_any(const u64 *sh, int i, int win) {
    switch (win) {
#define MT_WIN(W) \
    case W:       \
        return lds_window_argmin<W>(sh, i);
        MT_WIN(1) MT_WIN(2) MT_WIN(3) MT_WIN(4) MT_WIN(5) MT_WIN(6) MT_WIN(7) MT_WIN(8)
        MT_WIN(9) MT_WIN(10) MT_WIN(11) MT_WIN(12)
#undef MT_WIN
    default: {
        u64 bh = ~0ull;
        int best = -1;
        for (int t = 0; t < win; t++)
            if (sh[i + t] < bh) {
                bh = sh[i + t];
                best = i + t;
            }
        return best;
    }
    }
}

// One block per tile of TILE consecutive k-mer starts of one sequence.  The
// hashes of the tile plus a halo of w - 1 starts on each side go to LDS; every
// window that overlaps the tile picks its smallest (hash, position) among the
// valid k-mers, and picks inside the tile are marked.  The marks leave as one
// 64-bit word per 64 starts (tile_bits, TILE / 64 words per tile) with their
// count in tile_count.
template <int TPB, int TILE>
__global__ __launch_bounds__(TPB) void k_min_tiles(const u64x2 *__restrict__ lohi, const u64 *__restrict__ nbp,
                                                   const u64 *__restrict__ blk_off, const u64 *__restrict__ off,
                                                   const u64 *__restrict__ tile_off, const u32 *__restrict__ tile_map,
                                                   u64 n, u32 k, u32 w, u32 *__restrict__ tile_count,
                                                   u64 *__restrict__ tile_bits) {
    static_assert(TILE % TPB == 0 && TPB % 64 == 0, "tile of whole wavefront passes");
    static_assert((TILE + 2 * MAX_HALO) / TPB + 1 + 31 <= 64, "a thread's starts and k-mers fit its 64-base window");
    constexpr int SPAN = TILE + 2 * MAX_HALO;
    __shared__ u64 sh_h[SPAN];
    __shared__ u8 chosen[TILE];
    __shared__ u32 total;
    const u64 t = blockIdx.x;
    if (t >= tile_off[n]) return;
    const u32 s = tile_map[t];
    const i64 lt = (i64)(t - tile_off[s]);
    const i64 len = (i64)(off[s + 1] - off[s]);
    const i64 nk = len - (i64)k + 1;
    const i64 win = nk < (i64)w ? nk : (i64)w;
    const i64 t0 = lt * TILE, t1 = t0 + TILE < nk ? t0 + TILE : nk;
    const i64 h0 = t0 - win + 1 > 0 ? t0 - win + 1 : 0;
    const i64 h1 = t1 + win - 1 < nk ? t1 + win - 1 : nk;
    const u64x2 *ql = lohi + blk_off[s];
    const u64 *qn = nbp + blk_off[s];
    // Each thread hashes a run of consecutive starts: the first k-mer value
    // from its 64-base window, the next ones rolled in one base at a time.
    const u64 kmask = (1ull << k) - 1, xmask = (1ull << (2 * k)) - 1;
    const int span = (int)(h1 - h0);
    const int run = (span + TPB - 1) / TPB;  // at most (TILE + 2 * MAX_HALO) / TPB + 1 <= 64 - 31
    const int c0 = (int)threadIdx.x * run;
    if (c0 < span) {
        const Bits64 b = fetch_planes(ql, qn, h0 + c0);
        u64 x = kmer_value(b.lo, b.hi, k);
        const int cn = min(run, span - c0);
        for (int j = 0; j < cn; j++) {
            if (j > 0) {
                const u32 t = (u32)j + k - 1;  // the base entering the k-mer
                x = ((x << 2) | (((b.hi >> t) & 1ull) << 1) | ((b.lo >> t) & 1ull)) & xmask;
            }
            sh_h[c0 + j] = ((b.nb >> j) & kmask) == 0 ? mix64(x) : ~0ull;
        }
    }
    for (int i = threadIdx.x; i < TILE; i += TPB) chosen[i] = 0;
    if (threadIdx.x == 0) total = 0;
    __syncthreads();
    const i64 ws1 = t1 - 1 < nk - win ? t1 - 1 : nk - win;
    for (i64 ws = h0 + threadIdx.x; ws <= ws1; ws += TPB) {
        const int best = lds_window_argmin_any(sh_h, (int)(ws - h0), (int)win);
        if (best >= 0) {
            const i64 p = h0 + best;
            if (p >= t0 && p < t1) chosen[p - t0] = 1;
        }
    }
    __syncthreads();
    const u32 lane = threadIdx.x & 63;
#pragma unroll
    for (int u = 0; u < TILE / TPB; u++) {
        const int i = u * TPB + (int)threadIdx.x;  // 64 consecutive starts per wavefront
        const u64 m = __ballot(chosen[i] != 0);
        if (lane == 0) {
            tile_bits[t * (TILE / 64) + i / 64] = m;
            if (m) atomicAdd(&total, (u32)__popcll(m));
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) tile_count[t] = total;
}

// One wavefront per tile: the marked starts are first listed in LDS, then
// their k-mer values computed 64 at a time (one lane per start) and written in
// start order at the tile's output offset with sequence and position (each
// of those two outputs may be null).
constexpr int EMIT_WPB = 4;

template <int TILE>
__global__ __launch_bounds__(64 * EMIT_WPB) void k_min_emit(const u64x2 *__restrict__ lohi,
                                                            const u64 *__restrict__ nbp,
                                                            const u64 *__restrict__ blk_off,
                                                            const u64 *__restrict__ tile_off,
                                                            const u32 *__restrict__ tile_map, u64 n, u32 k,
                                                            const u64 *__restrict__ tile_bits,
                                                            const u64 *__restrict__ min_off, u64 *__restrict__ out_x,
                                                            u32 *__restrict__ out_seq, u32 *__restrict__ out_pos) {
    static_assert(TILE <= 65536, "starts within a tile fit 16 bits");
    __shared__ u16 list_all[EMIT_WPB][TILE];
    const u32 lane = threadIdx.x & 63;
    const u32 wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const u64 t = (u64)blockIdx.x * EMIT_WPB + wid;
    if (t >= tile_off[n]) return;
    u16 *list = list_all[wid];
    const u32 s = tile_map[t];
    const i64 t0 = (i64)(t - tile_off[s]) * TILE;
    const u64 below = lane ? (~0ull) >> (64 - lane) : 0ull;
    u32 nl = 0;
#pragma unroll 1
    for (int q = 0; q < TILE / 64; q++) {
        const u64 m = tile_bits[t * (TILE / 64) + q];
        if ((m >> lane) & 1) list[nl + (u32)__popcll(m & below)] = (u16)(64 * q + lane);
        nl += (u32)__popcll(m);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const u64x2 *ql = lohi + blk_off[s];
    const u64 *qn = nbp + blk_off[s];
    const u64 o = min_off[t];
#pragma unroll 1
    for (u32 b = 0; b < nl; b += 64) {
        if (b + lane < nl) {
            const i64 i = t0 + list[b + lane];
            const Bits64 bits = fetch_planes(ql, qn, i);
            out_x[o + b + lane] = kmer_value(bits.lo, bits.hi, k);
            if (out_seq) out_seq[o + b + lane] = s;
            if (out_pos) out_pos[o + b + lane] = (u32)i;
        }
    }
}

template <int TPB, int TILE>
static void launch_tiles(const mt_seqs &in, const PackedSeqs &ps, u32 k, u32 w, MinimizerPlan &mp, hipStream_t s) {
    k_min_tiles<TPB, TILE><<<grid_for(mp.tiles_cap, 1), TPB, 0, s>>>(ps.lohi.p, ps.nb.p, ps.blk_off.p, in.offsets,
                                                                      mp.tile_off.p, mp.tile_map.p, in.n, k, w,
                                                                      mp.tile_count.p, mp.tile_bits.p);
    MT_HIP(hipGetLastError());
}

template <int TILE>
static void launch_emit(const mt_seqs &in, const PackedSeqs &ps, u32 k, MinimizerPlan &mp, u64 *out_x,
                        u32 *out_seq, u32 *out_pos, hipStream_t s) {
    k_min_emit<TILE><<<grid_for(mp.tiles_cap, EMIT_WPB), 64 * EMIT_WPB, 0, s>>>(
        ps.lohi.p, ps.nb.p, ps.blk_off.p, mp.tile_off.p, mp.tile_map.p, in.n, k, mp.tile_bits.p, mp.min_off.p, out_x,
        out_seq, out_pos);
    MT_HIP(hipGetLastError());
}

void minimizer_plan(const mt_seqs &in, const PackedSeqs &ps, u32 k, u32 w, int tile, MinimizerPlan &mp,
                    hipStream_t s) {
    mp.tile = tile;
    mp.tiles_cap = in.total / (u64)tile + in.n + 1;
    mp.tile_off.alloc(in.n + 1);
    mp.tile_map.alloc(mp.tiles_cap);
    mp.tile_count.alloc(mp.tiles_cap);
    mp.min_off.alloc(mp.tiles_cap + 1);
    mp.tile_bits.alloc(mp.tiles_cap * (u64)(tile / 64));
    if (tile != 256 && tile != 1024) throw Error(MT_EINTERNAL, "unsupported minimizer tile");
    if (in.n == 0) {  // no tiles: every offset is 0 (callers read min_off[tiles_cap])
        MT_HIP(hipMemsetAsync(mp.tile_off.p, 0, sizeof(u64), s));
        MT_HIP(hipMemsetAsync(mp.min_off.p, 0, (mp.tiles_cap + 1) * sizeof(u64), s));
        return;
    }
    DBuf<u64> ntile(in.n);
    k_seq_tiles<<<grid_for(in.n, 256), 256, 0, s>>>(in.offsets, in.n, k, (u64)tile, ntile.p);
    MT_HIP(hipGetLastError());
    scan_u64(ntile.p, mp.tile_off.p, in.n, s);
    segment_map(mp.tile_off.p, in.n, mp.tile_map.p, mp.tiles_cap, s);
    MT_HIP(hipMemsetAsync(mp.tile_count.p, 0, mp.tiles_cap * sizeof(u32), s));
    if (tile == 1024)
        launch_tiles<256, 1024>(in, ps, k, w, mp, s);
    else
        launch_tiles<128, 256>(in, ps, k, w, mp, s);
    // min_off over the full tile bound: tiles past the real count hold 0.
    scan_u32(mp.tile_count.p, mp.min_off.p, mp.tiles_cap, s);
}

void minimizer_emit(const mt_seqs &in, const PackedSeqs &ps, u32 k, u32 w, MinimizerPlan &mp, u64 *out_x,
                    u32 *out_seq, u32 *out_pos, hipStream_t s) {
    (void)w;
    if (in.n == 0) return;
    if (mp.tile == 1024)
        launch_emit<1024>(in, ps, k, mp, out_x, out_seq, out_pos, s);
    else
        launch_emit<256>(in, ps, k, mp, out_x, out_seq, out_pos, s);
}

}  // namespace mt
