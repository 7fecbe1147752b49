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

// One block per tile of TILE consecutive k-mer starts of one sequence.  The
// hashes of the tile plus a halo of w - 1 starts on each side go to LDS; every
// window that overlaps the tile picks its smallest (hash, position) among the
// valid k-mers, and picks inside the tile are marked.  Pass 1 (out_x null)
// stores the tile's count; pass 2 writes (x, sequence, position) in order.
template <int TPB, int TILE>
__global__ __launch_bounds__(TPB) void k_min_tiles(const u64x2 *__restrict__ lohi, const u64 *__restrict__ nbp,
                                                   const u64 *__restrict__ blk_off, const u64 *__restrict__ off,
                                                   const u64 *__restrict__ tile_off, const u32 *__restrict__ tile_map,
                                                   u64 n, u32 k, u32 w, u32 *__restrict__ tile_count,
                                                   const u64 *__restrict__ min_off, u64 *__restrict__ out_x,
                                                   u32 *__restrict__ out_seq, u32 *__restrict__ out_pos) {
    constexpr int SPAN = TILE + 2 * MAX_HALO;
    __shared__ u64 sh_h[SPAN];
    __shared__ u64 sh_x[SPAN];
    __shared__ u8 sh_ok[SPAN];
    __shared__ u8 chosen[TILE];
    u64 t = blockIdx.x;
    if (t >= tile_off[n]) return;
    u32 s = tile_map[t];
    i64 lt = (i64)(t - tile_off[s]);
    i64 len = (i64)(off[s + 1] - off[s]);
    i64 nk = len - (i64)k + 1;
    i64 win = nk < (i64)w ? nk : (i64)w;
    i64 t0 = lt * TILE, t1 = t0 + TILE < nk ? t0 + TILE : nk;
    i64 h0 = t0 - win + 1 > 0 ? t0 - win + 1 : 0;
    i64 h1 = t1 + win - 1 < nk ? t1 + win - 1 : nk;
    const u64x2 *ql = lohi + blk_off[s];
    const u64 *qn = nbp + blk_off[s];
    u64 kmask = (1ull << k) - 1;
    for (i64 i = h0 + threadIdx.x; i < h1; i += TPB) {
        Bits64 b = fetch_planes(ql, qn, i);
        u64 x = kmer_value(b.lo, b.hi, k);
        int idx = (int)(i - h0);
        sh_x[idx] = x;
        sh_h[idx] = mix64(x);
        sh_ok[idx] = (b.nb & kmask) == 0;
    }
    for (int i = threadIdx.x; i < TILE; i += TPB) chosen[i] = 0;
    __syncthreads();
    i64 ws1 = t1 - 1 < nk - win ? t1 - 1 : nk - win;
    for (i64 ws = h0 + threadIdx.x; ws <= ws1; ws += TPB) {
        i64 best = -1;
        u64 bh = 0;
        for (i64 i = ws; i < ws + win; i++) {
            int idx = (int)(i - h0);
            if (!sh_ok[idx]) continue;
            u64 hv = sh_h[idx];
            if (best < 0 || hv < bh) {  // strict: the leftmost of equal hashes wins
                best = i;
                bh = hv;
            }
        }
        if (best >= t0 && best < t1) chosen[best - t0] = 1;
    }
    __syncthreads();
    constexpr int PER = TILE / TPB;
    u32 cnt = 0;
#pragma unroll
    for (int u = 0; u < PER; u++) cnt += chosen[threadIdx.x * PER + u];
    u32 total;
    u32 pre = block_exclusive_sum<TPB, u32>(cnt, &total);
    if (!out_x) {
        if (threadIdx.x == 0) tile_count[t] = total;
        return;
    }
    u64 o = min_off[t] + pre;
#pragma unroll
    for (int u = 0; u < PER; u++) {
        int li = threadIdx.x * PER + u;
        if (!chosen[li]) continue;
        i64 i = t0 + li;
        out_x[o] = sh_x[i - h0];
        out_seq[o] = s;
        out_pos[o] = (u32)i;
        o++;
    }
}

template <int TPB, int TILE>
static void launch_tiles(const mt_seqs &in, const PackedSeqs &ps, u32 k, u32 w, MinimizerPlan &mp, u64 *out_x,
                         u32 *out_seq, u32 *out_pos, hipStream_t s) {
    k_min_tiles<TPB, TILE><<<grid_for(mp.tiles_cap, 1), TPB, 0, s>>>(
        ps.lohi.p, ps.nb.p, ps.blk_off.p, in.offsets, mp.tile_off.p, mp.tile_map.p, in.n, k, w, mp.tile_count.p,
        mp.min_off.p, out_x, out_seq, out_pos);
    MT_HIP(hipGetLastError());
}

static void run_tiles(const mt_seqs &in, const PackedSeqs &ps, u32 k, u32 w, MinimizerPlan &mp, u64 *out_x,
                      u32 *out_seq, u32 *out_pos, hipStream_t s) {
    if (mp.tile == 1024)
        launch_tiles<256, 1024>(in, ps, k, w, mp, out_x, out_seq, out_pos, s);
    else if (mp.tile == 256)
        launch_tiles<128, 256>(in, ps, k, w, mp, out_x, out_seq, out_pos, s);
    else
        throw Error(MT_EINTERNAL, "unsupported minimizer tile");
}

void minimizer_plan(const mt_seqs &in, const PackedSeqs &ps, u32 k, u32 w, int tile, MinimizerPlan &mp,
                    hipStream_t s) {
    mp.tile = tile;
    mp.tiles_cap = in.total / (u64)tile + in.n + 1;
    mp.tile_off.alloc(in.n + 1);
    mp.tile_map.alloc(mp.tiles_cap);
    mp.tile_count.alloc(mp.tiles_cap);
    mp.min_off.alloc(mp.tiles_cap + 1);
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
    run_tiles(in, ps, k, w, mp, nullptr, nullptr, nullptr, s);
    // min_off over the full tile bound: tiles past the real count hold 0.
    scan_u32(mp.tile_count.p, mp.min_off.p, mp.tiles_cap, s);
}

void minimizer_emit(const mt_seqs &in, const PackedSeqs &ps, u32 k, u32 w, MinimizerPlan &mp, u64 *out_x,
                    u32 *out_seq, u32 *out_pos, hipStream_t s) {
    if (in.n == 0) return;
    run_tiles(in, ps, k, w, mp, out_x, out_seq, out_pos, s);
}

}  // namespace mt
