// Device helpers for the gfx950 kernels: base codes, the k-mer hash, 2-bit
// plane fetches, mismatch words and the wavefront-group obstacle walk.
//
// Sequence layout in HBM ("planes"): a sequence of length L owns
// ceil(L/64) + 1 blocks; block b holds bases [64b, 64b + 64) as three 64-bit
// words, base i at bit (i mod 64):
//   lo  bit 0 of the base code   (A=0, C=1, G=2, T=3)
//   hi  bit 1 of the base code
//   nb  1 where the base is N, or lies past the end of the sequence
// lo and hi of a block are stored together as one 16-byte word (u64x2) so a
// single load brings both; nb sits in its own array.  The extra block at the
// end lets a 64-bit funnel fetch at any position < L read block b + 1 without
// a bounds check.  With bit planes, one XOR per plane and one OR compare 64
// bases at once, so the neighbourhood map of the filter costs a handful of
// 64-bit VALU operations per 64 columns.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mt {
typedef uint8_t u8;
typedef uint16_t u16;
typedef uint32_t u32;
typedef uint64_t u64;
typedef int64_t i64;
}  // namespace mt
using namespace mt;

struct alignas(16) u64x2 {
    u64 lo, hi;
};

// Input-validation flags raised by kernels (OR-ed into one device word).
enum : u32 {
    ERR_BAD_BYTE = 1u,
    ERR_READ_TOO_LONG = 2u,
    ERR_E_TOO_LARGE = 4u,
    ERR_PAIR_RANGE = 8u,
    ERR_KEY_OVERFLOW = 16u,
    ERR_INTERNAL = 32u,
    ERR_OFFSETS = 64u,
};

// Offset added to a diagonal so that (genome, diagonal) packs into one
// unsigned 64-bit key: diagonal = q - p > -65536 for reads of <= 65535 bases.
constexpr i64 DIAG_BIAS = 65536;
constexpr u64 DIAG_MASK = (1ull << 33) - 1;

__host__ __device__ inline u64 cand_key(u32 genome, i64 diag) {
    return ((u64)genome << 33) | (u64)(diag + DIAG_BIAS);
}
__host__ __device__ inline u32 key_genome(u64 key) { return (u32)(key >> 33); }
__host__ __device__ inline i64 key_diag(u64 key) { return (i64)(key & DIAG_MASK) - DIAG_BIAS; }

// ASCII -> code: 0..3 for ACGT, 4 for N, 5 for any other byte (either case).
__device__ inline u32 base_code(u32 c) {
    u32 u = c & 0xDFu;  // upper-case letters
    u32 two = ((c >> 1) ^ (c >> 2)) & 3u;  // A->0, C->1, G->2, T->3
    bool acgt = (u == 'A') | (u == 'C') | (u == 'G') | (u == 'T');
    return acgt ? two : (u == 'N' ? 4u : 5u);
}

// splitmix64 finalizer (Steele, Lea and Flood 2014), a bijection on 64-bit words.
__host__ __device__ inline u64 mix64(u64 z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Spreads the low 32 bits of x to the even bit positions of a 64-bit word.
__device__ inline u64 spread_even(u64 x) {
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

// k-mer value sum code[t] * 4^(k-1-t) (first base most significant) from the
// lo / hi plane bits of bases t = 0..k-1 at bits 0..k-1 (k <= 31).
__device__ inline u64 kmer_value(u64 lo, u64 hi, u32 k) {
    u32 l = __brev((u32)lo) >> (32 - k);
    u32 h = __brev((u32)hi) >> (32 - k);
    return spread_even(l) | (spread_even(h) << 1);
}

__device__ inline u64 funnel(u64 a, u64 b, u32 s) {
    return s ? (a >> s) | (b << (64 - s)) : a;
}

// 64 bases from position p >= 0 of a sequence whose planes start at block 0
// of the given arrays (p must be < the sequence length, or < its padded
// length for the nb plane, so block p/64 + 1 exists).
struct Bits64 {
    u64 lo, hi, nb;
};

__device__ inline Bits64 fetch_planes(const u64x2 *__restrict__ lohi, const u64 *__restrict__ nb, i64 p) {
    u64 b = (u64)p >> 6;
    u32 s = (u32)p & 63u;
    u64x2 a = lohi[b], c = lohi[b + 1];
    Bits64 r;
    r.lo = funnel(a.lo, c.lo, s);
    r.hi = funnel(a.hi, c.hi, s);
    r.nb = funnel(nb[b], nb[b + 1], s);
    return r;
}

// 64 reference bases from signed position p of a genome of length L:
// bits of positions outside [0, L) come back with nb = 1 (never a match).
// has_n = 0 skips the N plane for genomes without N.
__device__ inline Bits64 fetch_ref(const u64x2 *__restrict__ lohi, const u64 *__restrict__ nb, i64 L, bool has_n,
                                   i64 p) {
    Bits64 r;
    if (p >= L || p <= -64) {
        r.lo = r.hi = 0;
        r.nb = ~0ull;
        return r;
    }
    i64 q = p < 0 ? 0 : p;
    u64 b = (u64)q >> 6;
    u32 s = (u32)q & 63u;
    u64x2 a = lohi[b], c = lohi[b + 1];
    r.lo = funnel(a.lo, c.lo, s);
    r.hi = funnel(a.hi, c.hi, s);
    r.nb = has_n ? funnel(nb[b], nb[b + 1], s) : 0ull;
    if (p < 0) {
        u32 sh = (u32)(-p);
        r.lo <<= sh;
        r.hi <<= sh;
        r.nb = (r.nb << sh) | ((1ull << sh) - 1);
    }
    i64 room = L - p;  // bases of the genome at or after p within this word
    if (room < 64) r.nb |= ~0ull << room;
    return r;
}

// Reference block blk (bases 64 blk .. 64 blk + 63) of a genome of length L
// with its bounds applied: a block before the genome or wholly past its end
// reads as invalid (nb = 1), and positions at or past L inside the last
// block get nb = 1.  has_n = 0 skips the N plane (the genome has no N).
__device__ inline Bits64 ref_block(const u64x2 *__restrict__ lohi, const u64 *__restrict__ nb, i64 L, bool has_n,
                                   i64 blk) {
    Bits64 r;
    if (blk < 0 || blk * 64 >= L) {
        r.lo = r.hi = 0;
        r.nb = ~0ull;
        return r;
    }
    const u64x2 a = lohi[blk];
    r.lo = a.lo;
    r.hi = a.hi;
    r.nb = has_n ? nb[blk] : 0ull;
    const i64 room = L - blk * 64;
    if (room < 64) r.nb |= ~0ull << room;
    return r;
}

// The mismatch words of one band row over read words 0..NW-1 (columns
// 64w .. 64w + 63), the row's reference starting at position p0 = diag + d
// (any sign): the NW + 1 reference blocks the row spans are each fetched once
// and every word is one funnel shift of two neighbouring blocks by p0 mod 64.
// The blocks are taken in order with only two of them live at a time (the
// caller's registers are scarce).  qword(w) gives the read's lo / hi / nb
// word w (nb 1 past the read's end, so the row's bits past column m are set).
template <int NW, class QWord>
__device__ inline void band_row(QWord qword, const u64x2 *__restrict__ rl, const u64 *__restrict__ rn, i64 L,
                                bool has_n, i64 p0, u64 (&row)[NW]) {
    const i64 blk = p0 >> 6;  // floor division: p0 may be negative
    const u32 s = (u32)p0 & 63u;
    Bits64 prev = ref_block(rl, rn, L, has_n, blk);
#pragma unroll
    for (int w = 0; w < NW; w++) {
        const Bits64 next = ref_block(rl, rn, L, has_n, blk + w + 1);
        const Bits64 q = qword(w);
        row[w] = (q.lo ^ funnel(prev.lo, next.lo, s)) | (q.hi ^ funnel(prev.hi, next.hi, s)) | q.nb |
                 funnel(prev.nb, next.nb, s);
        prev = next;
    }
}

// Word w of a row held in NW registers (all ones past the last word), by a
// chain of selects: a dynamically indexed array would go to scratch memory.
template <int NW>
__device__ inline u64 row_word(const u64 (&r)[NW], int w) {
    u64 v = ~0ull;
#pragma unroll
    for (int i = NW - 1; i >= 0; i--) v = w == i ? r[i] : v;
    return v;
}

// Obstacle-free run of a row held in registers from column j (the row's bits
// past the read's end are set, so the run stops by the end).
template <int NW>
__device__ inline int reg_run(const u64 (&r)[NW], int j) {
    int w = j >> 6;
    const u32 s = (u32)j & 63u;
    int run = 0;
    for (;;) {
        const u64 v = funnel(row_word<NW>(r, w), row_word<NW>(r, w + 1), s);
        if (v) return run + (int)__builtin_ctzll(v);
        run += 64;
        w += 1;
    }
}

// Mismatch ("obstacle") bits of 64 columns: 1 where the read base cannot match.
__device__ inline u64 mismatch(const Bits64 &q, const Bits64 &w) {
    return (q.lo ^ w.lo) | (q.hi ^ w.hi) | q.nb | w.nb;
}

// Max over the G lanes of an aligned group (G = 16, 32 or 64).  Within a
// 16-lane DPP row the max is spread by rotating the row by 1, 2, 4 and 8
// lanes (every lane ends up with the row max); wider groups then combine the
// row maxima read from lanes 0, 16, 32 and 48.  Every lane of the group must
// be active (the rows of inactive groups are read but never used).
template <int G>
__device__ inline int group_max(int v) {
    static_assert(G == 16 || G == 32 || G == 64, "group of 16, 32 or 64 lanes");
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x121, 0xF, 0xF, false));  // row_ror:1
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x122, 0xF, 0xF, false));  // row_ror:2
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x124, 0xF, 0xF, false));  // row_ror:4
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false));  // row_ror:8
    if (G > 16) {
        // row maxima sit in lanes 0, 16, 32 and 48; combine them per group
        int r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
        int r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
        if (G == 64) return max(max(r0, r1), max(r2, r3));
        return (threadIdx.x & 32) ? max(r2, r3) : max(r0, r1);
    }
    return v;
}

// Per-genome record, one 16-byte load: first plane block, length, taxon and
// whether the genome holds an N (top bit).
struct alignas(16) GenomeMeta {
    u64 blk;
    u32 len;
    u32 taxon_n;
};
__host__ __device__ inline u32 meta_taxon(const GenomeMeta &m) { return m.taxon_n & 0x7fffffffu; }
__host__ __device__ inline bool meta_has_n(const GenomeMeta &m) { return (m.taxon_n >> 31) != 0; }

// Read planes + reference planes of one (read, location) pair.
struct PairView {
    const u64x2 *qlohi;
    const u64 *qnb;
    int m;
    const u64x2 *rlohi;
    const u64 *rnb;
    i64 L;
    bool has_n;
    i64 diag;
};

// Length of the obstacle-free run of row d from column j (capped at m - j).
// The read's nb plane is 1 past its end, so the run always stops by column m.
__device__ inline int row_run(const PairView &v, int d, int j) {
    int run = 0;
    while (j + run < v.m) {
        Bits64 q = fetch_planes(v.qlohi, v.qnb, j + run);
        Bits64 w = fetch_ref(v.rlohi, v.rnb, v.L, v.has_n, v.diag + d + j + run);
        u64 mm = mismatch(q, w);
        if (mm) {
            run += (int)__builtin_ctzll(mm);
            break;
        }
        run += 64;
    }
    return min(run, v.m - j);
}

// The obstacle walk of one pair by a group of G lanes (lane = lane index in
// the group; all G lanes call it together).  Rows d = -E..E are dealt to the
// lanes round-robin; each step takes the longest run over all rows, then
// counts and skips the obstacle that ends it.  Returns min(count, E + 1).
template <int G>
__device__ inline int obstacle_walk(const PairView &v, int E, int lane) {
    int rows = 2 * E + 1;
    int j = 0, c = 0;
    for (;;) {
        int best = 0;
        for (int r = lane; r < rows; r += G) best = max(best, row_run(v, r - E, j));
        best = group_max<G>(best);
        j += best;
        if (j >= v.m) break;
        c += 1;
        if (c > E) break;
        j += 1;
    }
    return c < E + 1 ? c : E + 1;
}

// Table slot value: a single occurrence is (genome << 32 | position) with the
// top bit clear; several occurrences are MULTI | count << 40 | start into the
// occurrence array; count 0 marks a k-mer dropped by max_occ.
constexpr u64 SLOT_EMPTY_KEY = ~0ull;  // k-mer values are < 4^31
constexpr u64 SLOT_MULTI = 1ull << 63;
constexpr u64 SLOT_NONE = ~0ull;       // value of a slot still being built
constexpr u32 MAX_KEY_OCC = (1u << 23) - 1;

__device__ inline u32 slot_count(u64 val) { return (val & SLOT_MULTI) ? (u32)((val >> 40) & MAX_KEY_OCC) : 1u; }
__device__ inline u64 slot_start(u64 val) { return val & ((1ull << 40) - 1); }

// Bucket of k-mer x: 4 slots (64 bytes) per bucket, chosen by the top 32 bits
// of a salted second hash scaled to the bucket count (no power-of-two
// restriction).  The minimizer hash itself must not place keys: minimizers
// are window minima of it, so their hashes crowd toward zero and would pile
// into the first buckets.
__host__ __device__ inline u64 bucket_of(u64 x, u64 nbuckets) {
    return ((mix64(x ^ 0x632be59bd9b4e019ull) >> 32) * nbuckets) >> 32;
}

// Looks k-mer x up; returns the slot value or SLOT_NONE if absent.  The
// 4-slot bucket probe: all four slots are loaded before any compare, and
// the first slot (in slot order) that holds x or is empty decides, through a
// chain of selects rather than branches.  Slots fill in order, so a bucket
// with an empty slot and no x means x is absent; a full bucket without x
// sends the probe on to the next bucket.
__device__ inline u64 table_lookup(const u64x2 *__restrict__ table, u64 nbuckets, u64 x) {
    u64 b = bucket_of(x, nbuckets);
    for (;;) {
        const u64x2 *bk = table + b * 4;
        const u64x2 e0 = bk[0], e1 = bk[1], e2 = bk[2], e3 = bk[3];
        // Use every value here: otherwise the compiler loads only the keys in
        // the loop and fetches the chosen value afterwards, a second round
        // trip to memory per probe.
        asm volatile("" ::"v"(e0.hi), "v"(e1.hi), "v"(e2.hi), "v"(e3.hi));
        const bool d0 = e0.lo == x || e0.lo == SLOT_EMPTY_KEY, d1 = e1.lo == x || e1.lo == SLOT_EMPTY_KEY;
        const bool d2 = e2.lo == x || e2.lo == SLOT_EMPTY_KEY, d3 = e3.lo == x || e3.lo == SLOT_EMPTY_KEY;
        u64 v = e3.lo == x ? e3.hi : SLOT_NONE;
        v = d2 ? (e2.lo == x ? e2.hi : SLOT_NONE) : v;
        v = d1 ? (e1.lo == x ? e1.hi : SLOT_NONE) : v;
        v = d0 ? (e0.lo == x ? e0.hi : SLOT_NONE) : v;
        if (d0 | d1 | d2 | d3) return v;
        b = (b + 1 == nbuckets) ? 0 : b + 1;
    }
}

// Exclusive prefix sum of one value per thread over a block of TPB threads
// (TPB a multiple of 64); *total receives the block sum.  Contains barriers:
// every thread of the block must call it.
template <int TPB, class T>
__device__ inline T block_exclusive_sum(T v, T *total) {
    __shared__ T wave_tot[TPB / 64];
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wave_tot[wid] = x;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < TPB / 64; i++) {
        if (i < wid) before += wave_tot[i];
        all += wave_tot[i];
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}
