// Fused seed-count + filter path for short reads (Fig. 1 steps 2b-2d and 3a
// in one kernel).  One wavefront owns one read at a time:
//   1. its bytes (requested while the previous read was counted) become
//      lo / hi / N bit planes with ballots, kept in a per-read LDS slot, and a
//      big-endian 2-bit stream in LDS;
//   2. lane i hashes the k-mer at position i (per 64-position round) into a
//      per-wave LDS tile;
//   3. lane s scans window s for its smallest valid (hash, position); picks
//      are marked in LDS and compacted with ballot + popcount;
//   4. each minimizer lane probes one 64-byte table bucket (all four slots
//      loaded at once); a read's hits are counted in registers, one ballot
//      per distinct (genome, diagonal), when they fit one lane each, and in a
//      per-read LDS hash table otherwise;
//   5. locations with >= min_hits become candidates, and each candidate's
//      rank in (hits desc, genome, diagonal) order picks the top_n;
//   6. the kept candidates join a per-wave queue; a full queue is filtered by
//      groups of G lanes (G = 16, 32 or 64 by E), one band row d per lane:
//      the row's mismatch words are built from 64-base reference fetches,
//      parked in LDS, and the obstacle walk advances by ctz of the row bits
//      plus a max over the group;
//   7. a read whose candidates are all filtered gets its accept flag and its
//      per-taxon unique / multi count.
// Reads beyond the kernel's limits (longer than 256 bases, E above 31, more
// than 256 seed hits, or more than 8 candidates when every candidate is kept)
// are queued and finished by the per-stage kernels, so every read gets the
// same result as in per-stage mode; top_n above 8 runs per stage throughout.
#include <cstddef>
#include <type_traits>

#include "classify.hpp"

namespace mt {

constexpr int F_WPB = 4;         // wavefronts per block
constexpr int F_MAX_M = 256;     // longest read the fused kernel takes
constexpr int F_HIT_CAP = 256;   // seed hits per read (distinct locations fit the table)
constexpr int F_TSLOTS = 256;    // per-read LDS hash table of locations
constexpr int F_MAX_E = 31;      // 2E + 1 rows fit one wavefront
constexpr int F_MAX_TOPN = 8;  // staged candidates per read (top_n = 0 keeps up to this many)
constexpr int F_QCAP = 4;        // queued (read, candidate) pairs per wave: one per 16-lane group
constexpr int F_PCAP = 8;        // reads per wave waiting for their filter results
constexpr int F_WORDS = F_MAX_M / 16 + 2;  // 2-bit stream words (16 bases per word) + padding

enum : u32 { ST_READS, ST_BASES, ST_MINS, ST_WBLOCKS, ST_CANDS, ST_UNMAPPED, ST_OCC, ST_COUNT };

struct FusedArgs {
    const u8 *seq;
    const u64 *off;
    u64 n;
    u32 k, w, min_hits, top_n, e_mode, e_value;
    u32 ncap;  // staging slots per read: top_n, or F_MAX_TOPN when top_n = 0 (keep all)
    const u64x2 *table;
    u64 nbuckets;
    const u64 *occ;
    const GenomeMeta *meta;
    const u64x2 *ref_lohi;
    const u64 *ref_nb;
    // staging: top_n slots per read
    u32 *st_genome;
    i64 *st_diag;
    u32 *st_hits;
    u16 *st_approx;
    u8 *st_accept;
    u32 *ncand;
    u8 *read_accepted;
    u16 *read_E;
    unsigned long long *uniq, *multi, *unmapped;
    u32 *fb_list;
    u32 *fb_count;
    u32 *flags;
    const u32 *gate;  // offsets check result: nonzero skips the whole launch
    u64 *stats_part;  // ST_COUNT work counts per block
};
static_assert(std::is_standard_layout<FusedArgs>::value, "FusedArgs fields are read by offset");

// A field of the launch's arguments read from the kernel-argument segment
// where it is used rather than held in scalar registers throughout: the
// fields used once per read or per pair would otherwise crowd out the
// registers the loop needs, and spilled scalar registers cost a vector
// instruction at every use.  FusedArgs is the kernel's only argument, so it
// starts the segment.
//
// The segment's address exists only in the kernel itself: a function compiled
// apart from the kernel reads it as zero (and then faults), so this helper and
// every function that uses it are forced inline.
template <class T>
__device__ __attribute__((always_inline)) inline T karg_field(size_t off) {
    const __attribute__((address_space(4))) char *base =
        (const __attribute__((address_space(4))) char *)__builtin_amdgcn_kernarg_segment_ptr();
    return *(volatile const __attribute__((address_space(4))) T *)(base + off);
}
#define KA(field) karg_field<decltype(FusedArgs::field)>(offsetof(FusedArgs, field))

// A read whose candidates wait in the filter queue (per-wave LDS).
struct PendRead {
    u64 plane[12];   // lo[0..3], hi[0..3], nb[0..3] of the read
    u64 r;
    u32 nc, left;    // candidates, candidates not yet filtered
    u16 E, m;
    u16 apx[F_MAX_TOPN];
    u32 tax[F_MAX_TOPN];
};

// One queued (read, candidate) pair.
struct QEntry {
    u64 key;   // (genome, diagonal)
    u32 out;   // staging slot: read * top_n + candidate index
    u32 hits;
    u8 pend;   // PendRead slot
    u8 cidx;   // candidate index within the read
};

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline u64 ballot64(bool p) { return __ballot(p); }

// Value of v in lane l (l wave-uniform).
__device__ inline u64 readlane64(u64 v, int l) {
    const u32 lo = __builtin_amdgcn_readlane((u32)v, l), hi = __builtin_amdgcn_readlane((u32)(v >> 32), l);
    return ((u64)hi << 32) | lo;
}

// Number of set bits of m below this lane.
__device__ inline u32 lanes_below(u64 m, int lane) {
    return (u32)__popcll(lane ? m & ((~0ull) >> (64 - lane)) : 0ull);
}

// Slot of a location key in the per-read LDS table.
__device__ inline u32 tslot(u64 key) {
    u32 x = (u32)key ^ (u32)(key >> 29);
    return (x * 0x9E3779B1u) >> 24;
}

// Counts one seed hit of `key` in the per-read LDS table (linear probing; the
// table never holds more than F_HIT_CAP <= F_TSLOTS distinct keys).  A key's
// first hit also lists its slot (tlist, count *tn), so that the candidate
// scan visits only the slots in use.
__device__ inline void table_add(u64 *tkey, u32 *tcnt, u8 *tlist, u32 *tn, u64 key) {
    u32 s = tslot(key);
    for (int probe = 0; probe < F_TSLOTS; probe++, s = (s + 1) & (F_TSLOTS - 1)) {
        u64 cur = tkey[s];
        if (cur == ~0ull) {
            cur = atomicCAS((unsigned long long *)&tkey[s], ~0ull, (unsigned long long)key);
            if (cur == ~0ull) {
                cur = key;
                tlist[atomicAdd(tn, 1u)] = (u8)s;
            }
        }
        if (cur == key) {
            atomicAdd(&tcnt[s], 1u);
            return;
        }
    }
}

// k-mer value at position i from the big-endian 2-bit stream (base j at bits
// 30 - 2(j mod 16) of word j / 16): bits [2i, 2i + 2k) of the stream.
__device__ inline u64 stream_kmer(const u32 *st, int i, u32 k) {
    int w = i >> 4;
    u32 s = 2u * (u32)(i & 15);
    u64 hi = ((u64)st[w] << 32) | st[w + 1];
    u64 y = (hi << s) | (((u64)st[w + 2] << s) >> 32);
    return y >> (64 - 2 * k);
}

// Smallest hash of window [ws, ws + W) (leftmost on ties), all W hashes read
// before the compare chain; -1 when every hash reads ~0 (no valid k-mer in
// the window).  Unrolled for W <= 12 (the usual minimizer windows); wider
// windows take a loop.
template <int W>
__device__ inline int window_argmin(const u64 *hh, int ws) {
    u64 v[W];
#pragma unroll
    for (int t = 0; t < W; t++) v[t] = hh[ws + t];
    u64 bh = ~0ull;
    int bt = -1;  // offset of the best so far (a constant per step)
#pragma unroll
    for (int t = 0; t < W; t++)
        if (v[t] < bh) {
            bh = v[t];
            bt = t;
        }
    return bt < 0 ? -1 : ws + bt;
}

__device__ inline int window_argmin_any(const u64 *hh, int ws, int win) {
    switch (win) {
#define MT_WIN(W) \
    case W:       \
        return window_argmin<W>(hh, ws);
        MT_WIN(1) MT_WIN(2) MT_WIN(3) MT_WIN(4) MT_WIN(5) MT_WIN(6) MT_WIN(7) MT_WIN(8)
        MT_WIN(9) MT_WIN(10) MT_WIN(11) MT_WIN(12)
#undef MT_WIN
    default: {
        u64 bh = ~0ull;
        int best = -1;
        for (int t = 0; t < win; t++) {
            u64 hv = hh[ws + t];
            if (hv < bh) {
                bh = hv;
                best = ws + t;
            }
        }
        return best;
    }
    }
}

// Filters the first qn queued pairs, one pair per group of G lanes (lane_g <
// 2E+1 owns band row d = lane_g - E): the row's mismatch words over the read
// come from the read planes (LDS) and 64-base reference fetches, then the
// obstacle walk runs on registers.  Results go to the staging slot and to the
// pair's pending read.
// Obstacle-free run from column j of a row kept in LDS as four words (all
// ones past them; the row's bits past the read's end are set, so the run
// stops by the end).
__device__ inline int lds_run(const u64 *row, int j) {
    int w = j >> 6;
    const u32 s = (u32)j & 63u;
    int run = 0;
    for (;;) {
        const u64 lo = w < 4 ? row[w < 3 ? w : 3] : ~0ull;
        const u64 hi = w + 1 < 4 ? row[w + 1 < 3 ? w + 1 : 3] : ~0ull;
        const u64 v = funnel(lo, hi, s);
        if (v) return run + (int)__builtin_ctzll(v);
        run += 64;
        w += 1;
    }
}

template <int G>
__device__ __attribute__((always_inline)) inline void filter_batch(const FusedArgs &a, const QEntry *q, int qn, PendRead *pend, int lane,
                                    u64 *rowbuf) {
    const int gi = lane / G, lane_g = lane % G;
    if (gi >= qn) return;
    const QEntry e = q[gi];
    PendRead &pr = pend[e.pend];
    const int E = pr.E, m = pr.m;
    const u32 g = key_genome(e.key);
    const i64 diag = key_diag(e.key);
    const GenomeMeta gm = KA(meta)[g];
    u64 row[4] = {~0ull, ~0ull, ~0ull, ~0ull};
    if (lane_g < 2 * E + 1) {
        // four 64-base fetches per row (building the row from the five blocks it
        // spans, each fetched once, needs more live registers than this kernel
        // has to spare: it spilled four times as many)
        const i64 base = diag + (lane_g - E);
        const u64x2 *rl = KA(ref_lohi) + gm.blk;
        const u64 *rn = KA(ref_nb) + gm.blk;
        const i64 L = (i64)gm.len;
        const bool hn = meta_has_n(gm);
        const Bits64 w0 = fetch_ref(rl, rn, L, hn, base);
        const Bits64 w1 = fetch_ref(rl, rn, L, hn, base + 64);
        const Bits64 w2 = fetch_ref(rl, rn, L, hn, base + 128);
        const Bits64 w3 = fetch_ref(rl, rn, L, hn, base + 192);
        row[0] = (pr.plane[0] ^ w0.lo) | (pr.plane[4] ^ w0.hi) | pr.plane[8] | w0.nb;
        row[1] = (pr.plane[1] ^ w1.lo) | (pr.plane[5] ^ w1.hi) | pr.plane[9] | w1.nb;
        row[2] = (pr.plane[2] ^ w2.lo) | (pr.plane[6] ^ w2.hi) | pr.plane[10] | w2.nb;
        row[3] = (pr.plane[3] ^ w3.lo) | (pr.plane[7] ^ w3.hi) | pr.plane[11] | w3.nb;
    }
    // the row goes to this lane's four words of the per-read LDS table (empty
    // while candidates are filtered: 64 lanes x 4 words fill its 256 slots)
    // and is walked from there, which keeps registers free; the table is
    // emptied again afterwards
    u64 *myrow = rowbuf + 4 * lane;
    myrow[0] = row[0];
    myrow[1] = row[1];
    myrow[2] = row[2];
    myrow[3] = row[3];
    int j = 0, c = 0;
    for (;;) {
        int run = group_max<G>(lds_run(myrow, j));
        j += run;
        if (j >= m) break;
        c += 1;
        if (c > E) break;
        j += 1;
    }
    myrow[0] = myrow[1] = myrow[2] = myrow[3] = ~0ull;
    const int ap = c < E + 1 ? c : E + 1;
    if (lane_g == 0) {
        KA(st_genome)[e.out] = g;
        KA(st_diag)[e.out] = diag;
        KA(st_hits)[e.out] = e.hits;
        KA(st_approx)[e.out] = (u16)ap;
        KA(st_accept)[e.out] = ap <= E;
        pr.apx[e.cidx] = (u16)ap;
        pr.tax[e.cidx] = meta_taxon(gm);
    }
}

// Read accept flag and per-taxon counts of a read whose candidates are all
// filtered: the distinct taxa of its accepted candidates with the smallest
// count; one taxon is unique, several are multi-mapped.
__device__ __attribute__((always_inline)) inline void finalize_read(const FusedArgs &a, const PendRead &pr, u64 *wst) {
    const int nc = (int)pr.nc, E = pr.E;
    int best = 0x7fffffff;
    for (int c = 0; c < nc; c++)
        if (pr.apx[c] <= E && pr.apx[c] < best) best = pr.apx[c];
    if (best == 0x7fffffff) {
        KA(read_accepted)[pr.r] = 0;
        atomicAdd(&wst[ST_UNMAPPED], 1ull);  // the block adds its count once at the end
        return;
    }
    KA(read_accepted)[pr.r] = 1;
    int nt = 0;
    u32 first = 0;
    for (int c = 0; c < nc; c++) {
        if (pr.apx[c] != best) continue;
        bool seen = false;
        for (int b = 0; b < c; b++) seen |= pr.apx[b] == best && pr.tax[b] == pr.tax[c];
        if (seen) continue;
        if (nt == 0) first = pr.tax[c];
        nt++;
    }
    if (nt == 1) {
        atomicAdd(&KA(uniq)[first], 1ull);
        return;
    }
    for (int c = 0; c < nc; c++) {
        if (pr.apx[c] != best) continue;
        bool seen = false;
        for (int b = 0; b < c; b++) seen |= pr.apx[b] == best && pr.tax[b] == pr.tax[c];
        if (!seen) atomicAdd(&KA(multi)[pr.tax[c]], 1ull);
    }
}

// Runs the queued filter batch (group size by the queue's class), then
// finalizes every pending read whose last candidate it filtered.  Returns the
// new set of used pending slots.
template <int MAXG>
__device__ __attribute__((always_inline)) inline u32 flush_queue(const FusedArgs &a, QEntry *q, int &qn, int qG, PendRead *pend, u32 used,
                                  int lane, u64 *wst, u64 *rowbuf) {
    if (qn > 0) {
        if (MAXG == 16 || qG == 16)
            filter_batch<16>(a, q, qn, pend, lane, rowbuf);
        else if (MAXG == 32 || qG == 32)
            filter_batch<32>(a, q, qn, pend, lane, rowbuf);
        else
            filter_batch<64>(a, q, qn, pend, lane, rowbuf);
        wave_sync();
        if (lane == 0)
            for (int i = 0; i < qn; i++) pend[q[i].pend].left -= 1;
        wave_sync();
        qn = 0;
    }
    bool done = lane < F_PCAP && ((used >> lane) & 1u) && pend[lane].left == 0;
    if (done) finalize_read(a, pend[lane], wst);
    u32 fin = (u32)ballot64(done);
    wave_sync();
    return used & ~fin;
}

// The bytes of one read, one per lane for each 64-base round (reads longer
// than the kernel takes are not loaded).
struct ReadBytes {
    u64 beg;
    int m;
    u32 b[4];
};

__device__ inline void issue_read_bytes(const FusedArgs &a, u64 r, int lane, ReadBytes &rb) {
    rb.beg = a.off[r];
    rb.m = (int)(a.off[r + 1] - rb.beg);
#pragma unroll
    for (int q = 0; q < 4; q++) {
        int i = 64 * q + lane;
        rb.b[q] = (rb.m <= F_MAX_M && i < rb.m) ? (u32)a.seq[rb.beg + i] : (u32)'N';
    }
}

// Five wavefronts per SIMD (96 registers, a few spilled; the LDS of 4-wave
// blocks also allows five): the kernel waits on memory as much as it issues.
//
// MAXG: the widest filter group the launch needs (16 when every read's E is at
// most 7, 32 when at most 15, 64 in general); narrower instances hold fewer
// copies of the filter, which leaves the register allocator more room.
// REP: the index is repetitive (many k-mers occur in several genomes, as in a
// database of near-identical strains), so reads whose probes find several
// occurrences are also counted in registers; without it those reads use the
// per-read LDS table, and the instance spends no registers on that path.
template <int MAXG, bool REP>
__global__ __launch_bounds__(64 * F_WPB) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_fused(FusedArgs a) {
    __shared__ u64 sh_h[F_WPB][F_MAX_M];     // k-mer hashes (~0 when invalid); later candidate keys
    __shared__ u64 sh_tkey[F_WPB][F_TSLOTS]; // per-read hash table of (genome, diagonal) keys
    __shared__ u32 sh_tcnt[F_WPB][F_TSLOTS]; // ... and their seed-hit counts
    __shared__ u16 sh_pos[F_WPB][F_MAX_M];   // minimizer positions; later candidate hit counts
    __shared__ u8 sh_pick[F_WPB][F_MAX_M];   // window picks
    __shared__ u32 sh_st[F_WPB][F_WORDS];    // big-endian 2-bit stream of the read
    __shared__ u32 sh_sel[F_WPB][F_MAX_TOPN];
    __shared__ QEntry sh_q[F_WPB][F_QCAP];
    __shared__ PendRead sh_pend[F_WPB][F_PCAP];
    __shared__ u64 sh_stats[F_WPB][ST_COUNT];
    __shared__ u8 sh_tlist[F_WPB][F_TSLOTS];  // slots of the per-read table in use
    __shared__ u32 sh_tn[F_WPB];             // ... and their number

    // wid is wave-uniform; saying so keeps every per-read value (read index,
    // length, E, loop bounds) in scalar registers.
    if (*a.gate) return;  // malformed offsets: nothing may be read through them
    const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    u64 *hh = sh_h[wid];
    u64 *tkey = sh_tkey[wid];
    u32 *tcnt = sh_tcnt[wid];
    u16 *ccnt = sh_pos[wid];  // candidate hit counts reuse the minimizer positions (dead after the probes)
    u16 *mpos = sh_pos[wid];
    u8 *pick = sh_pick[wid];
    u32 *stream = sh_st[wid];
    u32 *sel = sh_sel[wid];
    QEntry *queue = sh_q[wid];
    PendRead *pend = sh_pend[wid];
    u64 *wst = sh_stats[wid];
    u8 *tlist = sh_tlist[wid];
    u32 *tn = &sh_tn[wid];
    if (lane < ST_COUNT) wst[lane] = 0;
    if (lane == 0) *tn = 0;
    // the table starts empty and every read leaves it empty
    for (int t = lane; t < F_TSLOTS; t += 64) {
        tkey[t] = ~0ull;
        tcnt[t] = 0;
    }

    const u32 k = a.k, T = a.min_hits ? a.min_hits : 1u, N = a.ncap;
    const u64 kmask = (1ull << k) - 1;
    const u64 stride = (u64)gridDim.x * F_WPB;
    u32 wflags = 0;
    int qn = 0, qG = 16;  // queued pairs and their group size
    u32 used = 0;         // pending-read slots in use

    u64 r = (u64)blockIdx.x * F_WPB + wid;
    ReadBytes cur;
    if (r < a.n) issue_read_bytes(a, r, lane, cur);
    for (; r < a.n; r += stride) {
        const u64 rn = r + stride;
        const int m = cur.m;
        u64 Ewide = KA(e_mode) == MT_E_FIXED ? KA(e_value)
                    : KA(e_mode) == MT_E_CEIL_PERMILLE ? ((u64)m * KA(e_value) + 999) / 1000
                                                     : ((u64)m * KA(e_value)) / 1000;
        if (Ewide > 65534) wflags |= ERR_E_TOO_LARGE;
        const int E = Ewide > 65535 ? 65535 : (int)Ewide;
        if (lane == 0) KA(read_E)[r] = (u16)E;
        if (m > F_MAX_M || E > F_MAX_E) {  // (2E + 1 <= MAXG here: the launch picks MAXG from the largest E)
            if (lane == 0) {
                KA(fb_list)[atomicAdd(KA(fb_count), 1u)] = (u32)r;
                KA(ncand)[r] = 0;  // until the per-stage kernels fill it in
            }
            if (rn < a.n) issue_read_bytes(a, rn, lane, cur);
            continue;
        }

        // 1. bit planes of the read (bases past m are N), written straight into
        // a free pending-read slot, and the read's big-endian 2-bit stream
        const int slot = __builtin_ctz(~used);
        PendRead &pr = pend[slot];
        if (lane < F_WORDS) stream[lane] = 0;
        bool bad = false;
        // the next read's offsets, its start in even lanes and its end in odd
        // ones: requested before the planes are built and read after them, so
        // the planes hide the load (a wave-uniform load would be waited for at
        // once, to move it to scalar registers)
        u64 noff = 0;
        if (rn < a.n) noff = a.off[rn + (u64)(lane & 1)];
        wave_sync();
#pragma unroll
        for (int q = 0; q < 4; q++) {
            int i = 64 * q + lane;
            u32 c = i < m ? base_code(cur.b[q]) : 4u;
            bad |= c == 5;
            u64 lo = ballot64(c < 4 && (c & 1u));
            u64 hi = ballot64(c < 4 && (c & 2u));
            u64 nb = ballot64(c >= 4);
            if (lane == 0) {
                pr.plane[q] = lo;
                pr.plane[4 + q] = hi;
                pr.plane[8 + q] = nb;
            }
            if (c < 4 && c > 0) atomicOr(&stream[i >> 4], c << (30 - 2 * (i & 15)));
        }
        // (the next read's bytes are requested after the probes)
        const u64 nbeg = readlane64(noff, 0), nend = readlane64(noff, 1);
        if (ballot64(bad)) {
            wflags |= ERR_BAD_BYTE;
            if (lane == 0) KA(ncand)[r] = 0;  // the call fails; its compaction still runs
            if (rn < a.n) issue_read_bytes(a, rn, lane, cur);
            continue;
        }
        wave_sync();

        // 2. k-mer hashes (~0 for k-mers with an N)
        const int nk = m - (int)k + 1;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            int i = 64 * q + lane;
            if (i < nk) {
                u64 nb = funnel(pr.plane[8 + q], q < 3 ? pr.plane[9 + q] : ~0ull, (u32)lane);
                hh[i] = (nb & kmask) == 0 ? mix64(stream_kmer(stream, i, k)) : ~0ull;
            }
            pick[i] = 0;
        }
        wave_sync();

        // 3. window minima: an invalid k-mer reads as ~0, a hash no valid k-mer
        // has (the hash is a bijection and the preimage of ~0 lies above every
        // 62-bit k-mer value), so a window of ~0 alone has no minimizer.
        int nmin = 0;
        if (nk > 0) {
            const int win = nk < (int)a.w ? nk : (int)a.w;
            const int nws = nk - win + 1;
#pragma unroll 1
            for (int q = 0; q < 4; q++) {
                int ws = 64 * q + lane;
                if (ws < nws) {
                    const int best = window_argmin_any(hh, ws, win);
                    if (best >= 0) pick[best] = 1;
                }
            }
            wave_sync();
#pragma unroll
            for (int q = 0; q < 4; q++) {
                int i = 64 * q + lane;
                bool chosen = i < nk && pick[i];
                u64 cm = ballot64(chosen);
                if (chosen) mpos[nmin + lanes_below(cm, lane)] = (u16)i;
                nmin += __popcll(cm);
            }
            wave_sync();
        }

        // 4. table probes -> seed hits.  When every minimizer fits one round
        // and the hits fit one lane each (at most 64 of them, at most 15 per
        // probe), they are counted in registers: one ballot per distinct
        // location; otherwise they go through the per-read LDS table.  With
        // one occurrence per probe (the usual case) a probe's lane holds its
        // hit; otherwise every probe lists its hits in the (empty) table at
        // its prefix offset and lane h takes hit h, the occurrences of all
        // probes being read in one round trip.
        int H = 0, C = 0, nocc = 0;  // nocc: entries read from the multi-occurrence array
        bool overflow = false, counted = false;
        for (int t0 = 0; t0 < nmin; t0 += 64) {
            int j = t0 + lane;
            u64 v = SLOT_NONE;
            int p = 0;
            u32 cnt = 0;
            if (j < nmin) {
                p = mpos[j];
                v = table_lookup(a.table, a.nbuckets, stream_kmer(stream, p, k));
                cnt = v == SLOT_NONE ? 0u : slot_count(v);
            }
            const bool single = cnt == 1 && !(v & SLOT_MULTI);
            const u64 sm = ballot64(single);
            const u64 mm = ballot64(cnt != 0 && !single);  // probes with several occurrences
            bool inreg = false;
            u64 key = 0, hm = 0;  // this lane's hit and the lanes holding one
            if (t0 == 0 && nmin <= 64 && mm == 0) {
                key = single ? cand_key((u32)(v >> 32), (i64)(u32)v - p) : 0ull;
                hm = sm;
                H = __popcll(sm);
                inreg = true;
            } else if (REP && t0 == 0 && nmin <= 64 && ballot64(cnt > 15u) == 0) {
                // exclusive prefix sum of cnt over the lanes, bit by bit
                u32 off = 0, tot = 0;
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    const u64 bm = ballot64((cnt >> b) & 1u);
                    off += lanes_below(bm, lane) << b;
                    tot += (u32)__popcll(bm) << b;
                }
                if (tot <= 64) {
                    // per hit: the slot value (one occurrence) or the index of
                    // the occurrence, and the minimizer position with bit 16
                    // marking an index
                    for (u32 u = 0; u < cnt; u++) {
                        tkey[off + u] = single ? v : slot_start(v) + u;
                        tcnt[off + u] = (u32)p | (single ? 0u : 0x10000u);
                    }
                    wave_sync();
                    const bool has = lane < (int)tot;
                    u64 gv = has ? tkey[lane] : 0ull;
                    const u32 f = has ? tcnt[lane] : 0u;
                    if (has) {  // the table is left empty again
                        tkey[lane] = ~0ull;
                        tcnt[lane] = 0;
                    }
                    if (f & 0x10000u) gv = KA(occ)[gv];
                    key = has ? cand_key((u32)(gv >> 32), (i64)(u32)gv - (i64)(f & 0xffffu)) : 0ull;
                    hm = ballot64(has);
                    H = (int)tot;
                    nocc += (int)tot - __popcll(sm);
                    inreg = true;
                }
            }
            if (inreg) {
                const bool mine = REP ? (bool)((hm >> lane) & 1u) : single;
                for (u64 rem = hm; rem;) {
                    const int ld = __builtin_amdgcn_readfirstlane(__builtin_ctzll(rem));
                    const u64 kl = readlane64(key, ld);
                    const u64 eq = ballot64(mine && key == kl);
                    const u32 c = (u32)__popcll(eq);
                    if (c >= T) {
                        if (lane == 0) {
                            hh[C] = kl;
                            ccnt[C] = (u16)c;
                        }
                        C++;
                    }
                    rem &= ~eq;
                }
                counted = true;
                break;
            }
            u32 tot = (u32)__popcll(sm);
            for (u64 rem = mm; rem; rem &= rem - 1)
                tot += __builtin_amdgcn_readlane(cnt, __builtin_amdgcn_readfirstlane(__builtin_ctzll(rem)));
            nocc += (int)(tot - (u32)__popcll(sm));
            if (H + (int)tot > F_HIT_CAP) {
                overflow = true;
                break;
            }
            if (cnt) {
                if (!(v & SLOT_MULTI)) {
                    table_add(tkey, tcnt, tlist, tn, cand_key((u32)(v >> 32), (i64)(u32)v - p));
                } else {  // several occurrences: four loads in flight at a time
                    const u64 st = slot_start(v);
                    for (u32 u0 = 0; u0 < cnt; u0 += 4) {
                        u64 gp[4];
#pragma unroll
                        for (int t = 0; t < 4; t++) gp[t] = u0 + t < cnt ? KA(occ)[st + u0 + t] : 0ull;
#pragma unroll
                        for (int t = 0; t < 4; t++)
                            if (u0 + t < cnt) table_add(tkey, tcnt, tlist, tn, cand_key((u32)(gp[t] >> 32), (i64)(u32)gp[t] - p));
                    }
                }
            }
            H += (int)tot;
        }
        // the next read's bytes arrive while this one is counted and filtered
        ReadBytes nxt;
        if (rn < a.n) {
            nxt.beg = nbeg;
            nxt.m = (int)(nend - nbeg);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                int i = 64 * q + lane;
                nxt.b[q] = (nxt.m <= F_MAX_M && i < nxt.m) ? (u32)a.seq[nbeg + i] : (u32)'N';
            }
        }
        wave_sync();
        if (overflow) {
            for (int t = lane; t < F_TSLOTS; t += 64) {
                tkey[t] = ~0ull;
                tcnt[t] = 0;
            }
            if (lane == 0) {
                *tn = 0;
                KA(fb_list)[atomicAdd(KA(fb_count), 1u)] = (u32)r;
                KA(ncand)[r] = 0;
            }
            cur = nxt;
            wave_sync();
            continue;
        }

        // 5. locations with >= min_hits hits become candidates (the table is
        // emptied as it is read), then top_n by rank
        if (!counted && H > 0) {
            const int nd = (int)*tn;  // distinct keys: the listed slots
            for (int q0 = 0; q0 < nd; q0 += 64) {
                const bool in = q0 + lane < nd;
                const int t = in ? tlist[q0 + lane] : 0;
                const u64 key = in ? tkey[t] : ~0ull;
                const u32 c = in ? tcnt[t] : 0u;
                const bool is_c = key != ~0ull && c >= T;
                if (in) {
                    tkey[t] = ~0ull;
                    tcnt[t] = 0;
                }
                const u64 cm = ballot64(is_c);
                if (is_c) {
                    const int s2 = C + (int)lanes_below(cm, lane);
                    hh[s2] = key;
                    ccnt[s2] = (u16)c;
                }
                C += __popcll(cm);
            }
        }
        wave_sync();
        if (lane == 0) *tn = 0;
        if (a.top_n == 0 && C > (int)N) {
            // keep-all with more candidates than staging slots: per-stage finish
            if (lane == 0) {
                KA(fb_list)[atomicAdd(KA(fb_count), 1u)] = (u32)r;
                KA(ncand)[r] = 0;
            }
            cur = nxt;
            wave_sync();
            continue;
        }
        const int nc = C < (int)N ? C : (int)N;
        for (int t0 = 0; t0 < C; t0 += 64) {
            int cidx = t0 + lane;
            if (cidx < C) {
                u64 kc = hh[cidx];
                u32 hc = ccnt[cidx];
                int rank = 0;
#pragma unroll 4
                for (int b = 0; b < C; b++) {
                    u32 hb = ccnt[b];
                    rank += hb > hc || (hb == hc && hh[b] < kc);
                }
                if (rank < nc) sel[rank] = (u32)cidx;
            }
        }
        wave_sync();

        // 6. queue the kept candidates for batched filtering
        if (lane == 0) KA(ncand)[r] = (u32)nc;
        if (nc == 0) {
            if (lane == 0) {
                KA(read_accepted)[r] = 0;
                atomicAdd(&wst[ST_UNMAPPED], 1ull);
            }
        } else {
            const int rows = 2 * E + 1;
            const int G = (MAXG == 16 || rows <= 16) ? 16 : (MAXG == 32 || rows <= 32) ? 32 : 64;
            used |= 1u << slot;
            if (lane == 0) {
                pr.r = r;
                pr.nc = (u32)nc;
                pr.left = (u32)nc;
                pr.E = (u16)E;
                pr.m = (u16)m;
            }
            wave_sync();
            // one flush site: the queue is flushed when it is full or holds
            // pairs of another group size; the candidates that fit are queued
            // together, one lane each
            for (int c0 = 0; c0 < nc;) {
                if (qn > 0 && (qn == 64 / qG || qG != G))
                    used = flush_queue<MAXG>(a, queue, qn, qG, pend, used, lane, wst, tkey);
                qG = G;
                const int room = 64 / G - qn;
                const int take = nc - c0 < room ? nc - c0 : room;
                if (lane < take) {
                    const int c = c0 + lane;
                    const u32 si = sel[c];
                    queue[qn + lane] = QEntry{hh[si], (u32)(r * N + (u64)c), ccnt[si], (u8)slot, (u8)c};
                }
                qn += take;
                c0 += take;
                wave_sync();
            }
        }
        if (lane == 0) {  // work counts, kept in LDS to spare registers
            wst[ST_READS] += 1;
            wst[ST_BASES] += (u64)m;
            wst[ST_MINS] += (u64)nmin;
            wst[ST_CANDS] += (u64)nc;
            wst[ST_WBLOCKS] += (u64)nc * (u64)((m + 2 * E + 63) / 64);
            wst[ST_OCC] += (u64)nocc;
        }
        cur = nxt;
        wave_sync();
    }
    used = flush_queue<MAXG>(a, queue, qn, qG, pend, used, lane, wst, tkey);
    if (lane == 0) {
        if (used) wflags |= ERR_INTERNAL;  // every queued read is finalized by now
        if (wflags) atomicOr(KA(flags), wflags);
    }
    // work counts: one record per block, summed by k_fused_summary
    __syncthreads();
    if (threadIdx.x < ST_COUNT) {
        u64 t = 0;
        for (int w = 0; w < F_WPB; w++) t += sh_stats[w][threadIdx.x];
        KA(stats_part)[(u64)blockIdx.x * ST_COUNT + threadIdx.x] = t;
        // unmapped reads: one global atomic per block instead of one per read
        if (threadIdx.x == ST_UNMAPPED && t) atomicAdd(KA(unmapped), (unsigned long long)t);
    }
}

// Control words of one fused call: [0] offsets check, [1] run flags,
// [2] fallback count.
constexpr int CTL_GATE = 0, CTL_FLAGS = 1, CTL_FB = 2, CTL_WORDS = 4;

// Host-visible summary of one fused call, read back with a single copy.
struct FusedSummary {
    u32 gate, flags, nfb, pad;
    u64 n_cands;
    u64 stats[ST_COUNT];
};

__global__ void k_fused_init(u32 *__restrict__ ctl) {
    if (threadIdx.x < CTL_WORDS) ctl[threadIdx.x] = 0;
}

// Block s < ST_COUNT sums work count s over the kernel's blocks; block 0
// also copies the control words and the candidate total.
constexpr int SUM_TPB = 1024;
__global__ __launch_bounds__(SUM_TPB) void k_fused_summary(const u32 *__restrict__ ctl,
                                                           const u64 *__restrict__ cand_end,
                                                           const u64 *__restrict__ stats_part, u32 blocks,
                                                           FusedSummary *__restrict__ out) {
    __shared__ u64 part[SUM_TPB / 64];
    const int st = blockIdx.x, t = threadIdx.x;
    u64 acc = 0;
    if (!ctl[CTL_GATE])
        for (u32 b = t; b < blocks; b += SUM_TPB) acc += stats_part[(u64)b * ST_COUNT + st];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((t & 63) == 0) part[t >> 6] = acc;
    __syncthreads();
    if (t == 0) {
        u64 v = 0;
        for (int i = 0; i < SUM_TPB / 64; i++) v += part[i];
        out->stats[st] = v;
        if (st == 0) {
            out->gate = ctl[CTL_GATE];
            out->flags = ctl[CTL_FLAGS];
            out->nfb = ctl[CTL_FB];
            out->pad = 0;
            out->n_cands = ctl[CTL_GATE] ? 0 : *cand_end;
        }
    }
}

// Offsets check for the fused path (it reads the ASCII bytes directly).
__global__ void k_check_reads(const u64 *__restrict__ off, u64 n, u64 total, u32 *__restrict__ flags) {
    u64 s = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    u64 a = off[s], b = off[s + 1];
    u32 f = 0;
    if (b < a || b > total || (s == 0 && a != 0) || (s == n - 1 && b != total)) f |= ERR_OFFSETS;
    else if (b - a > 65535) f |= ERR_READ_TOO_LONG;
    if (f) atomicOr(flags, f);
}

// Subset of reads (the fallback list) gathered into a contiguous batch.
__global__ void k_subset_lengths(const u64 *__restrict__ off, const u32 *__restrict__ list, u64 n,
                                 u64 *__restrict__ len) {
    u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) len[i] = off[list[i] + 1] - off[list[i]];
}

__global__ void k_subset_copy(const u8 *__restrict__ seq, const u64 *__restrict__ off, const u32 *__restrict__ list,
                              u64 n, const u64 *__restrict__ sub_off, u8 *__restrict__ sub_seq) {
    u64 i = blockIdx.x;
    if (i >= n) return;
    u64 src = off[list[i]], dst = sub_off[i], len = sub_off[i + 1] - dst;
    for (u64 t = threadIdx.x; t < len; t += blockDim.x) sub_seq[dst + t] = seq[src + t];
}

__global__ void k_subset_scatter(const u32 *__restrict__ list, u64 n, u32 stride, const u64 *__restrict__ sub_off,
                                 const u8 *__restrict__ sub_acc, const u32 *__restrict__ sg,
                                 const i64 *__restrict__ sd, const u32 *__restrict__ sh,
                                 const u16 *__restrict__ sa, const u8 *__restrict__ sc, u32 *__restrict__ ncand,
                                 u8 *__restrict__ read_accepted, u32 *__restrict__ st_genome,
                                 i64 *__restrict__ st_diag, u32 *__restrict__ st_hits, u16 *__restrict__ st_approx,
                                 u8 *__restrict__ st_accept) {
    u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    u64 r = list[i];
    u64 b = sub_off[i], e = sub_off[i + 1];
    ncand[r] = (u32)(e - b);
    read_accepted[r] = sub_acc[i];
    for (u64 c = b; c < e && c - b < stride; c++) {  // the rest (keep-all) is placed by k_subset_place
        u64 o = r * stride + (c - b);
        st_genome[o] = sg[c];
        st_diag[o] = sd[c];
        st_hits[o] = sh[c];
        st_approx[o] = sa[c];
        st_accept[o] = sc[c];
    }
}

// Candidates of the per-stage finished reads straight into the final arrays
// (keep-all reads may have more candidates than staging slots).
__global__ void k_subset_place(const u32 *__restrict__ list, u64 n, const u64 *__restrict__ sub_off,
                               const u32 *__restrict__ sg, const i64 *__restrict__ sd, const u32 *__restrict__ sh,
                               const u16 *__restrict__ sa, const u8 *__restrict__ sc,
                               const u64 *__restrict__ cand_off, u64 cap, u32 *__restrict__ genome,
                               i64 *__restrict__ diag, u32 *__restrict__ hits, u16 *__restrict__ approx,
                               u8 *__restrict__ accept) {
    u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u64 r = list[i], b = sub_off[i], e = sub_off[i + 1], o = cand_off[r];
    if (o + (e - b) > cap) return;  // never past the candidate capacity
    for (u64 c = b; c < e; c++) {
        genome[o + c - b] = sg[c];
        diag[o + c - b] = sd[c];
        hits[o + c - b] = sh[c];
        approx[o + c - b] = sa[c];
        accept[o + c - b] = sc[c];
    }
}

__global__ void k_add_u64(unsigned long long *__restrict__ dst, const u64 *__restrict__ src, u64 n) {
    u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] += src[i];
}

__global__ void k_compact_staged(const u32 *__restrict__ gate, const u64 *__restrict__ cand_off, u64 n, u32 top_n,
                                 u64 cap,
                                 const u32 *__restrict__ st_genome, const i64 *__restrict__ st_diag,
                                 const u32 *__restrict__ st_hits, const u16 *__restrict__ st_approx,
                                 const u8 *__restrict__ st_accept, u32 *__restrict__ genome, i64 *__restrict__ diag,
                                 u32 *__restrict__ hits, u16 *__restrict__ approx, u8 *__restrict__ accept) {
    u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n || *gate) return;
    u64 o = cand_off[r], c = cand_off[r + 1] - o;
    if (c > top_n) c = top_n;
    if (o > cap || c > cap - o) return;  // never past the candidate capacity
    for (u64 i = 0; i < c; i++) {
        u64 s = r * top_n + i;
        genome[o + i] = st_genome[s];
        diag[o + i] = st_diag[s];
        hits[o + i] = st_hits[s];
        approx[o + i] = st_approx[s];
        accept[o + i] = st_accept[s];
    }
}

// The launches of one fused call once its buffers exist: no host
// synchronization and no memset, so the sequence can also be captured and
// replayed as one HIP graph.
struct FusedLaunch {
    FusedArgs a;
    u32 *ctl;
    u64 n;
    u32 N;
    unsigned blocks;
    u64 total;
    mt_result *res;
    FusedSummary *sum;
    bool rep;  // repetitive index: the kernel instance with register counting of repeated k-mers
};

static void enqueue_fused(const FusedLaunch &L, Timer *tm, hipStream_t s) {
    const FusedArgs &a = L.a;
    k_fused_init<<<1, 64, 0, s>>>(L.ctl);
    k_check_reads<<<grid_for(L.n, 256), 256, 0, s>>>(a.off, L.n, L.total, L.ctl + CTL_GATE);
    if (tm) tm->mark("check");
    // the widest filter group any read can need: E is fixed, or grows with the
    // length, which is at most F_MAX_M in the kernel (longer reads take the
    // per-stage path), so every fused read's 2E + 1 rows fit the instance's
    // widest group
    u64 maxE = a.e_mode == MT_E_FIXED           ? a.e_value
               : a.e_mode == MT_E_CEIL_PERMILLE ? ((u64)F_MAX_M * a.e_value + 999) / 1000
                                                : ((u64)F_MAX_M * a.e_value) / 1000;
    if (maxE > (u64)F_MAX_E) maxE = F_MAX_E;
    if (L.rep) {
        if (maxE <= 7)
            k_fused<16, true><<<L.blocks, 64 * F_WPB, 0, s>>>(a);
        else if (maxE <= 15)
            k_fused<32, true><<<L.blocks, 64 * F_WPB, 0, s>>>(a);
        else
            k_fused<64, true><<<L.blocks, 64 * F_WPB, 0, s>>>(a);
    } else {
        if (maxE <= 7)
            k_fused<16, false><<<L.blocks, 64 * F_WPB, 0, s>>>(a);
        else if (maxE <= 15)
            k_fused<32, false><<<L.blocks, 64 * F_WPB, 0, s>>>(a);
        else
            k_fused<64, false><<<L.blocks, 64 * F_WPB, 0, s>>>(a);
    }
    if (tm) tm->mark("fused");
    scan_u32(a.ncand, L.res->cand_off.p, L.n, s);
    k_compact_staged<<<grid_for(L.n, 256), 256, 0, s>>>(L.ctl + CTL_GATE, L.res->cand_off.p, L.n, L.N, L.res->cap,
                                                        a.st_genome,
                                                        a.st_diag, a.st_hits, a.st_approx, a.st_accept,
                                                        L.res->genome.p, L.res->diag.p, L.res->hits.p,
                                                        L.res->approx.p, L.res->accept.p);
    k_fused_summary<<<ST_COUNT, SUM_TPB, 0, s>>>(L.ctl, L.res->cand_off.p + L.n, a.stats_part, L.blocks, L.sum);
    MT_HIP(hipGetLastError());
    if (tm) tm->mark("compact");
}

// One executable graph per host thread, updated in place when a new capture
// has the same shape (only kernel arguments differ) and rebuilt otherwise.
struct GraphCache {
    hipGraphExec_t exec = nullptr;
    ~GraphCache() {
        if (exec) (void)hipGraphExecDestroy(exec);
    }
};
static thread_local GraphCache g_graph;

static void launch_fused_graph(const FusedLaunch &L, hipStream_t s) {
    if (s == nullptr) throw Error(MT_EINVAL, "the graph form needs a stream other than the null stream");
    hipGraph_t graph = nullptr;
    MT_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    try {
        enqueue_fused(L, nullptr, s);
    } catch (...) {
        (void)hipStreamEndCapture(s, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
    }
    MT_HIP(hipStreamEndCapture(s, &graph));
    bool updated = false;
    if (g_graph.exec) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult ur;
        updated = hipGraphExecUpdate(g_graph.exec, graph, &err_node, &ur) == hipSuccess &&
                  ur == hipGraphExecUpdateSuccess;
        if (!updated) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(g_graph.exec);
            g_graph.exec = nullptr;
        }
    }
    hipError_t e = hipSuccess;
    if (!updated) e = hipGraphInstantiate(&g_graph.exec, graph, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipGraphLaunch(g_graph.exec, s);
    (void)hipGraphDestroy(graph);
    MT_HIP(e);
}

void classify_fused(const mt_index &ix, const mt_query_params &q, const mt_seqs &reads, ReadBatch &rb,
                    mt_result &res, Timer &tm, hipStream_t s, bool graph) {
    if (q.filter != MT_FILTER_OBSTACLE || q.strands == 2) {  // the fused kernel: obstacle walk, forward strand
        classify_staged(ix, q, reads, rb, res, tm, s);
        return;
    }
    const u64 n = reads.n;
    // staging slots per read: top_n, or F_MAX_TOPN for keep-all (top_n = 0;
    // reads with more candidates are finished per stage)
    const u32 N = q.top_n ? q.top_n : (u32)F_MAX_TOPN;
    if (q.top_n > (u32)F_MAX_TOPN) {
        // Long candidate lists: the per-stage kernels handle them.
        rb.prepare(reads, q.e_mode, q.e_value, s);
        MT_HIP(hipMemcpyAsync(res.read_E.p, rb.read_E.p, (n ? n : 1) * sizeof(u16), hipMemcpyDeviceToDevice, s));
        tm.mark("pack");
        classify_per_stage(ix, q, reads, rb, res, tm, s);
        u32 f = 0;
        read_back(s, rb.flags.p, &f, sizeof f);
        check_flags(f);
        read_back(s, res.cand_off.p + n, &res.n_cands, sizeof(u64));
        return;
    }
    rb.n = n;
    if (n == 0) {
        res.n_cands = 0;
        return;
    }

    int dev = 0, cus = 0;
    MT_HIP(hipGetDevice(&dev));
    MT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    u64 blocks = (n + F_WPB - 1) / F_WPB;
    const u64 cap = (u64)cus * 64;  // many short blocks: resident blocks finish together
    if (blocks > cap) blocks = cap;

    DBuf<u32> st_genome(n * N), st_hits(n * N), ncand(n), fb_list(n), ctl(CTL_WORDS);
    DBuf<i64> st_diag(n * N);
    DBuf<u16> st_approx(n * N);
    DBuf<u8> st_accept(n * N);
    DBuf<u64> stats_part(blocks * ST_COUNT);
    DBuf<FusedSummary> sum(1);
    res.alloc_cands(n * N);

    FusedLaunch L{};
    FusedArgs &a = L.a;
    a.seq = (const u8 *)reads.seq;
    a.off = reads.offsets;
    a.n = n;
    a.k = ix.k;
    a.w = ix.w;
    a.min_hits = q.min_hits;
    a.top_n = q.top_n;
    a.ncap = N;
    a.e_mode = q.e_mode;
    a.e_value = q.e_value;
    a.table = ix.table.p;
    a.nbuckets = ix.nbuckets;
    a.occ = ix.occ.p;
    a.meta = ix.meta.p;
    a.ref_lohi = ix.ref.lohi.p;
    a.ref_nb = ix.ref.nb.p;
    a.st_genome = st_genome.p;
    a.st_diag = st_diag.p;
    a.st_hits = st_hits.p;
    a.st_approx = st_approx.p;
    a.st_accept = st_accept.p;
    a.ncand = ncand.p;
    a.read_accepted = res.read_accepted.p;
    a.read_E = res.read_E.p;
    a.uniq = (unsigned long long *)res.uniq.p;
    a.multi = (unsigned long long *)res.multi.p;
    a.unmapped = (unsigned long long *)res.unmapped.p;
    a.fb_list = fb_list.p;
    a.fb_count = ctl.p + CTL_FB;
    a.flags = ctl.p + CTL_FLAGS;
    a.gate = ctl.p + CTL_GATE;
    a.stats_part = stats_part.p;
    L.ctl = ctl.p;
    L.n = n;
    L.N = N;
    L.blocks = (unsigned)blocks;
    L.total = reads.total;
    L.res = &res;
    L.sum = sum.p;
    // repetitive: at least one occurrence in eight belongs to a k-mer found in
    // several places
    L.rep = ix.n_multi_occ * 8 >= ix.n_minimizers && ix.n_multi_occ > 0;

    if (graph) {
        launch_fused_graph(L, s);
        tm.mark("graph");
    } else {
        enqueue_fused(L, &tm, s);
    }
    FusedSummary h{};
    read_back(s, sum.p, &h, sizeof h);
    check_flags(h.gate | h.flags);
    mt_stats &ls = last_stats();
    ls.fused_reads += h.stats[ST_READS];
    ls.fused_bases += h.stats[ST_BASES];
    ls.fused_minimizers += h.stats[ST_MINS];
    ls.fused_window_blocks += h.stats[ST_WBLOCKS];
    ls.fused_cands += h.stats[ST_CANDS];
    ls.fused_occ += h.stats[ST_OCC];
    ls.n_minimizers += h.stats[ST_MINS];
    // Every read's count is at most N (k_fused writes one count per read), so
    // the total fits the staged capacity; a result never claims more
    // candidates than its arrays hold.
    if (h.n_cands > res.cap) throw Error(MT_EINTERNAL, "fused candidate count exceeds the staged capacity");
    res.n_cands = h.n_cands;
    const u32 nfb = h.nfb;
    if (nfb == 0) return;

    // Reads past the fused kernel's limits: finish them per stage on a
    // gathered subset, scatter the results into the staging slots, and
    // compact again.
    DBuf<u64> sub_len(nfb), sub_off(nfb + 1);
    k_subset_lengths<<<grid_for(nfb, 256), 256, 0, s>>>(reads.offsets, fb_list.p, nfb, sub_len.p);
    MT_HIP(hipGetLastError());
    scan_u64(sub_len.p, sub_off.p, nfb, s);
    u64 sub_total = 0;
    read_back(s, sub_off.p + nfb, &sub_total, sizeof sub_total);
    DBuf<u8> sub_seq(sub_total);
    k_subset_copy<<<nfb, 256, 0, s>>>((const u8 *)reads.seq, reads.offsets, fb_list.p, nfb, sub_off.p, sub_seq.p);
    MT_HIP(hipGetLastError());
    mt_seqs sub{(const char *)sub_seq.p, sub_off.p, nfb, sub_total};
    mt_result tmp;
    mt_result_init(tmp, nfb, ix.n_taxa, s);
    ReadBatch srb;
    srb.prepare(sub, q.e_mode, q.e_value, s);
    classify_per_stage(ix, q, sub, srb, tmp, tm, s);
    u32 f2 = 0;
    read_back(s, srb.flags.p, &f2, sizeof f2);
    check_flags(f2);
    k_subset_scatter<<<grid_for(nfb, 256), 256, 0, s>>>(fb_list.p, nfb, N, tmp.cand_off.p, tmp.read_accepted.p,
                                                        tmp.genome.p, tmp.diag.p, tmp.hits.p, tmp.approx.p,
                                                        tmp.accept.p, ncand.p, res.read_accepted.p, st_genome.p,
                                                        st_diag.p, st_hits.p, st_approx.p, st_accept.p);
    MT_HIP(hipGetLastError());
    if (ix.n_taxa) {
        k_add_u64<<<grid_for(ix.n_taxa, 256), 256, 0, s>>>((unsigned long long *)res.uniq.p, tmp.uniq.p, ix.n_taxa);
        k_add_u64<<<grid_for(ix.n_taxa, 256), 256, 0, s>>>((unsigned long long *)res.multi.p, tmp.multi.p,
                                                           ix.n_taxa);
    }
    k_add_u64<<<1, 64, 0, s>>>((unsigned long long *)res.unmapped.p, tmp.unmapped.p, 1);
    scan_u32(ncand.p, res.cand_off.p, n, s);
    u64 total = 0;
    read_back(s, res.cand_off.p + n, &total, sizeof total);
    if (total > res.cap) res.alloc_cands(total);  // keep-all reads with many candidates
    k_compact_staged<<<grid_for(n, 256), 256, 0, s>>>(ctl.p + CTL_GATE, res.cand_off.p, n, N, res.cap, st_genome.p,
                                                      st_diag.p, st_hits.p, st_approx.p, st_accept.p, res.genome.p,
                                                      res.diag.p, res.hits.p, res.approx.p, res.accept.p);
    MT_HIP(hipGetLastError());
    if (q.top_n == 0) {
        // the finished reads' full lists, after the compaction (which copied
        // at most N staged entries of theirs)
        k_subset_place<<<grid_for(nfb, 256), 256, 0, s>>>(fb_list.p, nfb, tmp.cand_off.p, tmp.genome.p, tmp.diag.p,
                                                          tmp.hits.p, tmp.approx.p, tmp.accept.p, res.cand_off.p,
                                                          res.cap, res.genome.p, res.diag.p, res.hits.p,
                                                          res.approx.p, res.accept.p);
        MT_HIP(hipGetLastError());
    }
    res.n_cands = total;
    tm.mark("fallback");
}

// ------------------------------------------------------ containment search --

// Containment search (Fig. 1 steps 1a-1c) for reads of up to F_MAX_M bases,
// one wavefront per read: its N plane by ballot and its 2-bit stream in LDS,
// k-mer hashes and window minima as in k_fused (steps 1-3), then one table
// probe per minimizer lane adding one hit to the genome of every occurrence.
// Up to CF_LDS_GENOMES genomes a block counts in LDS and adds its nonzero
// counters to the global ones when it ends; with more genomes the hits go to
// the global counters directly.  Longer reads are listed for the per-stage
// chain.
struct ContainArgs {
    const u8 *seq;
    const u64 *off;
    u64 n;
    u32 k, w;
    const u64x2 *table;
    u64 nbuckets;
    const u64 *occ;
    u64 n_genomes;
    unsigned long long *hits;
    u32 *fb_list;
    u32 *fb_count;
    u32 *flags;
    const u32 *gate;  // offsets check result: nonzero skips the whole launch
};

constexpr u64 CF_LDS_GENOMES = 2048;  // 64-bit counters, at most 16 KB per block

__global__ __launch_bounds__(64 * F_WPB) void k_contain_fused(ContainArgs a) {
    __shared__ u64 sh_h[F_WPB][F_MAX_M];
    __shared__ u16 sh_pos[F_WPB][F_MAX_M];
    __shared__ u8 sh_pick[F_WPB][F_MAX_M];
    __shared__ u32 sh_st[F_WPB][F_WORDS];
    __shared__ u64 sh_nb[F_WPB][4];
    extern __shared__ unsigned long long cnt[];  // one counter per genome when they fit (sized at launch)
    if (*a.gate) return;  // malformed offsets: the whole grid leaves
    const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    u64 *hh = sh_h[wid];
    u16 *mpos = sh_pos[wid];
    u8 *pick = sh_pick[wid];
    u32 *stream = sh_st[wid];
    u64 *nbp = sh_nb[wid];
    const bool in_lds = a.n_genomes <= CF_LDS_GENOMES;  // uniform over the grid
    unsigned long long *dst = in_lds ? cnt : a.hits;
    if (in_lds)
        for (u64 g = threadIdx.x; g < a.n_genomes; g += blockDim.x) cnt[g] = 0;
    __syncthreads();
    const u32 k = a.k;
    const u64 kmask = (1ull << k) - 1;
    u32 wflags = 0;
    const u64 stride = (u64)gridDim.x * F_WPB;
    u64 r = (u64)blockIdx.x * F_WPB + wid;
    // the read in hand: its length and its bytes, one per lane per 64-base
    // round (the next read's are requested while this one is probed)
    int m = 0;
    u32 b[4];
    if (r < a.n) {
        const u64 beg = a.off[r];
        m = (int)(a.off[r + 1] - beg);
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int i = 64 * q + lane;
            b[q] = (m <= F_MAX_M && i < m) ? (u32)a.seq[beg + i] : (u32)'N';
        }
    }
    for (; r < a.n; r += stride) {
        const u64 rn = r + stride;
        // the next read's offsets, its start in even lanes and its end in odd
        // ones (read after the minimizers; a wave-uniform load would be waited
        // for at once)
        u64 noff = 0;
        if (rn < a.n) noff = a.off[rn + (u64)(lane & 1)];
        if (m > F_MAX_M) {
            if (lane == 0) a.fb_list[atomicAdd(a.fb_count, 1u)] = (u32)r;
            const u64 nbeg = readlane64(noff, 0);
            m = (int)(readlane64(noff, 1) - nbeg);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int i = 64 * q + lane;
                b[q] = (rn < a.n && m <= F_MAX_M && i < m) ? (u32)a.seq[nbeg + i] : (u32)'N';
            }
            continue;
        }
        // 1. N plane and big-endian 2-bit stream
        if (lane < F_WORDS) stream[lane] = 0;
        wave_sync();
        bool bad = false;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int i = 64 * q + lane;
            const u32 c = i < m ? base_code(b[q]) : 4u;
            bad |= c == 5;
            const u64 nb = ballot64(c >= 4);
            if (lane == 0) nbp[q] = nb;
            if (c < 4 && c > 0) atomicOr(&stream[i >> 4], c << (30 - 2 * (i & 15)));
        }
        if (ballot64(bad)) {
            wflags |= ERR_BAD_BYTE;  // the call fails; the grid still reads no further bytes
            wave_sync();
            break;
        }
        wave_sync();
        // 2. k-mer hashes (~0 for k-mers with an N)
        const int nk = m - (int)k + 1;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int i = 64 * q + lane;
            if (i < nk) {
                const u64 nb = funnel(nbp[q], q < 3 ? nbp[q + 1] : ~0ull, (u32)lane);
                hh[i] = (nb & kmask) == 0 ? mix64(stream_kmer(stream, i, k)) : ~0ull;
            }
            pick[i] = 0;
        }
        wave_sync();
        // 3. window minima (~0 marks an invalid k-mer, as in k_fused) and their
        // positions in order
        int nmin = 0;
        if (nk > 0) {
            const int win = nk < (int)a.w ? nk : (int)a.w;
            const int nws = nk - win + 1;
#pragma unroll 1
            for (int q = 0; q < 4; q++) {
                const int ws = 64 * q + lane;
                if (ws < nws) {
                    const int best = window_argmin_any(hh, ws, win);
                    if (best >= 0) pick[best] = 1;
                }
            }
            wave_sync();
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int i = 64 * q + lane;
                const bool chosen = i < nk && pick[i];
                const u64 cm = ballot64(chosen);
                if (chosen) mpos[nmin + lanes_below(cm, lane)] = (u16)i;
                nmin += __popcll(cm);
            }
            wave_sync();
        }
        // the next read's bytes, requested ahead of the probes
        {
            const u64 nbeg = readlane64(noff, 0);
            const int nm = (int)(readlane64(noff, 1) - nbeg);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int i = 64 * q + lane;
                b[q] = (rn < a.n && nm <= F_MAX_M && i < nm) ? (u32)a.seq[nbeg + i] : (u32)'N';
            }
            m = rn < a.n ? nm : 0;
        }
        // 4. one probe per minimizer; one hit per occurrence to its genome
        for (int t0 = 0; t0 < nmin; t0 += 64) {
            const int j = t0 + lane;
            if (j >= nmin) continue;
            const u64 v = table_lookup(a.table, a.nbuckets, stream_kmer(stream, mpos[j], k));
            if (v == SLOT_NONE) continue;
            if (!(v & SLOT_MULTI)) {
                atomicAdd(&dst[v >> 32], 1ull);
                continue;
            }
            const u32 c = slot_count(v);  // 0 for a k-mer above max_occ
            const u64 st = slot_start(v);
            for (u32 u = 0; u < c; u++) atomicAdd(&dst[a.occ[st + u] >> 32], 1ull);
        }
        wave_sync();  // the next read reuses the wavefront's LDS
    }
    if (lane == 0 && wflags) atomicOr(a.flags, wflags);
    if (in_lds) {
        __syncthreads();
        for (u64 g = threadIdx.x; g < a.n_genomes; g += blockDim.x)
            if (cnt[g]) atomicAdd(&a.hits[g], cnt[g]);
    }
}

void containment(const mt_index &ix, const mt_seqs &reads, u64 *hits, hipStream_t s) {
    const u64 n = reads.n;
    if (n == 0 || ix.n_genomes == 0) return;
    DBuf<u32> ctl(CTL_WORDS), fb_list(n);
    k_fused_init<<<1, 64, 0, s>>>(ctl.p);
    MT_HIP(hipGetLastError());
    k_check_reads<<<grid_for(n, 256), 256, 0, s>>>(reads.offsets, n, reads.total, ctl.p + CTL_GATE);
    MT_HIP(hipGetLastError());
    int dev = 0, cus = 0;
    MT_HIP(hipGetDevice(&dev));
    MT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // the genome counters take only the LDS the index needs, so more blocks fit
    // a CU (eight wavefronts per SIMD for a few hundred genomes); enough blocks
    // to fill them
    const u64 blocks = std::min<u64>(grid_for(n, F_WPB), (u64)std::max(cus, 1) * 32);
    const size_t lds = ix.n_genomes <= CF_LDS_GENOMES ? ix.n_genomes * sizeof(unsigned long long) : 0;
    ContainArgs a{(const u8 *)reads.seq, reads.offsets, n, ix.k, ix.w, ix.table.p, ix.nbuckets, ix.occ.p,
                  ix.n_genomes, (unsigned long long *)hits, fb_list.p, ctl.p + CTL_FB, ctl.p + CTL_FLAGS,
                  ctl.p + CTL_GATE};
    k_contain_fused<<<(unsigned)blocks, 64 * F_WPB, lds, s>>>(a);
    MT_HIP(hipGetLastError());
    u32 h[CTL_WORDS];
    read_back(s, ctl.p, h, sizeof h);
    check_flags(h[CTL_GATE] | h[CTL_FLAGS]);
    const u32 nfb = h[CTL_FB];
    if (nfb == 0) return;
    // longer reads: the per-stage chain on a gathered subset, adding to hits
    DBuf<u64> sub_len(nfb), sub_off(nfb + 1);
    k_subset_lengths<<<grid_for(nfb, 256), 256, 0, s>>>(reads.offsets, fb_list.p, nfb, sub_len.p);
    MT_HIP(hipGetLastError());
    scan_u64(sub_len.p, sub_off.p, nfb, s);
    u64 sub_total = 0;
    read_back(s, sub_off.p + nfb, &sub_total, sizeof sub_total);
    DBuf<u8> sub_seq(sub_total);
    k_subset_copy<<<nfb, 256, 0, s>>>((const u8 *)reads.seq, reads.offsets, fb_list.p, nfb, sub_off.p, sub_seq.p);
    MT_HIP(hipGetLastError());
    const mt_seqs sub{(const char *)sub_seq.p, sub_off.p, nfb, sub_total};
    containment_per_stage(ix, sub, hits, s);
}

}  // namespace mt
