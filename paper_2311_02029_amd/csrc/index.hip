// Seed index over the reference genomes (Fig. 1 step 2a; "Reference Database
// Organisation and Index Construction & Querying").
//
// Built entirely on the device:
//   1. the genomes are packed into bit planes (kept: the filter reads its
//      reference windows from them);
//   2. every genome's minimizers (the same k, w and hash as the reads) are
//      extracted tile by tile;
//   3. each minimizer's k-mer is inserted into a bucketed open-addressing
//      table (4 slots of {k-mer, value} = one 64-byte line per bucket) and
//      its occurrences are counted;
//   4. k-mers occurring once keep their (genome, position) inline in the slot,
//      so the common lookup costs one random 64-byte line; k-mers occurring
//      several times point into an occurrence array; k-mers occurring more
//      than max_occ times are marked as never seeding.
// The table is sized for a load of at most 1/2 of its slots, so a lookup
// nearly always ends in its first bucket.  Buckets come from a second,
// salted hash of the k-mer (see bucket_of).
#include <cstring>
#include <vector>

#include "index.hpp"
#include "seq.hpp"

namespace mt {

__global__ void k_genome_meta(const u64 *__restrict__ off, u64 n, const u64 *__restrict__ blk_off,
                              const u32 *__restrict__ has_n, const u32 *__restrict__ taxon, u64 *__restrict__ glen,
                              GenomeMeta *__restrict__ meta) {
    u64 g = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    u64 len = off[g + 1] - off[g];
    glen[g] = len;
    meta[g] = GenomeMeta{blk_off[g], (u32)len, taxon[g] | (has_n[g] ? 0x80000000u : 0u)};
}

__global__ void k_insert(const u64 *__restrict__ xs, u64 n, u64x2 *__restrict__ table, u64 nbuckets,
                         u32 *__restrict__ cnt, unsigned long long *__restrict__ n_keys) {
    u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    u64 x = xs[i];
    u64 b = bucket_of(x, nbuckets);
    for (;;) {
        u64x2 *bk = table + b * 4;
        for (int s = 0; s < 4; s++) {
            unsigned long long *kp = (unsigned long long *)&bk[s].lo;
            u64 cur = __hip_atomic_load(kp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (cur == SLOT_EMPTY_KEY) {
                u64 old = atomicCAS(kp, (unsigned long long)SLOT_EMPTY_KEY, (unsigned long long)x);
                if (old == SLOT_EMPTY_KEY) {
                    atomicAdd(n_keys, 1ull);
                    cur = x;
                } else {
                    cur = old;
                }
            }
            if (cur == x) {
                atomicAdd(&cnt[b * 4 + s], 1u);
                return;
            }
        }
        b = (b + 1 == nbuckets) ? 0 : b + 1;
    }
}

// Multi-occurrence sizes; marks k-mers above max_occ as never seeding.
__global__ void k_slot_sizes(const u32 *__restrict__ cnt, u64 nslots, u32 max_occ, u64x2 *__restrict__ table,
                             u32 *__restrict__ size, u32 *__restrict__ flags) {
    u64 s = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslots) return;
    u32 c = cnt[s];
    u32 sz = 0;
    if (c > 0) {
        if (max_occ && c > max_occ) {
            table[s].hi = SLOT_MULTI;  // count 0: never a seed
        } else {
            if (c > MAX_KEY_OCC) atomicOr(flags, ERR_KEY_OVERFLOW);
            sz = c >= 2 ? c : 0;
        }
    }
    size[s] = sz;
}

__device__ inline u64 find_slot(const u64x2 *table, u64 nbuckets, u64 x) {
    u64 b = bucket_of(x, nbuckets);
    for (;;) {
        for (int s = 0; s < 4; s++)
            if (table[b * 4 + s].lo == x) return b * 4 + s;
        b = (b + 1 == nbuckets) ? 0 : b + 1;
    }
}

__global__ void k_fill(const u64 *__restrict__ xs, const u32 *__restrict__ gs, const u32 *__restrict__ ps, u64 n,
                       u64x2 *__restrict__ table, u64 nbuckets, u32 *__restrict__ cnt, const u64 *__restrict__ start,
                       u64 *__restrict__ occ) {
    u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    u64 s = find_slot(table, nbuckets, xs[i]);
    u64 gp = ((u64)gs[i] << 32) | ps[i];
    u64 sz = start[s + 1] - start[s];
    if (sz > 0) {
        u32 k = atomicSub(&cnt[s], 1u) - 1u;
        occ[start[s] + k] = gp;
    } else if (table[s].hi != SLOT_MULTI) {
        table[s].hi = gp;  // the only occurrence, stored inline
    }
}

__global__ void k_finalize(u64x2 *__restrict__ table, u64 nslots, const u64 *__restrict__ start) {
    u64 s = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslots) return;
    u64 sz = start[s + 1] - start[s];
    if (sz >= 2) table[s].hi = SLOT_MULTI | (sz << 40) | start[s];
}

void build_index(mt_index &ix, const mt_index_params &p, const mt_seqs &g, const uint32_t *taxon, uint32_t n_taxa,
                 hipStream_t s) {
    Timer tm;
    tm.begin(s);
    MT_REQUIRE(p.k >= 1 && p.k <= 31, "k must be in 1..31");
    MT_REQUIRE(p.w >= 1 && p.w <= 255, "w must be in 1..255");
    MT_REQUIRE(p.reserved == 0, "reserved field must be 0");
    MT_REQUIRE(g.n < (1ull << 31), "at most 2^31 - 1 genomes");
    MT_REQUIRE(n_taxa < (1u << 31), "at most 2^31 - 1 taxa");
    MT_REQUIRE(g.n == 0 || (g.seq && g.offsets), "null genome arrays");
    std::vector<u32> tax(g.n);
    for (u64 i = 0; i < g.n; i++) {
        tax[i] = taxon ? taxon[i] : (u32)i;
        MT_REQUIRE(tax[i] < n_taxa, "taxon id out of range");
    }
    ix.k = p.k;
    ix.w = p.w;
    ix.max_occ = p.max_occ;
    ix.n_taxa = n_taxa;
    ix.n_genomes = g.n;
    ix.total_bases = g.total;

    DBuf<u32> flags(1);
    MT_HIP(hipMemsetAsync(flags.p, 0, sizeof(u32), s));
    ix.has_n.alloc(g.n);
    MT_HIP(hipMemsetAsync(ix.has_n.p, 0, (g.n ? g.n : 1) * sizeof(u32), s));
    pack_sequences(g, 4294901759ull, ERR_READ_TOO_LONG, "genome length must be below 2^32 - 2^16", ix.ref,
                   flags.p, ix.has_n.p, s);
    ix.taxon.alloc(g.n);
    if (g.n) MT_HIP(hipMemcpyAsync(ix.taxon.p, tax.data(), g.n * sizeof(u32), hipMemcpyHostToDevice, s));
    ix.glen.alloc(g.n);
    ix.meta.alloc(g.n);
    if (g.n) {
        k_genome_meta<<<grid_for(g.n, 256), 256, 0, s>>>(g.offsets, g.n, ix.ref.blk_off.p, ix.has_n.p, ix.taxon.p,
                                                          ix.glen.p, ix.meta.p);
        MT_HIP(hipGetLastError());
    }
    tm.mark("index_pack");

    MinimizerPlan mp;
    minimizer_plan(g, ix.ref, p.k, p.w, 1024, mp, s);
    u32 f0 = 0;
    read_back(s, flags.p, &f0, sizeof(u32));
    check_flags(f0);
    u64 n_min = 0;
    read_back(s, mp.min_off.p + mp.tiles_cap, &n_min, sizeof(u64));
    ix.n_minimizers = n_min;
    tm.mark("index_min_count");

    DBuf<u64> ex(n_min);
    DBuf<u32> eg(n_min), ep(n_min);
    minimizer_emit(g, ix.ref, p.k, p.w, mp, ex.p, eg.p, ep.p, s);
    tm.mark("index_min_emit");

    u64 nbuckets = (n_min + 1) / 2;
    if (nbuckets < 1) nbuckets = 1;
    ix.nbuckets = nbuckets;
    u64 nslots = nbuckets * 4;
    ix.table.alloc(nslots);
    MT_HIP(hipMemsetAsync(ix.table.p, 0xFF, nslots * sizeof(u64x2), s));
    DBuf<u32> cnt(nslots);
    MT_HIP(hipMemsetAsync(cnt.p, 0, nslots * sizeof(u32), s));
    DBuf<unsigned long long> nkeys(1);
    MT_HIP(hipMemsetAsync(nkeys.p, 0, sizeof(u64), s));
    if (n_min) {
        k_insert<<<grid_for(n_min, 256), 256, 0, s>>>(ex.p, n_min, ix.table.p, nbuckets, cnt.p, nkeys.p);
        MT_HIP(hipGetLastError());
    }
    tm.mark("index_insert");
    DBuf<u32> size(nslots);
    k_slot_sizes<<<grid_for(nslots, 256), 256, 0, s>>>(cnt.p, nslots, p.max_occ, ix.table.p, size.p, flags.p);
    MT_HIP(hipGetLastError());
    DBuf<u64> start(nslots + 1);
    scan_u32(size.p, start.p, nslots, s);
    u64 n_multi = 0;
    read_back(s, start.p + nslots, &n_multi, sizeof(u64));
    read_back(s, nkeys.p, &ix.n_keys, sizeof(u64));
    u32 f1 = 0;
    read_back(s, flags.p, &f1, sizeof(u32));
    check_flags(f1);
    ix.n_multi_occ = n_multi;
    tm.mark("index_sizes");
    ix.occ.alloc(n_multi);
    if (n_min) {
        k_fill<<<grid_for(n_min, 256), 256, 0, s>>>(ex.p, eg.p, ep.p, n_min, ix.table.p, nbuckets, cnt.p, start.p,
                                                    ix.occ.p);
        MT_HIP(hipGetLastError());
    }
    k_finalize<<<grid_for(nslots, 256), 256, 0, s>>>(ix.table.p, nslots, start.p);
    MT_HIP(hipGetLastError());
    tm.mark("index_fill");
    MT_HIP(hipStreamSynchronize(s));
    tm.finish();
}

u64 index_device_bytes(const mt_index &ix) {
    return ix.ref.lohi.n * sizeof(u64x2) + ix.ref.nb.n * sizeof(u64) + ix.ref.blk_off.n * sizeof(u64) +
           ix.glen.n * sizeof(u64) + ix.has_n.n * sizeof(u32) + ix.taxon.n * sizeof(u32) +
           ix.meta.n * sizeof(GenomeMeta) +
           ix.table.n * sizeof(u64x2) + ix.occ.n * sizeof(u64);
}

}  // namespace mt

// ---------------------------------------------------------------------- ABI --

using mt::Error;

extern "C" int mt_index_build(const mt_index_params *params, const mt_seqs *genomes,
                              const uint32_t *taxon_of_genome, uint32_t n_taxa, void *stream, mt_index **out) {
    if (!params || !genomes || !out) {
        mt::set_last_error("mt_index_build: null argument");
        return MT_EINVAL;
    }
    *out = nullptr;
    mt_index *ix = nullptr;
    try {
        ix = new mt_index();
        MT_HIP(hipGetDevice(&ix->device));
        {
            mt::CallScope scope((hipStream_t)stream);
            mt::build_index(*ix, *params, *genomes, taxon_of_genome, n_taxa, (hipStream_t)stream);
        }
        mt::pool_trim();  // the build's scratch (several times the index) is not needed again
        *out = ix;
        mt::set_last_error("");
        return MT_OK;
    } catch (const Error &e) {
        delete ix;
        mt::set_last_error(e.what());
        return e.status;
    } catch (const std::exception &e) {
        delete ix;
        mt::set_last_error(e.what());
        return MT_EINTERNAL;
    }
}

extern "C" int mt_index_free(mt_index *index) {
    delete index;
    return MT_OK;
}

extern "C" int mt_index_get_info(const mt_index *ix, mt_index_info *info) {
    if (!ix || !info) {
        mt::set_last_error("mt_index_get_info: null argument");
        return MT_EINVAL;
    }
    std::memset(info, 0, sizeof *info);
    info->n_genomes = ix->n_genomes;
    info->total_bases = ix->total_bases;
    info->n_minimizers = ix->n_minimizers;
    info->n_keys = ix->n_keys;
    info->n_slots = ix->nbuckets * 4;
    info->n_multi_occ = ix->n_multi_occ;
    info->device_bytes = mt::index_device_bytes(*ix);
    info->k = ix->k;
    info->w = ix->w;
    info->max_occ = ix->max_occ;
    info->n_taxa = ix->n_taxa;
    return MT_OK;
}
