// The device-resident seed index (an opaque mt_index at the ABI).
#pragma once

#include "seq.hpp"

struct mt_index {
    int device = 0;
    uint32_t k = 0, w = 0, max_occ = 0, n_taxa = 0;
    uint64_t n_genomes = 0, total_bases = 0;
    uint64_t n_minimizers = 0, n_keys = 0, n_multi_occ = 0;
    mt::PackedSeqs ref;          // reference bit planes, genome g at block ref.blk_off[g]
    mt::DBuf<mt::u64> glen;      // genome lengths
    mt::DBuf<mt::u32> has_n;     // 1 if the genome contains N
    mt::DBuf<mt::u32> taxon;     // taxon of each genome
    mt::DBuf<GenomeMeta> meta;   // per-genome record used by the filter
    mt::DBuf<u64x2> table;     // nbuckets * 4 slots {k-mer, value}
    mt::u64 nbuckets = 0;
    mt::DBuf<mt::u64> occ;       // occurrences (genome << 32 | position) of multi-occurrence k-mers
};

namespace mt {
void build_index(mt_index &ix, const mt_index_params &p, const mt_seqs &g, const uint32_t *taxon, uint32_t n_taxa,
                 hipStream_t s);
u64 index_device_bytes(const mt_index &ix);
}  // namespace mt
