// Read classification: the result handle and the per-stage / fused drivers.
#pragma once

#include "index.hpp"

struct mt_result {
    mt::u64 n_reads = 0, n_cands = 0, cap = 0;
    mt::u32 n_taxa = 0;
    mt::DBuf<mt::u64> cand_off;       // n_reads + 1
    mt::DBuf<mt::u8> read_accepted;   // n_reads
    mt::DBuf<mt::u16> read_E;         // n_reads
    mt::DBuf<mt::u32> genome;         // candidates (capacity cap)
    mt::DBuf<mt::i64> diag;
    mt::DBuf<mt::u32> hits;
    mt::DBuf<mt::u16> approx;
    mt::DBuf<mt::u8> accept;
    mt::DBuf<mt::u64> uniq, multi;    // n_taxa
    mt::DBuf<mt::u64> unmapped;       // 1
    void alloc_cands(mt::u64 c);
};

namespace mt {

// Per-call read state shared by both execution forms.
struct ReadBatch {
    u64 n = 0;
    DBuf<u32> flags;   // validation flags
    DBuf<u32> maxE;    // largest E of the batch
    DBuf<u16> read_E;  // E per read
    PackedSeqs planes; // read bit planes
    void prepare(const mt_seqs &reads, u32 e_mode, u32 e_value, hipStream_t s);
};

void validate_query(const mt_query_params &q);
void mt_result_init(mt_result &res, u64 n, u32 n_taxa, hipStream_t s);
void classify_per_stage(const mt_index &ix, const mt_query_params &q, const mt_seqs &reads, ReadBatch &rb,
                        mt_result &res, Timer &tm, hipStream_t s);
void classify_fused(const mt_index &ix, const mt_query_params &q, const mt_seqs &reads, ReadBatch &rb,
                    mt_result &res, Timer &tm, hipStream_t s);
void launch_max_u16(const u16 *v, u64 n, u32 *out, hipStream_t s);

}  // namespace mt
