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
    mt::DBuf<mt::u8> strand;          // both-strand results only (else empty)
    mt::DBuf<mt::u64> uniq, multi;    // n_taxa
    mt::DBuf<mt::u64> unmapped;       // 1
    void alloc_cands(mt::u64 c);
    // Served results live in host memory (the DBufs above stay empty).
    bool on_host = false;
    struct Host {
        std::vector<mt::u64> cand_off;
        std::vector<mt::u8> read_accepted;
        std::vector<mt::u16> read_E;
        std::vector<mt::u32> genome;
        std::vector<mt::i64> diag;
        std::vector<mt::u32> hits;
        std::vector<mt::u16> approx;
        std::vector<mt::u8> accept;
        std::vector<mt::u8> strand;   // both-strand results only (else empty)
        std::vector<mt::u64> counts;  // unique[n_taxa], multi[n_taxa], unmapped
    } h;
    mt::u64 submit_ns = 0, done_ns = 0;
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

// Pair lists handed to the filter kernels.
struct FilterArgs {
    const u32 *pair_read;
    const u32 *pair_genome;
    const i64 *pair_diag;
    const u16 *pair_E;   // per-pair E, or null to use read_E
    const u16 *read_E;
    const u64 *n_dev;    // pair count on the device, or null to use n_host
    u64 n_host;
    u64 n_reads;
    const u64 *read_off;  // ASCII offsets (lengths)
    const u64 *read_blk;
    const u64x2 *read_lohi;
    const u64 *read_nb;
    u64 n_genomes;
    const GenomeMeta *meta;
    const u64x2 *ref_lohi;
    const u64 *ref_nb;
    u16 *approx;
    u8 *accept;
    u32 *flags;
};

// Filters pairs [0, n) (n = *n_dev if set, else n_host; n_cap bounds it):
// pairs are bucketed by their E (one synchronization to size the buckets),
// then each bucket runs the kernel shaped for it.
void launch_filter(const FilterArgs &a, u64 n_cap, u32 max_E, hipStream_t s, Timer *tm = nullptr);
// Pairs [0, count) through the Hamming (MT_FILTER_HAMMING), base-counting
// (MT_FILTER_BASE_COUNT), q-gram (MT_FILTER_QGRAM) or shifted Hamming (MT_FILTER_SHD)
// filter; count = *n_dev if set, else n_host, at most n.
void launch_filter_simple(const FilterArgs &a, u64 n, u32 kind, hipStream_t s);

// Filter variants per bucket (see filter.hip) and their autotuner.
void autotune_filter(const FilterArgs &a, u64 n_pairs, u32 reps, hipStream_t s);
int tune_buckets();
void tune_info(int bucket, mt_tune_bucket &out);
void tune_set(int bucket, int variant);
void tune_reset();

void validate_query(const mt_query_params &q);
void mt_result_init(mt_result &res, u64 n, u32 n_taxa, hipStream_t s);
void classify_per_stage(const mt_index &ix, const mt_query_params &q, const mt_seqs &reads, ReadBatch &rb,
                        mt_result &res, Timer &tm, hipStream_t s);
// Fused form.  Checks the call's flags and sets res.n_cands before it
// returns; graph = launch the sequence as one captured HIP graph.
// Containment search: adds every genome's seed hits over `reads` to hits
// (device, n_genomes).  containment runs reads of up to 256 bases in one
// fused kernel and the rest through containment_per_stage.
void containment(const mt_index &ix, const mt_seqs &reads, u64 *hits, hipStream_t s);
void containment_per_stage(const mt_index &ix, const mt_seqs &reads, u64 *hits, hipStream_t s);

// The per-stage form end to end: packing and validation, classify_per_stage,
// flags, candidate count.
void classify_staged(const mt_index &ix, const mt_query_params &q, const mt_seqs &reads, ReadBatch &rb,
                     mt_result &res, Timer &tm, hipStream_t s);
void classify_fused(const mt_index &ix, const mt_query_params &q, const mt_seqs &reads, ReadBatch &rb,
                    mt_result &res, Timer &tm, hipStream_t s, bool graph);
// The taxon step of a batch that holds several requests: reads
// [slot_off[s], slot_off[s+1]) add into counts[s] = {unique[n_taxa],
// multi[n_taxa], unmapped} (device arrays; slot_off and counts on the device).
void launch_reduce_slots(const mt_result &res, const mt_index &ix, const u64 *slot_off, u32 n_slots,
                         unsigned long long *const *counts, hipStream_t s);

}  // namespace mt
