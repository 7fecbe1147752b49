/*
 * metatrinity.h — C ABI of the MI355X (gfx950) seed-count + approximate edit
 * distance read classifier (MetaTrinity, Gollwitzer et al., arXiv 2311.02029,
 * stage 2 "Heuristic read mapping" and the read counts of stage 3a).
 *
 * The problem (Methods, problem statement): given reference sequences R and
 * query reads Q over {A, C, G, T, N}, find the mapping locations of each Q.
 * The library does it the paper's heuristic way (Fig. 1, steps 2a-2d; read
 * mapping Evaluation Methodology; Empirically Determined Parameters):
 *   2a  an HBM-resident minimizer seed index over the reference genomes,
 *   2b  minimizer seeds of every read looked up in the index; every seed match
 *       votes for a location (genome, diagonal),
 *   2c  locations with fewer than min_hits votes are dropped, the rest sorted
 *       by votes and cut to the top_n,
 *   2d  each surviving (read, location) pair gets an approximate edit count
 *       (the obstacle count of the pigeonhole filter family of Table 1) and is
 *       accepted when the count is at most the read's threshold E,
 *   3a  accepted reads are counted per taxon as unique or multi-mapped.
 *
 * Conventions for every entry point:
 *   - Every call returns an mt_status; MT_OK is 0.  Nothing aborts and no
 *     exception crosses the ABI.  mt_last_error() describes the last failure
 *     on the calling thread.
 *   - "device" arguments are pointers to GPU memory on the current HIP device
 *     (hipMalloc, or a torch CUDA tensor's data_ptr()).  "host" arguments are
 *     ordinary CPU memory.  All inputs are borrowed for the duration of the
 *     call and never retained.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work of a call is enqueued on it, and the call synchronizes that
 *     stream before it returns (device-side input validation is reported
 *     through the return code), so on return every output is complete.
 *   - Handles (mt_index, mt_result) are owned by the library and released
 *     with their *_free call.  Device pointers returned by accessors stay valid
 *     until their handle is freed.  Free a result only once no device work
 *     that reads its arrays is pending on any stream.
 *   - An mt_index is immutable after mt_index_build and may be used from
 *     several host threads (each with its own stream) at once.
 *   - Bases are ASCII A, C, G, T, N in either case; any other byte makes the
 *     call fail with MT_EINVAL.  A k-mer containing N is never a seed, and an
 *     N (in a read or the reference) never matches anything, not even an N.
 *   - Limits: 1 <= k <= 31, 1 <= w <= 255; read length <= 65535; genome
 *     length < 2^32 - 2^16; fewer than 2^31 genomes; E <= 65534; at most
 *     2^23 - 1 occurrences of one k-mer in the index (use max_occ above that).
 */
#ifndef METATRINITY_H
#define METATRINITY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MT_ABI_VERSION 1

typedef enum mt_status {
    MT_OK = 0,
    MT_EINVAL = -1,      /* bad argument or input byte; limits exceeded */
    MT_ENOMEM = -2,      /* device or host allocation failed */
    MT_EDEVICE = -3,     /* a HIP runtime call failed */
    MT_EAGAIN = -4,      /* reserved: admission refused, try later */
    MT_ETIMEDOUT = -5,   /* reserved: wait timed out */
    MT_ECANCELED = -6,   /* reserved: request canceled */
    MT_EINTERNAL = -7    /* library bug: an internal invariant failed */
} mt_status;

/* A set of sequences: concatenated ASCII plus CSR offsets. */
typedef struct mt_seqs {
    const char *seq;          /* device: all bases back to back */
    const uint64_t *offsets;  /* device: n + 1 non-decreasing offsets, offsets[0] = 0 */
    uint64_t n;               /* number of sequences */
    uint64_t total;           /* host copy of offsets[n] (sizes device buffers) */
} mt_seqs;

typedef struct mt_index_params {
    uint32_t k;        /* k-mer length of the seeds */
    uint32_t w;        /* minimizer window: w consecutive k-mer starts */
    uint32_t max_occ;  /* k-mers occurring more than this often are never seeds; 0 = no cap */
    uint32_t reserved; /* must be 0 */
} mt_index_params;

/* How a read's edit threshold E follows from its length m. */
enum {
    MT_E_FIXED = 0,          /* E = e_value */
    MT_E_CEIL_PERMILLE = 1,  /* E = ceil(m * e_value / 1000)  (e.g. 50 = 5%) */
    MT_E_FLOOR_PERMILLE = 2  /* E = floor(m * e_value / 1000) */
};

/* Execution form; every form gives bit-identical results. */
enum {
    MT_MODE_PER_STAGE = 0,   /* one kernel launch per step of the path */
    MT_MODE_FUSED = 1,       /* one fused seed-count + filter kernel for short reads,
                                per-stage kernels for the rest */
    MT_MODE_FUSED_GRAPH = 2  /* MT_MODE_FUSED with its launches captured and replayed as
                                one HIP graph (needs a stream other than NULL) */
};

typedef struct mt_query_params {
    uint32_t min_hits;   /* keep locations with at least this many seed hits (paper: 3) */
    uint32_t top_n;      /* keep the top_n locations per read (paper: 3); 0 keeps all */
    uint32_t e_mode;     /* MT_E_* */
    uint32_t e_value;    /* E, or permille of the read length */
    uint32_t mode;       /* MT_MODE_* */
    uint32_t filter;     /* MT_FILTER_* (0: the obstacle walk).  The other filters
                            run in the per-stage form whatever the mode. */
    uint32_t strands;    /* 0 or 1: the forward strand of each genome; 2: both
                            strands (see mt_result_strands).  Two strands run in
                            the per-stage form whatever the mode. */
    uint32_t reserved;   /* must be 0 */
} mt_query_params;

typedef struct mt_index_info {
    uint64_t n_genomes;
    uint64_t total_bases;
    uint64_t n_minimizers;   /* reference minimizer occurrences (all genomes) */
    uint64_t n_keys;         /* distinct k-mers among them */
    uint64_t n_slots;        /* hash-table slots (16 bytes each) */
    uint64_t n_multi_occ;    /* entries in the multi-occurrence array */
    uint64_t device_bytes;   /* HBM held by the index */
    uint32_t k, w, max_occ, n_taxa;
} mt_index_info;

typedef struct mt_index mt_index;
typedef struct mt_result mt_result;

/*
 * Builds the seed index (Fig. 1 step 2a) over `genomes` on the device:
 * 2-bit packed reference planes, the minimizers of every genome, and a
 * bucketed hash table from k-mer to its occurrences (genome, position).
 *   params          host; k, w, max_occ as above.
 *   genomes         host struct with device seq/offsets.
 *   taxon_of_genome host array of genomes->n entries, each < n_taxa; NULL
 *                   maps genome i to taxon i (then n_taxa must be >= n).
 *   out             receives the handle (owned; release with mt_index_free).
 * Errors: MT_EINVAL (bad parameters, byte, or limit), MT_ENOMEM, MT_EDEVICE.
 */
int mt_index_build(const mt_index_params *params, const mt_seqs *genomes,
                   const uint32_t *taxon_of_genome, uint32_t n_taxa,
                   void *stream, mt_index **out);
int mt_index_free(mt_index *index);
int mt_index_get_info(const mt_index *index, mt_index_info *info);

/*
 * Classifies `reads` against the index (Fig. 1 steps 2b-2d and 3a).
 *   params  host; min_hits, top_n, E rule and execution mode.
 *   reads   host struct with device seq/offsets.
 *   out     receives the result handle (owned; release with mt_result_free).
 * Candidates of each read appear in the canonical order: seed hits
 * descending, then genome ascending, then diagonal ascending.
 * Errors: MT_EINVAL (bad parameter or byte, read > 65535 bases, E > 65534),
 * MT_ENOMEM, MT_EDEVICE.
 */
int mt_classify(const mt_index *index, const mt_query_params *params,
                const mt_seqs *reads, void *stream, mt_result **out);

/* Per-read outputs (device arrays of n_reads entries, cand_offsets n_reads+1):
 * cand_offsets  CSR into the candidate arrays;
 * read_accepted 1 if at least one candidate of the read is accepted;
 * read_E        the read's threshold E. */
int mt_result_reads(const mt_result *res, uint64_t *n_reads, const uint64_t **cand_offsets,
                    const uint8_t **read_accepted, const uint16_t **read_E);

/* Per-candidate outputs (device arrays of n_cands entries):
 * genome, diag (reference position of read base 0; may be negative),
 * hits (seed hits on that diagonal), approx (obstacle count, saturated at
 * E + 1), accept (approx <= E). */
int mt_result_cands(const mt_result *res, uint64_t *n_cands, const uint32_t **genome,
                    const int64_t **diag, const uint32_t **hits, const uint16_t **approx,
                    const uint8_t **accept);

/* Per-taxon read counts (device arrays of n_taxa entries, unmapped: one entry):
 * a read's mapped taxa are the taxa of its accepted candidates with the
 * smallest approx; one such taxon counts as unique, several as multi-mapped
 * for each; a read with no accepted candidate is unmapped. */
int mt_result_taxa(const mt_result *res, uint32_t *n_taxa, const uint64_t **unique_reads,
                   const uint64_t **multi_reads, const uint64_t **unmapped);

/* Strand of every candidate (device array of n_cands entries, or host for a
 * served result): 0 forward, 1 reverse.  *strand is NULL for a result of a
 * one-strand query (every candidate is forward) and for a served result
 * without candidates.
 *
 * Both strands (Fig. 1 step 2b: reads come from either strand of a genome,
 * and the mapper the paper builds on maps both): the reverse strand is met by
 * the reverse complement R of the read (reversed, A<->T and C<->G swapped, N
 * kept) against the forward genome.  A reverse candidate's seeds are the
 * minimizers of R in the same forward index, its diag is the reference
 * position of R's first base, and its filter value is computed on R.  The
 * candidates of both strands are ordered together by (hits descending, genome,
 * diag, strand ascending) and one top_n cut applies to the union. */
int mt_result_strands(const mt_result *res, const uint8_t **strand);

/* Relative abundance of the taxa (Fig. 1 step 3b) from a classification
 * result made with this index (device or served).  The paper takes the
 * apportionment of multi-mapped reads from Metalign without stating it; the
 * rule here: with u_t the unique reads of taxon t and T(r) the mapped taxa of
 * a multi-mapped read r (mt_result_taxa's rule),
 *   counts[t] = 2^32 u_t + sum over multi-mapped r with t in T(r) of
 *               floor(2^32 u_t / U_r),  U_r = sum of u over T(r)
 *               (floor(2^32 / |T(r)|) when U_r = 0),
 * in units of 2^-32 read (exact integers); a taxon is kept iff
 * counts[t] * cutoff_den >= (sum of counts) * cutoff_num (the paper drops taxa
 * below 0.01%: 1 / 10000); abundance[t] = counts[t] / (sum of kept counts) as
 * the nearest double of the exact ratio (rounded once, ties to even, also when
 * the sum needs more than 53 bits), 0 for dropped taxa and when no read is
 * mapped.  The sums are 64-bit: up to 2^32 mapped reads per result.
 * counts (uint64) and abundance (double): device arrays of n_taxa entries;
 * *n_kept (host) receives the number of kept taxa.  Errors: null arguments,
 * cutoff_den = 0, a result whose taxon count differs from the index's. */
int mt_abundance(const mt_index *index, const mt_result *res, uint64_t cutoff_num, uint64_t cutoff_den,
                 uint64_t *counts, double *abundance, uint64_t *n_kept, void *stream);
int mt_result_free(mt_result *res);

/* Per-launch kernel timings of the last mt_classify on this thread (ms,
 * measured with HIP events on the call's stream).  names/ms: host arrays of
 * `cap` entries; *n receives the number of entries written. */
int mt_last_timings(const char **names, float *ms, uint32_t cap, uint32_t *n);
/* Enables (1) or disables (0, default) the event timing above. */
int mt_set_timing(int enabled);

/* Work counts of the last mt_classify on this thread. */
typedef struct mt_stats {
    uint64_t n_reads;
    uint64_t n_minimizers;        /* read minimizers looked up */
    uint64_t n_hits;              /* (minimizer, occurrence) seed matches */
    uint64_t n_cands;             /* (read, location) pairs filtered */
    uint64_t fused_reads;         /* reads the fused kernel finished */
    uint64_t fused_bases;         /* their bases */
    uint64_t fused_minimizers;    /* their minimizers */
    uint64_t fused_window_blocks; /* 64-base reference blocks their filter read */
    uint64_t fused_cands;         /* their candidates */
    uint64_t fused_occ;           /* entries their probes read from the multi-occurrence array */
} mt_stats;
int mt_last_stats(mt_stats *out);

/*
 * The filter alone (Fig. 1 step 2d) over explicit (read, location) pairs.
 *   reads        host struct with device seq/offsets.
 *   pair_read    device, n_pairs read indices (< reads->n).
 *   pair_genome  device, n_pairs genome indices (< number of genomes).
 *   pair_diag    device, n_pairs diagonals (reference position of read base 0).
 *   pair_E       device, n_pairs thresholds.
 *   approx_out   device, n_pairs outputs: obstacle count saturated at E + 1.
 *   accept_out   device, n_pairs outputs: approx <= E.
 * Errors: MT_EINVAL (index out of range, bad byte, read > 65535, E > 65534).
 */
int mt_filter_pairs(const mt_index *index, const mt_seqs *reads, const uint32_t *pair_read,
                    const uint32_t *pair_genome, const int64_t *pair_diag, const uint16_t *pair_E,
                    uint64_t n_pairs, uint16_t *approx_out, uint8_t *accept_out, void *stream);

/*
 * Other filters of Table 1 on the same pair stream, the runtime/accuracy knob
 * of the filter choice (same arguments and errors as mt_filter_pairs, plus
 * MT_EINVAL for an unknown kind):
 *   MT_FILTER_OBSTACLE    the obstacle walk over the 2E+1 band rows (as
 *                         mt_filter_pairs);
 *   MT_FILTER_HAMMING     the Hamming distance: mismatching columns of the
 *                         diagonal itself (row 0 alone), N and positions
 *                         outside the genome mismatching;
 *   MT_FILTER_BASE_COUNT  base counting: ceil(sum over A, C, G, T of |count in
 *                         the read - count in reference [diag, diag + m)| / 2),
 *                         a lower bound of the Hamming distance;
 *   MT_FILTER_QGRAM       q-grams (q = 5): ceil((m - 4 - shared) / 5), shared =
 *                         the multiset intersection of the read's q-grams and
 *                         those of reference [diag - E, diag + m + E) (q-grams
 *                         with N or outside positions excluded); 0 for m < 5;
 *                         a lower bound of the banded edit distance;
 *   MT_FILTER_SHD         shifted Hamming distance: the band rows' mismatch
 *                         masks, each with runs of one or two zeros between
 *                         ones set, ANDed; the value counts the ones.
 * Each value saturates at E + 1; accept is value <= E.
 */
enum { MT_FILTER_OBSTACLE = 0, MT_FILTER_HAMMING = 1, MT_FILTER_BASE_COUNT = 2, MT_FILTER_QGRAM = 3,
       MT_FILTER_SHD = 4 };
int mt_filter_pairs_kind(const mt_index *index, const mt_seqs *reads, const uint32_t *pair_read,
                         const uint32_t *pair_genome, const int64_t *pair_diag, const uint16_t *pair_E,
                         uint64_t n_pairs, uint32_t kind, uint16_t *approx_out, uint8_t *accept_out, void *stream);

/*
 * Containment search (Fig. 1 steps 1a-1c; section "Containment Search"): the
 * seed-hit count of every genome of the index over the whole read set -- one
 * hit per (read minimizer, occurrence of its k-mer among the genome's
 * minimizers), k-mers above max_occ skipped, summed over all reads (the
 * stage-2 seed matches of every read summed over its locations).
 *   index  the resident index (the counts run on it, no other copy is made).
 *   reads  host struct with device seq/offsets, as for mt_classify.
 *   hits   device, n_genomes 64-bit counts, overwritten; owned by the caller.
 * The call returns when the counts are written.  Errors: MT_EINVAL (null
 * argument, byte outside ACGTN, read longer than 65535), MT_ENOMEM,
 * MT_EDEVICE.
 */
int mt_containment(const mt_index *index, const mt_seqs *reads, uint64_t *hits, void *stream);

/*
 * Subset-database selection (Fig. 1 step 1d; the normalised seed-hit cutoff
 * of the containment evaluation): with M the largest count, genome g is kept
 * when hits[g] / M exceeds cutoff_num / cutoff_den (the paper: 1 / 10000),
 * decided exactly as hits[g] * cutoff_den > M * cutoff_num in 128-bit
 * arithmetic; M = 0 keeps none.  For an index split into shards, pass the
 * per-genome maximum over the shards' counts (the paper's merge rule).
 *   hits        device, n_genomes counts (e.g. from mt_containment).
 *   selected    device, n_genomes capacity: the kept genome indices, ascending.
 *   n_selected  host: how many were kept.   max_hits  host: M.
 * The call waits for its stream.  Errors: MT_EINVAL (null argument,
 * cutoff_den 0), MT_EDEVICE.
 */
int mt_select_genomes(const uint64_t *hits, uint64_t n_genomes, uint64_t cutoff_num, uint64_t cutoff_den,
                      uint32_t *selected, uint64_t *n_selected, uint64_t *max_hits, void *stream);

/*
 * mt_select_genomes for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Same arguments, results and errors as mt_select_genomes, plus
 * MT_EINVAL for n_genomes above 1,048,576.  It allocates nothing: its scratch
 * (the maximum, per-genome keep flags and offsets, the scan's block sums) is
 * a static device array of the library, about 12.6 MB, which every GPU the
 * library runs on holds until the process ends.  All calls on one GPU share
 * that array, so calls that overlap on one GPU race: issue them one at a
 * time (one stream, or wait for the previous call).  The call waits for its
 * stream (it returns n_selected and max_hits on the host).
 */
int mt_select_genomes_noalloc(const uint64_t *hits, uint64_t n_genomes, uint64_t cutoff_num, uint64_t cutoff_den,
                              uint32_t *selected, uint64_t *n_selected, uint64_t *max_hits, void *stream);

/*
 * Serving loop: continuous batching of classification requests on one GPU
 * with the index resident in HBM.  Requests that arrive while others run are
 * admitted as batch slots and device memory free up; reads of several
 * requests with the same query parameters share a device batch, and a large
 * request is split across batches.  n_streams worker threads each own a HIP
 * stream, so the upload of one batch overlaps the classification of another.
 * Each request gets exactly what mt_classify gives for its reads alone
 * (Fig. 1 steps 2b-2d, and the taxon counts of step 3a over its own reads).
 */
typedef struct mt_server mt_server;

typedef struct mt_server_params {
    uint64_t mem_budget_bytes;      /* device bytes admitted at once; 0 = a quarter of the device
                                       memory free when the server is created (at least 256 MiB) */
    uint64_t max_batch_reads;       /* reads per device batch; 0 = 262,144 (smaller batches
                                       cut the latency tail, larger ones raise throughput) */
    uint32_t n_streams;             /* batches in flight (worker threads); 0 = 4 */
    uint32_t max_queued_requests;   /* submitted and not yet waited for; 0 = 4096 */
    uint64_t pinned_arena_bytes;    /* pinned host memory for queued reads; 0 = 1 GiB */
    uint32_t reserved[4];           /* must be 0 */
} mt_server_params;

/* Creates the server (threads start at once).  The index must outlive it. */
int mt_server_create(const mt_index *index, const mt_server_params *params, mt_server **out);

/*
 * Queues one request.  seq / offsets are HOST memory (offsets: n + 1
 * non-decreasing entries, offsets[0] = 0), validated and copied into the
 * server's pinned arena before the call returns.  params->mode is ignored (the
 * fused form runs, with the same per-stage handling of reads past its limits
 * as mt_classify).  *request_id receives the id to wait for.
 * Errors: MT_EINVAL (bad parameter, offset or byte, read > 65535 bases,
 * E > 65534, request larger than the arena), MT_EAGAIN (max_queued_requests
 * not yet waited for, or the arena is full: retry after a wait), MT_ECANCELED
 * (server shutting down), MT_ENOMEM, MT_EDEVICE.
 */
int mt_server_submit(mt_server *server, const mt_query_params *params, const char *seq, const uint64_t *offsets,
                     uint64_t n, uint64_t *request_id);

/*
 * Waits up to timeout_us (< 0: forever) for a request and hands over its
 * result: a handle like mt_classify's, but its arrays are HOST memory
 * (mt_result_on_host) and its taxon counts cover this request only.
 * A finished request is handed over once; *out is NULL on error.
 * Errors: MT_ETIMEDOUT (not finished yet; wait again), MT_EINVAL (unknown id,
 * already handed over, or waited for by another thread), and the error of a
 * device batch that held the request (MT_EDEVICE, MT_ENOMEM).
 */
int mt_server_wait(mt_server *server, uint64_t request_id, int64_t timeout_us, mt_result **out);

/* Stops accepting requests, finishes the queued ones, joins the threads.
 * Results not yet waited for are released; results already handed over stay
 * valid.  No other call on this server may be in progress or follow. */
int mt_server_destroy(mt_server *server);

/* Counters of a server since its creation (host struct): batches run and
 * the reads in them; batches that the memory budget cut short (admission
 * control held reads back until memory of running batches was released);
 * the largest estimated device bytes and the most batches in flight at once;
 * the budget and batch cap in force (defaults resolved); and, from HIP events
 * recorded on the worker streams around each batch's kernels (after its
 * upload, before its download), the device time of those kernels summed over
 * the batches, the time covered by at least one of them, and the time during
 * which the kernels of two or more batches were running at once (ms). */
typedef struct mt_server_counters {
    uint64_t batches;
    uint64_t reads;
    uint64_t budget_limited;
    uint64_t peak_inflight_bytes;
    uint64_t mem_budget_bytes;
    uint64_t max_batch_reads;
    uint32_t peak_batches;
    uint32_t reserved;
    uint64_t timed_batches;
    double kernel_ms_sum;
    double kernel_ms_union;
    double kernel_ms_overlap;
} mt_server_counters;
int mt_server_stats(mt_server *server, mt_server_counters *out);

/* 1 if the result's arrays live in host memory (served results), 0 if on
 * the device (mt_classify). */
int mt_result_on_host(const mt_result *res);

/* Submit and completion times of a served request (steady clock, ns). */
int mt_result_times(const mt_result *res, uint64_t *submit_ns, uint64_t *done_ns);

/*
 * Autotuning of the filter step (Fig. 1 step 2d; the E-dependent band of 2E+1
 * rows of Table 1's pigeonhole filters).  Filter pairs are bucketed by E
 * (<= 7, <= 15, <= 31) and, for larger E, by the 64-base blocks of read and
 * reference window they stage in LDS (<= 96, 192, 384, 768); each bucket has
 * variants: lanes per pair (pairs per wavefront) for small E, the LDS tile
 * with 1/2/4/8 wavefronts per block or a rows-in-lanes layout reading global
 * memory for large E.  Every variant gives bit-identical results; the choice
 * is process-wide and applies to mt_classify (per-stage form and the fused
 * form's per-stage finish) and mt_filter_pairs.
 */
#define MT_TUNE_MAX_VARIANTS 6

typedef struct mt_tune_bucket {
    const char *name;                                 /* e.g. "E<=7", "long<=384" */
    uint32_t n_variants;
    uint32_t current;                                 /* variant in use */
    const char *variant_names[MT_TUNE_MAX_VARIANTS];  /* NULL past n_variants */
    float ms[MT_TUNE_MAX_VARIANTS];                   /* last autotune time per variant (0: not timed) */
    uint64_t pairs;                                   /* pairs the last autotune timed in this bucket */
} mt_tune_bucket;

/* Number of buckets (*n) and the state of one bucket (host structs; the
 * strings are static). */
int mt_tune_buckets(uint32_t *n);
int mt_tune_info(uint32_t bucket, mt_tune_bucket *out);
/* Selects a variant for a bucket.  Errors: MT_EINVAL (no such bucket or
 * variant, or a variant whose LDS does not fit a workgroup). */
int mt_tune_set(uint32_t bucket, uint32_t variant);
/* Back to the built-in defaults. */
int mt_tune_reset(void);
/*
 * Classifies `reads` (host struct with device arrays) in the per-stage form to
 * obtain their filter pairs, then times every variant of every bucket that
 * holds pairs on those pairs (best of `reps` launches, HIP events on
 * `stream`) and selects the fastest.  Results: mt_tune_info.
 */
int mt_autotune(const mt_index *index, const mt_query_params *params, const mt_seqs *reads, uint32_t reps,
                void *stream);
/* Writes / reads the selection as JSON ({"arch": ..., "buckets": {name: variant}}).
 * mt_tune_load fails with MT_EINVAL for a file made on another GPU
 * architecture or naming unknown buckets or variants. */
int mt_tune_save(const char *path);
int mt_tune_load(const char *path);

/*
 * Device memory of the library.  Every device buffer the library holds -- an
 * index, a result's arrays, per-call scratch, a server's batches and request
 * counters -- comes from one allocator.  By default it is the library's own
 * caching pool (hipMalloc'd blocks kept on free lists for reuse).
 *
 * mt_set_allocator installs the caller's allocator instead (the binding
 * installs PyTorch's caching allocator, so that one allocator owns HBM and
 * its statistics cover the library): from then on every device allocation is
 * alloc(bytes, stream, ctx) and every release free_(ptr, ctx), and the library
 * keeps no cache of its own (its idle pool blocks are released by the call).
 *   alloc   returns device memory of at least `bytes` bytes (256-byte aligned
 *           or better), or NULL when none is left (the library call then
 *           fails with MT_ENOMEM).  `stream` is the hipStream_t (as void*,
 *           NULL = the null stream) on which the library first uses the
 *           memory; a stream-ordered allocator may hand out memory whose
 *           earlier use on that stream is still queued.  Called from any
 *           host thread, including the server's workers.
 *   free_   takes back a pointer alloc returned.  The library calls it only
 *           after its own work on the memory is complete.
 *   ctx     passed through to both.
 * alloc and free_ both NULL restore the built-in pool.  Blocks keep the
 * allocator that made them: memory allocated before a switch is released
 * to its own allocator.  The hook must stay valid while any block it made
 * is alive.  Errors: MT_EINVAL (exactly one of alloc and free_ is NULL).
 * (The paper leaves memory management open; this is the boundary's hook for
 * a host framework that owns device memory.)
 */
int mt_set_allocator(void *(*alloc)(size_t bytes, void *stream, void *ctx), void (*free_)(void *ptr, void *ctx),
                     void *ctx);

/* Allocation counters since the library was loaded (host struct). */
typedef struct mt_mem_stats {
    uint64_t device_mallocs;  /* hipMalloc calls made by the built-in pool */
    uint64_t hook_allocs;     /* allocations made through an mt_set_allocator hook */
    uint64_t live_bytes;      /* device bytes held by live blocks (handles and calls in progress) */
    uint64_t cached_bytes;    /* idle bytes on the built-in pool's free lists */
    uint32_t hooked;          /* 1 while a hook is installed */
    uint32_t reserved;
} mt_mem_stats;
int mt_memory_stats(mt_mem_stats *out);

/* Releases device memory cached by the library's allocator (not held by any handle). */
int mt_trim(void);
/* Description of the last error on the calling thread ("" if none). */
const char *mt_last_error(void);
int mt_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* METATRINITY_H */
