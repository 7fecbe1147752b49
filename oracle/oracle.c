/*
 * CPU oracle for the seed-count + edit-distance-approximation read classifier
 * of MetaTrinity (Gollwitzer et al., arXiv 2311.02029).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the GPU path computes.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code,
 * header, table or helper with the HIP library, and it includes none of it.
 *
 * Every step follows the paper's order:
 *   stage 2a  a seed index over the (subset) reference database   (Fig. 1, 2a)
 *   stage 2b  read seeding and seed matches                       (Fig. 1, 2b; "Alignment-free read-mapping")
 *   stage 2c  drop locations below the seed-hit minimum, sort by
 *             seed hits, keep the top locations                   (Fig. 1, 2c; "Empirically Determined Parameters")
 *   stage 2d  approximate edit distance per (read, location) pair,
 *             accept when it is within the threshold E            (Fig. 1, 2d; read-mapping Evaluation Methodology)
 *   stage 3a  per-taxon unique / multi-mapped read counts         (Fig. 1, 3a)
 * The approximation is the pigeonhole-family filter the paper rates best
 * (SneakySnake, Table 1 and the Discussion of accuracy): the 2E+1 diagonals of
 * the band around a location are turned into rows of mismatch bits ("obstacles")
 * and a greedy walk from the read's first to its last base counts how many
 * obstacles it has to cross, stopping once the count exceeds E.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   O1  codes A0 C1 G2 T3, N4, case-insensitive; any other byte is an error.
 *       A k-mer containing N is never a seed.  N never matches anything (not
 *       even N); a reference position outside the genome never matches.
 *   O2  k-mer value x = sum code[i+t] * 4^(k-1-t) (first base most
 *       significant); its hash is the splitmix64 finalizer (Steele, Lea and
 *       Flood, OOPSLA 2014), a bijection of 64-bit words.
 *   O3  minimizers: every window of w consecutive k-mer start positions picks
 *       the valid position with the smallest (hash, position); the minimizer
 *       set is the union of picks.  Fewer than w k-mers: one window over all.
 *   O4  a mapping location is an exact diagonal (genome, q - p) of a seed
 *       match; its seed-hit count is the number of (read minimizer, reference
 *       minimizer occurrence) pairs with equal k-mer on that diagonal.  Keys
 *       with more than max_occ occurrences are skipped (max_occ 0: no cap).
 *   O5  keep hits >= min_hits; order by (hits desc, genome asc, diag asc);
 *       keep the first top_n (0 keeps all).
 *   O6  row d in [-E, E], column j in [0, m): obstacle iff Q[j] differs from
 *       reference position diag + j + d (N / outside counts as different).
 *       Walk: j = 0, c = 0; repeat { l = longest obstacle-free run starting at
 *       column j over all rows (capped at m - j); j += l; stop if j >= m;
 *       c += 1; stop if c > E; j += 1 }.  approx = min(c, E + 1).
 *   O7  accept iff approx <= E.
 *   O8  a read is accepted iff one of its candidates is.  Its mapped taxa are
 *       the taxa of accepted candidates whose approx equals the smallest
 *       accepted approx of the read; one taxon -> unique[t] += 1, several ->
 *       multi[t] += 1 for each; none -> unmapped += 1.
 *   O9  stage 1 (containment search): the seed-hit count of genome g over a
 *       read set is the number of (read minimizer, minimizer occurrence in g)
 *       pairs with equal k-mer, summed over all reads, keys above max_occ
 *       skipped -- the O4 matches of every read summed over its diagonals.
 *   O10 subset database: with M the largest seed-hit count over the genomes,
 *       genome g is kept iff hits[g] / M exceeds the cutoff num / den
 *       (strictly: "above" / "surpasses"), decided exactly as
 *       hits[g] * den > M * num; M = 0 keeps no genome.
 *   O11 Hamming-distance filter (Table 1; the simplest pigeonhole method): the
 *       number of columns j in [0, m) where Q[j] and reference position
 *       diag + j differ under O1 (row 0 of the O6 band alone), saturated at
 *       E + 1; accept iff <= E.
 *   O12 base-counting filter (the frequency comparison of the Table 1
 *       discussion): with n_Q(c) and n_W(c) the counts of base c in {A, C,
 *       G, T} in the read and in the reference window [diag, diag + m)
 *       (N and positions outside the genome count as no base), the value is
 *       ceil(sum_c |n_Q(c) - n_W(c)| / 2), saturated at E + 1; accept iff
 *       <= E.  It never exceeds the Hamming distance of O11.
 *   O13 q-gram filter (Table 1's q-gram family, q = 5): with the read's
 *       m - 4 q-grams and the reference window [diag - E, diag + m + E) of
 *       the band, shared = the size of the multiset intersection of the
 *       q-grams free of N and of positions outside the genome, missing =
 *       (m - 4) - shared, value = ceil(missing / 5) (0 for m < 5), saturated
 *       at E + 1; accept iff <= E.  Each edit destroys at most q of the read's
 *       q-grams, so the value never exceeds the banded edit distance.
 *   O14 shifted Hamming distance (SHD, Table 1): for each row d in [-E, E] the
 *       mismatch mask H_d[j] = O6 obstacle at column j; in each mask a run of
 *       one or two zeros with a one on both sides (inside [0, m)) becomes
 *       ones; the value is the number of columns where every amended mask is
 *       one, saturated at E + 1; accept iff <= E.
 *   O15 both strands (reads come from either strand; minimap2 maps both): the
 *       reverse strand of a genome is met by the reverse complement R of the
 *       read (Q reversed, A<->T and C<->G swapped, N kept) against the forward
 *       genome.  Strand-1 seeds are the O3 minimizers of R looked up in the
 *       same forward index; a location is (genome, strand, diag) with diag =
 *       q - p for the position p in R.  O5 counts both strands together:
 *       (hits desc, genome asc, diag asc, strand asc), one top_n over the
 *       union.  The filter of a strand-1 location runs on R.  With one strand
 *       (the default) only strand 0 exists.
 *   O16 relative abundance (Fig. 1 step 3b; PARITY UNPINNED: the paper takes
 *       the apportionment from Metalign and does not state it): with T(r) the
 *       mapped taxa of read r (O8) and u_t the unique-read count of taxon t,
 *       the count of t in units of 2^-32 read is 2^32 * u_t plus, for every
 *       multi-mapped read r with t in T(r), floor(2^32 * u_t / U_r) where U_r
 *       is the sum of u over T(r), or floor(2^32 / |T(r)|) when U_r = 0 (one
 *       proportional step from the unique evidence).  With C the sum of the
 *       counts, taxon t is kept iff count_t * den >= C * num (the paper drops
 *       taxa below 0.01%: num/den = 1/10^4), and its abundance is count_t / K
 *       in double precision with K the sum over kept taxa; dropped taxa (and
 *       every taxon when C = 0) get 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)

#define MAX_READ_LEN 65535u

/* ------------------------------------------------------------ threads ---- */

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the parallel loops use from now on (n < 1: the default, which
 * OMP_NUM_THREADS sets, else every processor); returns the number that will
 * be used.  Built without OpenMP, always 1. */
int or_set_threads(int n)
{
#ifdef _OPENMP
    static int dflt = 0;
    if (dflt == 0) dflt = omp_get_max_threads();
    omp_set_num_threads(n >= 1 ? n : dflt);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ---------------------------------------------------------------- O1 ---- */

static int base_code(uint8_t c)
{
    switch (c) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    case 'N': case 'n': return 4;
    default: return -1;
    }
}

/* Codes of seq[0, len) into out; returns OR_EINVAL on a byte outside ACGTN. */
static int encode(const uint8_t *seq, int64_t len, uint8_t *out)
{
    for (int64_t i = 0; i < len; i++) {
        int c = base_code(seq[i]);
        if (c < 0) return OR_EINVAL;
        out[i] = (uint8_t)c;
    }
    return OR_OK;
}

/* ---------------------------------------------------------------- O2 ---- */

uint64_t or_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* ---------------------------------------------------------------- O3 ---- */

/*
 * Minimizers of one encoded sequence.  Writes the selected positions (in
 * increasing order) and their k-mer values; returns how many were selected.
 * pos_out / x_out must hold max(len - k + 1, 0) entries.
 */
static int64_t minimizers_of_codes(const uint8_t *code, int64_t len, int k, int w,
                                   int64_t *pos_out, uint64_t *x_out)
{
    int64_t nk = len - k + 1;
    if (nk <= 0) return 0;
    uint64_t *x = malloc((size_t)nk * sizeof *x);
    uint64_t *h = malloc((size_t)nk * sizeof *h);
    uint8_t *valid = malloc((size_t)nk);
    uint8_t *chosen = calloc((size_t)nk, 1);
    for (int64_t i = 0; i < nk; i++) {
        uint64_t v = 0;
        int ok = 1;
        for (int t = 0; t < k; t++) {
            uint8_t c = code[i + t];
            if (c == 4) ok = 0;
            v = v * 4 + (c & 3);
        }
        x[i] = v;
        h[i] = or_mix64(v);
        valid[i] = (uint8_t)ok;
    }
    int64_t win = nk < w ? nk : w;           /* one window over all k-mers if fewer than w */
    for (int64_t s = 0; s + win <= nk; s++) {
        int64_t best = -1;
        for (int64_t i = s; i < s + win; i++) {
            if (!valid[i]) continue;
            if (best < 0 || h[i] < h[best]) best = i;   /* strict '<': leftmost of equal hashes */
        }
        if (best >= 0) chosen[best] = 1;
    }
    int64_t n = 0;
    for (int64_t i = 0; i < nk; i++) {
        if (chosen[i]) {
            pos_out[n] = i;
            x_out[n] = x[i];
            n++;
        }
    }
    free(x); free(h); free(valid); free(chosen);
    return n;
}

/* Minimizers of an ASCII sequence (returns -1 on an invalid byte). */
int64_t or_minimizers(const uint8_t *seq, int64_t len, int k, int w,
                      int64_t *pos_out, uint64_t *x_out)
{
    uint8_t *code = malloc((size_t)(len > 0 ? len : 1));
    if (encode(seq, len, code) != OR_OK) { free(code); return -1; }
    int64_t n = minimizers_of_codes(code, len, k, w, pos_out, x_out);
    free(code);
    return n;
}

/* ------------------------------------------------------ stage 2a index ---- */

typedef struct {
    uint64_t x;
    uint32_t genome;
    uint32_t pos;
} occ_t;

typedef struct or_index {
    int k, w;
    uint32_t max_occ;
    uint64_t n_genomes;
    uint8_t **gcode;          /* encoded genomes */
    int64_t *glen;
    uint32_t *taxon;          /* taxon of each genome */
    uint32_t n_taxa;
    occ_t *occ;               /* all reference minimizers, sorted by (x, genome, pos) */
    int64_t n_occ;
} or_index;

static int cmp_occ(const void *a, const void *b)
{
    const occ_t *p = a, *q = b;
    if (p->x != q->x) return p->x < q->x ? -1 : 1;
    if (p->genome != q->genome) return p->genome < q->genome ? -1 : 1;
    if (p->pos != q->pos) return p->pos < q->pos ? -1 : 1;
    return 0;
}

void or_index_free(or_index *ix)
{
    if (!ix) return;
    if (ix->gcode)
        for (uint64_t g = 0; g < ix->n_genomes; g++) free(ix->gcode[g]);
    free(ix->gcode); free(ix->glen); free(ix->taxon); free(ix->occ);
    free(ix);
}

/*
 * Builds the index over genomes given as ASCII with offsets[n+1].
 * taxon: n entries (NULL = genome i is taxon i).  Returns NULL on error
 * (bad byte, k outside 1..31, w outside 1..255, genome length >= 2^32 - 2^16).
 *
 * Genomes are independent, so their encoding and their minimizers may be
 * computed on several threads (OpenMP); every genome writes only its own
 * arrays.  The occurrence array is then put in (x, genome, pos) order by one
 * pass that deals the occurrences into buckets by the top bits of x (bucket
 * b holds the x with x >> shift == b, so the buckets follow each other in x
 * order) and a qsort with the full comparison inside every bucket.
 */
or_index *or_index_build(const uint8_t *seq, const uint64_t *offsets, uint64_t n,
                         int k, int w, uint32_t max_occ,
                         const uint32_t *taxon, uint32_t n_taxa)
{
    if (k < 1 || k > 31 || w < 1 || w > 255) return NULL;
    or_index *ix = calloc(1, sizeof *ix);
    ix->k = k; ix->w = w; ix->max_occ = max_occ; ix->n_genomes = n;
    ix->gcode = calloc(n ? n : 1, sizeof *ix->gcode);
    ix->glen = calloc(n ? n : 1, sizeof *ix->glen);
    ix->taxon = calloc(n ? n : 1, sizeof *ix->taxon);
    ix->n_taxa = n_taxa;
    int64_t maxlen = 1;
    for (uint64_t g = 0; g < n; g++) {
        int64_t len = (int64_t)(offsets[g + 1] - offsets[g]);
        if (len >= (int64_t)4294901760LL) { or_index_free(ix); return NULL; }
        ix->glen[g] = len;
        ix->taxon[g] = taxon ? taxon[g] : (uint32_t)g;
        if (ix->taxon[g] >= n_taxa) { or_index_free(ix); return NULL; }
        if (len > maxlen) maxlen = len;
    }
    int bad = 0;
    #pragma omp parallel for schedule(dynamic, 1) reduction(|:bad)
    for (int64_t g = 0; g < (int64_t)n; g++) {
        ix->gcode[g] = malloc((size_t)(ix->glen[g] > 0 ? ix->glen[g] : 1));
        if (encode(seq + offsets[g], ix->glen[g], ix->gcode[g]) != OR_OK) bad = 1;
    }
    if (bad) { or_index_free(ix); return NULL; }

    /* the minimizers of every genome (stage 2a) */
    occ_t **per = calloc(n ? n : 1, sizeof *per);
    int64_t *cnt = calloc(n ? n : 1, sizeof *cnt);
    #pragma omp parallel
    {
        int64_t *pos = malloc((size_t)maxlen * sizeof *pos);
        uint64_t *x = malloc((size_t)maxlen * sizeof *x);
        #pragma omp for schedule(dynamic, 1)
        for (int64_t g = 0; g < (int64_t)n; g++) {
            int64_t c = minimizers_of_codes(ix->gcode[g], ix->glen[g], k, w, pos, x);
            per[g] = malloc((size_t)(c > 0 ? c : 1) * sizeof *per[g]);
            for (int64_t i = 0; i < c; i++) {
                occ_t o = { x[i], (uint32_t)g, (uint32_t)pos[i] };
                per[g][i] = o;
            }
            cnt[g] = c;
        }
        free(pos); free(x);
    }

    /* sort by (x, genome, pos): buckets by the top bits of x, then qsort each */
    int bits = 2 * k < 12 ? 2 * k : 12;
    int shift = 2 * k - bits;
    int64_t nb = (int64_t)1 << bits;
    int64_t *bstart = calloc((size_t)nb + 1, sizeof *bstart);
    int64_t total = 0;
    for (uint64_t g = 0; g < n; g++) {
        for (int64_t i = 0; i < cnt[g]; i++) bstart[(per[g][i].x >> shift) + 1]++;
        total += cnt[g];
    }
    for (int64_t b = 0; b < nb; b++) bstart[b + 1] += bstart[b];
    ix->occ = malloc((size_t)(total > 0 ? total : 1) * sizeof *ix->occ);
    ix->n_occ = total;
    int64_t *fill = malloc((size_t)nb * sizeof *fill);
    memcpy(fill, bstart, (size_t)nb * sizeof *fill);
    for (uint64_t g = 0; g < n; g++) {
        for (int64_t i = 0; i < cnt[g]; i++) ix->occ[fill[per[g][i].x >> shift]++] = per[g][i];
        free(per[g]);
    }
    free(per); free(cnt); free(fill);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < nb; b++)
        qsort(ix->occ + bstart[b], (size_t)(bstart[b + 1] - bstart[b]), sizeof *ix->occ, cmp_occ);
    free(bstart);
    return ix;
}

int64_t or_index_n_occ(const or_index *ix) { return ix->n_occ; }

/* Copies the occurrence array (x, genome, pos), in its sorted order. */
void or_index_copy_occ(const or_index *ix, uint64_t *x, uint32_t *genome, uint32_t *pos)
{
    for (int64_t i = 0; i < ix->n_occ; i++) {
        x[i] = ix->occ[i].x;
        genome[i] = ix->occ[i].genome;
        pos[i] = ix->occ[i].pos;
    }
}

/* First index in occ with occ.x >= x. */
static int64_t lower_bound(const occ_t *occ, int64_t n, uint64_t x)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (occ[mid].x < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* -------------------------------------------------------- O6 filter ---- */

/* Is reference position p of genome g a mismatch for read code qc? */
static int obstacle(uint8_t qc, const uint8_t *gcode, int64_t glen, int64_t p)
{
    if (qc == 4) return 1;
    if (p < 0 || p >= glen) return 1;
    uint8_t rc = gcode[p];
    if (rc == 4) return 1;
    return qc != rc;
}

/*
 * Approximate edit distance of read q[0,m) at location (genome, diag) with
 * threshold E: the obstacle count of O6, saturated at E + 1.
 */
static int approx_codes(const uint8_t *q, int64_t m, const uint8_t *gcode, int64_t glen,
                        int64_t diag, int E)
{
    int64_t rows = 2 * (int64_t)E + 1;
    uint8_t *M = malloc((size_t)(rows * (m > 0 ? m : 1)));
    for (int64_t r = 0; r < rows; r++) {
        int64_t d = r - E;
        for (int64_t j = 0; j < m; j++)
            M[r * m + j] = (uint8_t)obstacle(q[j], gcode, glen, diag + j + d);
    }
    int64_t j = 0;
    int c = 0;
    for (;;) {
        int64_t best = 0;
        for (int64_t r = 0; r < rows; r++) {
            int64_t run = 0;
            while (j + run < m && M[r * m + j + run] == 0) run++;
            if (run > best) best = run;
        }
        j += best;
        if (j >= m) break;
        c += 1;
        if (c > E) break;
        j += 1;
    }
    free(M);
    return c < E + 1 ? c : E + 1;
}

/* The filter on ASCII inputs: read q[0,m), reference ref[0,L).  -1 on a bad byte. */
int or_approx(const uint8_t *q, int64_t m, const uint8_t *ref, int64_t L, int64_t diag, int E)
{
    uint8_t *qc = malloc((size_t)(m > 0 ? m : 1));
    uint8_t *rc = malloc((size_t)(L > 0 ? L : 1));
    int r = -1;
    if (encode(q, m, qc) == OR_OK && encode(ref, L, rc) == OR_OK)
        r = approx_codes(qc, m, rc, L, diag, E);
    free(qc); free(rc);
    return r;
}

/* ---------------------------------------------------- classification ---- */

/* E of a read of length m: mode 0 fixed, 1 ceil(m*v/1000), 2 floor(m*v/1000). */
int or_read_E(int64_t m, uint32_t e_mode, uint32_t e_value)
{
    if (e_mode == 0) return (int)e_value;
    uint64_t num = (uint64_t)m * e_value;
    if (e_mode == 1) return (int)((num + 999) / 1000);
    return (int)(num / 1000);
}

typedef struct { uint32_t genome; int64_t diag; uint8_t strand; } hit_t;
typedef struct { uint32_t genome; int64_t diag; uint32_t hits; uint8_t strand; } cand_t;

static int cmp_hit(const void *a, const void *b)
{
    const hit_t *p = a, *q = b;
    if (p->genome != q->genome) return p->genome < q->genome ? -1 : 1;
    if (p->diag != q->diag) return p->diag < q->diag ? -1 : 1;
    if (p->strand != q->strand) return p->strand < q->strand ? -1 : 1;
    return 0;
}

/* O5 order: hits descending, then genome ascending, then diagonal ascending,
 * then strand ascending (O15). */
static int cmp_cand(const void *a, const void *b)
{
    const cand_t *p = a, *q = b;
    if (p->hits != q->hits) return p->hits > q->hits ? -1 : 1;
    if (p->genome != q->genome) return p->genome < q->genome ? -1 : 1;
    if (p->diag != q->diag) return p->diag < q->diag ? -1 : 1;
    if (p->strand != q->strand) return p->strand < q->strand ? -1 : 1;
    return 0;
}

/* O15: codes of the reverse complement of q[0, m) (A0<->T3, C1<->G2, N4 kept). */
static void reverse_complement_codes(const uint8_t *q, int64_t m, uint8_t *out)
{
    for (int64_t j = 0; j < m; j++) {
        uint8_t c = q[m - 1 - j];
        out[j] = c == 4 ? 4 : (uint8_t)(3 - c);
    }
}

typedef struct or_result {
    uint64_t n_reads;
    uint64_t *cand_offsets;    /* n_reads + 1 */
    uint8_t *read_accepted;    /* n_reads */
    uint16_t *read_E;          /* n_reads */
    uint64_t n_cands;
    uint32_t *genome;
    int64_t *diag;
    uint32_t *hits;
    uint16_t *approx;
    uint8_t *accept;
    uint8_t *strand;
    uint32_t n_taxa;
    uint64_t *unique_reads;
    uint64_t *multi_reads;
    uint64_t unmapped;
    uint64_t cap;
} or_result;

void or_result_free(or_result *r)
{
    if (!r) return;
    free(r->cand_offsets); free(r->read_accepted); free(r->read_E);
    free(r->genome); free(r->diag); free(r->hits); free(r->approx); free(r->accept); free(r->strand);
    free(r->unique_reads); free(r->multi_reads);
    free(r);
}

static void push_cand(or_result *r, const cand_t *c)
{
    if (r->n_cands == r->cap) {
        r->cap = r->cap ? 2 * r->cap : 1024;
        r->genome = realloc(r->genome, r->cap * sizeof *r->genome);
        r->diag = realloc(r->diag, r->cap * sizeof *r->diag);
        r->hits = realloc(r->hits, r->cap * sizeof *r->hits);
        r->approx = realloc(r->approx, r->cap * sizeof *r->approx);
        r->accept = realloc(r->accept, r->cap * sizeof *r->accept);
        r->strand = realloc(r->strand, r->cap * sizeof *r->strand);
    }
    r->genome[r->n_cands] = c->genome;
    r->strand[r->n_cands] = c->strand;
    r->diag[r->n_cands] = c->diag;
    r->hits[r->n_cands] = c->hits;
    r->n_cands++;
}

static int hamming_codes(const uint8_t *q, int64_t m, const uint8_t *gcode, int64_t glen, int64_t diag, int E);
static int base_count_codes(const uint8_t *q, int64_t m, const uint8_t *gcode, int64_t glen, int64_t diag, int E);
static int qgram_codes(const uint8_t *q, int64_t m, const uint8_t *gcode, int64_t glen, int64_t diag, int E);
static int shd_codes(const uint8_t *q, int64_t m, const uint8_t *gcode, int64_t glen, int64_t diag, int E);

/* The filter of kind 0 (O6 obstacle walk), 1 (O11 Hamming), 2 (O12 base
 * counting), 3 (O13 q-grams) or 4 (O14 SHD) on one pair. */
static int filter_codes(uint32_t kind, const uint8_t *q, int64_t m, const uint8_t *gcode, int64_t glen,
                        int64_t diag, int E)
{
    switch (kind) {
    case 1: return hamming_codes(q, m, gcode, glen, diag, E);
    case 2: return base_count_codes(q, m, gcode, glen, diag, E);
    case 3: return qgram_codes(q, m, gcode, glen, diag, E);
    case 4: return shd_codes(q, m, gcode, glen, diag, E);
    default: return approx_codes(q, m, gcode, glen, diag, E);
    }
}

/* Stages 2b-2d of one read: its candidates in O5 order (top_n applied) with
 * their filter values.  Reads are independent, so several threads may run
 * this at once; each call writes only its own record. */
typedef struct {
    int err;            /* nonzero: bad byte, read longer than 65535 or E above 65534 */
    int E;
    int64_t nc;
    cand_t *cand;
    uint16_t *approx;
    uint8_t *accept;
} read_out_t;

static void classify_read(const or_index *ix, const uint8_t *ascii, int64_t m, uint32_t min_hits, uint32_t top_n,
                          uint32_t e_mode, uint32_t e_value, uint32_t kind, uint32_t strands, read_out_t *out)
{
    memset(out, 0, sizeof *out);
    int E = or_read_E(m, e_mode, e_value);
    if (m > (int64_t)MAX_READ_LEN || E > 65534) { out->err = 1; return; }
    out->E = E;
    /* the read (strand 0) and its reverse complement (strand 1, O15) */
    uint8_t *oriented[2];
    oriented[0] = malloc((size_t)(m > 0 ? m : 1));
    oriented[1] = malloc((size_t)(m > 0 ? m : 1));
    if (encode(ascii, m, oriented[0]) != OR_OK) {
        free(oriented[0]); free(oriented[1]); out->err = 1; return;
    }
    reverse_complement_codes(oriented[0], m, oriented[1]);

    /* stage 2b: read minimizers and their seed matches -> (genome, diag, strand) hits */
    int64_t nk = m - ix->k + 1 > 0 ? m - ix->k + 1 : 0;
    int64_t *mpos = malloc((size_t)(nk ? nk : 1) * sizeof *mpos);
    uint64_t *mx = malloc((size_t)(nk ? nk : 1) * sizeof *mx);
    int64_t nh = 0, hcap = 64;
    hit_t *hit = malloc((size_t)hcap * sizeof *hit);
    for (uint32_t st = 0; st < strands; st++) {
        int64_t nmin = minimizers_of_codes(oriented[st], m, ix->k, ix->w, mpos, mx);
        for (int64_t i = 0; i < nmin; i++) {
            int64_t lo = lower_bound(ix->occ, ix->n_occ, mx[i]);
            int64_t hi = lo;
            while (hi < ix->n_occ && ix->occ[hi].x == mx[i]) hi++;
            if (ix->max_occ > 0 && hi - lo > (int64_t)ix->max_occ) continue;
            for (int64_t o = lo; o < hi; o++) {
                if (nh == hcap) { hcap *= 2; hit = realloc(hit, (size_t)hcap * sizeof *hit); }
                hit[nh].genome = ix->occ[o].genome;
                hit[nh].diag = (int64_t)ix->occ[o].pos - mpos[i];
                hit[nh].strand = (uint8_t)st;
                nh++;
            }
        }
    }
    free(mpos); free(mx);

    /* stage 2b/2c: seed hits per location, minimum, order, top N */
    qsort(hit, (size_t)nh, sizeof *hit, cmp_hit);
    cand_t *cand = malloc((size_t)(nh ? nh : 1) * sizeof *cand);
    int64_t nc = 0;
    for (int64_t i = 0; i < nh;) {
        int64_t j = i;
        while (j < nh && hit[j].genome == hit[i].genome && hit[j].diag == hit[i].diag &&
               hit[j].strand == hit[i].strand)
            j++;
        if ((uint64_t)(j - i) >= min_hits) {
            cand[nc].genome = hit[i].genome;
            cand[nc].diag = hit[i].diag;
            cand[nc].strand = hit[i].strand;
            cand[nc].hits = (uint32_t)(j - i);
            nc++;
        }
        i = j;
    }
    free(hit);
    qsort(cand, (size_t)nc, sizeof *cand, cmp_cand);
    if (top_n > 0 && nc > (int64_t)top_n) nc = top_n;

    /* stage 2d: approximate edit distance + accept per pair */
    out->nc = nc;
    out->cand = cand;
    out->approx = malloc((size_t)(nc ? nc : 1) * sizeof *out->approx);
    out->accept = malloc((size_t)(nc ? nc : 1));
    for (int64_t c = 0; c < nc; c++) {
        uint32_t g = cand[c].genome;
        int a = filter_codes(kind, oriented[cand[c].strand], m, ix->gcode[g], ix->glen[g], cand[c].diag, E);
        out->approx[c] = (uint16_t)a;
        out->accept[c] = (uint8_t)(a <= E);
    }
    free(oriented[0]); free(oriented[1]);
}

static void read_out_free(read_out_t *o)
{
    free(o->cand); free(o->approx); free(o->accept);
}

#define READ_BLOCK 65536

/*
 * Classifies reads (ASCII + offsets[n+1]) on one strand or both (O15).
 * Returns NULL on an invalid input (bad byte, read longer than 65535, E above
 * 65534, unknown filter kind, strands other than 1 or 2).
 *
 * The reads of a block go through stages 2b-2d on all threads at once
 * (classify_read); the block's results are then appended in read order and
 * counted per taxon (stage 3a) on one thread.
 */
or_result *or_classify_strands(const or_index *ix, const uint8_t *seq, const uint64_t *offsets, uint64_t n,
                               uint32_t min_hits, uint32_t top_n, uint32_t e_mode, uint32_t e_value,
                               uint32_t kind, uint32_t strands)
{
    if (kind > 4 || strands < 1 || strands > 2) return NULL;
    or_result *res = calloc(1, sizeof *res);
    res->n_reads = n;
    res->cand_offsets = calloc(n + 1, sizeof *res->cand_offsets);
    res->read_accepted = calloc(n ? n : 1, 1);
    res->read_E = calloc(n ? n : 1, sizeof *res->read_E);
    res->n_taxa = ix->n_taxa;
    res->unique_reads = calloc(ix->n_taxa ? ix->n_taxa : 1, sizeof(uint64_t));
    res->multi_reads = calloc(ix->n_taxa ? ix->n_taxa : 1, sizeof(uint64_t));
    uint8_t *taxon_seen = calloc(ix->n_taxa ? ix->n_taxa : 1, 1);
    read_out_t *outs = malloc(sizeof *outs * (n < READ_BLOCK ? (n ? n : 1) : READ_BLOCK));

    for (uint64_t r0 = 0; r0 < n; r0 += READ_BLOCK) {
        int64_t nb = (int64_t)(n - r0 < READ_BLOCK ? n - r0 : READ_BLOCK);
        #pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = 0; i < nb; i++) {
            uint64_t r = r0 + (uint64_t)i;
            classify_read(ix, seq + offsets[r], (int64_t)(offsets[r + 1] - offsets[r]), min_hits, top_n, e_mode,
                          e_value, kind, strands, &outs[i]);
        }
        int failed = 0;
        for (int64_t i = 0; i < nb; i++) failed |= outs[i].err;
        if (failed) {
            for (int64_t i = 0; i < nb; i++) read_out_free(&outs[i]);
            free(outs); free(taxon_seen); or_result_free(res);
            return NULL;
        }
        for (int64_t i = 0; i < nb; i++) {
            uint64_t r = r0 + (uint64_t)i;
            read_out_t *o = &outs[i];
            int E = o->E;
            res->read_E[r] = (uint16_t)E;
            uint64_t first = res->n_cands;
            int best = -1;
            for (int64_t c = 0; c < o->nc; c++) {
                push_cand(res, &o->cand[c]);
                int a = o->approx[c];
                res->approx[res->n_cands - 1] = o->approx[c];
                res->accept[res->n_cands - 1] = o->accept[c];
                if (a <= E && (best < 0 || a < best)) best = a;
            }
            res->cand_offsets[r + 1] = res->n_cands;
            read_out_free(o);

            /* stage 3a: per-taxon unique / multi-mapped counts */
            if (best < 0) {
                res->unmapped++;
                continue;
            }
            res->read_accepted[r] = 1;
            uint32_t ntax = 0, only = 0;
            for (uint64_t c = first; c < res->n_cands; c++) {
                if (!res->accept[c] || res->approx[c] != best) continue;
                uint32_t t = ix->taxon[res->genome[c]];
                if (!taxon_seen[t]) { taxon_seen[t] = 1; ntax++; only = t; }
            }
            for (uint64_t c = first; c < res->n_cands; c++) {
                if (!res->accept[c] || res->approx[c] != best) continue;
                uint32_t t = ix->taxon[res->genome[c]];
                if (taxon_seen[t]) {
                    taxon_seen[t] = 0;
                    if (ntax > 1) res->multi_reads[t]++;
                }
            }
            if (ntax == 1) res->unique_reads[only]++;
        }
    }
    free(outs);
    free(taxon_seen);
    return res;
}

/* Classification on the forward strand with the filter of the given kind. */
or_result *or_classify_kind(const or_index *ix, const uint8_t *seq, const uint64_t *offsets, uint64_t n,
                            uint32_t min_hits, uint32_t top_n, uint32_t e_mode, uint32_t e_value, uint32_t kind)
{
    return or_classify_strands(ix, seq, offsets, n, min_hits, top_n, e_mode, e_value, kind, 1);
}

/* Classification with the obstacle filter (kind 0). */
or_result *or_classify(const or_index *ix, const uint8_t *seq, const uint64_t *offsets, uint64_t n,
                       uint32_t min_hits, uint32_t top_n, uint32_t e_mode, uint32_t e_value)
{
    return or_classify_kind(ix, seq, offsets, n, min_hits, top_n, e_mode, e_value, 0);
}

uint64_t or_result_n_cands(const or_result *r) { return r->n_cands; }

/* Copies a result into caller arrays (sizes from or_result_n_cands / n_reads / n_taxa). */
void or_result_copy(const or_result *r, uint64_t *cand_offsets, uint8_t *read_accepted, uint16_t *read_E,
                    uint32_t *genome, int64_t *diag, uint32_t *hits, uint16_t *approx, uint8_t *accept,
                    uint64_t *unique_reads, uint64_t *multi_reads, uint64_t *unmapped)
{
    memcpy(cand_offsets, r->cand_offsets, (r->n_reads + 1) * sizeof *cand_offsets);
    memcpy(read_accepted, r->read_accepted, r->n_reads);
    memcpy(read_E, r->read_E, r->n_reads * sizeof *read_E);
    if (r->n_cands) {
        memcpy(genome, r->genome, r->n_cands * sizeof *genome);
        memcpy(diag, r->diag, r->n_cands * sizeof *diag);
        memcpy(hits, r->hits, r->n_cands * sizeof *hits);
        memcpy(approx, r->approx, r->n_cands * sizeof *approx);
        memcpy(accept, r->accept, r->n_cands);
    }
    memcpy(unique_reads, r->unique_reads, r->n_taxa * sizeof *unique_reads);
    memcpy(multi_reads, r->multi_reads, r->n_taxa * sizeof *multi_reads);
    *unmapped = r->unmapped;
}

/* The strand of every candidate (O15). */
void or_result_strand(const or_result *r, uint8_t *strand)
{
    if (r->n_cands) memcpy(strand, r->strand, r->n_cands);
}

/* O11: mismatching columns of row 0, saturated at E + 1. */
static int hamming_codes(const uint8_t *q, int64_t m, const uint8_t *gcode, int64_t glen, int64_t diag, int E)
{
    int64_t c = 0;
    for (int64_t j = 0; j < m; j++) c += obstacle(q[j], gcode, glen, diag + j);
    return c < E + 1 ? (int)c : E + 1;
}

/* O12: half the L1 distance of the base counts, rounded up, saturated at E + 1. */
static int base_count_codes(const uint8_t *q, int64_t m, const uint8_t *gcode, int64_t glen, int64_t diag, int E)
{
    int64_t nq[4] = {0, 0, 0, 0}, nw[4] = {0, 0, 0, 0};
    for (int64_t j = 0; j < m; j++) {
        if (q[j] < 4) nq[q[j]]++;
        int64_t p = diag + j;
        if (p >= 0 && p < glen && gcode[p] < 4) nw[gcode[p]]++;
    }
    int64_t l1 = 0;
    for (int c = 0; c < 4; c++) l1 += nq[c] > nw[c] ? nq[c] - nw[c] : nw[c] - nq[c];
    int64_t v = (l1 + 1) / 2;
    return v < E + 1 ? (int)v : E + 1;
}

#define QGRAM_Q 5

/* O13: the q-gram lower bound over the band's window, saturated at E + 1. */
static int qgram_codes(const uint8_t *q, int64_t m, const uint8_t *gcode, int64_t glen, int64_t diag, int E)
{
    if (m < QGRAM_Q) return 0;
    uint32_t *cw = calloc(1u << (2 * QGRAM_Q), sizeof *cw);
    for (int64_t p = diag - E; p + QGRAM_Q <= diag + m + E; p++) {
        int v = 0, ok = 1;
        for (int t = 0; t < QGRAM_Q && ok; t++) {
            int64_t x = p + t;
            if (x < 0 || x >= glen || gcode[x] == 4) ok = 0;
            else v = v * 4 + gcode[x];
        }
        if (ok) cw[v]++;
    }
    int64_t shared = 0;
    for (int64_t j = 0; j + QGRAM_Q <= m; j++) {
        int v = 0, ok = 1;
        for (int t = 0; t < QGRAM_Q && ok; t++) {
            if (q[j + t] == 4) ok = 0;
            else v = v * 4 + q[j + t];
        }
        if (ok && cw[v] > 0) { cw[v]--; shared++; }
    }
    free(cw);
    int64_t missing = (m - QGRAM_Q + 1) - shared;
    int64_t val = (missing + QGRAM_Q - 1) / QGRAM_Q;
    return val < E + 1 ? (int)val : E + 1;
}

/* O14: ones of the AND over the band of the amended mismatch masks. */
static int shd_codes(const uint8_t *q, int64_t m, const uint8_t *gcode, int64_t glen, int64_t diag, int E)
{
    if (m == 0) return 0;
    uint8_t *F = malloc((size_t)m), *H = malloc((size_t)m);
    memset(F, 1, (size_t)m);
    for (int64_t d = -(int64_t)E; d <= E; d++) {
        for (int64_t j = 0; j < m; j++) H[j] = (uint8_t)obstacle(q[j], gcode, glen, diag + j + d);
        for (int64_t j = 0; j < m;) {
            if (H[j]) { F[j] &= 1; j++; continue; }
            int64_t k = j;
            while (k < m && !H[k]) k++;              /* zeros [j, k) */
            int amend = j > 0 && k < m && k - j <= 2;  /* a short match between two mismatches */
            for (int64_t t = j; t < k; t++) F[t] &= (uint8_t)amend;
            j = k;
        }
    }
    int64_t c = 0;
    for (int64_t j = 0; j < m; j++) c += F[j];
    free(F); free(H);
    return c < E + 1 ? (int)c : E + 1;
}

/*
 * One filter of kind 0 (O6 obstacle walk), 1 (O11 Hamming), 2 (O12 base
 * counting), 3 (O13 q-grams) or 4 (O14 SHD) over explicit pairs, as
 * or_filter_pairs.  Returns OR_EINVAL on a bad byte, an out-of-range index or
 * an unknown kind.
 */
int or_filter_pairs_kind(const or_index *ix, const uint8_t *seq, const uint64_t *offsets, uint64_t n_reads,
                         const uint32_t *pair_read, const uint32_t *pair_genome, const int64_t *pair_diag,
                         const uint16_t *pair_E, uint64_t n_pairs, uint32_t kind, uint16_t *approx_out,
                         uint8_t *accept_out)
{
    if (kind > 4) return OR_EINVAL;
    int bad = 0;
    /* pairs are independent: several threads may filter at once */
    #pragma omp parallel for schedule(dynamic, 64) reduction(|:bad)
    for (int64_t pi = 0; pi < (int64_t)n_pairs; pi++) {
        uint64_t p = (uint64_t)pi;
        if (pair_read[p] >= n_reads || pair_genome[p] >= ix->n_genomes) { bad = 1; continue; }
        uint64_t r = pair_read[p];
        int64_t m = (int64_t)(offsets[r + 1] - offsets[r]);
        uint8_t *q = malloc((size_t)(m > 0 ? m : 1));
        if (encode(seq + offsets[r], m, q) != OR_OK) { free(q); bad = 1; continue; }
        uint32_t g = pair_genome[p];
        int E = pair_E[p];
        int a = filter_codes(kind, q, m, ix->gcode[g], ix->glen[g], pair_diag[p], E);
        approx_out[p] = (uint16_t)a;
        accept_out[p] = (uint8_t)(a <= E);
        free(q);
    }
    return bad ? OR_EINVAL : OR_OK;
}

/* The obstacle filter alone over explicit pairs (pair_read indexes the reads). */
int or_filter_pairs(const or_index *ix, const uint8_t *seq, const uint64_t *offsets, uint64_t n_reads,
                    const uint32_t *pair_read, const uint32_t *pair_genome, const int64_t *pair_diag,
                    const uint16_t *pair_E, uint64_t n_pairs, uint16_t *approx_out, uint8_t *accept_out)
{
    return or_filter_pairs_kind(ix, seq, offsets, n_reads, pair_read, pair_genome, pair_diag, pair_E, n_pairs, 0,
                                approx_out, accept_out);
}

/* ----------------------------------------- stage 1 containment search ---- */

/*
 * Containment search (Fig. 1 steps 1a-1c, "Containment Search"): seeds
 * every read (ASCII + offsets[n+1]) and adds to hits[g] one per seed match in
 * genome g (reading O9).  hits: n_genomes entries, overwritten.  Returns
 * OR_EINVAL on a bad byte or a read longer than 65535.
 */
int or_containment(const or_index *ix, const uint8_t *seq, const uint64_t *offsets, uint64_t n, uint64_t *hits)
{
    for (uint64_t g = 0; g < ix->n_genomes; g++) hits[g] = 0;
    int bad = 0;
    /* reads are independent: each thread counts into its own array, and the
     * arrays are summed into hits at the end */
    #pragma omp parallel reduction(|:bad)
    {
        uint64_t *local = calloc(ix->n_genomes ? ix->n_genomes : 1, sizeof *local);
        #pragma omp for schedule(dynamic, 64)
        for (int64_t ri = 0; ri < (int64_t)n; ri++) {
            uint64_t r = (uint64_t)ri;
            int64_t m = (int64_t)(offsets[r + 1] - offsets[r]);
            if (m > (int64_t)MAX_READ_LEN) { bad = 1; continue; }
            uint8_t *q = malloc((size_t)(m > 0 ? m : 1));
            if (encode(seq + offsets[r], m, q) != OR_OK) { free(q); bad = 1; continue; }
            int64_t nk = m - ix->k + 1 > 0 ? m - ix->k + 1 : 0;
            int64_t *mpos = malloc((size_t)(nk ? nk : 1) * sizeof *mpos);
            uint64_t *mx = malloc((size_t)(nk ? nk : 1) * sizeof *mx);
            int64_t nmin = minimizers_of_codes(q, m, ix->k, ix->w, mpos, mx);
            for (int64_t i = 0; i < nmin; i++) {
                int64_t lo = lower_bound(ix->occ, ix->n_occ, mx[i]);
                int64_t hi = lo;
                while (hi < ix->n_occ && ix->occ[hi].x == mx[i]) hi++;
                if (ix->max_occ && (uint64_t)(hi - lo) > ix->max_occ) continue; /* O4 cap */
                for (int64_t o = lo; o < hi; o++) local[ix->occ[o].genome] += 1;
            }
            free(mpos); free(mx); free(q);
        }
        #pragma omp critical
        for (uint64_t g = 0; g < ix->n_genomes; g++) hits[g] += local[g];
        free(local);
    }
    return bad ? OR_EINVAL : OR_OK;
}

/*
 * Subset database selection (Fig. 1 step 1d; the normalised seed-hit cutoff of
 * the containment Evaluation Methodology): reading O10 with exact 128-bit
 * products.  selected receives the kept genome indices in ascending order and
 * *max_out the largest count.  Returns the number kept, or -1 when den is 0.
 */
int64_t or_select_genomes(const uint64_t *hits, uint64_t n, uint64_t num, uint64_t den, uint32_t *selected,
                          uint64_t *max_out)
{
    if (den == 0) return -1;
    uint64_t M = 0;
    for (uint64_t g = 0; g < n; g++) if (hits[g] > M) M = hits[g];
    *max_out = M;
    int64_t c = 0;
    for (uint64_t g = 0; g < n; g++)
        if ((unsigned __int128)hits[g] * den > (unsigned __int128)M * num) selected[c++] = (uint32_t)g;
    return c;
}

/* ------------------------------------------------ stage 3b abundance ---- */

/*
 * num / den as the nearest double, ties to even (0 <= num <= den, den > 0,
 * den < 2^127): the quotient's binary expansion by schoolbook long division,
 * its first 53 significant bits rounded with the next bit and whether any
 * remainder is left.  Converting num and den to double first and dividing
 * would round twice once den needs more than 53 bits.
 */
static double div_nearest(unsigned __int128 num, unsigned __int128 den)
{
    if (num == 0) return 0.0;
    if (num >= den) return 1.0;
    int e = 0;                        /* num / den lies in [2^-e, 2^(1-e)) */
    unsigned __int128 r = num;
    while (r < den) { r <<= 1; e++; }
    r -= den;                         /* the leading quotient bit, weight 2^-e */
    uint64_t q = 1;
    for (int i = 1; i < 53; i++) {
        r <<= 1;
        q <<= 1;
        if (r >= den) { r -= den; q |= 1; }
    }
    r <<= 1;                          /* the next bit, then the rest */
    int half = r >= den;
    if (half) r -= den;
    if (half && (r != 0 || (q & 1))) q++;
    return ldexp((double)q, -e - 52);  /* q <= 2^53: exact */
}

/*
 * Relative abundance from a classification's candidates (reading O16):
 * cand_offsets[n_reads + 1], genome / approx / accept per candidate,
 * taxon_of_genome.  counts (n_taxa, units of 2^-32 read) and abund (n_taxa)
 * receive the results.  Returns the number of kept taxa, -1 when den is 0.
 */
int64_t or_abundance(uint64_t n_reads, const uint64_t *cand_offsets, const uint32_t *genome, const uint16_t *approx,
                     const uint8_t *accept, const uint32_t *taxon_of_genome, uint32_t n_taxa, uint64_t num,
                     uint64_t den, uint64_t *counts, double *abund)
{
    if (den == 0) return -1;
    uint64_t *unique = calloc(n_taxa ? n_taxa : 1, sizeof *unique);
    uint32_t *set = malloc(sizeof *set * (n_taxa ? n_taxa : 1));
    memset(counts, 0, sizeof *counts * n_taxa);
    for (int pass = 0; pass < 2; pass++) {
        for (uint64_t r = 0; r < n_reads; r++) {
            /* the read's mapped taxa (O8): distinct taxa of accepted candidates at the best value */
            int best = -1;
            for (uint64_t c = cand_offsets[r]; c < cand_offsets[r + 1]; c++)
                if (accept[c] && (best < 0 || approx[c] < best)) best = approx[c];
            if (best < 0) continue;
            uint32_t nt = 0;
            for (uint64_t c = cand_offsets[r]; c < cand_offsets[r + 1]; c++) {
                if (!accept[c] || approx[c] != best) continue;
                uint32_t t = taxon_of_genome[genome[c]], seen = 0;
                for (uint32_t i = 0; i < nt; i++) seen |= set[i] == t;
                if (!seen) set[nt++] = t;
            }
            if (pass == 0) {                 /* unique-read counts u_t */
                if (nt == 1) unique[set[0]]++;
                continue;
            }
            if (nt == 1) {
                counts[set[0]] += (uint64_t)1 << 32;
                continue;
            }
            uint64_t U = 0;
            for (uint32_t i = 0; i < nt; i++) U += unique[set[i]];
            for (uint32_t i = 0; i < nt; i++)
                counts[set[i]] += U ? (uint64_t)(((unsigned __int128)unique[set[i]] << 32) / U)
                                    : ((uint64_t)1 << 32) / nt;
        }
    }
    unsigned __int128 C = 0, K = 0;
    for (uint32_t t = 0; t < n_taxa; t++) C += counts[t];
    int64_t kept = 0;
    for (uint32_t t = 0; t < n_taxa; t++) {
        int keep = C > 0 && (unsigned __int128)counts[t] * den >= C * num;
        if (keep) { K += counts[t]; kept++; }
    }
    for (uint32_t t = 0; t < n_taxa; t++) {
        int keep = C > 0 && (unsigned __int128)counts[t] * den >= C * num;
        abund[t] = keep ? div_nearest(counts[t], K) : 0.0;
    }
    free(unique);
    free(set);
    return kept;
}
