// Serving loop: continuous batching of classification requests against one
// HBM-resident index.
//
// mt_server_submit validates a request on the host and copies it into a
// pinned host arena, so its upload can run as an asynchronous DMA.  Worker
// threads, each owning a HIP stream, repeatedly form a device batch from the
// queued requests: requests with the same query parameters, in arrival order,
// a large request split across batches, admitted while the estimated device
// bytes of all batches in flight stay within the memory budget.  A batch is
// uploaded, classified by the fused form, its taxon step (Fig. 1 step 3a) is
// run once more per request slot into each request's own device counters,
// and its per-read and per-candidate outputs are copied back and sliced per
// request.  Every read is classified independently of the reads around it,
// so a served result is the same as classifying the request alone.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "classify.hpp"

namespace mt {
namespace serve {

inline u64 now_ns() {
    return (u64)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

constexpr u64 ARENA_ALIGN = 256;
constexpr u32 MAX_SLOTS = 256;  // requests per device batch

// First-fit allocator over one pinned host block.
class PinnedArena {
  public:
    void init(u64 bytes) {
        MT_HIP(hipHostMalloc((void **)&base_, bytes, hipHostMallocDefault));
        size_ = bytes;
        free_[0] = bytes;
    }
    ~PinnedArena() {
        if (base_) (void)hipHostFree(base_);
    }
    u8 *base() const { return base_; }
    u64 size() const { return size_; }
    static u64 granule(u64 b) { return std::max<u64>(ARENA_ALIGN, (b + ARENA_ALIGN - 1) / ARENA_ALIGN * ARENA_ALIGN); }
    // Offset of a free block of `bytes`, or ~0 if no free range is large enough.
    u64 alloc(u64 bytes) {
        bytes = granule(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const u64 off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            return off;
        }
        return ~0ull;
    }
    void release(u64 off, u64 bytes) {
        bytes = granule(bytes);
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }

  private:
    u8 *base_ = nullptr;
    u64 size_ = 0;
    std::map<u64, u64> free_;  // offset -> length
};

// Pinned host buffer that grows on demand (per worker).
struct Pinned {
    u8 *p = nullptr;
    u64 cap = 0;
    void ensure(u64 bytes) {
        if (bytes <= cap) return;
        if (p) MT_HIP(hipHostFree(p));
        p = nullptr;
        cap = 0;
        const u64 want = std::max<u64>(bytes, 1ull << 20) * 5 / 4;
        MT_HIP(hipHostMalloc((void **)&p, want, hipHostMallocDefault));
        cap = want;
    }
    ~Pinned() {
        if (p) (void)hipHostFree(p);
    }
};

// Outputs of reads [r0, r0 + len) of one request, as classified in one batch.
struct Piece {
    u64 len = 0;
    std::vector<u64> cand_off;  // len + 1, from 0
    std::vector<u8> read_accepted;
    std::vector<u16> read_E;
    std::vector<u32> genome;
    std::vector<i64> diag;
    std::vector<u32> hits;
    std::vector<u16> approx;
    std::vector<u8> accept;
    std::vector<u8> strand;  // both-strand queries only
};

struct Request {
    u64 id = 0;
    mt_query_params q{};
    u64 n = 0, bases = 0;
    u64 arena_off = 0, arena_bytes = 0;
    const u64 *off = nullptr;  // n + 1 offsets, in the arena
    const u8 *seq = nullptr;   // bases, in the arena
    u64 next = 0;              // first read not yet in a batch
    u32 open = 0;              // batches holding reads of this request
    unsigned long long *counts = nullptr;  // device: unique[n_taxa], multi[n_taxa], unmapped
    hipEvent_t zeroed = nullptr;           // recorded on the control stream once counts are zero
    std::map<u64, Piece> pieces;           // by first read
    int status = MT_OK;
    std::string error;
    bool done = false, waiting = false;
    u64 submit_ns = 0;
    std::unique_ptr<mt_result> result;
};

struct Slice {
    Request *req;
    u64 r0, len;  // reads of the request
    u64 b0;       // first read in the batch
};

struct Batch {
    std::vector<Slice> slices;
    mt_query_params q{};
    u64 reads = 0, bases = 0, est = 0;
};

inline bool same_query(const mt_query_params &a, const mt_query_params &b) {
    return a.min_hits == b.min_hits && a.top_n == b.top_n && a.e_mode == b.e_mode && a.e_value == b.e_value &&
           a.filter == b.filter && (a.strands == 2) == (b.strands == 2);
}

// Device bytes a batch holds while it runs: bases and offsets, the read planes
// and outputs, and the staged and final candidate arrays (19 bytes each, top_n
// per read; lists without a bound are priced at 32 candidates plus the
// per-stage form's minimizer and hit arrays, about 24 bytes per base).
inline u64 batch_bytes(u64 reads, u64 bases, const mt_query_params &q) {
    const u64 per_cand = 19;
    const bool bounded = q.top_n >= 1 && q.top_n <= 4;
    const u64 cands = bounded ? q.top_n : 32;
    u64 b = 2 * bases + reads * (64 + 2 * per_cand * cands) + (1ull << 20);
    if (!bounded) b += 24 * bases;
    // both strands: the two-strand read set and its per-stage arrays
    if (q.strands == 2) b = 2 * b + 2 * bases + 24 * 2 * bases;
    return b;
}

// Copies n bases and reports whether each is A, C, G, T or N in either case.
#define MT_COPY_BASES_BODY                                                                                  \
    u8 bad = 0;                                                                                              \
    for (u64 i = 0; i < n; i++) {                                                                            \
        const u8 c = src[i];                                                                                 \
        const u8 u = c & 0xDF; /* upper case; no other byte maps onto these letters */                      \
        bad |= (u8)((u != 'A') & (u != 'C') & (u != 'G') & (u != 'T') & (u != 'N'));                        \
        dst[i] = c;                                                                                          \
    }                                                                                                        \
    return bad == 0;

__attribute__((target("avx2"))) static bool copy_bases_avx2(u8 *__restrict__ dst, const u8 *__restrict__ src,
                                                             u64 n) {
    MT_COPY_BASES_BODY
}
static bool copy_bases_plain(u8 *__restrict__ dst, const u8 *__restrict__ src, u64 n) { MT_COPY_BASES_BODY }
#undef MT_COPY_BASES_BODY

inline bool copy_bases(u8 *dst, const u8 *src, u64 n) {
    static const bool avx2 = __builtin_cpu_supports("avx2");
    return avx2 ? copy_bases_avx2(dst, src, n) : copy_bases_plain(dst, src, n);
}

}  // namespace serve
}  // namespace mt

using namespace mt::serve;
using mt::u16;
using mt::u32;
using mt::u64;
using mt::u8;

struct mt_server {
    const mt_index *ix = nullptr;
    mt_server_params p{};
    int device = 0;
    PinnedArena arena;
    hipStream_t ctl = nullptr;  // zeroes request counters at submit
    std::mutex mu;
    std::vector<hipEvent_t> free_events;  // guarded by mu
    std::condition_variable cv_work, cv_done;
    std::unordered_map<u64, std::unique_ptr<Request>> reqs;
    std::deque<Request *> queue;  // requests with reads not yet in a batch
    u64 next_id = 1;
    u64 inflight = 0;             // estimated device bytes of the batches in flight
    u32 running = 0;              // batches in flight
    mt_server_counters stats{};   // guarded by mu
    hipEvent_t ref_ev = nullptr;  // recorded on the control stream at creation: the time origin
    std::vector<std::pair<float, float>> spans;  // device time of every batch's kernels (ms); guarded by mu
    bool stopping = false;
    std::vector<std::thread> workers;

    // Takes reads from the queue into b (lock held).  False if nothing can be
    // admitted now.
    bool form_batch(Batch &b) {
        if (queue.empty()) return false;
        bool limited = false;
        const u64 budget = p.mem_budget_bytes;
        const u64 avail = budget > inflight ? budget - inflight : 0;
        b.q = queue.front()->q;
        for (auto it = queue.begin(); it != queue.end();) {
            if (b.reads >= p.max_batch_reads || b.slices.size() >= MAX_SLOTS) break;
            Request *r = *it;
            if (!same_query(r->q, b.q)) {
                ++it;
                continue;
            }
            const u64 r0 = r->next;
            u64 hi = std::min(p.max_batch_reads - b.reads, r->n - r0), lo = 0;
            auto fits = [&](u64 take) {
                return batch_bytes(b.reads + take, b.bases + (r->off[r0 + take] - r->off[r0]), b.q) <= avail;
            };
            if (!fits(hi)) {  // largest number of reads that fits the budget
                limited = true;
                while (hi - lo > 1) {
                    const u64 mid = lo + (hi - lo) / 2;
                    if (fits(mid)) lo = mid; else hi = mid;
                }
                hi = lo;
            }
            if (hi == 0) {
                // Nothing more fits.  With no batch in flight, one read is
                // taken anyway so that every request makes progress.
                if (!b.slices.empty() || inflight != 0) break;
                hi = 1;
            }
            b.slices.push_back(Slice{r, r0, hi, b.reads});
            b.reads += hi;
            b.bases += r->off[r0 + hi] - r->off[r0];
            r->next += hi;
            r->open++;
            if (r->next < r->n) break;  // the batch is full
            it = queue.erase(it);
        }
        if (limited) stats.budget_limited++;
        if (b.slices.empty()) return false;
        b.est = batch_bytes(b.reads, b.bases, b.q);
        inflight += b.est;
        running++;
        stats.batches++;
        stats.reads += b.reads;
        stats.peak_inflight_bytes = std::max<u64>(stats.peak_inflight_bytes, inflight);
        stats.peak_batches = std::max<u32>(stats.peak_batches, running);
        return true;
    }

    void run_batch(Batch &b, hipStream_t s, Pinned &h_in, Pinned &h_out, std::vector<Piece> &pieces,
                   hipEvent_t ev_a, hipEvent_t ev_b);
    void worker();
    // Completes a request whose reads are all classified; counts = its taxon
    // counts already on the host (2 * n_taxa + 1 values; unused on error).
    void finish(Request *r, const u64 *counts);
};

void mt_server::run_batch(Batch &b, hipStream_t s, Pinned &h_in, Pinned &h_out, std::vector<Piece> &pieces,
                          hipEvent_t ev_a, hipEvent_t ev_b) {
    using namespace mt;
    const u64 n = b.reads;
    const u32 ns = (u32)b.slices.size();
    CallScope scope(s);
    // Host side of the batch: read offsets, slot offsets, counter pointers.
    const u64 in_bytes = (n + 1) * 8 + (ns + 1) * 8 + ns * 8;
    h_in.ensure(in_bytes);
    u64 *h_off = (u64 *)h_in.p;
    u64 *h_slot = h_off + n + 1;
    unsigned long long **h_cnt = (unsigned long long **)(h_slot + ns + 1);
    DBuf<u8> d_seq(b.bases);
    DBuf<u64> d_in(in_bytes / 8);
    u64 base = 0;
    h_off[0] = 0;
    for (u32 i = 0; i < ns; i++) {
        const Slice &sl = b.slices[i];
        const u64 *ro = sl.req->off + sl.r0;
        for (u64 j = 0; j < sl.len; j++) h_off[sl.b0 + j + 1] = base + (ro[j + 1] - ro[0]);
        const u64 bytes = ro[sl.len] - ro[0];
        if (bytes)
            MT_HIP(hipMemcpyAsync(d_seq.p + base, sl.req->seq + ro[0], bytes, hipMemcpyHostToDevice, s));
        base += bytes;
        h_slot[i] = sl.b0;
        h_cnt[i] = sl.req->counts;
    }
    h_slot[ns] = n;
    MT_HIP(hipMemcpyAsync(d_in.p, h_in.p, in_bytes, hipMemcpyHostToDevice, s));
    const u64 *d_off = d_in.p;
    const u64 *d_slot = d_in.p + n + 1;
    unsigned long long *const *d_cnt = (unsigned long long *const *)(d_in.p + n + 1 + ns + 1);

    mt_seqs seqs{(const char *)d_seq.p, d_off, n, b.bases};
    if (ev_a) MT_HIP(hipEventRecord(ev_a, s));  // the batch's kernels start after its upload
    mt_query_params q = b.q;
    q.mode = MT_MODE_FUSED;
    mt_result res;
    ReadBatch rb;
    Timer tm;
    tm.stream = s;
    mt_result_init(res, n, ix->n_taxa, s);
    classify_fused(*ix, q, seqs, rb, res, tm, s, false);
    const u64 nc = res.n_cands;
    for (u32 i = 0; i < ns; i++) MT_HIP(hipStreamWaitEvent(s, b.slices[i].req->zeroed, 0));
    launch_reduce_slots(res, *ix, d_slot, ns, d_cnt, s);
    if (ev_b) MT_HIP(hipEventRecord(ev_b, s));  // ... and end before its download

    // Outputs back to the host in one pinned block.
    const bool with_strand = res.strand.p != nullptr;
    const u64 out_bytes = (n + 1) * 8 + nc * (8 + 4 + 4 + 2 + 1 + 1) + n * (2 + 1) + 64;
    h_out.ensure(out_bytes);
    u8 *o = h_out.p;
    u64 *co = (u64 *)o;
    i64 *dg = (i64 *)(co + n + 1);
    u32 *gn = (u32 *)(dg + nc);
    u32 *ht = gn + nc;
    u16 *ap = (u16 *)(ht + nc);
    u16 *re = ap + nc;
    u8 *ac = (u8 *)(re + n);
    u8 *ra = ac + nc;
    u8 *sd = ra + n;
    MT_HIP(hipMemcpyAsync(co, res.cand_off.p, (n + 1) * 8, hipMemcpyDeviceToHost, s));
    if (nc) {
        MT_HIP(hipMemcpyAsync(dg, res.diag.p, nc * 8, hipMemcpyDeviceToHost, s));
        MT_HIP(hipMemcpyAsync(gn, res.genome.p, nc * 4, hipMemcpyDeviceToHost, s));
        MT_HIP(hipMemcpyAsync(ht, res.hits.p, nc * 4, hipMemcpyDeviceToHost, s));
        MT_HIP(hipMemcpyAsync(ap, res.approx.p, nc * 2, hipMemcpyDeviceToHost, s));
        MT_HIP(hipMemcpyAsync(ac, res.accept.p, nc, hipMemcpyDeviceToHost, s));
        if (with_strand) MT_HIP(hipMemcpyAsync(sd, res.strand.p, nc, hipMemcpyDeviceToHost, s));
    }
    MT_HIP(hipMemcpyAsync(re, res.read_E.p, n * 2, hipMemcpyDeviceToHost, s));
    MT_HIP(hipMemcpyAsync(ra, res.read_accepted.p, n, hipMemcpyDeviceToHost, s));
    MT_HIP(hipStreamSynchronize(s));
    if (ev_a && ev_b && ref_ev) {
        float t0 = 0, t1 = 0;
        if (hipEventElapsedTime(&t0, ref_ev, ev_a) == hipSuccess && hipEventElapsedTime(&t1, ref_ev, ev_b) == hipSuccess) {
            std::lock_guard<std::mutex> lk(mu);
            if (spans.size() < (1u << 20)) spans.emplace_back(t0, t1);
        } else {
            (void)hipGetLastError();
        }
    }

    pieces.resize(ns);
    for (u32 i = 0; i < ns; i++) {
        const Slice &sl = b.slices[i];
        Piece &pc = pieces[i];
        pc.len = sl.len;
        const u64 c0 = co[sl.b0], c1 = co[sl.b0 + sl.len];
        pc.cand_off.resize(sl.len + 1);
        for (u64 j = 0; j <= sl.len; j++) pc.cand_off[j] = co[sl.b0 + j] - c0;
        pc.read_accepted.assign(ra + sl.b0, ra + sl.b0 + sl.len);
        pc.read_E.assign(re + sl.b0, re + sl.b0 + sl.len);
        pc.genome.assign(gn + c0, gn + c1);
        pc.diag.assign(dg + c0, dg + c1);
        pc.hits.assign(ht + c0, ht + c1);
        pc.approx.assign(ap + c0, ap + c1);
        pc.accept.assign(ac + c0, ac + c1);
        if (with_strand) pc.strand.assign(sd + c0, sd + c1);
    }
}

// Completes a request whose reads are all classified (lock not held; no
// other thread touches the request until done is set).
void mt_server::finish(Request *r, const u64 *counts) {
    using namespace mt;
    std::unique_ptr<mt_result> res;
    if (r->status == MT_OK) {
        try {
            res.reset(new mt_result());
            res->on_host = true;
            res->n_reads = r->n;
            res->n_taxa = ix->n_taxa;
            res->submit_ns = r->submit_ns;
            auto &h = res->h;
            h.counts.assign(counts, counts + 2 * (u64)ix->n_taxa + 1);
            u64 nc = 0;
            for (auto &kv : r->pieces) nc += kv.second.genome.size();
            res->n_cands = nc;
            if (r->pieces.size() == 1) {
                Piece &pc = r->pieces.begin()->second;
                h.cand_off = std::move(pc.cand_off);
                h.read_accepted = std::move(pc.read_accepted);
                h.read_E = std::move(pc.read_E);
                h.genome = std::move(pc.genome);
                h.diag = std::move(pc.diag);
                h.hits = std::move(pc.hits);
                h.approx = std::move(pc.approx);
                h.accept = std::move(pc.accept);
                h.strand = std::move(pc.strand);
            } else {
                h.cand_off.reserve(r->n + 1);
                h.cand_off.push_back(0);
                for (auto &kv : r->pieces) {
                    Piece &pc = kv.second;
                    const u64 base = h.cand_off.back();
                    for (u64 j = 1; j <= pc.len; j++) h.cand_off.push_back(base + pc.cand_off[j]);
                    h.read_accepted.insert(h.read_accepted.end(), pc.read_accepted.begin(), pc.read_accepted.end());
                    h.read_E.insert(h.read_E.end(), pc.read_E.begin(), pc.read_E.end());
                    h.genome.insert(h.genome.end(), pc.genome.begin(), pc.genome.end());
                    h.diag.insert(h.diag.end(), pc.diag.begin(), pc.diag.end());
                    h.hits.insert(h.hits.end(), pc.hits.begin(), pc.hits.end());
                    h.approx.insert(h.approx.end(), pc.approx.begin(), pc.approx.end());
                    h.accept.insert(h.accept.end(), pc.accept.begin(), pc.accept.end());
                    h.strand.insert(h.strand.end(), pc.strand.begin(), pc.strand.end());
                }
            }
            if (h.cand_off.size() != r->n + 1) throw Error(MT_EINTERNAL, "served pieces do not cover the request");
        } catch (const Error &e) {
            r->status = e.status;
            r->error = e.what();
            res.reset();
        } catch (const std::bad_alloc &) {
            r->status = MT_ENOMEM;
            r->error = "host allocation failed";
            res.reset();
        }
    }
    r->pieces.clear();
    if (r->counts) {
        // the zero fill is long done unless a batch failed before waiting on it
        if (r->zeroed) (void)hipEventSynchronize(r->zeroed);
        pool_free(r->counts);
    }
    r->counts = nullptr;
    std::lock_guard<std::mutex> lk(mu);
    if (r->zeroed) free_events.push_back(r->zeroed);
    r->zeroed = nullptr;
    arena.release(r->arena_off, r->arena_bytes);
    if (res) res->done_ns = now_ns();
    r->result = std::move(res);
    r->done = true;
    cv_done.notify_all();
    cv_work.notify_all();  // arena space freed
}

void mt_server::worker() {
    using namespace mt;
    hipStream_t s = nullptr;
    std::string setup_error;
    if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        setup_error = "worker stream creation failed";
        s = nullptr;
    }
    Pinned h_in, h_out, h_cnt;
    hipEvent_t ev_a = nullptr, ev_b = nullptr;  // device timestamps around each batch's kernels
    if (s && (hipEventCreate(&ev_a) != hipSuccess || hipEventCreate(&ev_b) != hipSuccess)) {
        (void)hipGetLastError();
        if (ev_a) (void)hipEventDestroy(ev_a);
        ev_a = ev_b = nullptr;
    }
    for (;;) {
        Batch b;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                if (form_batch(b)) break;
                if (stopping && queue.empty()) goto out;
                cv_work.wait(lk);
            }
        }
        std::vector<Piece> pieces;
        int status = MT_OK;
        std::string error;
        try {
            if (!s) throw Error(MT_EDEVICE, setup_error);
            run_batch(b, s, h_in, h_out, pieces, ev_a, ev_b);
        } catch (const Error &e) {
            status = e.status;
            error = e.what();
        } catch (const std::bad_alloc &) {
            status = MT_ENOMEM;
            error = "host allocation failed";
        } catch (const std::exception &e) {
            status = MT_EINTERNAL;
            error = e.what();
        }
        std::vector<Request *> closed;
        {
            std::lock_guard<std::mutex> lk(mu);
            inflight -= b.est;
            running--;
            for (size_t i = 0; i < b.slices.size(); i++) {
                Request *r = b.slices[i].req;
                if (status != MT_OK && r->status == MT_OK) {
                    r->status = status;
                    r->error = error;
                    if (r->next < r->n) {  // stop batching the rest of it
                        r->next = r->n;
                        queue.erase(std::remove(queue.begin(), queue.end(), r), queue.end());
                    }
                }
                if (status == MT_OK && r->status == MT_OK) r->pieces[b.slices[i].r0] = std::move(pieces[i]);
                if (--r->open == 0 && r->next == r->n) closed.push_back(r);
            }
        }
        cv_work.notify_all();
        // the closed requests' counters: one pinned download and one wait
        const u64 nt = 2 * (u64)ix->n_taxa + 1;
        bool got = false;
        if (!closed.empty() && s) {
            try {
                h_cnt.ensure(closed.size() * nt * 8);
                for (size_t i = 0; i < closed.size(); i++)
                    if (closed[i]->status == MT_OK)
                        MT_HIP(hipMemcpyAsync(h_cnt.p + i * nt * 8, closed[i]->counts, nt * 8, hipMemcpyDeviceToHost,
                                              s));
                MT_HIP(hipStreamSynchronize(s));
                got = true;
            } catch (const Error &e) {
                for (Request *r : closed)
                    if (r->status == MT_OK) {
                        r->status = e.status;
                        r->error = e.what();
                    }
            }
        }
        for (size_t i = 0; i < closed.size(); i++)
            finish(closed[i], got ? (const u64 *)(h_cnt.p + i * nt * 8) : nullptr);
    }
out:
    if (ev_a) (void)hipEventDestroy(ev_a);
    if (ev_b) (void)hipEventDestroy(ev_b);
    if (s) (void)hipStreamDestroy(s);
}

// ---------------------------------------------------------------------- ABI --

extern "C" int mt_server_stats(mt_server *server, mt_server_counters *out) {
    if (!server || !out) {
        mt::set_last_error("mt_server_stats: null argument");
        return MT_EINVAL;
    }
    std::vector<std::pair<float, float>> sp;
    {
        std::lock_guard<std::mutex> lk(server->mu);
        *out = server->stats;
        out->mem_budget_bytes = server->p.mem_budget_bytes;
        out->max_batch_reads = server->p.max_batch_reads;
        sp = server->spans;
    }
    // device time of the batches' kernels: their sum, their union, and the
    // time during which two or more batches' kernels were running at once
    std::vector<std::pair<float, int>> ev;
    double sum = 0;
    for (auto &x : sp) {
        if (x.second < x.first) continue;
        sum += x.second - x.first;
        ev.emplace_back(x.first, 1);
        ev.emplace_back(x.second, -1);
    }
    std::sort(ev.begin(), ev.end(), [](const std::pair<float, int> &a, const std::pair<float, int> &b) {
        return a.first < b.first || (a.first == b.first && a.second < b.second);
    });
    double uni = 0, ovl = 0;
    int depth = 0;
    for (size_t i = 0; i < ev.size(); i++) {
        if (i > 0) {
            const double dt = ev[i].first - ev[i - 1].first;
            if (depth >= 1) uni += dt;
            if (depth >= 2) ovl += dt;
        }
        depth += ev[i].second;
    }
    out->timed_batches = sp.size();
    out->kernel_ms_sum = sum;
    out->kernel_ms_union = uni;
    out->kernel_ms_overlap = ovl;
    return MT_OK;
}

extern "C" int mt_server_create(const mt_index *index, const mt_server_params *params, mt_server **out) {
    if (!index || !out) {
        mt::set_last_error("mt_server_create: null argument");
        return MT_EINVAL;
    }
    *out = nullptr;
    std::unique_ptr<mt_server> sv;
    int rc = mt::guarded("mt_server_create", [&] {
        mt_server_params p{};
        if (params) p = *params;
        MT_REQUIRE(p.reserved[0] == 0 && p.reserved[1] == 0 && p.reserved[2] == 0 && p.reserved[3] == 0,
                   "reserved fields must be 0");
        if (!p.mem_budget_bytes) {
            size_t free_b = 0, total_b = 0;
            MT_HIP(hipMemGetInfo(&free_b, &total_b));
            p.mem_budget_bytes = std::max<u64>(free_b / 4, 256ull << 20);
        }
        if (!p.max_batch_reads) p.max_batch_reads = 1ull << 18;
        if (!p.n_streams) p.n_streams = 4;
        if (!p.max_queued_requests) p.max_queued_requests = 4096;
        if (!p.pinned_arena_bytes) p.pinned_arena_bytes = 1ull << 30;
        MT_REQUIRE(p.n_streams <= 16, "n_streams must be at most 16");
        sv.reset(new mt_server());
        sv->ix = index;
        sv->p = p;
        MT_HIP(hipGetDevice(&sv->device));
        sv->arena.init(p.pinned_arena_bytes);
        MT_HIP(hipStreamCreateWithFlags(&sv->ctl, hipStreamNonBlocking));
        MT_HIP(hipEventCreate(&sv->ref_ev));
        MT_HIP(hipEventRecord(sv->ref_ev, sv->ctl));
        for (u32 i = 0; i < p.n_streams; i++) sv->workers.emplace_back([s = sv.get()] { s->worker(); });
    });
    if (rc != MT_OK) {
        if (sv) {
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                sv->stopping = true;
            }
            sv->cv_work.notify_all();
            for (auto &t : sv->workers) t.join();
            if (sv->ref_ev) (void)hipEventDestroy(sv->ref_ev);
            if (sv->ctl) (void)hipStreamDestroy(sv->ctl);
        }
        return rc;
    }
    *out = sv.release();
    return MT_OK;
}

extern "C" int mt_server_submit(mt_server *sv, const mt_query_params *params, const char *seq,
                                const uint64_t *offsets, uint64_t n, uint64_t *request_id) {
    using namespace mt;
    if (!sv || !params || !offsets || !request_id || (n && !seq && offsets[n] != 0)) {
        set_last_error("mt_server_submit: null argument");
        return MT_EINVAL;
    }
    return guarded("mt_server_submit", [&] {
        mt_query_params q = *params;
        q.mode = MT_MODE_FUSED;
        validate_query(q);
        MT_REQUIRE(offsets[0] == 0, "offsets[0] must be 0");
        u64 max_len = 0;
        for (u64 i = 0; i < n; i++) {
            MT_REQUIRE(offsets[i + 1] >= offsets[i], "offsets must never decrease");
            max_len = std::max<u64>(max_len, offsets[i + 1] - offsets[i]);
        }
        MT_REQUIRE(max_len <= 65535, "read longer than 65535 bases");
        if (q.e_mode != MT_E_FIXED)
            MT_REQUIRE((max_len * q.e_value + 999) / 1000 <= 65534, "edit threshold E above 65534");
        const u64 total = offsets[n];
        const u64 off_bytes = (n + 1) * 8;
        const u64 bytes = off_bytes + total;
        std::unique_ptr<Request> r(new Request());
        r->q = q;
        r->n = n;
        r->bases = total;
        r->submit_ns = now_ns();
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            if (sv->stopping) throw Error(MT_ECANCELED, "server is shutting down");
            if (sv->reqs.size() >= sv->p.max_queued_requests) throw Error(MT_EAGAIN, "request queue is full");
            MT_REQUIRE(PinnedArena::granule(bytes) <= sv->arena.size(), "request larger than the pinned arena");
            r->arena_off = sv->arena.alloc(bytes);
            if (r->arena_off == ~0ull) throw Error(MT_EAGAIN, "pinned arena is full");
            r->arena_bytes = bytes;
        }
        auto give_back = [&] {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->arena.release(r->arena_off, r->arena_bytes);
        };
        u8 *dst = sv->arena.base() + r->arena_off;
        std::memcpy(dst, offsets, off_bytes);
        if (!copy_bases(dst + off_bytes, (const u8 *)seq, total)) {
            give_back();
            throw Error(MT_EINVAL, "sequence byte outside A, C, G, T, N (either case)");
        }
        r->off = (const u64 *)dst;
        r->seq = dst + off_bytes;
        const u64 nt = sv->ix->n_taxa;
        if (n) {  // zeroed asynchronously; workers wait for the event before adding
            try {
                {
                    std::lock_guard<std::mutex> lk(sv->mu);
                    if (!sv->free_events.empty()) {
                        r->zeroed = sv->free_events.back();
                        sv->free_events.pop_back();
                    }
                }
                if (!r->zeroed) MT_HIP(hipEventCreateWithFlags(&r->zeroed, hipEventDisableTiming));
                r->counts = (unsigned long long *)pool_alloc_on((2 * nt + 1) * 8, sv->ctl);
                MT_HIP(hipMemsetAsync(r->counts, 0, (2 * nt + 1) * 8, sv->ctl));
                MT_HIP(hipEventRecord(r->zeroed, sv->ctl));
            } catch (...) {
                if (r->counts) pool_free(r->counts);
                if (r->zeroed) (void)hipEventDestroy(r->zeroed);
                give_back();
                throw;
            }
        }
        Request *rp = r.get();
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            rp->id = sv->next_id++;
            *request_id = rp->id;
            sv->reqs.emplace(rp->id, std::move(r));
            if (n) sv->queue.push_back(rp);
        }
        if (n == 0) {
            const std::vector<u64> zeros(2 * nt + 1, 0);
            sv->finish(rp, zeros.data());  // nothing to classify
        } else {
            sv->cv_work.notify_one();
        }
    });
}

extern "C" int mt_server_wait(mt_server *sv, uint64_t request_id, int64_t timeout_us, mt_result **out) {
    if (!sv || !out) {
        mt::set_last_error("mt_server_wait: null argument");
        return MT_EINVAL;
    }
    *out = nullptr;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(request_id);
    if (it == sv->reqs.end() || it->second->waiting) {
        mt::set_last_error("mt_server_wait: unknown request id (or already waited for)");
        return MT_EINVAL;
    }
    Request *r = it->second.get();
    r->waiting = true;
    auto ready = [&] { return r->done; };
    if (timeout_us < 0)
        sv->cv_done.wait(lk, ready);
    else
        sv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
    if (!r->done) {
        r->waiting = false;
        mt::set_last_error("mt_server_wait: timed out");
        return MT_ETIMEDOUT;
    }
    const int status = r->status;
    const std::string error = r->error;
    *out = r->result.release();
    sv->reqs.erase(it);
    lk.unlock();
    sv->cv_work.notify_all();
    mt::set_last_error(status == MT_OK ? "" : "mt_server_wait: " + error);
    return status;
}

extern "C" int mt_server_destroy(mt_server *sv) {
    if (!sv) return MT_OK;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stopping = true;
    }
    sv->cv_work.notify_all();
    for (auto &t : sv->workers) t.join();
    for (auto &kv : sv->reqs) {
        if (kv.second->counts) mt::pool_free(kv.second->counts);
        if (kv.second->zeroed) (void)hipEventDestroy(kv.second->zeroed);
    }
    sv->reqs.clear();
    for (hipEvent_t e : sv->free_events) (void)hipEventDestroy(e);
    if (sv->ref_ev) (void)hipEventDestroy(sv->ref_ev);
    if (sv->ctl) (void)hipStreamDestroy(sv->ctl);
    delete sv;
    return MT_OK;
}
