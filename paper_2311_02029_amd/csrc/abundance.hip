// Relative abundance (Fig. 1 step 3b): every taxon's share of the mapped
// reads, multi-mapped reads split in proportion to the unique-read counts of
// their taxa, taxa below the cutoff (0.01% in the paper) dropped and the rest
// renormalised.  The paper takes the apportionment from Metalign without
// stating it; the rule here is one proportional step from the unique evidence:
//
//   count_t = 2^32 * u_t + sum over multi-mapped reads r with t in T(r) of
//             floor(2^32 * u_t / U_r), U_r = sum of u over T(r)
//             (floor(2^32 / |T(r)|) when U_r = 0),
//
// in units of 2^-32 read, so that the counts are exact integers whatever the
// order of the atomic additions; keep t iff count_t * den >= total * num;
// abundance_t = count_t / (sum of kept counts), correctly rounded doubles.
#include "classify.hpp"

namespace mt {

constexpr int AB_TPB = 256;
constexpr u32 AB_LDS_TAXA = 4096;  // taxa counted per block in LDS (64-bit, 32 KB)
constexpr u64 AB_ONE = 1ull << 32;

// The mapped taxa of read r (Fig. 1 step 3a: accepted candidates at the
// smallest value, distinct taxa) and its additions to the counts.
template <class Add>
__device__ inline void abundance_read(u64 cs, u64 ce, const u32 *__restrict__ genome, const u16 *__restrict__ approx,
                                      const u8 *__restrict__ accept, const u32 *__restrict__ taxon,
                                      const u64 *__restrict__ uniq, const Add &add) {
    u32 best = 0xFFFFFFFFu;
    for (u64 c = cs; c < ce; c++)
        if (accept[c] && approx[c] < best) best = approx[c];
    if (best == 0xFFFFFFFFu) return;
    auto first_of_taxon = [&](u64 c, u32 t) {
        for (u64 d = cs; d < c; d++)
            if (accept[d] && approx[d] == best && taxon[genome[d]] == t) return false;
        return true;
    };
    u32 nt = 0, only = 0;
    u64 U = 0;
    for (u64 c = cs; c < ce; c++) {
        if (!accept[c] || approx[c] != best) continue;
        const u32 t = taxon[genome[c]];
        if (!first_of_taxon(c, t)) continue;
        only = t;
        nt++;
        U += uniq[t];
    }
    if (nt == 1) {
        add(only, AB_ONE);
        return;
    }
    for (u64 c = cs; c < ce; c++) {
        if (!accept[c] || approx[c] != best) continue;
        const u32 t = taxon[genome[c]];
        if (!first_of_taxon(c, t)) continue;
        // u_t < 2^32 (reads per call < 2^31), so u_t * 2^32 fits 64 bits
        add(t, U ? (uniq[t] << 32) / U : AB_ONE / nt);
    }
}

// Grid-stride over the reads; up to AB_LDS_TAXA taxa each block adds in LDS
// and flushes its nonzero counters once at the end.
__global__ __launch_bounds__(AB_TPB) void k_abundance(const u64 *__restrict__ cand_off, u64 n,
                                                      const u32 *__restrict__ genome, const u16 *__restrict__ approx,
                                                      const u8 *__restrict__ accept, const u32 *__restrict__ taxon,
                                                      const u64 *__restrict__ uniq, u32 n_taxa,
                                                      unsigned long long *__restrict__ counts) {
    __shared__ unsigned long long cnt[AB_LDS_TAXA];
    const u64 stride = (u64)gridDim.x * AB_TPB;
    if (n_taxa > AB_LDS_TAXA) {
        auto add = [&](u32 t, u64 v) { atomicAdd(&counts[t], (unsigned long long)v); };
        for (u64 r = (u64)blockIdx.x * AB_TPB + threadIdx.x; r < n; r += stride)
            abundance_read(cand_off[r], cand_off[r + 1], genome, approx, accept, taxon, uniq, add);
        return;
    }
    for (u32 i = threadIdx.x; i < n_taxa; i += AB_TPB) cnt[i] = 0;
    __syncthreads();
    auto add = [&](u32 t, u64 v) { atomicAdd(&cnt[t], (unsigned long long)v); };
    for (u64 r = (u64)blockIdx.x * AB_TPB + threadIdx.x; r < n; r += stride)
        abundance_read(cand_off[r], cand_off[r + 1], genome, approx, accept, taxon, uniq, add);
    __syncthreads();
    for (u32 i = threadIdx.x; i < n_taxa; i += AB_TPB)
        if (cnt[i]) atomicAdd(&counts[i], cnt[i]);
}

constexpr int AF_TPB = 1024;

__device__ inline u64 block_sum(u64 v, u64 *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = AF_TPB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const u64 r = sh[0];
    __syncthreads();
    return r;
}

// a * b >= c * d on 128-bit products.
__device__ inline bool ge128(u64 a, u64 b, u64 c, u64 d) {
    const u64 lh = __umul64hi(a, b), ll = a * b, rh = __umul64hi(c, d), rl = c * d;
    return lh > rh || (lh == rh && ll >= rl);
}

// num / den as the nearest double, ties to even (0 <= num <= den, den > 0):
// the quotient's bits by long division (the remainder doubled with its carry
// out of 64 bits kept), 53 significant bits rounded with the next bit and
// whether a remainder is left.  Dividing the two converted doubles would
// round twice once den needs more than 53 bits.
__device__ inline double div_nearest(u64 num, u64 den) {
    if (num == 0) return 0.0;
    if (num >= den) return 1.0;
    int e = 0;  // num / den lies in [2^-e, 2^(1-e))
    u64 r = num;
    for (;;) {  // double r until it reaches den (a carry out of 64 bits means it has)
        const bool carry = (r >> 63) != 0;
        r <<= 1;
        e++;
        if (carry || r >= den) break;
    }
    r -= den;  // the true 2r - den is below den: the wrapped difference is exact
    u64 q = 1;
    for (int i = 1; i < 53; i++) {
        const bool carry = (r >> 63) != 0;
        r <<= 1;
        q <<= 1;
        if (carry || r >= den) {
            r -= den;  // the true 2r - den is below den: the wrapped difference is exact
            q |= 1;
        }
    }
    const bool carry = (r >> 63) != 0;
    r <<= 1;
    const bool half = carry || r >= den;
    if (half) r -= den;
    if (half && (r != 0 || (q & 1))) q++;
    return ldexp((double)q, -e - 52);
}

// One block: the total, the cutoff, the kept total, the abundances.
// out[0] = kept taxa.
__global__ __launch_bounds__(AF_TPB) void k_abundance_final(const u64 *__restrict__ counts, u32 n_taxa, u64 num,
                                                            u64 den, double *__restrict__ abund,
                                                            u64 *__restrict__ out) {
    __shared__ u64 sh[AF_TPB];
    u64 part = 0;
    for (u32 t = threadIdx.x; t < n_taxa; t += AF_TPB) part += counts[t];
    const u64 C = block_sum(part, sh);
    u64 kept = 0, K = 0;
    for (u32 t = threadIdx.x; t < n_taxa; t += AF_TPB)
        if (C && ge128(counts[t], den, C, num)) {
            kept++;
            K += counts[t];
        }
    kept = block_sum(kept, sh);
    K = block_sum(K, sh);
    for (u32 t = threadIdx.x; t < n_taxa; t += AF_TPB) {
        const bool keep = C && ge128(counts[t], den, C, num);
        abund[t] = keep ? div_nearest(counts[t], K) : 0.0;
    }
    if (threadIdx.x == 0) out[0] = kept;
}

}  // namespace mt

using namespace mt;

extern "C" int mt_abundance(const mt_index *index, const mt_result *res, uint64_t cutoff_num, uint64_t cutoff_den,
                            uint64_t *counts, double *abundance, uint64_t *n_kept, void *stream) {
    if (!index || !res || !n_kept || ((!counts || !abundance) && index->n_taxa)) {
        set_last_error("mt_abundance: null argument");
        return MT_EINVAL;
    }
    if (cutoff_den == 0) {
        set_last_error("mt_abundance: cutoff denominator must be nonzero");
        return MT_EINVAL;
    }
    if (res->n_taxa != index->n_taxa) {
        set_last_error("mt_abundance: the result was not made with this index (taxon counts differ)");
        return MT_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    return guarded("mt_abundance", [&] {
        *n_kept = 0;
        const u32 nt = index->n_taxa;
        if (nt == 0) return;
        CallScope scope(s);
        const u64 n = res->n_reads, nc = res->n_cands;
        // a served result lives in host memory: its arrays go up first
        DBuf<u64> h_off, h_uniq;
        DBuf<u32> h_genome;
        DBuf<u16> h_approx;
        DBuf<u8> h_accept;
        const u64 *off = res->cand_off.p, *uniq = res->uniq.p;
        const u32 *genome = res->genome.p;
        const u16 *approx = res->approx.p;
        const u8 *accept = res->accept.p;
        if (res->on_host) {
            h_off.alloc(n + 1);
            h_uniq.alloc(nt);
            h_genome.alloc(nc);
            h_approx.alloc(nc);
            h_accept.alloc(nc);
            MT_HIP(hipMemcpyAsync(h_off.p, res->h.cand_off.data(), (n + 1) * 8, hipMemcpyHostToDevice, s));
            MT_HIP(hipMemcpyAsync(h_uniq.p, res->h.counts.data(), (u64)nt * 8, hipMemcpyHostToDevice, s));
            if (nc) {
                MT_HIP(hipMemcpyAsync(h_genome.p, res->h.genome.data(), nc * 4, hipMemcpyHostToDevice, s));
                MT_HIP(hipMemcpyAsync(h_approx.p, res->h.approx.data(), nc * 2, hipMemcpyHostToDevice, s));
                MT_HIP(hipMemcpyAsync(h_accept.p, res->h.accept.data(), nc, hipMemcpyHostToDevice, s));
            }
            off = h_off.p;
            uniq = h_uniq.p;
            genome = h_genome.p;
            approx = h_approx.p;
            accept = h_accept.p;
        }
        MT_HIP(hipMemsetAsync(counts, 0, (u64)nt * 8, s));
        if (n) {
            int dev = 0, cus = 0;
            MT_HIP(hipGetDevice(&dev));
            MT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            const unsigned blocks = (unsigned)std::max<u64>(1, std::min<u64>(grid_for(n, AB_TPB),
                                                                             (u64)std::max(cus, 1) * 4));
            k_abundance<<<blocks, AB_TPB, 0, s>>>(off, n, genome, approx, accept, index->taxon.p, uniq, nt,
                                                  (unsigned long long *)counts);
            MT_HIP(hipGetLastError());
        }
        DBuf<u64> out(1);
        k_abundance_final<<<1, AF_TPB, 0, s>>>(counts, nt, cutoff_num, cutoff_den, abundance, out.p);
        MT_HIP(hipGetLastError());
        read_back(s, out.p, n_kept, sizeof(u64));
    });
}
