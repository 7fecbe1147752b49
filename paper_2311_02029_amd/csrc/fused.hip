// Fused seed-count + filter path (placeholder until the fused kernel lands).
#include "classify.hpp"

namespace mt {

__global__ void k_max_u16(const u16 *__restrict__ v, u64 n, u32 *__restrict__ out) {
    u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicMax(out, (u32)v[i]);
}

void launch_max_u16(const u16 *v, u64 n, u32 *out, hipStream_t s) {
    k_max_u16<<<grid_for(n, 256), 256, 0, s>>>(v, n, out);
    MT_HIP(hipGetLastError());
}

void classify_fused(const mt_index &, const mt_query_params &, const mt_seqs &, ReadBatch &, mt_result &, Timer &,
                    hipStream_t) {
    throw Error(MT_EINVAL, "fused mode is not available in this build");
}

}  // namespace mt
