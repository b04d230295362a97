// HBM bandwidth probes, run in the same process as the benchmark to give
// the achievable bandwidth beside the published peak: a read-only sweep
// (16-byte loads, one partial per workgroup so nothing is optimised away)
// and a copy (16-byte loads and stores).
#include "internal.h"

namespace stag {

constexpr int kProbeBlock = 256;

__global__ void __launch_bounds__(kProbeBlock) k_probe_read(const float4 *src, int64_t n, float *out) {
    float acc = 0.f;
    for (int64_t j = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kProbeBlock) {
        const float4 v = src[j];
        acc += (v.x + v.y) + (v.z + v.w);
    }
    if (acc == 1.2345f) out[blockIdx.x * kProbeBlock + threadIdx.x] = acc;  // never true for the probe's data
}

__global__ void __launch_bounds__(kProbeBlock) k_probe_copy(const float4 *src, float4 *dst, int64_t n) {
    for (int64_t j = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kProbeBlock)
        dst[j] = src[j];
}

}  // namespace stag

using namespace stag;

extern "C" stag_status stag_hbm_probe(const void *src, void *dst, int64_t bytes, int kind, void *stream) {
    if (!src || !dst || bytes < 16 || (bytes & 15)) return invalid("probe needs two buffers and a size that is a multiple of 16");
    if (kind != 0 && kind != 1) return invalid("probe kind must be 0 (read) or 1 (copy)");
    const int64_t n = bytes / 16;
    const int grid = 8192;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (kind == 0)
        hipLaunchKernelGGL(k_probe_read, dim3(grid), dim3(kProbeBlock), 0, s, static_cast<const float4 *>(src), n,
                           static_cast<float *>(dst));
    else
        hipLaunchKernelGGL(k_probe_copy, dim3(grid), dim3(kProbeBlock), 0, s, static_cast<const float4 *>(src),
                           static_cast<float4 *>(dst), n);
    STAG_HIP(hipGetLastError());
    return STAG_OK;
}
