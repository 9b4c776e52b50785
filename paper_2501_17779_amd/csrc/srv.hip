// Square-root-velocity transform of section 3: q = beta' / |beta'|^(1/2) for
// the closed polygon through n nodes at t_k = k / n, piecewise constant on
// the segments: beta'_k = n (z[k+1] - z[k]), q_k = beta'_k |beta'_k|^(-1/2).
#include "common.hpp"
#include "launch.hpp"

namespace ca {

// One wave per curve, curves strided over a persistent grid.  Each lane
// reads its node and the next one (the second read hits the cache lines of
// the first), so HBM sees one read and one write per node.
__global__ __launch_bounds__(256) void k_srv(const cf* __restrict__ z, const int64_t* __restrict__ offsets,
                                             int n_uniform, int64_t count, cf* __restrict__ q) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t c = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); c < count; c += waves) {
        int64_t base;
        int64_t n;
        if (offsets) {
            base = offsets[c];
            n = offsets[c + 1] - base;
        } else {
            n = n_uniform;
            base = c * n;
        }
        const float fn = (float)n;
        for (int64_t k = lane; k < n; k += 64) {
            const cf a = z[base + k];
            const cf b = z[base + (k + 1 == n ? 0 : k + 1)];
            const float dx = fn * (b.x - a.x), dy = fn * (b.y - a.y);
            const float s = fmaf(dx, dx, dy * dy);
            // |d|^(-1/2) = rsqrt(sqrt(|d|^2)); a zero-length segment gives q = 0
            const float f = s > 0.0f ? __builtin_amdgcn_rsqf(sqrtf(s)) : 0.0f;
            q[base + k] = cf{dx * f, dy * f};
        }
    }
}

hipError_t launch_srv(const void* z, const int64_t* offsets, int n, int64_t count, void* q, int num_cus,
                      hipStream_t s) {
    int64_t blocks = (count + 3) / 4;
    const int64_t cap = (int64_t)num_cus * 8;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(k_srv, dim3((unsigned)blocks), dim3(256), 0, s, (const cf*)z, offsets, n, count, (cf*)q);
    return hipGetLastError();
}

}  // namespace ca
