// Hand-off to an elastic shape-distance solver (section 3): the rigid optimum
// in the paper's notation, t0* and R(theta_p) of section 2.
#include "common.hpp"
#include "launch.hpp"

namespace ca {

__global__ __launch_bounds__(256) void k_to_initializer(const ca_result_t* __restrict__ res, int n_uniform,
                                                        const int64_t* __restrict__ offsets, int64_t count,
                                                        double* __restrict__ t0, double* __restrict__ rot) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const ca_result_t r = res[i];
    const int64_t n = offsets ? offsets[i + 1] - offsets[i] : n_uniform;
    // start index m = (n - s) mod n; curve 2 is read from t0 = m / n on
    int64_t m = 0;
    if (n > 0) {
        m = (n - (int64_t)r.shift) % n;
        if (m < 0) m += n;
    }
    t0[i] = n > 0 ? (double)m / (double)n : 0.0;
    // theta_p = -theta: R(theta_p) = [[cos, -sin theta], [sin theta, cos]]
    double sn, cs;
    sincos(r.theta, &sn, &cs);
    double* R = rot + 4 * i;
    R[0] = cs;
    R[1] = -sn;
    R[2] = sn;
    R[3] = cs;
}

hipError_t launch_initializer(const ca_result_t* res, int n, const int64_t* offsets, int64_t count,
                              double* t0, double* rot, hipStream_t s) {
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(k_to_initializer, dim3((unsigned)blocks), dim3(256), 0, s, res, n, offsets, count, t0,
                       rot);
    return hipGetLastError();
}

}  // namespace ca
