// Device-side helpers shared by the gfx950 kernels: complex arithmetic,
// team/wave/block reductions, the result record and numeric constants.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/curvealign.h"

namespace ca {

constexpr int kMaxN = CA_MAX_N;
constexpr int kCandCap = 32;           // FP64 re-scoring candidates per pair
constexpr double kNearTie = 1e-6;      // relative gap that counts as a near-tie
// Multiplier of u * log2(n) in the FP32 error bound of |C|:
//   |C32(s) - C(s)| <= kErrScale * u32 * log2(n) * n * sqrt(n1 n2)
// (the n sqrt(n1 n2) factor is the Cauchy-Schwarz bound on |C|).
constexpr double kErrScale = 2.0;

template <typename R> struct __attribute__((aligned(2 * sizeof(R)))) cpx { R x, y; };
using cf = cpx<float>;
using cd = cpx<double>;

template <typename R> __device__ __forceinline__ cpx<R> mk(R x, R y) { return cpx<R>{x, y}; }
template <typename R> __device__ __forceinline__ cpx<R> add(cpx<R> a, cpx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R> __device__ __forceinline__ cpx<R> sub(cpx<R> a, cpx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R> __device__ __forceinline__ cpx<R> mul(cpx<R> a, cpx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// conj(a) * b
template <typename R> __device__ __forceinline__ cpx<R> cjmul(cpx<R> a, cpx<R> b) {
    return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
template <typename R> __device__ __forceinline__ cpx<R> scale(cpx<R> a, R s) { return {a.x * s, a.y * s}; }
// -i * a
template <typename R> __device__ __forceinline__ cpx<R> mul_mi(cpx<R> a) { return {a.y, -a.x}; }
// +i * a
template <typename R> __device__ __forceinline__ cpx<R> mul_pi(cpx<R> a) { return {-a.y, a.x}; }
template <typename R> __device__ __forceinline__ R norm2(cpx<R> a) { return a.x * a.x + a.y * a.y; }

template <typename R> struct num;
template <> struct num<float> { static constexpr double u = 5.9604644775390625e-08; };   // 2^-24
template <> struct num<double> { static constexpr double u = 1.1102230246251565e-16; };  // 2^-53

// Result record, identical layout to ca_result_t.
static_assert(sizeof(ca_result_t) == 32, "ca_result_t must be 32 bytes");

// Ordering of the LDS accesses of one wave: the fences stop the compiler from
// moving LDS reads above LDS writes (and back); a wave's LDS operations are
// executed in issue order, so no hardware barrier is needed within a wave.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Argmax combine: larger value wins, the smaller index on equal values.
__device__ __forceinline__ void argmax_combine(float& v, int& i, float ov, int oi) {
    if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
}
__device__ __forceinline__ void argmax_combine(double& v, int& i, double ov, int oi) {
    if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
}

// Reductions across the W lanes of an aligned team (W a power of two <= 64).
template <int W, typename V> __device__ __forceinline__ V team_sum(V v) {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
    return v;
}
template <int W, typename V> __device__ __forceinline__ void team_argmax(V& v, int& i) {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) {
        V ov = __shfl_xor(v, o, W);
        int oi = __shfl_xor(i, o, W);
        argmax_combine(v, i, ov, oi);
    }
}

// Block-wide reductions for the one-pair-per-workgroup kernels.  `scratch`
// must hold 2 * (blockDim / 64) doubles; results are returned to every thread.
template <int NT> __device__ __forceinline__ double block_sum(double v, double* scratch) {
    v = team_sum<64>(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) scratch[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) s += scratch[k];
    return s;
}
template <int NT, typename V> __device__ __forceinline__ void block_argmax(V& v, int& i, double* scratch) {
    team_argmax<64>(v, i);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) { scratch[2 * w] = (double)v; scratch[2 * w + 1] = (double)i; }
    __syncthreads();
    V bv = (V)scratch[0];
    int bi = (int)scratch[1];
#pragma unroll
    for (int k = 1; k < NT / 64; ++k) argmax_combine(bv, bi, (V)scratch[2 * k], (int)scratch[2 * k + 1]);
    v = bv; i = bi;
}

__device__ __forceinline__ int ilog2_ceil(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

}  // namespace ca
