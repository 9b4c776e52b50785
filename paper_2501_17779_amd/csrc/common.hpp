// Device-side helpers shared by the gfx950 kernels: complex arithmetic,
// team/wave/block reductions, the result record and numeric constants.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/curvealign.h"

namespace ca {

constexpr int kMaxN = CA_MAX_N;
constexpr int kMaxM = 2 * CA_MAX_N;   // largest transform size (zero-padded correlation)
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

// Cross-lane moves.  Inside a row of 16 lanes the data-parallel-primitive
// (DPP) forms exchange at VALU latency: quad_perm [1,0,3,2] and [2,3,0,1]
// pair lanes i ^ 1 and i ^ 2, row_half_mirror pairs i with 7 - i inside each
// group of 8, row_mirror pairs i with 15 - i.  After the quad steps every
// lane of a quad holds the quad result, so the mirror steps complete groups
// of 8 and 16.  Rows are then combined through v_readlane of lanes 0, 16,
// 32, 48 (wave-uniform values).  Every lane of a team ends with the same
// value, computed in the same order.
enum { kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140 };

template <int CTRL> __device__ __forceinline__ int dpp32(int x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
template <int CTRL> __device__ __forceinline__ float dpp(float x) {
    return __int_as_float(dpp32<CTRL>(__float_as_int(x)));
}
template <int CTRL> __device__ __forceinline__ int dpp(int x) { return dpp32<CTRL>(x); }
template <int CTRL> __device__ __forceinline__ double dpp(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = dpp32<CTRL>((int)(b & 0xffffffffll));
    const int hi = dpp32<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float rdlane(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ int rdlane(int x, int l) { return __builtin_amdgcn_readlane(x, l); }
__device__ __forceinline__ double rdlane(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Reductions across the W lanes of an aligned team (W a power of two <= 64)
// with a commutative operation.
template <int W, typename V, typename Op> __device__ __forceinline__ V team_reduce(V v, Op op) {
    if constexpr (W >= 2) v = op(v, dpp<kDppXor1>(v));
    if constexpr (W >= 4) v = op(v, dpp<kDppXor2>(v));
    if constexpr (W >= 8) v = op(v, dpp<kDppHalfMirror>(v));
    if constexpr (W >= 16) v = op(v, dpp<kDppMirror>(v));
    if constexpr (W == 32) {
        const V a = op(rdlane(v, 0), rdlane(v, 16)), b = op(rdlane(v, 32), rdlane(v, 48));
        v = (threadIdx.x & 32) ? b : a;
    } else if constexpr (W == 64) {
        v = op(op(rdlane(v, 0), rdlane(v, 16)), op(rdlane(v, 32), rdlane(v, 48)));
    }
    return v;
}
template <int W, typename V> __device__ __forceinline__ V team_sum(V v) {
    return team_reduce<W>(v, [](V a, V b) { return a + b; });
}
template <int W> __device__ __forceinline__ float team_max(float v) {
    return team_reduce<W>(v, [](float a, float b) { return fmaxf(a, b); });
}
template <int W> __device__ __forceinline__ int team_max(int v) {
    return team_reduce<W>(v, [](int a, int b) { return max(a, b); });
}
template <int W> __device__ __forceinline__ int team_min(int v) {
    return team_reduce<W>(v, [](int a, int b) { return min(a, b); });
}
template <int W, typename V> __device__ __forceinline__ void team_argmax(V& v, int& i) {
    auto step = [&](V ov, int oi) { argmax_combine(v, i, ov, oi); };
    if constexpr (W >= 2) step(dpp<kDppXor1>(v), dpp<kDppXor1>(i));
    if constexpr (W >= 4) step(dpp<kDppXor2>(v), dpp<kDppXor2>(i));
    if constexpr (W >= 8) step(dpp<kDppHalfMirror>(v), dpp<kDppHalfMirror>(i));
    if constexpr (W >= 16) step(dpp<kDppMirror>(v), dpp<kDppMirror>(i));
    if constexpr (W >= 32) {
        V a = rdlane(v, 0), b = rdlane(v, 32);
        int ia = rdlane(i, 0), ib = rdlane(i, 32);
        argmax_combine(a, ia, rdlane(v, 16), rdlane(i, 16));
        argmax_combine(b, ib, rdlane(v, 48), rdlane(i, 48));
        if constexpr (W == 64) {
            argmax_combine(a, ia, b, ib);
            v = a;
            i = ia;
        } else {
            const bool hi = (threadIdx.x & 32) != 0;
            v = hi ? b : a;
            i = hi ? ib : ia;
        }
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
// Two sums at once (one pair of barriers); scratch holds 2 * (blockDim / 64) doubles.
template <int NT> __device__ __forceinline__ void block_sum2(double& a, double& b, double* scratch) {
    a = team_sum<64>(a);
    b = team_sum<64>(b);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) { scratch[2 * w] = a; scratch[2 * w + 1] = b; }
    __syncthreads();
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) { sa += scratch[2 * k]; sb += scratch[2 * k + 1]; }
    a = sa;
    b = sb;
}
// Four sums at once (one pair of barriers); scratch holds 4 * (blockDim / 64) doubles.
template <int NT> __device__ __forceinline__ void block_sum4(double& a, double& b, double& c, double& d,
                                                            double* scratch) {
    a = team_sum<64>(a);
    b = team_sum<64>(b);
    c = team_sum<64>(c);
    d = team_sum<64>(d);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        scratch[4 * w] = a;
        scratch[4 * w + 1] = b;
        scratch[4 * w + 2] = c;
        scratch[4 * w + 3] = d;
    }
    __syncthreads();
    double sa = 0.0, sb = 0.0, sc = 0.0, sd = 0.0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) {
        sa += scratch[4 * k];
        sb += scratch[4 * k + 1];
        sc += scratch[4 * k + 2];
        sd += scratch[4 * k + 3];
    }
    a = sa;
    b = sb;
    c = sc;
    d = sd;
}
__device__ __forceinline__ int ilog2_ceil(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

}  // namespace ca
