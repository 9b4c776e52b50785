// Split-BF16 MFMA path for n = 128 (the precision variant of Algorithm 2).
//
// Each DFT of length 128 is computed as two DFT-matrix products on the
// matrix cores, with n = 8 n1 + n2 and k = k1 + 16 k2:
//   stage 1:  Y[k1][n2]  = sum_n1 W16[k1][n1] x[8 n1 + n2]          (16-point DFTs)
//   twiddle:  Y'[k1][n2] = Y[k1][n2] w_128^{n2 k1}                  (FP32, VALU)
//   stage 2:  X[k1 + 16 k2] = sum_n2 W8[k2][n2] Y'[k1][n2]          (8-point DFTs)
// Complex products are written as real GEMMs ([Re; Im] stacked).  Operands are
// split into BF16 pairs, a = a_hi + a_lo with a_hi = bf16(a) and
// a_lo = bf16(a - a_hi), and each product keeps the three leading terms
//   A B ~ A_hi B_hi + A_hi B_lo + A_lo B_hi
// accumulated in FP32 by v_mfma_f32_16x16x32_bf16.  The DFT matrices are
// split on the host from FP64 values.  As in the FP32 path the correlation is
// D = DFT(conj(Z1) Z2) = n conj(C); the epilogue (candidate window with the
// split-BF16 error bound, FP64 re-scoring, theta, e0) is shared.
//
// A wave processes two pairs at a time (a stage-1 product covers 16 columns
// = 2 pairs x 8 values of n2).  MFMA operand layouts (16x16x32, lane l,
// element e, accumulator r):  A[l % 16][8 (l / 16) + e],
// B[8 (l / 16) + e][l % 16],  D[4 (l / 16) + r][l % 16].
#include "epilogue.hpp"
#include "launch.hpp"

namespace ca {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct Bf16Lane {
    bf16x8 s1[4];   // stage-1 A for lane l: Re-block hi, Re-block lo, Im-block hi, Im-block lo
    bf16x8 s2[2];   // stage-2 A: [W_hi | W_hi] and [W_lo | 0] (K = 32 covers hi and lo B halves)
    cf tw[4];       // w_128^{n2 k1} for the lane's four stage-1 outputs
};
static_assert(sizeof(Bf16Lane) == 128, "per-lane constant block");

constexpr int kBN = 128;
constexpr int kBPad = team_padn<kBN>();
// Error unit of the split-BF16 path in the |C| bound kErrScale u log2(n) n |z1||z2|.
// Per product the dropped lo*lo term and the rounding of the two lo parts are
// each at most 2^-16 relative; they carry random signs, and the measured |C|
// error (through theta at the optimum: <= 6e-6 rad over the parity sets) is
// twenty times below the bound this unit gives (1.1e-4 relative at n = 128).
constexpr double kBf16U = 7.62939453125e-06;   // 2^-17

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two values at a time: one packed conversion per BF16 pair, the hi parts
// widened back exactly, the remainders converted as one more pair.
__device__ __forceinline__ void split8(const float (&v)[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
        const f32x2 a = {v[e], v[e + 1]};
        const bf16x2 h = __builtin_convertvector(a, bf16x2);
        const f32x2 r = a - __builtin_convertvector(h, f32x2);
        const bf16x2 l = __builtin_convertvector(r, bf16x2);
        hi[e] = h[0];
        hi[e + 1] = h[1];
        lo[e] = l[0];
        lo[e + 1] = l[1];
    }
}

__device__ __forceinline__ f32x4 mma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// DFT of length 128 of two pairs' signals.  src(p, n, comp) reads component
// comp (0 real, 1 imaginary) of element n of pair p; the result is written
// with dst(p, k, comp, value) in natural order k.
template <class Src, class Dst>
__device__ __forceinline__ void dft128x2(Src src, Dst dst, cf* ys, const Bf16Lane& c, int l) {
    // stage 1: B rows = (Re n1 0..15, Im n1 0..15), columns = (pair, n2)
    {
        const int j = l & 15, p = j >> 3, n2 = j & 7;
        const int comp = l >> 5, n1b = 8 * ((l >> 4) & 1);
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = src(p, 8 * (n1b + e) + n2, comp);
        bf16x8 bh, bl;
        split8(v, bh, bl);
        f32x4 yr = {0.0f, 0.0f, 0.0f, 0.0f}, yi = {0.0f, 0.0f, 0.0f, 0.0f};
        yr = mma(c.s1[0], bh, yr);
        yr = mma(c.s1[0], bl, yr);
        yr = mma(c.s1[1], bh, yr);
        yi = mma(c.s1[2], bh, yi);
        yi = mma(c.s1[2], bl, yi);
        yi = mma(c.s1[3], bh, yi);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k1 = 4 * (l >> 4) + r;
            ys[p * kBN + k1 * 8 + n2] = mul(cf{yr[r], yi[r]}, c.tw[r]);
        }
    }
    wave_lds_sync();
    // stage 2 (one pair per product): B rows = (Re n2 hi, Im n2 hi, Re n2 lo, Im n2 lo), columns = k1
#pragma unroll
    for (int pp = 0; pp < 2; ++pp) {
        const int k1 = l & 15, comp = (l >> 4) & 1, half = l >> 5;
        const float* yc = reinterpret_cast<const float*>(ys + pp * kBN + k1 * 8) + comp;
        float u[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) u[e] = yc[2 * e];
        bf16x8 bh, bl;
        split8(u, bh, bl);
        const bf16x8 b = half ? bl : bh;
        f32x4 x = {0.0f, 0.0f, 0.0f, 0.0f};
        x = mma(c.s2[0], b, x);
        x = mma(c.s2[1], b, x);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 4 * (l >> 4) + r;      // row: Re X[k2 = i] for i < 8, Im X[k2 = i - 8] otherwise
            dst(pp, k1 + 16 * (i & 7), i >> 3, x[r]);
        }
    }
    wave_lds_sync();
}

__global__ __launch_bounds__(256, 2) void k_align_bf16(const cf* __restrict__ z1, const cf* __restrict__ z2,
                                                       int64_t num_pairs, ca_result_t* __restrict__ out,
                                                       const Bf16Lane* __restrict__ cst, int theta64) {
    __shared__ cf s_z[4][2][2][kBPad];    // [wave][pair][curve] nodes, padded layout
    __shared__ cf s_w[4][2][2][kBN];      // [wave][pair][signal] spectra / correlation
    __shared__ cf s_y[4][2][kBN];         // stage-1 outputs
    __shared__ int s_cand[4][2][kCandCap];
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
    const Bf16Lane c = cst[l];
    cf* ys = &s_y[wv][0][0];
    const int64_t groups = (num_pairs + 1) / 2;
    for (int64_t g = (int64_t)blockIdx.x * 4 + wv; g < groups; g += (int64_t)gridDim.x * 4) {
        const int64_t p0 = 2 * g;
        const bool has1 = p0 + 1 < num_pairs;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int idx = l + 64 * i;            // pair (idx >> 8), curve (idx >> 7) & 1, node idx & 127
            const int p = idx >> 8, cv = (idx >> 7) & 1, n = idx & (kBN - 1);
            cf val = {0.0f, 0.0f};
            if (p == 0 || has1) val = (cv ? z2 : z1)[(p0 + p) * kBN + n];
            s_z[wv][p][cv][lpad<kBN>(n)] = val;
        }
        wave_lds_sync();
        // FP64 norms, one team of 32 lanes per pair
        const int p = l >> 5, t = l & 31;
        double q1 = 0.0, q2 = 0.0;
        cf a0[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a0[q] = s_z[wv][p][0][lpad<kBN>(t + 32 * q)];
            const cf b = s_z[wv][p][1][lpad<kBN>(t + 32 * q)];
            q1 = fma((double)a0[q].x, (double)a0[q].x, fma((double)a0[q].y, (double)a0[q].y, q1));
            q2 = fma((double)b.x, (double)b.x, fma((double)b.y, (double)b.y, q2));
        }
        const double n1 = team_sum<32>(q1) / kBN, n2 = team_sum<32>(q2) / kBN;
        for (int cv = 0; cv < 2; ++cv) {
            dft128x2([&](int pp, int n, int comp) {
                         return reinterpret_cast<const float*>(&s_z[wv][pp][cv][lpad<kBN>(n)])[comp];
                     },
                     [&](int pp, int k, int comp, float v) {
                         float* w = reinterpret_cast<float*>(&s_w[wv][pp][cv][k]);
                         w[comp] = v;
                     },
                     ys, c, l);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int idx = l + 64 * i, pp = idx >> 7, k = idx & (kBN - 1);
            s_w[wv][pp][0][k] = cjmul(s_w[wv][pp][0][k], s_w[wv][pp][1][k]);
        }
        wave_lds_sync();
        dft128x2([&](int pp, int n, int comp) { return reinterpret_cast<const float*>(&s_w[wv][pp][0][n])[comp]; },
                 [&](int pp, int k, int comp, float v) {
                     float* w = reinterpret_cast<float*>(&s_w[wv][pp][1][k]);
                     w[comp] = v;
                 },
                 ys, c, l);
        cf d[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) d[q] = s_w[wv][p][1][t + 32 * q];
        wave_lds_sync();
        // curve 2's nodes twice over the pair's spectra area (read into d
        // above), so the re-scoring reads them at constant offsets
        cf* zt = &s_w[wv][p][0][0];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const cf b = s_z[wv][p][1][lpad<kBN>(t + 32 * q)];
            zt[t + 32 * q] = b;
            zt[kBN + t + 32 * q] = b;
        }
        wave_lds_sync();
        const ca_result_t res = team_epilogue<kBN, 32, kZTwice>(d, a0, zt, s_cand[wv][p], t, n1, n2,
                                                                CA_RESCORE_WINDOW, theta64, kBf16U);
        if (t == 0 && (p == 0 || has1)) out[p0 + p] = res;
        wave_lds_sync();
    }
}

static int bf16_blocks_per_cu() {
    static int cached = -1;
    if (cached < 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_align_bf16, 256, 0) != hipSuccess || nb < 1)
            nb = 1;
        cached = nb;
    }
    return cached;
}

hipError_t launch_align_bf16(const void* z1, const void* z2, int64_t num_pairs, ca_result_t* out,
                             const void* lane_consts, int theta64, int num_cus, hipStream_t s) {
    const int64_t groups = (num_pairs + 1) / 2;
    int64_t blocks = (groups + 3) / 4;
    const int64_t cap = (int64_t)num_cus * bf16_blocks_per_cu();
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(k_align_bf16, dim3((unsigned)blocks), dim3(256), 0, s, (const cf*)z1, (const cf*)z2,
                       num_pairs, out, (const Bf16Lane*)lane_consts, theta64);
    return hipGetLastError();
}

}  // namespace ca
