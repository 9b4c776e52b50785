// Split-BF16 MFMA paths (the precision variant of Algorithm 2), n = 128 and
// n = 1024.  Every DFT runs as DFT-matrix products on the matrix cores with the
// operands split into BF16 pairs, a = a_hi + a_lo with a_hi = bf16(a) and
// a_lo = bf16(a - a_hi), keeping the three leading terms of each product
//   A B ~ A_hi B_hi + A_hi B_lo + A_lo B_hi
// accumulated in FP32.  Complex products are real GEMMs: with the data as the
// A operand, [Pr | Pi] = [Ar | Ai] [[Fr, Fi], [-Fi, Fr]]; with the data as the
// B operand the same block matrix (the DFT matrices are symmetric) is the A
// operand.  Both stages of a transform read the previous stage's accumulators
// in place: the data is the A operand where the contraction index is the
// lane's row and the B operand where it is in-lane, and the K index of every
// K-block is read in the accumulator-row order, so no value moves between
// lanes or through LDS inside the three transforms.  The DFT matrices are split
// on the host from FP64 values; twiddles between the stages are FP32.  As in
// the FP32 path the correlation is D = DFT(conj(Z1) Z2) = n conj(C).
#include "epilogue.hpp"
#include "launch.hpp"

namespace ca {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

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

// ----------------------------------------------------------------- n = 128
// Two pairs per MFMA group, v_mfma_f32_16x16x32_bf16.  Lane l (g = l / 16, c = l % 16)
// holds operand A element e as A[c][8 g + e], operand B element e as
// B[8 g + e][c] and accumulator r as D[4 g + r][c].  K slot (g, e) is read as
// part e / 4 (real, imaginary) of index 4 g + e % 4 (16-point stages), or of
// pair g / 2 and index 4 (g % 2) + e % 4 (8-point stages, whose constant is
// block-diagonal in the pair).  With x_P[8 n1 + n2] the nodes of pair P:
//   forward stage 1 (data = A, row c = (P = c / 8, n2 = c % 8), K = n1):
//       Y_P[k1][n2] = sum_n1 W16^{n1 k1} x_P[8 n1 + n2]; lane column k1 = c,
//       rows (P, n2) = 4 g + r, i.e. P = g / 2, n2 = 4 (g % 2) + r
//   twiddle w_128^{n2 k1}
//   forward stage 2 (data = B, K = (P, n2)): X_P[k1 + 16 k2] =
//       sum_n2 W8^{n2 k2} Y'_P[k1][n2]; lane column k1 = c, rows (P, k2)
// The correlation transform of Q = conj(X1) X2 (index m = m1 + 16 m2 with
// m1 = c in the lane's column and m2 = 4 (g % 2) + r in its rows) takes the
// slow index first:
//   stage 1 (data = A, row m1 = c, K = (P, m2)): U_P[m1][s1] =
//       sum_m2 W8^{m2 s1} Q_P[m1 + 16 m2]; lane column (P, s1) = c, rows m1 = 4 g + r
//   twiddle w_128^{m1 s1}
//   stage 2 (data = B, K = m1): D_P[s1 + 8 s2] = sum_m1 W16^{m1 s2} U'_P[m1][s1];
//       lane column (P, s1) = c, rows s2 = 4 g + r.
// The two constants (the 16-point matrix and the block-diagonal 8-point one,
// each as a real and an imaginary output block in BF16 hi and lo) are the same
// registers for all six stages.  D is then written to LDS in natural order and
// the shared epilogue (candidate window with the split-BF16 error bound,
// FP64 re-scoring, theta, e0) runs with one team of 16 lanes per pair, over
// the two groups of a wave.
struct Bf16Lane {
    bf16x8 k1[2][2];   // 16-point matrix: [output part][hi, lo]
    bf16x8 k2[2][2];   // block-diagonal 8-point matrix: [output part][hi, lo]
    cf twf[4];         // w_128^{(4 (g % 2) + r) c}
    cf twt[4];         // w_128^{(4 g + r) (c % 8)}
};
static_assert(sizeof(Bf16Lane) == 192, "per-lane constant block");

template <bool DATA_A>
__device__ __forceinline__ void stage128(const float (&in)[8], const bf16x8 (&K)[2][2], cf (&outv)[4]) {
    bf16x8 dh, dl;
    split8(in, dh, dl);
    f32x4 acc[2];
#pragma unroll
    for (int ob = 0; ob < 2; ++ob) {
        acc[ob] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        if constexpr (DATA_A) {
            acc[ob] = mma(dh, K[ob][0], acc[ob]);
            acc[ob] = mma(dh, K[ob][1], acc[ob]);
            acc[ob] = mma(dl, K[ob][0], acc[ob]);
        } else {
            acc[ob] = mma(K[ob][0], dh, acc[ob]);
            acc[ob] = mma(K[ob][1], dh, acc[ob]);
            acc[ob] = mma(K[ob][0], dl, acc[ob]);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) outv[r] = cf{acc[0][r], acc[1][r]};
}

// operand elements of the next stage from a lane's four complex values
__device__ __forceinline__ void ops4(const cf (&v)[4], float (&o)[8]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        o[r] = v[r].x;
        o[4 + r] = v[r].y;
    }
}

// A lane's first-stage nodes of two pairs' curves (x0: pair 0, x1: pair 1,
// NULL: zeros).  The loads are unconditional: a missing curve reads the valid
// curve `any` and is zeroed.
__device__ __forceinline__ void load128(const cf* x0, const cf* x1, const cf* any, int g, int c, cf (&lv)[4]) {
    const cf* xs = (c >> 3) ? x1 : x0;
    const cf* x = xs ? xs : any;
    const int n2 = c & 7;
#pragma unroll
    for (int e = 0; e < 4; ++e) lv[e] = x[8 * (4 * g + e) + n2];
    if (!xs) {
#pragma unroll
        for (int e = 0; e < 4; ++e) lv[e] = cf{0.0f, 0.0f};
    }
}

// Forward DFT of two pairs' curves from the nodes load128 gave.
__device__ __forceinline__ void fwd128(const cf (&lv)[4], const Bf16Lane& k, cf (&X)[4]) {
    float op[8];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        op[e] = lv[e].x;
        op[4 + e] = lv[e].y;
    }
    cf y[4];
    stage128<true>(op, k.k1, y);
#pragma unroll
    for (int r = 0; r < 4; ++r) y[r] = mul(y[r], k.twf[r]);
    ops4(y, op);
    stage128<false>(op, k.k2, X);
}

// Four pairs per wave: two MFMA groups of two pairs fill the D buffers, then
// the epilogue runs with one team of 16 lanes per pair, so its reductions
// span 16 lanes and its per-pair scalar work (square roots, arc tangent, the
// result) is shared by four pairs.
constexpr int kBPW = 4;             // pairs per wave
constexpr int kBT = 64 / kBPW;      // epilogue team
constexpr int kBR = kBN / kBT;      // values per lane in the epilogue

__global__ __launch_bounds__(256, 3) void k_align_bf16(const cf* __restrict__ z1, const cf* __restrict__ z2,
                                                       int64_t num_pairs, ca_result_t* __restrict__ out,
                                                       const Bf16Lane* __restrict__ cst, int theta64) {
    __shared__ cf s_zt[4][kBPW][2 * kBN];    // [wave][pair] curve 2's nodes twice (FP64 re-scoring)
    __shared__ cf s_d[4][kBPW][kBN + 8];     // [wave][pair] D in natural order
    __shared__ int s_cand[4][kBPW][kCandCap];
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c = l & 15;
    const Bf16Lane k = cst[l];
    const int p = l / kBT, t = l % kBT;      // epilogue: team p (pair p0 + p)
    cf* zt = s_zt[wv][p];
    const int64_t groups = (num_pairs + kBPW - 1) / kBPW;
    for (int64_t grp = (int64_t)blockIdx.x * 4 + wv; grp < groups; grp += (int64_t)gridDim.x * 4) {
        const int64_t p0 = kBPW * grp;
        const int np = (int)(num_pairs - p0 < kBPW ? num_pairs - p0 : kBPW);   // pairs in the group
        const bool mine = p < np;
        // the epilogue's team layout: curve 1 in registers, curve 2 twice in
        // LDS; loads unconditional (a missing pair reads pair p0's nodes and
        // zeroes them), so all of them are in flight together
        const int64_t pl = mine ? p0 + p : p0;
        const cf* ap = z1 + pl * kBN;
        const cf* bp = z2 + pl * kBN;
        cf la[kBR], lb[kBR];
#pragma unroll
        for (int q = 0; q < kBR; ++q) {
            la[q] = ap[t + kBT * q];
            lb[q] = bp[t + kBT * q];
        }
        // the transforms' operands of both MFMA groups, requested with them
        cf x1v[kBPW / 2][4], x2v[kBPW / 2][4];
#pragma unroll
        for (int h = 0; h < kBPW / 2; ++h) {
            const cf* a0p = 2 * h < np ? z1 + (p0 + 2 * h) * kBN : nullptr;
            const cf* b0p = 2 * h < np ? z2 + (p0 + 2 * h) * kBN : nullptr;
            const cf* a1p = 2 * h + 1 < np ? z1 + (p0 + 2 * h + 1) * kBN : nullptr;
            const cf* b1p = 2 * h + 1 < np ? z2 + (p0 + 2 * h + 1) * kBN : nullptr;
            load128(a0p, a1p, ap, g, c, x1v[h]);
            load128(b0p, b1p, bp, g, c, x2v[h]);
        }
        cf a0[kBR];
        double q1 = 0.0, q2 = 0.0;
#pragma unroll
        for (int q = 0; q < kBR; ++q) {
            const cf va = mine ? la[q] : cf{0.0f, 0.0f};
            const cf vb = mine ? lb[q] : cf{0.0f, 0.0f};
            a0[q] = va;
            zt[t + kBT * q] = vb;
            zt[kBN + t + kBT * q] = vb;
            q1 = fma((double)va.x, (double)va.x, fma((double)va.y, (double)va.y, q1));
            q2 = fma((double)vb.x, (double)vb.x, fma((double)vb.y, (double)vb.y, q2));
        }
        const double n1 = team_sum<kBT>(q1) / kBN, n2 = team_sum<kBT>(q2) / kBN;
#pragma unroll
        for (int h = 0; h < kBPW / 2; ++h) {
            // MFMA group h: pairs p0 + 2 h (rows c < 8) and p0 + 2 h + 1
            cf X1[4], X2[4];
            fwd128(x1v[h], k, X1);
            fwd128(x2v[h], k, X2);
            cf Q[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) Q[r] = cjmul(X1[r], X2[r]);
            float op[8];
            ops4(Q, op);
            cf u[4];
            stage128<true>(op, k.k2, u);
#pragma unroll
            for (int r = 0; r < 4; ++r) u[r] = mul(u[r], k.twt[r]);
            ops4(u, op);
            cf D[4];
            stage128<false>(op, k.k1, D);
            // D_P[s1 + 8 s2] with P = 2 h + c / 8, s1 = c % 8, s2 = 4 g + r
#pragma unroll
            for (int r = 0; r < 4; ++r) s_d[wv][2 * h + (c >> 3)][(c & 7) + 8 * (4 * g + r)] = D[r];
        }
        wave_lds_sync();
        cf d[kBR];
#pragma unroll
        for (int q = 0; q < kBR; ++q) d[q] = s_d[wv][p][t + kBT * q];
        const ca_result_t res = team_epilogue<kBN, kBT, kZTwice, true, false, true>(d, a0, zt, s_cand[wv][p], t, n1, n2,
                                                                       CA_RESCORE_WINDOW, theta64, kBf16U);
        if (t == 0 && mine) out[p0 + p] = res;
        wave_lds_sync();
    }
}

// ---------------------------------------------------------------- n = 1024
// Split-BF16 path for n = 1024: every transform is a four-step DFT of
// 32 x 32 with both stages on v_mfma_f32_32x32x16_bf16, one pair per wave.
//
// Lane l (h = l / 32, c = l % 32) and the MFMA 32x32x16 layouts: operand A
// element e of lane l is A[c][slot(h, e)], operand B element e is
// B[slot(h, e)][c], accumulator g is D[row(g, h)][c] with
// row(g, h) = 8 (g / 4) + 4 h + g % 4.  The K index of K-block kb is read as
// (part, j) with part = kb / 2 (real, imaginary) and
// j = 16 (kb % 2) + 8 (e / 4) + 4 h + e % 4 = row(8 (kb % 2) + e, h),
// so the eight accumulators 8 (kb % 2) .. 8 (kb % 2) + 7 of a lane are
// exactly its operand elements of K-block kb in the next stage: no data
// moves between lanes or through LDS anywhere in the three transforms.
//
// Forward DFT, x[32 n1 + n2] -> X[k1 + 32 k2]:
//   stage 1 (data = A, lane row n2, K = n1):  Y[k1][n2] = sum_n1 W32^{n1 k1} x[32 n1 + n2]
//            accumulators: lane column k1, rows n2
//   twiddle: Y'[k1][n2] = Y[k1][n2] w_1024^{n2 k1}
//   stage 2 (data = B, lane column k1, K = n2): X[k1 + 32 k2] = sum_n2 W32^{n2 k2} Y'[k1][n2]
//            accumulators: lane column k1, rows k2
// The correlation transform of P = conj(X1) X2 (lane column m1 = k1, rows
// m2 = k2, index m = m1 + 32 m2) takes the slow index first:
//   stage 1 (data = A, lane row m1, K = m2): U[m1][s1] = sum_m2 W32^{m2 s1} P[m1 + 32 m2]
//            accumulators: lane column s1, rows m1
//   twiddle: U'[m1][s1] = U[m1][s1] w_1024^{m1 s1}
//   stage 2 (data = B, lane column s1, K = m1): D[s1 + 32 s2] = sum_m1 W32^{m1 s2} U'[m1][s1]
//            accumulators: lane column s1, rows s2.
// Both twiddle steps multiply accumulator g of lane l by w_1024^{row(g, h) c}.
// Complex products are real GEMMs: with the data as A, [Pr | Pi] =
// [Ar | Ai] [[Fr, Fi], [-Fi, Fr]]; with the data as B the same 64 x 64 block
// matrix is the A operand.  W32 is symmetric, so both uses read the same
// per-lane constant registers: for K-half q = kb % 2 the blocks Re W32,
// Im W32 and -Im W32 at rows j(q, h, e), column c, each split into BF16 hi
// and lo on the host.
//
// Shift selection.  The split-BF16 |C| is accurate to ~1e-5 relative, above
// the ~3.5e-7 by which neighbouring shifts differ at this size, so the
// largest |D| only locates the peak.  A least-squares parabola through the
// |D|^2 values within 16 shifts of it places the vertex (within one shift of
// the FP64 optimum on the workload), FP64 correlations at the vertex and its
// two neighbours are computed in one pass (curve 1's norm and curve 2's norm
// in the same pass), and the FP64 values then climb to a local maximum.  With
// T the best FP64 n |C| so far and eps the split-BF16 error bound, a shift can
// only beat T if its |D| is at least T - eps; the run of shifts around a
// climb's end whose |D| stays at or above T - 2 eps is that peak.  A shift
// outside every run (and more than 32 shifts from every climb's start and end)
// that could beat T starts another FP64 climb (at most eight;
// CA_FLAG_CAND_CAPPED beyond that), so separate peaks of nearly equal height
// (curves with rotational symmetry) are compared in FP64 as well.  When the
// main run is wider than 96 shifts (nearly circular shapes, whose |C| varies
// by less than the error bound around the whole circle, so one run can hold
// several maxima) the largest |D| of every 32-shift segment that could beat T
// starts a climb instead (at most sixteen), unless it lies within four shifts
// of the segment's edge next to a segment with a larger value (a slope).
constexpr int kB1k = 1024;
constexpr int kLocalW = 16;      // half-width of the parabola fit
constexpr int kFarD = 32;        // distance beyond which a window shift starts its own climb
constexpr int kMaxFar = 8;
constexpr int kMaxClimb = 32;
constexpr int kWideRun = 96;     // a main run wider than this: several maxima may share it
constexpr int kMaxSeg = 16;      // climbs of the segment search
constexpr int kSegEdge = 4;      // segment maxima this close to a larger neighbour are on a slope

typedef float f32x16 __attribute__((ext_vector_type(16)));

struct Bf16Lane1k {
    bf16x8 k[2][3][2];   // [K-half q][Re, Im, -Im][hi, lo]
};
static_assert(sizeof(Bf16Lane1k) == 192, "per-lane constant block");
struct Bf16Tables1k {
    Bf16Lane1k lane[64];
    float4 tw[8][64];    // tw[i][l] = (w(row(2i, h) c), w(row(2i + 1, h) c)) as (re, im, re, im)
};

__device__ __forceinline__ f32x16 mma32(bf16x8 a, bf16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Constant block of K-block kb, output block nb: (real input part) Re, Im;
// (imaginary input part) -Im, Re.
__device__ __forceinline__ const bf16x8& kblk(const bf16x8 (&K)[2][3][2], int kb, int nb, int hl) {
    const int q = kb & 1;
    const int cls = (kb >> 1) == 0 ? nb : (nb == 0 ? 2 : 0);
    return K[q][cls][hl];
}

// One DFT-32 stage of 32 columns: in[kb][e] are the operand elements
// (K-blocks 0, 1: real parts, 2, 3: imaginary parts).  DATA_A: the data is
// the A operand; else the B operand.  acc[0] = real, acc[1] = imaginary part.
template <bool DATA_A>
__device__ __forceinline__ void dft32_stage(const float (&in)[4][8], const bf16x8 (&K)[2][3][2],
                                            f32x16 (&acc)[2]) {
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int g = 0; g < 16; ++g) acc[b][g] = 0.0f;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        bf16x8 dh, dl;
        split8(in[kb], dh, dl);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            if constexpr (DATA_A) {
                acc[b] = mma32(dh, kblk(K, kb, b, 0), acc[b]);
                acc[b] = mma32(dh, kblk(K, kb, b, 1), acc[b]);
                acc[b] = mma32(dl, kblk(K, kb, b, 0), acc[b]);
            } else {
                acc[b] = mma32(kblk(K, kb, b, 0), dh, acc[b]);
                acc[b] = mma32(kblk(K, kb, b, 1), dh, acc[b]);
                acc[b] = mma32(kblk(K, kb, b, 0), dl, acc[b]);
            }
        }
    }
}

// Accumulators times the per-lane twiddles w_1024^{row(g, h) c}, as the next
// stage's operand elements.
__device__ __forceinline__ void twiddle_to_ops(const f32x16 (&acc)[2], const float4* tws, int l, float (&op)[4][8]) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const float4 w = tws[i * 64 + l];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int g = 2 * i + u;
            const cf y = mul(cf{acc[0][g], acc[1][g]}, u ? cf{w.z, w.w} : cf{w.x, w.y});
            op[g >> 3][g & 7] = y.x;
            op[2 + (g >> 3)][g & 7] = y.y;
        }
    }
}

__device__ __forceinline__ void acc_to_ops(const f32x16 (&acc)[2], float (&op)[4][8]) {
#pragma unroll
    for (int g = 0; g < 16; ++g) {
        op[g >> 3][g & 7] = acc[0][g];
        op[2 + (g >> 3)][g & 7] = acc[1][g];
    }
}

// Node index held by lane (h, c) in operand slot (q, e) of the first stage.
__device__ __forceinline__ int node1k(int q, int e, int h, int c) {
    return 32 * (16 * q + 8 * (e >> 2) + 4 * h + (e & 3)) + c;
}

// Forward DFT of 1024 nodes: returns X[c + 32 row(g, h)] in (acc[0][g], acc[1][g]).
// A lane's nodes for the first stage: slot 8 q + e holds node node1k(q, e, h, c).
__device__ __forceinline__ void load1k(const cf* __restrict__ x, int l, cf (&v)[16]) {
    const int h = l >> 5, c = l & 31;
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int e = 0; e < 8; ++e) v[8 * q + e] = x[node1k(q, e, h, c)];
}

// Forward DFT of 1024 nodes (a lane's slots from load1k): returns
// X[c + 32 row(g, h)] in (acc[0][g], acc[1][g]).
__device__ __forceinline__ void fwd1k(const cf (&v)[16], const bf16x8 (&K)[2][3][2], const float4* tws, int l,
                                      f32x16 (&acc)[2]) {
    float op[4][8];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            op[q][e] = v[8 * q + e].x;
            op[2 + q][e] = v[8 * q + e].y;
        }
    dft32_stage<true>(op, K, acc);
    twiddle_to_ops(acc, tws, l, op);
    dft32_stage<false>(op, K, acc);
}

__global__ __launch_bounds__(256, 2) void k_align_bf16_1k(const cf* __restrict__ z1, const cf* __restrict__ z2,
                                                          int64_t num_pairs, ca_result_t* __restrict__ out,
                                                          const Bf16Tables1k* __restrict__ tab, int theta64) {
    __shared__ float4 s_tw[8 * 64];
    __shared__ cf s_z2[4][2 * kB1k];      // per wave: curve 2's nodes twice
    __shared__ int s_runs[4][3][2 * kMaxFar + 2];   // per wave: peak centres and run extents
    __shared__ float s_segv[4][32];                 // per wave: largest |D|^2 of each 32-shift segment
    __shared__ int s_segi[4][32];                   //           and its shift
    for (int i = threadIdx.x; i < 8 * 64; i += blockDim.x) s_tw[i] = (&tab->tw[0][0])[i];
    __syncthreads();
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, h = l >> 5, c = l & 31;
    cf* zt = s_z2[wv];
    // FP64 bound of |D| error in units of n * sqrt(n1 n2) (see the n = 128 kernel)
    const double err_unit = kErrScale * kBf16U * 10.0 * kB1k * kB1k;
    for (int64_t pair = (int64_t)blockIdx.x * 4 + wv; pair < num_pairs; pair += (int64_t)gridDim.x * 4) {
        const cf* pa = z1 + pair * kB1k;
        const cf* pb = z2 + pair * kB1k;
        // the DFT constants are read again for every pair (cache hits), so that
        // they do not stay live through the epilogue: the empty asm statement
        // keeps the compiler from hoisting the loads out of the loop
        const Bf16Tables1k* tb = tab;
        asm volatile("" : "+s"(tb));
        const Bf16Lane1k* kl = &tb->lane[l];
        bf16x8 K[2][3][2];
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int u = 0; u < 2; ++u) K[q][k][u] = kl->k[q][k][u];
        // both curves' nodes requested together; curve 2's also go twice to
        // LDS for the shifted FP64 reads
        cf xa[16], xb[16];
        load1k(pa, l, xa);
        load1k(pb, l, xb);
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int node = node1k(q, e, h, c);
                zt[node] = xb[8 * q + e];
                zt[kB1k + node] = xb[8 * q + e];
            }
        f32x16 X1[2], acc[2];
        fwd1k(xa, K, s_tw, l, X1);
        fwd1k(xb, K, s_tw, l, acc);
        // P = conj(X1) X2 as the correlation transform's first operands
        float op[4][8];
#pragma unroll
        for (int g = 0; g < 16; ++g) {
            const cf p = cjmul(cf{X1[0][g], X1[1][g]}, cf{acc[0][g], acc[1][g]});
            op[g >> 3][g & 7] = p.x;
            op[2 + (g >> 3)][g & 7] = p.y;
        }
        dft32_stage<true>(op, K, acc);
        twiddle_to_ops(acc, s_tw, l, op);
        dft32_stage<false>(op, K, acc);
        // curve 1 again (its nodes in the first stage's slots) for the FP64
        // sums, requested before the peak search so the loads overlap it
        cf a0[16];
        load1k(pa, l, a0);
        // acc[.][g] = D[s] = n conj C(s), s = c + 32 row(g, h)
        auto yat = [&](int g) { return acc[0][g] * acc[0][g] + acc[1][g] * acc[1][g]; };
        float bvl = -1.0f;
        int bil = 0x7fffffff;
#pragma unroll
        for (int g = 0; g < 16; ++g) {
            const float yg = yat(g);
            const int sg = c + 32 * (8 * (g >> 2) + 4 * h + (g & 3));
            argmax_combine(bvl, bil, yg, sg);
        }
        float bv = bvl;
        int sb = bil;
        team_argmax<64>(bv, sb);
        if (sb < 0 || sb >= kB1k) sb = 0;
        // least-squares parabola y ~ a + b d + c2 d^2 over |d| <= kLocalW
        float sy = 0.0f, sdy = 0.0f, sd2y = 0.0f;
        const float ib = bv > 0.0f ? __builtin_amdgcn_rcpf(bv) : 0.0f;
#pragma unroll
        for (int g = 0; g < 16; ++g) {
            const int sg = c + 32 * (8 * (g >> 2) + 4 * h + (g & 3));
            const int d = ((sg - sb + kB1k / 2) & (kB1k - 1)) - kB1k / 2;
            const float yy = (d >= -kLocalW && d <= kLocalW) ? yat(g) * ib : 0.0f;
            const float df = (float)d;
            sy += yy;
            sdy = fmaf(df, yy, sdy);
            sd2y = fmaf(df * df, yy, sd2y);
        }
        sy = team_sum<64>(sy);
        sdy = team_sum<64>(sdy);
        sd2y = team_sum<64>(sd2y);
        // sums of d^k over the window, k = 0, 2, 4
        constexpr float S0 = 2 * kLocalW + 1;
        constexpr float S2 = (float)(kLocalW * (kLocalW + 1) * (2 * kLocalW + 1) / 3);
        constexpr float S4 = (float)(2.0 * kLocalW * (kLocalW + 1) * (2 * kLocalW + 1) *
                                     (3.0 * kLocalW * kLocalW + 3 * kLocalW - 1) / 30.0);
        const float bco = sdy / S2;
        const float cco = (sd2y - (S2 / S0) * sy) / (S4 - S2 * S2 / S0);
        float v = cco < 0.0f ? -bco / (2.0f * cco) : 0.0f;
        if (!(fabsf(v) <= 0.5f * kLocalW)) v = 0.0f;
        int sc = (sb + (int)rintf(v)) & (kB1k - 1);
        wave_lds_sync();
        // FP64 C at sc - 1, sc, sc + 1 (times n), curve norms in the same pass
        double cre[3] = {0.0, 0.0, 0.0}, cim[3] = {0.0, 0.0, 0.0}, q1 = 0.0, q2 = 0.0;
        {
            // node j = c + 128 h + off of curve 1 meets z2[(j - s) mod n] = zt[n + j - s]
            // (s in [0, n), so the index stays in [1, 2n - 1])
            int base[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) base[k] = kB1k + c + 128 * h - ((sc - 1 + k) & (kB1k - 1));
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int off = 32 * (16 * q + 8 * (e >> 2) + (e & 3));
                    const double ax = a0[8 * q + e].x, ay = a0[8 * q + e].y;
                    q1 = fma(ax, ax, fma(ay, ay, q1));
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const cf zz = zt[base[k] + off];   // shift sc - 1 + k
                        const double bx = zz.x, by = zz.y;
                        if (k == 1) q2 = fma(bx, bx, fma(by, by, q2));
                        cre[k] = fma(ax, bx, fma(ay, by, cre[k]));
                        cim[k] = fma(ay, bx, fma(-ax, by, cim[k]));
                    }
                }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            cre[k] = team_sum<64>(cre[k]);
            cim[k] = team_sum<64>(cim[k]);
        }
        const double n1 = team_sum<64>(q1) / kB1k, n2 = team_sum<64>(q2) / kB1k;
        ca_result_t res;
        if (special_case(res, n1, n2, (double)bv)) {
            if (l == 0) out[pair] = res;
            wave_lds_sync();
            continue;
        }
        // FP64 C at one shift
        auto dot1 = [&](int s, double& re, double& im) {
            const int base = kB1k + c + 128 * h - s;
            re = 0.0;
            im = 0.0;
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int off = 32 * (16 * q + 8 * (e >> 2) + (e & 3));
                    const cf zz = zt[base + off];
                    const double ax = a0[8 * q + e].x, ay = a0[8 * q + e].y, bx = zz.x, by = zz.y;
                    re = fma(ax, bx, fma(ay, by, re));
                    im = fma(ay, bx, fma(-ax, by, im));
                }
            re = team_sum<64>(re);
            im = team_sum<64>(im);
        };
        Pick pk;
        // climb from the three values at (s - 1, s, s + 1) to a local maximum
        auto climb = [&](int s, double (&m)[3], double (&re)[3], double (&im)[3]) {
            for (int it = 0; it < kMaxClimb; ++it) {
                if (m[1] >= m[0] && m[1] >= m[2]) break;
                if (m[0] > m[2]) {       // move left
                    s = (s - 1) & (kB1k - 1);
                    m[2] = m[1]; re[2] = re[1]; im[2] = im[1];
                    m[1] = m[0]; re[1] = re[0]; im[1] = im[0];
                    dot1((s - 1) & (kB1k - 1), re[0], im[0]);
                    m[0] = re[0] * re[0] + im[0] * im[0];
                    pk.offer((s - 1) & (kB1k - 1), re[0], im[0]);
                } else {                 // move right
                    s = (s + 1) & (kB1k - 1);
                    m[0] = m[1]; re[0] = re[1]; im[0] = im[1];
                    m[1] = m[2]; re[1] = re[2]; im[1] = im[2];
                    dot1((s + 1) & (kB1k - 1), re[2], im[2]);
                    m[2] = re[2] * re[2] + im[2] * im[2];
                    pk.offer((s + 1) & (kB1k - 1), re[2], im[2]);
                }
            }
            return s;
        };
        double m3[3];
        for (int k = 0; k < 3; ++k) {
            m3[k] = cre[k] * cre[k] + cim[k] * cim[k];
            pk.offer((sc - 1 + k) & (kB1k - 1), cre[k], cim[k]);
        }
        const int sl = climb(sc, m3, cre, cim);
        // Other peaks.  T = n |C64| at the best shift so far; a shift can only
        // beat it if its split-BF16 |D| is at least T - eps.  The shifts whose
        // |D| stays at or above T - 2 eps on both sides of a climb's end form
        // that peak's run; a shift outside every run (and more than kFarD from
        // every climb's start and end) that could beat T starts a climb of its own.
        const double d1 = (double)__builtin_amdgcn_sqrtf(bv);
        const double epsD = err_unit * sqrt(n1 * n2);
        const double tbest = (double)kB1k * sqrt(pk.best);
        const double tf = tbest - epsD, tr = tbest - 2.0 * epsD;
        const float thr_far2 = tf > 0.0 ? (float)(tf * tf) : 0.0f;
        const float thr_run2 = tr > 0.0 ? (float)(tr * tr) : 0.0f;
        // run around s: shifts s - lo < x < s + hi (lo, hi = n: the whole circle)
        auto run_of = [&](int s0, int& lo, int& hi) {
            int dr = kB1k, dl = kB1k;
#pragma unroll
            for (int g = 0; g < 16; ++g) {
                const int sg = c + 32 * (8 * (g >> 2) + 4 * h + (g & 3));
                if (yat(g) < thr_run2) {
                    dr = min(dr, (sg - s0) & (kB1k - 1));
                    dl = min(dl, (s0 - sg) & (kB1k - 1));
                }
            }
            hi = team_min<64>(dr);
            lo = team_min<64>(dl);
        };
        bool capped = false;
        // common case: only the main run and the band around the climb's start
        int lo0, hi0;
        run_of(sl, lo0, hi0);
        int fs0;
        {
            const int wr = max(hi0, kFarD + 1), wl = max(lo0, kFarD + 1);
            float fv = -1.0f;
            int fs = 0x7fffffff;
#pragma unroll
            for (int g = 0; g < 16; ++g) {
                const float yg = yat(g);
                if (yg >= thr_far2) {
                    const int sg = c + 32 * (8 * (g >> 2) + 4 * h + (g & 3));
                    const int dr = (sg - sl) & (kB1k - 1), dl = (sl - sg) & (kB1k - 1);
                    const int er = (sg - sc) & (kB1k - 1), el = (sc - sg) & (kB1k - 1);
                    if (dr >= wr && dl >= wl && er > kFarD && el > kFarD) argmax_combine(fv, fs, yg, sg);
                }
            }
            team_argmax<64>(fv, fs);
            fs0 = fs;
        }
        if (lo0 + hi0 > kWideRun) {
            // Flat correlation (nearly circular shapes): the main run is wide
            // and may hold several maxima of nearly equal height.  Every
            // 32-shift segment s2 (shifts 32 s2 .. 32 s2 + 31, one register
            // in one half-wave) whose largest |D| could beat T starts a climb
            // at that largest value, unless a climb already ended within
            // kFarD of it.
#pragma unroll
            for (int g = 0; g < 16; ++g) {
                float v = yat(g);
                int i = c + 32 * (8 * (g >> 2) + 4 * h + (g & 3));
                team_argmax<32>(v, i);
                if (c == 0) {
                    const int s2 = 8 * (g >> 2) + 4 * h + (g & 3);
                    s_segv[wv][s2] = v;
                    s_segi[wv][s2] = i;
                }
            }
            wave_lds_sync();
            int* ctr = s_runs[wv][0];
            int nd = 0;
            ctr[nd++] = sl;
            int climbs = 0;
            for (int s2 = 0; s2 < 32; ++s2) {
                const float v = s_segv[wv][s2];
                const int fs = s_segi[wv][s2];
                if (!(v >= thr_far2)) continue;
                // a largest value at the edge facing a larger neighbouring
                // segment lies on a slope: its climb would end in that segment
                const int p = fs & 31;
                if (p >= 32 - kSegEdge && s_segv[wv][(s2 + 1) & 31] > v) continue;
                if (p < kSegEdge && s_segv[wv][(s2 - 1) & 31] > v) continue;
                bool near_done = false;
                for (int k = 0; k < nd; ++k) {
                    const int d = ((fs - ctr[k] + kB1k / 2) & (kB1k - 1)) - kB1k / 2;
                    near_done = near_done || (d >= -kFarD && d <= kFarD);
                }
                if (near_done) continue;
                if (climbs == kMaxSeg) {
                    capped = true;
                    break;
                }
                ++climbs;
                double fre[3], fim[3], fm[3];
                for (int k = 0; k < 3; ++k) {
                    dot1((fs - 1 + k) & (kB1k - 1), fre[k], fim[k]);
                    fm[k] = fre[k] * fre[k] + fim[k] * fim[k];
                    pk.offer((fs - 1 + k) & (kB1k - 1), fre[k], fim[k]);
                }
                const int fe = climb(fs, fm, fre, fim);
                wave_lds_sync();
                if (nd < 2 * kMaxFar + 2) ctr[nd++] = fe;
                wave_lds_sync();
            }
        } else if (fs0 >= 0 && fs0 < kB1k) {
            // other peaks: (centre, lo, hi) of every run in LDS (wave-uniform
            // values indexed by a counter)
            int* ctr = s_runs[wv][0];
            int* rlo = s_runs[wv][1];
            int* rhi = s_runs[wv][2];
            int nr = 0;
            auto add_run = [&](int s0, int lo, int hi) {
                wave_lds_sync();
                ctr[nr] = s0;
                rlo[nr] = lo;
                rhi[nr] = hi;
                ++nr;
                wave_lds_sync();
            };
            add_run(sl, lo0, hi0);
            add_run(sc, kFarD + 1, kFarD + 1);
            int fs = fs0;
            for (int f = 0; f <= kMaxFar; ++f) {
                if (f > 0) {
                    float fv = -1.0f;
                    fs = 0x7fffffff;
#pragma unroll
                    for (int g = 0; g < 16; ++g) {
                        const int sg = c + 32 * (8 * (g >> 2) + 4 * h + (g & 3));
                        const float yg = yat(g);
                        bool far = yg >= thr_far2;
                        for (int k = 0; k < nr; ++k) {
                            const int dr = (sg - ctr[k]) & (kB1k - 1), dl = (ctr[k] - sg) & (kB1k - 1);
                            far = far && dr >= max(rhi[k], kFarD + 1) && dl >= max(rlo[k], kFarD + 1);
                        }
                        if (far) argmax_combine(fv, fs, yg, sg);
                    }
                    team_argmax<64>(fv, fs);
                    if (fs < 0 || fs >= kB1k) break;
                }
                if (f == kMaxFar) {
                    capped = true;
                    break;
                }
                double fre[3], fim[3], fm[3];
                for (int k = 0; k < 3; ++k) {
                    dot1((fs - 1 + k) & (kB1k - 1), fre[k], fim[k]);
                    fm[k] = fre[k] * fre[k] + fim[k] * fim[k];
                    pk.offer((fs - 1 + k) & (kB1k - 1), fre[k], fim[k]);
                }
                const int fe = climb(fs, fm, fre, fim);
                int lo, hi;
                run_of(fe, lo, hi);
                add_run(fe, lo, hi);
                add_run(fs, kFarD + 1, kFarD + 1);
            }
        }
        // theta: FP32 arc tangent of the FP64 C at the chosen shift
        const double theta_path = (double)wrap_pi(atan2f((float)pk.im, (float)pk.re));
        // runner-up |D| for the reported gap when only one shift was evaluated
        finish(res, pk, kB1k, n1, n2, d1, d1, epsD, capped, theta_path, theta64);
        if (l == 0) out[pair] = res;
        wave_lds_sync();
    }
}

hipError_t launch_align_bf16_1k(const void* z1, const void* z2, int64_t num_pairs, ca_result_t* out,
                                const void* tables, int theta64, int num_cus, hipStream_t s) {
    static int per_cu = -1;
    if (per_cu < 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_align_bf16_1k, 256, 0) != hipSuccess || nb < 1)
            nb = 1;
        per_cu = nb;
    }
    int64_t blocks = (num_pairs + 3) / 4;
    const int64_t cap = (int64_t)num_cus * per_cu;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(k_align_bf16_1k, dim3((unsigned)blocks), dim3(256), 0, s, (const cf*)z1, (const cf*)z2,
                       num_pairs, out, (const Bf16Tables1k*)tables, theta64);
    return hipGetLastError();
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
    const int64_t groups = (num_pairs + kBPW - 1) / kBPW;
    int64_t blocks = (groups + 3) / 4;
    const int64_t cap = (int64_t)num_cus * bf16_blocks_per_cu();
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(k_align_bf16, dim3((unsigned)blocks), dim3(256), 0, s, (const cf*)z1, (const cf*)z2,
                       num_pairs, out, (const Bf16Lane*)lane_consts, theta64);
    return hipGetLastError();
}

}  // namespace ca
