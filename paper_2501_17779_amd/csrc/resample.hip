// Uniform arc-length resampling of closed polygons (section 2: Eq.
// arc-length-param, then cubic-spline interpolation evaluated at the uniform
// parameters t_n = n/N), followed by scaling to unit length and centering on
// the node mean.  Two kernels: a fast path with one wave per curve (below),
// and a general path for the curves it rejects, one workgroup per listed
// curve, persistent over the list, each owning a slot of global scratch for
// the cleaned vertex list and the per-knot quantities.
//
// Spline: the periodic C2 cubic through (s_j, Q_j) has second derivatives
// M_j solving the cyclic tridiagonal system
//   h_{j-1} M_{j-1} + 2 (h_{j-1} + h_j) M_j + h_j M_{j+1} = 6 (D_j - D_{j-1}),
//   D_j = (Q_{j+1} - Q_j) / h_j.
// After Jacobi scaling its eigenvalues lie in [1/2, 3/2], so the inverse
// decays at least like ((sqrt 3 - 1)/(sqrt 3 + 1))^d = 0.268^d with distance d.
// Each chunk of kRsC consecutive knots is therefore solved on the periodic
// extension truncated kRsW knots to either side (forward elimination from the
// left end, backward elimination from the right end, meeting at the chunk's
// right edge, then back substitution): the truncation changes M by at most
// ~0.268^W relative for a window of W knots.  A node moves by h^2 / 6 times
// the change of the moments around it (h the chord parameter step), so even
// a relative change of 1e-3 moves nodes far less than FP32 rounding of the
// curve when h is small: the general kernel uses W = kRsW = 12 (3e-7), the
// fast kernel W = kFtW = 6 (3.7e-4) for curves of at least kFtBigM = 256
// vertices (h <= 1/256) and W = 12 below.
#include <math.h>

#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace ca {

constexpr int kRsNT = 256;
constexpr int kRsW = 12;
constexpr int kRsC = 16;
constexpr int kRsMCap = CA_RESAMPLE_MAX_RAW;   // raw vertices per curve

struct RsSlot {
    cf* Q;        // cleaned vertices            [cap]
    double* s;    // knot parameters s_j in [0,1) [cap + 1]
    float* h;     // normalised chord lengths     [cap]
    cf* rhs;      // 6 (D_j - D_{j-1})            [cap]
    cf* M;        // spline second derivatives    [cap]
};

__host__ __device__ inline int64_t rs_slot_bytes() {
    return (int64_t)kRsMCap * (8 + 8 + 4 + 8 + 8) + 8 + 256;
}

__device__ __forceinline__ RsSlot rs_slot(unsigned char* base) {
    RsSlot s;
    s.s = reinterpret_cast<double*>(base);
    s.Q = reinterpret_cast<cf*>(s.s + kRsMCap + 1);
    s.rhs = s.Q + kRsMCap;
    s.M = s.rhs + kRsMCap;
    s.h = reinterpret_cast<float*>(s.M + kRsMCap);
    return s;
}

__device__ __forceinline__ int wrapk(int i, int K) {
    i %= K;
    return i < 0 ? i + K : i;
}

// Block-wide reductions/scans on 256 threads (4 waves).
__device__ __forceinline__ double rs_sum(double v, double* sh) {
    v = team_sum<64>(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return sh[0] + sh[1] + sh[2] + sh[3];
}
__device__ __forceinline__ int rs_max(int v, int* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return max(max(sh[0], sh[1]), max(sh[2], sh[3]));
}
// Exclusive scan of doubles over the block; returns this thread's prefix and
// the block total.
__device__ __forceinline__ double rs_exscan(double v, double* sh, double& total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    __syncthreads();
    if (lane == 63) sh[w] = incl;
    __syncthreads();
    double off = 0.0;
    for (int k = 0; k < w; ++k) off += sh[k];
    total = sh[0] + sh[1] + sh[2] + sh[3];
    return off + incl - v;
}

// Local solve for knots [a0, a0 + kRsC) (indices mod K).
__device__ void rs_local_solve(const RsSlot& S, int K, int a0) {
    float al[kRsC];
    cf de[kRsC];
    // forward elimination from a0 - W (natural truncation M = 0 outside)
    float hprev = S.h[wrapk(a0 - kRsW - 1, K)];
    float alpha = 0.0f, cprev = 0.0f;
    cf delta = {0.0f, 0.0f};
#pragma unroll
    for (int i = 0; i < kRsW + kRsC; ++i) {
        const int j = wrapk(a0 - kRsW + i, K);
        const float hj = S.h[j];
        const cf d = S.rhs[j];
        const float b = 2.0f * (hprev + hj);
        if (i == 0) {
            alpha = b;
            delta = d;
        } else {
            const float f = hprev / alpha;     // a_j / alpha_{j-1}, a_j = h_{j-1}
            alpha = b - f * cprev;             // c_{j-1} = h_{j-1}
            delta = {d.x - f * delta.x, d.y - f * delta.y};
        }
        cprev = hj;
        hprev = hj;
        if (i >= kRsW) { al[i - kRsW] = alpha; de[i - kRsW] = delta; }
    }
    // backward elimination from e + W - 1 down to e = a0 + C
    const int e = a0 + kRsC;
    float hnext = S.h[wrapk(e + kRsW - 1, K)];   // h_{last}
    float beta = 0.0f, anext = 0.0f;
    cf eps = {0.0f, 0.0f};
#pragma unroll
    for (int i = kRsW - 1; i >= 0; --i) {
        const int j = wrapk(e + i, K);
        const float hj = S.h[j];
        const float hjm = S.h[wrapk(e + i - 1, K)];
        const cf d = S.rhs[j];
        const float b = 2.0f * (hjm + hj);
        if (i == kRsW - 1) {
            beta = b;
            eps = d;
        } else {
            const float g = hj / beta;          // c_j / beta_{j+1}, c_j = h_j
            beta = b - g * anext;               // a_{j+1} = h_j
            eps = {d.x - g * eps.x, d.y - g * eps.y};
        }
        anext = hjm;   // a_j = h_{j-1}, used by the next (smaller) j
        (void)hnext;
    }
    // meet at e: a_e M_{e-1} + beta_e M_e = eps_e, alpha_{e-1} M_{e-1} + c_{e-1} M_e = delta_{e-1}
    const float ae = S.h[wrapk(e - 1, K)];       // a_e = h_{e-1} = c_{e-1}
    const float ce1 = ae;
    const float aL = al[kRsC - 1];
    const cf dL = de[kRsC - 1];
    const float den = beta - ae * ce1 / aL;
    cf Me = {(eps.x - ae * dL.x / aL) / den, (eps.y - ae * dL.y / aL) / den};
    cf Mnext = Me;
#pragma unroll
    for (int i = kRsC - 1; i >= 0; --i) {
        const int j = a0 + i;
        const float cj = S.h[wrapk(j, K)];
        const cf Mi = {(de[i].x - cj * Mnext.x) / al[i], (de[i].y - cj * Mnext.y) / al[i]};
        if (j < K) S.M[j] = Mi;
        Mnext = Mi;
    }
}

__global__ __launch_bounds__(kRsNT) void k_resample(const cf* __restrict__ raw, const int64_t* __restrict__ raw_off,
                                                    int64_t num_curves, const int64_t* __restrict__ out_off,
                                                    cf* __restrict__ out, double* __restrict__ norms,
                                                    uint32_t* __restrict__ flags, int mode,
                                                    unsigned char* __restrict__ scratch, int64_t slot_bytes,
                                                    const int* __restrict__ list_count,
                                                    const int* __restrict__ list) {
    __shared__ double shd[4];
    __shared__ int shi[4];
    const RsSlot S = rs_slot(scratch + (int64_t)blockIdx.x * slot_bytes);
    const int tid = threadIdx.x;
    const int64_t count = list_count ? (int64_t)*list_count : num_curves;
    for (int64_t li = blockIdx.x; li < count; li += gridDim.x) {
        const int64_t c = list ? (int64_t)list[li] : li;
        const int64_t r0 = raw_off[c];
        const int64_t mraw = raw_off[c + 1] - r0;
        const int64_t o0 = out_off[c];
        const int N = (int)(out_off[c + 1] - o0);
        cf* o = out + o0;
        uint32_t fl = 0;
        if (mraw < 1 || mraw > kRsMCap) fl = CA_FLAG_UNSUPPORTED_N;
        const cf* P = raw + r0;
        int M = (int)(fl ? 0 : mraw);

        // non-finite check and trailing copies of the first vertex
        int last = 0, bad = 0;
        const cf P0 = M > 0 ? P[0] : cf{0.0f, 0.0f};
        for (int j = tid; j < M; j += kRsNT) {
            const cf p = P[j];
            if (!(isfinite(p.x) && isfinite(p.y))) bad = 1;
            if (p.x != P0.x || p.y != P0.y) last = max(last, j);
        }
        if (rs_max(bad, shi)) fl |= CA_FLAG_NONFINITE;
        const int mt = rs_max(last, shi) + 1;

        // compaction: keep j iff j == 0 or P_j != P_{j-1}
        int K = 0;
        if (!fl) {
            for (int base = 0; base < mt; base += kRsNT) {
                const int j = base + tid;
                bool keep = false;
                cf p = {0.0f, 0.0f};
                if (j < mt) {
                    p = P[j];
                    if (j == 0) keep = true;
                    else { const cf pp = P[j - 1]; keep = (p.x != pp.x || p.y != pp.y); }
                }
                const uint64_t msk = __ballot(keep);
                const int lane = tid & 63;
                const int pre = __popcll(msk & ((1ull << lane) - 1ull));
                __syncthreads();
                if (lane == 0) shi[tid >> 6] = __popcll(msk);
                __syncthreads();
                int woff = 0;
                for (int k = 0; k < (tid >> 6); ++k) woff += shi[k];
                if (keep) S.Q[K + woff + pre] = p;
                K += shi[0] + shi[1] + shi[2] + shi[3];
            }
        }
        if (!fl && K < 3) fl = CA_FLAG_DEGENERATE;
        __syncthreads();

        // chord lengths and their FP64 exclusive scan: L_j = sum_{i<j} |Q_{i+1} - Q_i|
        double L = 0.0;
        double area2 = 0.0;                    // twice the signed area of the cleaned polygon
        if (!fl) {
            double carry = 0.0;
            const cf q0 = S.Q[0];
            for (int base = 0; base < K; base += kRsNT) {
                const int j = base + tid;
                double hj = 0.0;
                if (j < K) {
                    const cf a = S.Q[j], b = S.Q[j + 1 < K ? j + 1 : 0];
                    const float dx = b.x - a.x, dy = b.y - a.y;
                    const float hf = sqrtf(dx * dx + dy * dy);
                    hj = hf;
                    S.h[j] = hf;
                    area2 += (double)(a.x - q0.x) * dy - (double)(a.y - q0.y) * dx;
                }
                double tot;
                const double pre = rs_exscan(hj, shd, tot);
                if (j < K) S.s[j] = carry + pre;
                carry += tot;
            }
            L = carry;
            if (!(L > 0.0)) fl = CA_FLAG_DEGENERATE;
            area2 = rs_sum(area2, shd);
        }
        __syncthreads();
        const double invL = fl ? 0.0 : 1.0 / L;
        if (!fl) {
            for (int j = tid; j < K; j += kRsNT) {
                S.s[j] *= invL;
                S.h[j] = (float)((double)S.h[j] * invL);
            }
            if (tid == 0) S.s[K] = 1.0;
        }
        __syncthreads();
        if (!fl && mode == CA_RESAMPLE_SPLINE) {
            // right-hand sides 6 (D_j - D_{j-1})
            for (int j = tid; j < K; j += kRsNT) {
                const int jm = j > 0 ? j - 1 : K - 1, jp = j + 1 < K ? j + 1 : 0;
                const cf qm = S.Q[jm], q = S.Q[j], qp = S.Q[jp];
                const float hm = S.h[jm], hj = S.h[j];
                const float Dx = (qp.x - q.x) / hj, Dy = (qp.y - q.y) / hj;
                const float Dmx = (q.x - qm.x) / hm, Dmy = (q.y - qm.y) / hm;
                S.rhs[j] = {6.0f * (Dx - Dmx), 6.0f * (Dy - Dmy)};
            }
            __syncthreads();
            const int nchunks = (K + kRsC - 1) / kRsC;
            for (int g = tid; g < nchunks; g += kRsNT) rs_local_solve(S, K, g * kRsC);
            __syncthreads();
        }

        // evaluation at t_n = n/N: thread owns knots [a, b) and the nodes in [s_a N, s_b N)
        double sx = 0.0, sy = 0.0;
        if (!fl) {
            const int per = (K + kRsNT - 1) / kRsNT;
            const int a = tid * per;
            const int b = min(a + per, K);
            const float il = (float)invL;
            if (a < b) {
                const double dN = (double)N;
                const int nlo = (int)ceil(S.s[a] * dN);
                const int nhi = (b == K) ? N : (int)ceil(S.s[b] * dN);
                int j = a;
                for (int nn = nlo; nn < nhi; ++nn) {
                    while (j + 1 < b && S.s[j + 1] * dN <= (double)nn) ++j;
                    const int jp = j + 1 < K ? j + 1 : 0;
                    const float hj = S.h[j];
                    const float bb = (float)((double)nn / dN - S.s[j]);
                    const float aa = hj - bb;
                    const cf qj = S.Q[j], qp = S.Q[jp];
                    cf z;
                    if (mode == CA_RESAMPLE_SPLINE) {
                        const cf mj = S.M[j], mp = S.M[jp];
                        const float ih = 1.0f / hj;
                        const float ca = aa * aa * aa * ih * (1.0f / 6.0f);
                        const float cb = bb * bb * bb * ih * (1.0f / 6.0f);
                        const float h6 = hj * hj * (1.0f / 6.0f);
                        const float ua = aa * ih, ub = bb * ih;
                        z.x = mj.x * ca + mp.x * cb + (qj.x - mj.x * h6) * ua + (qp.x - mp.x * h6) * ub;
                        z.y = mj.y * ca + mp.y * cb + (qj.y - mj.y * h6) * ua + (qp.y - mp.y * h6) * ub;
                    } else {
                        const float ub = bb / hj, ua = 1.0f - ub;
                        z.x = qj.x * ua + qp.x * ub;
                        z.y = qj.y * ua + qp.y * ub;
                    }
                    z.x *= il;
                    z.y *= il;
                    o[nn] = z;
                    sx += z.x;
                    sy += z.y;
                }
            }
        }
        sx = rs_sum(sx, shd);
        sy = rs_sum(sy, shd);
        const float mx = (float)(sx / N), my = (float)(sy / N);
        double q2 = 0.0;
        for (int nn = tid; nn < N; nn += kRsNT) {
            cf z;
            if (fl) {
                z = {0.0f, 0.0f};
            } else {
                z = o[nn];
                z.x -= mx;
                z.y -= my;
            }
            o[nn] = z;
            q2 = fma((double)z.x, (double)z.x, fma((double)z.y, (double)z.y, q2));
        }
        q2 = rs_sum(q2, shd);
        if (tid == 0) {
            if (norms) norms[c] = q2 / N;
            if (flags) flags[c] = fl ? fl : (area2 < 0.0 ? CA_FLAG_CLOCKWISE : 0u);
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------- fast path
// One wave per curve, no workgroup barriers.  Pass 1 streams the polygon once
// for the perimeter (FP64) and rejects curves that need the general path
// (duplicate or non-finite vertices, fewer than 3 or more than the cap).
// Pass 2 walks the curve in tiles of kFtK knots (consecutive tiles share one
// knot): the tile and a halo of kRsW + 1 knots on each side are staged in
// LDS, chord lengths, right-hand sides, tile-relative arc-length parameters
// and the local spline solves are computed there, and every output node
// whose parameter falls in the tile is evaluated by the lane that owns its
// segment (a binary search over the tile's knots only for tiles with many
// nodes per knot).  Pass 3 centres the nodes and accumulates their norm.
constexpr int kFtC = 7;                    // knots per lane in the local solve
constexpr int kFtW = 6;                    // solve window on each side, curves of >= kFtBigM vertices
constexpr int kFtBigM = 256;
constexpr int kFtK = 64 * kFtC;            // knots per tile
constexpr int kFtH = kRsW + 1;             // halo on each side (the widest window + 1)
constexpr int kFtP = kFtK + 2 * kFtH;      // staged knots
constexpr int kFtSegMax = 24;              // most nodes per lane for lane-owned segments
// Per-knot LDS arrays are not padded: the local solve and the scan give lane
// l the knots [7 l, 7 l + 7), a stride coprime to the bank count.  The
// spline moments share the right-hand sides' array (the solve's sweeps read
// every right-hand side before the back substitution writes a moment), which
// with 7 knots per lane keeps a wave's LDS at ~11 KB: three waves per SIMD.
constexpr int kFtPP = kFtP;
constexpr int kFtKP = kFtK + 1;
__device__ __forceinline__ int kp(int i) { return i; }

__device__ __forceinline__ int wrapm(int i, int m) {
    while (i < 0) i += m;
    while (i >= m) i -= m;
    return i;
}

__device__ __forceinline__ double wave_sum_d(double v) { return team_sum<64>(v); }

// Hardware reciprocal (1 ulp): the spline quantities are positive, finite and
// far from the denormal range on the fast path.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
// Hardware square root (1 ulp), for chord lengths of the fast path: their
// squares are positive normal numbers there, and a zero or non-finite chord
// sends the curve to the general kernel.
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
// Lane i receives lane (i + 1) mod 64, resp. (i - 1) mod 64 (DPP wave
// rotations; the whole wave must be active, so every lane is written and no
// previous value is kept).
__device__ __forceinline__ float wave_rol1(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x134, 0xF, 0xF, false));
}
__device__ __forceinline__ float wave_ror1(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x13C, 0xF, 0xF, false));
}
__device__ __forceinline__ cf wave_rol1(cf z) { return {wave_rol1(z.x), wave_rol1(z.y)}; }
__device__ __forceinline__ cf wave_ror1(cf z) { return {wave_ror1(z.x), wave_ror1(z.y)}; }

// Inclusive scan of a double over the wave: shifts by 1, 2, 4, 8 inside each
// row of 16 lanes (DPP row_shr; lanes without a source add 0), then the row
// totals read from lanes 15, 31, 47.  The whole wave must be active.
template <int CTRL> __device__ __forceinline__ double dpp_shr_d(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double wave_incl_scan(double x, int lane) {
    x += dpp_shr_d<0x111>(x);
    x += dpp_shr_d<0x112>(x);
    x += dpp_shr_d<0x114>(x);
    x += dpp_shr_d<0x118>(x);
    const double r0 = rdlane(x, 15), r1 = rdlane(x, 31), r2 = rdlane(x, 47);
    const int row = lane >> 4;
    const double off = row == 0 ? 0.0 : (row == 1 ? r0 : (row == 2 ? r0 + r1 : (r0 + r1) + r2));
    return x + off;
}

__global__ __launch_bounds__(64, 3) void k_resample_fast(const cf* __restrict__ raw, const int64_t* __restrict__ raw_off,
                                                      int64_t num_curves, const int64_t* __restrict__ out_off,
                                                      cf* __restrict__ out, double* __restrict__ norms,
                                                      uint32_t* __restrict__ flags, int mode,
                                                      int* __restrict__ slow_count, int* __restrict__ slow_list) {
    __shared__ cf sP[kFtPP];
    __shared__ float sH[kFtPP];
    __shared__ cf sR[kFtPP > kFtKP ? kFtPP : kFtKP];
    __shared__ float sS[kFtKP];
    cf* const sM = sR;                         // moments over the right-hand sides
    const int64_t c = blockIdx.x;
    if (c >= num_curves) return;
    const int lane = threadIdx.x;
    const int64_t r0 = raw_off[c];
    const int64_t mraw = raw_off[c + 1] - r0;
    const int64_t o0 = out_off[c];
    const int N = (int)(out_off[c + 1] - o0);
    cf* o = out + o0;
    const cf* P = raw + r0;
    bool general = (mraw < 3 || mraw > kRsMCap || N < 1);
    const int M = general ? 0 : (int)mraw;

    // pass 1: perimeter, duplicates, non-finite values.  Eight vertices per
    // lane per group of 512, loads issued together; the successor of vertex j
    // comes from the next lane through a wave rotation (lane 63: the first
    // lane of the next group), so only the vertex after the group is loaded
    // twice.  Groups that end before the last vertex skip the range checks.
    // The per-lane order of the chord sum is j = lane, lane + 64, ...
    double Ls = 0.0;
    float ar = 0.0f;
    int bad = 0;
    constexpr int kP1 = 8;
    const cf p0 = M > 0 ? P[0] : cf{0.0f, 0.0f};
    auto group = [&](auto full, int j0) {
        constexpr bool kFull = decltype(full)::value;
        cf a[kP1 + 1], rot[kP1 + 1];
#pragma unroll
        for (int u = 0; u < kP1; ++u) {
            const int j = j0 + lane + 64 * u;
            a[u] = P[(kFull || j < M) ? j : 0];
        }
        a[kP1] = P[(kFull || j0 + 64 * kP1 < M) ? j0 + 64 * kP1 : 0];   // the same on every lane
#pragma unroll
        for (int u = 0; u < kP1; ++u) rot[u] = wave_rol1(a[u]);
        rot[kP1] = a[kP1];
#pragma unroll
        for (int u = 0; u < kP1; ++u) {
            const int j = j0 + lane + 64 * u;
            // lane 63's successor is lane 0's vertex of the next step, which
            // the rotation of that step has put in lane 63
            cf b = lane == 63 ? rot[u + 1] : rot[u];
            if (!kFull && j + 1 == M) b = p0;  // closing chord back to vertex 0
            if (kFull || j < M) {
                const float dx = b.x - a[u].x, dy = b.y - a[u].y;
                const float h = fsqrt(dx * dx + dy * dy);
                if (!(h > 0.0f) || !isfinite(h)) bad = 1;
                Ls += (double)h;
                // twice the signed area: sum of (a - p0) x (b - a) over the chords
                ar = fmaf(a[u].x - p0.x, dy, fmaf(-(a[u].y - p0.y), dx, ar));
            }
        }
    };
    for (int j0 = 0; j0 < M; j0 += 64 * kP1) {
        if (j0 + 64 * kP1 < M) group(std::true_type{}, j0);
        else group(std::false_type{}, j0);
    }
    general = general || (__ballot(bad) != 0ull);
    if (general) {
        if (lane == 0) {
            const int pos = atomicAdd(slow_count, 1);
            slow_list[pos] = (int)c;
        }
        return;
    }
    const double L = wave_sum_d(Ls);
    const double area2 = wave_sum_d((double)ar);
    const double invL = 1.0 / L;
    const double uN = L / (double)N;           // arc length between output nodes
    // node index of an arc length, up to rounding: the tile bounds below are
    // the same expression of the same carry for consecutive tiles, so every
    // node is placed exactly once whatever the rounding
    const double inv_uN = (double)N / L;

    // pass 2: tiles of kFtK knots starting at a; segments [a, a + kFtK - 1)
    double carry = 0.0;                        // arc length at knot a
    double sx = 0.0, sy = 0.0;
    constexpr int kStage = (kFtP + 63) / 64;   // staged vertices per lane
    cf pre[kStage] = {};                       // next tile's vertices, loaded ahead
    // staged knot j of the tile at a reads vertex a - kFtH + j (cyclic); with
    // M >= kFtP one correction by M suffices
    const bool wide = M >= kFtP;
    auto vert = [&](int j) { return wide ? (j < 0 ? j + M : (j >= M ? j - M : j)) : wrapm(j, M); };
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
        const int i = lane + 64 * u;
        if (64 * (u + 1) <= kFtP || i < kFtP) pre[u] = P[vert(i - kFtH)];
    }
    // LDS index of staged knot lane + 64 u
    const int kpl = kp(lane);
    for (int a = 0; a < M; a += kFtK - 1) {
        const bool last = (a + kFtK - 1 >= M);
        const int kt = last ? (M - a + 1) : kFtK;       // knots in this tile incl. the right end
        // stage knots a - kFtH .. a + kFtK + kFtH - 1 (cyclic) with their chord
        // lengths and, for the spline, the right-hand sides 6 (D_i - D_{i-1}),
        // all from registers: the successor of staged knot lane + 64 u is the
        // next lane's (lane 63: lane 0 of u + 1), the slope D_{i-1} the
        // previous lane's (lane 0: lane 63 of u - 1)
        // (a rotation of step u + 1 puts lane 0's knot in lane 63, one of step
        // u - 1 lane 63's slope in lane 0)
        auto stage = [&](auto spline) {
            constexpr bool kSpline = decltype(spline)::value;
            cf rot[kStage];
#pragma unroll
            for (int u = 0; u < kStage; ++u) rot[u] = wave_rol1(pre[u]);
            cf dmprev = {0.0f, 0.0f};
#pragma unroll
            for (int u = 0; u < kStage; ++u) {
                const int i = lane + 64 * u;
                // every step but the last stages only knots below kFtP - 1
                const bool kInside = 64 * (u + 1) <= kFtP - 1;   // folds once the loop is unrolled
                const cf q = (u + 1 < kStage && lane == 63) ? rot[u + 1 < kStage ? u + 1 : u] : rot[u];
                const float dx = q.x - pre[u].x, dy = q.y - pre[u].y;
                const float h = fsqrt(dx * dx + dy * dy);
                if (kInside || i < kFtP) sP[kpl + kp(64 * u)] = pre[u];
                if (kInside || i < kFtP - 1) sH[kpl + kp(64 * u)] = h;
                if constexpr (kSpline) {
                    const float ih = frcp(h);
                    const cf d = {dx * ih, dy * ih};
                    const cf dr = wave_ror1(d);
                    const cf dm = lane == 0 ? dmprev : dr;
                    if ((u > 0 || i >= 1) && (kInside || i < kFtP - 1))
                        sR[kpl + kp(64 * u)] = {6.0f * (d.x - dm.x), 6.0f * (d.y - dm.y)};
                    dmprev = dr;
                }
            }
        };
        if (mode == CA_RESAMPLE_SPLINE) stage(std::true_type{});
        else stage(std::false_type{});
        // start loading the next tile's vertices (no wrap-around except near the end)
        if (!last) {
            const int b0 = a + kFtK - 1 - kFtH;
            if (b0 + kFtP <= M) {
#pragma unroll
                for (int u = 0; u < kStage; ++u) {
                    const int i = lane + 64 * u;
                    if (64 * (u + 1) <= kFtP || i < kFtP) pre[u] = P[b0 + i];
                }
            } else {
#pragma unroll
                for (int u = 0; u < kStage; ++u) {
                    const int i = lane + 64 * u;
                    if (64 * (u + 1) <= kFtP || i < kFtP) pre[u] = P[vert(b0 + i)];
                }
            }
        }
        wave_lds_sync();
        // tile-relative arc length: lane owns local knots [kFtC lane, kFtC lane + kFtC)
        float loc[kFtC];
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < kFtC; ++k) {
            loc[k] = (float)acc;
            acc += (double)sH[kp(kFtH + kFtC * lane + k)];
        }
        const double base = wave_incl_scan(acc, lane) - acc;   // arc length from knot a to knot a + kFtC lane
#pragma unroll
        for (int k = 0; k < kFtC; ++k) sS[kp(kFtC * lane + k)] = (float)(base + (double)loc[k]);
        // arc length from knot a to knot a + kt - 1 (tile end), exact in FP64
        double span;
        {
            const int e = kt - 1;              // local index of the right end
            const int el = e / kFtC, ek = e % kFtC;
            double part = 0.0;                 // same on every lane (el is wave-uniform)
#pragma unroll
            for (int k = 0; k < kFtC; ++k)
                if (k < ek) part += (double)sH[kp(kFtH + kFtC * el + k)];
            span = rdlane(base, el) + part;
        }
        wave_lds_sync();
        if (mode == CA_RESAMPLE_SPLINE) {
            // local solve for knots [kFtC lane, kFtC (lane + 1)), window W each
            // side: W = kFtW for curves of at least kFtBigM vertices (parameter
            // step h <= 1/kFtBigM), the full halo otherwise (the truncation
            // reaches the nodes through h^2)
            auto solve = [&](auto win) {
                constexpr int W = decltype(win)::value;
                float al[kFtC];
                cf de[kFtC];
                const int i0 = kFtH + kFtC * lane;           // staged index of the chunk's first knot
                float hprev = sH[kp(i0 - W - 1)];
                float alpha = 0.0f;
                cf delta = {0.0f, 0.0f};
#pragma unroll
                for (int i = 0; i < W + kFtC; ++i) {
                    const int j = i0 - W + i;
                    const float hj = sH[kp(j)];
                    const cf d = sR[kp(j)];
                    const float b = 2.0f * (hprev + hj);
                    if (i == 0) {
                        alpha = b;
                        delta = d;
                    } else {
                        const float f = hprev * frcp(alpha);
                        alpha = b - f * hprev;
                        delta = {d.x - f * delta.x, d.y - f * delta.y};
                    }
                    hprev = hj;
                    if (i >= W) { al[i - W] = alpha; de[i - W] = delta; }
                }
                const int e = i0 + kFtC;
                float beta = 0.0f, anext = 0.0f;
                cf eps = {0.0f, 0.0f};
#pragma unroll
                for (int i = W - 1; i >= 0; --i) {
                    const int j = e + i;
                    const float hj = sH[kp(j)], hjm = sH[kp(j - 1)];
                    const cf d = sR[kp(j)];
                    const float b = 2.0f * (hjm + hj);
                    if (i == W - 1) {
                        beta = b;
                        eps = d;
                    } else {
                        const float g = hj * frcp(beta);
                        beta = b - g * anext;
                        eps = {d.x - g * eps.x, d.y - g * eps.y};
                    }
                    anext = hjm;
                }
                const float ae = sH[kp(e - 1)];
                const float aL = al[kFtC - 1];
                const cf dL = de[kFtC - 1];
                const float iaL = frcp(aL);
                const float iden = frcp(beta - ae * ae * iaL);
                cf Mn = {(eps.x - ae * dL.x * iaL) * iden, (eps.y - ae * dL.y * iaL) * iden};
                wave_lds_sync();                   // every right-hand side is read before moments overwrite them
#pragma unroll
                for (int i = kFtC - 1; i >= 0; --i) {
                    const float cj = sH[kp(i0 + i)];
                    const float ia = frcp(al[i]);
                    const cf Mi = {(de[i].x - cj * Mn.x) * ia, (de[i].y - cj * Mn.y) * ia};
                    sM[kp(kFtC * lane + i)] = Mi;
                    Mn = Mi;
                }
            };
            if (M >= kFtBigM) solve(std::integral_constant<int, kFtW>{});
            else solve(std::integral_constant<int, kRsW>{});
        }
        wave_lds_sync();
        // output nodes with arc length in [carry, carry + span) (up to N on the last tile)
        const int nlo = (int)ceil(carry * inv_uN);
        const int nhi = last ? N : min(N, (int)ceil((carry + span) * inv_uN));
        const float il = (float)invL;
        auto upar = [&](int nn) { return (float)((double)nn * uN - carry); };
        // Node nn lies on segment j = the largest j in [0, kt - 2] with
        // sS[j] <= upar(nn) (j = 0 below sS[0]).  Since upar and sS are
        // non-decreasing, the nodes of lane l's segments [kFtC l, kFtC (l + 1)) are the
        // contiguous range [first(kFtC l), first(kFtC (l + 1))), first(j) being the
        // smallest node at or after sS[j]; each lane places its own range with
        // one LDS round trip per node.  Tiles with many nodes per knot fall
        // back to one node per lane and a binary search.
        const int j0 = kFtC * lane;
        int ns = nhi;
        if (j0 == 0) {
            ns = nlo;
        } else if (j0 <= kt - 2) {
            const float s0 = sS[kp(j0)];
            int e = (int)ceil((carry + (double)s0) * inv_uN);
            e = max(nlo, min(nhi, e));
            while (e > nlo && upar(e - 1) >= s0) --e;
            while (e < nhi && upar(e) < s0) ++e;
            ns = e;
        }
        int ne = __shfl_down(ns, 1, 64);
        if (lane == 63) ne = nhi;
        const bool seg = team_max<64>(ne - ns) <= kFtSegMax;
        float sk[kFtC];                        // this lane's knot parameters
#pragma unroll
        for (int k = 1; k < kFtC; ++k) {
            const float v = sS[kp(j0 + k)];    // j0 + k <= kFtK - 1: inside sS
            sk[k] = (j0 + k <= kt - 2) ? v : 3.0e38f;
        }
        const int nbeg = seg ? ns : nlo + lane, nend = seg ? ne : nhi, nstep = seg ? 1 : 64;
        for (int nn = nbeg; nn < nend; nn += nstep) {
            const float u = upar(nn);
            int j;
            if (seg) {
                j = j0;
#pragma unroll
                for (int k = 1; k < kFtC; ++k) j += sk[k] <= u ? 1 : 0;
            } else {
                int lo = 0, hi = kt - 2;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (sS[kp(mid)] <= u) lo = mid; else hi = mid - 1;
                }
                j = lo;
            }
            const float hj = sH[kp(kFtH + j)];
            const float bb = u - sS[kp(j)];
            const float aa = hj - bb;
            const cf qj = sP[kp(kFtH + j)], qp = sP[kp(kFtH + j + 1)];
            cf z;
            if (mode == CA_RESAMPLE_SPLINE) {
                const cf mj = sM[kp(j)], mp = sM[kp(j + 1)];
                const float ih = frcp(hj);
                const float ca = aa * aa * aa * ih * (1.0f / 6.0f);
                const float cb = bb * bb * bb * ih * (1.0f / 6.0f);
                const float h6 = hj * hj * (1.0f / 6.0f);
                const float ua = aa * ih, ub = bb * ih;
                z.x = mj.x * ca + mp.x * cb + (qj.x - mj.x * h6) * ua + (qp.x - mp.x * h6) * ub;
                z.y = mj.y * ca + mp.y * cb + (qj.y - mj.y * h6) * ua + (qp.y - mp.y * h6) * ub;
            } else {
                const float ub = bb * frcp(hj), ua = 1.0f - ub;
                z.x = qj.x * ua + qp.x * ub;
                z.y = qj.y * ua + qp.y * ub;
            }
            z.x *= il;
            z.y *= il;
            o[nn] = z;
            sx += z.x;
            sy += z.y;
        }
        carry += span;
        wave_lds_sync();
    }
    // pass 3: centre on the node mean, norms (other lanes wrote these nodes)
    __syncthreads();
    sx = wave_sum_d(sx);
    sy = wave_sum_d(sy);
    const float mx = (float)(sx / N), my = (float)(sy / N);
    double q2 = 0.0;
    // eight loads in flight per lane; groups that end before N skip the range checks
    auto centre = [&](auto full, int n0) {
        constexpr bool kFull = decltype(full)::value;
        cf zz[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int nn = n0 + lane + 64 * u;
            if (kFull || nn < N) zz[u] = o[nn];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int nn = n0 + lane + 64 * u;
            if (kFull || nn < N) {
                cf z = zz[u];
                z.x -= mx;
                z.y -= my;
                o[nn] = z;
                q2 = fma((double)z.x, (double)z.x, fma((double)z.y, (double)z.y, q2));
            }
        }
    };
    for (int n0 = 0; n0 < N; n0 += 64 * 8) {
        if (n0 + 64 * 8 <= N) centre(std::true_type{}, n0);
        else centre(std::false_type{}, n0);
    }
    q2 = wave_sum_d(q2);
    if (lane == 0) {
        if (norms) norms[c] = q2 / N;
        if (flags) flags[c] = area2 < 0.0 ? CA_FLAG_CLOCKWISE : 0u;
    }
}

__global__ void k_zero_int(int* p) { *p = 0; }

hipError_t launch_resample(const void* raw, const int64_t* raw_off, int64_t num_curves,
                           const int64_t* out_off, void* out, double* norms, uint32_t* flags, int mode,
                           void* scratch, int64_t slot_bytes, int64_t slots, int* slow_count, int* slow_list,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, s, slow_count);
    hipLaunchKernelGGL(k_resample_fast, dim3((unsigned)num_curves), dim3(64), 0, s, (const cf*)raw, raw_off,
                       num_curves, out_off, (cf*)out, norms, flags, mode, slow_count, slow_list);
    const int64_t grid = num_curves < slots ? num_curves : slots;
    hipLaunchKernelGGL(k_resample, dim3((unsigned)grid), dim3(kRsNT), 0, s, (const cf*)raw, raw_off,
                       num_curves, out_off, (cf*)out, norms, flags, mode, (unsigned char*)scratch,
                       slot_bytes, (const int*)slow_count, (const int*)slow_list);
    return hipGetLastError();
}

int64_t resample_slot_bytes() { return rs_slot_bytes(); }
int resample_max_raw() { return kRsMCap; }

}  // namespace ca
