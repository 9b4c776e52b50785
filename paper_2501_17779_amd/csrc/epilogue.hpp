// Shared epilogue of the alignment kernels: candidate selection, FP64
// re-scoring of C at the candidate shifts, theta and e0 (Algorithm 2's final
// step, with the FP64 energy of Eq. disc-energy).
#pragma once

#include <math.h>

#include "fft_engines.hpp"

namespace ca {

// ------------------------------------------------------------ shared epilogue
// Selection state of the FP64 re-scoring: best |C64|^2 (smallest shift on
// equal values), its C64, and the second best value.
struct Pick {
    double best = -1.0, second = -1.0, re = 0.0, im = 0.0;
    int shift = -1, count = 0;
    __device__ __forceinline__ void offer(int c, double r, double i) {
        const double m = r * r + i * i;
        if (m > best || (m == best && c < shift)) {
            second = best; best = m; shift = c; re = r; im = i;
        } else if (m > second) {
            second = m;
        }
        ++count;
    }
};

__device__ __forceinline__ float wrap_pi(float a) {
    const float pi = 3.14159265358979323846f;
    return (a <= -pi) ? pi : a;
}
__device__ __forceinline__ double wrap_pi(double a) {
    const double pi = 3.14159265358979323846;
    return (a <= -pi) ? pi : a;
}

// FP64 arc tangent for the opt-in FP64 theta, kept out of line: inlined, its
// polynomial constants are hoisted into registers for the whole persistent
// loop (and spilled), although only pairs with theta_fp64 set use them.
__device__ __attribute__((noinline)) double atan2_fp64(double y, double x) { return atan2(y, x); }

__device__ __forceinline__ void finish(ca_result_t& res, const Pick& pk, int n, double n1, double n2,
                                       double d1, double d2, double epsD, bool capped,
                                       double theta_path, int theta64) {
    uint32_t flags = 0;
    const double c64 = sqrt(pk.best);
    if (pk.count > 1) flags |= CA_FLAG_RESCORED;
    if (capped) flags |= CA_FLAG_CAND_CAPPED;
    // relative gap (c - s) / c = (c^2 - s^2) / (c^2 + c s): the difference of
    // the squares is formed in FP64, the rest only needs FP32
    float gap;
    if (pk.count > 1 && pk.second >= 0.0)
        gap = (float)(pk.best - pk.second) *
              __builtin_amdgcn_rcpf((float)(pk.best + c64 * (double)__builtin_amdgcn_sqrtf((float)pk.second)));
    else
        gap = (float)(d1 - d2) * __builtin_amdgcn_rcpf((float)d1);
    if (gap < kNearTie) flags |= CA_FLAG_NEAR_TIE;
    double th = theta_path;
    if (theta64) {
        th = wrap_pi(atan2_fp64(pk.im, pk.re));
        flags |= CA_FLAG_THETA_FP64;
    }
    res.shift = pk.shift;
    res.flags = flags;
    res.theta = th;
    res.err_est = 2.0f * (float)epsD * __builtin_amdgcn_rcpf((float)d1);
    res.gap = gap;
    res.e0 = n1 + n2 - c64 * (2.0 / (double)n);
}

__device__ __forceinline__ bool special_case(ca_result_t& res, double n1, double n2, double bv) {
    res.shift = 0;
    res.theta = 0.0;
    res.err_est = 0.0f;
    res.gap = 0.0f;
    if (!(isfinite(n1) && isfinite(n2) && isfinite(bv))) {
        res.flags = CA_FLAG_NONFINITE;
        res.e0 = __builtin_nan("");
        return true;
    }
    if (!(n1 > 0.0) || !(n2 > 0.0) || !(bv > 0.0)) {
        res.flags = CA_FLAG_DEGENERATE;
        res.e0 = n1 + n2;
        return true;
    }
    return false;
}

// --------------------------------------------------------------- team engine
// Layouts of the LDS copy of curve 2's nodes read by the FP64 re-scoring:
// kZPad: node i at lpad<N>(i); kZTwice: node i at i and at N + i, so that the
// shifted reads (t + T q - c) mod N become one base plus constant offsets.
enum { kZPad = 0, kZTwice = 1 };

// Epilogue of one pair held by a team: d[q] = D[t + T q] (D = n conj C),
// a0[q] = z1[t + T q] (FP32 nodes of curve 1), zb = LDS copy of curve 2's
// nodes in layout ZL, cand = the team's candidate list in LDS.
// With OWN_NORMS the n1 and n2 arguments are ignored and n1 = (1/n) sum |z1|^2
// and n2 = (1/n) sum |z2|^2 are formed here: under the top-two rule in the
// pass that re-scores the best shift, whose FP64 conversions of both curves'
// nodes they share (n2 then sums curve 2's nodes in the shifted order that
// pass reads them).  With FUSE2 the window's candidates are re-scored two per
// pass; with PRUNE (window rule) the argmax and its two neighbours are
// re-scored in one pass and only the window shifts whose bound can still reach
// the best value after it.
// Returns the finished result (every lane).
template <int N, int T, int ZL = kZPad, bool FUSE2 = false, bool OWN_NORMS = false, bool PRUNE = false>
__device__ __forceinline__ ca_result_t team_epilogue(const cf (&d)[N / T], const cf (&a0)[N / T],
                                                     const cf* zb, int* cand, int t, double n1, double n2,
                                                     int rescore, int theta64,
                                                     double err_u = num<float>::u) {
    constexpr int R = N / T;
    constexpr int kNone = 0x7fffffff;
    // |D|^2, and per lane the largest and second largest value
    float m2[R];
    float b1 = -1.0f, b2 = -1.0f;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        m2[q] = norm2(d[q]);
        // new second largest = median of (largest, second largest, value)
        b2 = __builtin_amdgcn_fmed3f(b1, b2, m2[q]);
        b1 = fmaxf(b1, m2[q]);
    }
    // best value, then the smallest shift holding it
    const float bv = team_max<T>(b1);
    int bl = kNone;
#pragma unroll
    for (int q = R - 1; q >= 0; --q)
        if (m2[q] == bv) bl = t + T * q;
    int bi = team_min<T>(bl);
    if (bi == kNone) bi = 0;     // no finite maximum: flagged by special_case
    // runner-up value over every other shift: the lane holding bi offers its
    // second largest value, the others their largest
    const float cv = team_max<T>((bi & (T - 1)) == t ? b2 : b1);
    auto runner_up = [&]() {
        int cl = kNone;
#pragma unroll
        for (int q = R - 1; q >= 0; --q) {
            const int idx = t + T * q;
            if (m2[q] == cv && idx != bi) cl = idx;
        }
        const int c = team_min<T>(cl);
        return c == kNone ? ((bi + 1) & (N - 1)) : c;
    };

    auto zat = [&](int c, int q) {
        return (ZL == kZTwice) ? zb[((t - c) & (N - 1)) + T * q] : zb[lpad<N>((t + T * q - c) & (N - 1))];
    };
    // FP64 C at shift c (times n): sum over k of conj(z1[k]) z2[k + c]
    auto dot64 = [&](int c, double& re, double& im) {
        re = 0.0;
        im = 0.0;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const cf zz = zat(c, q);
            const double ax = a0[q].x, ay = a0[q].y, bx = zz.x, by = zz.y;
            re = fma(ax, bx, fma(ay, by, re));
            im = fma(ay, bx, fma(-ax, by, im));
        }
        re = team_sum<T>(re);
        im = team_sum<T>(im);
    };
    // theta in FP32 from the FP64 re-scored C at the chosen shift (every lane
    // holds it: no selection of the transform's value across registers and
    // lanes, and no less accurate than arg of the transform's C)
    auto theta_of = [](const Pick& pk) { return (double)wrap_pi(atan2f((float)pk.im, (float)pk.re)); };

    ca_result_t res;
    if (OWN_NORMS && rescore != CA_RESCORE_WINDOW) {
        // top-two rule: the best shift is re-scored before the norms are
        // needed, and the same pass sums |z1|^2 and |z2|^2
        double re = 0.0, im = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const cf zz = zat(bi, q);
            const double ax = a0[q].x, ay = a0[q].y, bx = zz.x, by = zz.y;
            s1 = fma(ax, ax, fma(ay, ay, s1));
            s2 = fma(bx, bx, fma(by, by, s2));
            re = fma(ax, bx, fma(ay, by, re));
            im = fma(ay, bx, fma(-ax, by, im));
        }
        re = team_sum<T>(re);
        im = team_sum<T>(im);
        n1 = team_sum<T>(s1) / N;
        n2 = team_sum<T>(s2) / N;
        if (special_case(res, n1, n2, (double)bv)) return res;
        const double d1 = (double)__builtin_amdgcn_sqrtf(bv), d2 = (double)__builtin_amdgcn_sqrtf(fmaxf(cv, 0.0f));
        const double epsD = (double)((float)(kErrScale * err_u * (double)ilog2_ceil(N) * N * N) *
                                     __builtin_amdgcn_sqrtf((float)(n1 * n2)));
        Pick pk;
        pk.offer(bi, re, im);
        if (d1 - d2 < 2.0 * epsD) {
            const int ci = runner_up();
            dot64(ci, re, im);
            pk.offer(ci, re, im);
        }
        finish(res, pk, N, n1, n2, d1, d2, epsD, false, theta_of(pk), theta64);
        return res;
    }
    if (OWN_NORMS) {
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const cf zz = zat(0, q);
            const double ax = a0[q].x, ay = a0[q].y, bx = zz.x, by = zz.y;
            s1 = fma(ax, ax, fma(ay, ay, s1));
            s2 = fma(bx, bx, fma(by, by, s2));
        }
        n1 = team_sum<T>(s1) / N;
        n2 = team_sum<T>(s2) / N;
    }
    if (special_case(res, n1, n2, (double)bv)) return res;
    // |D| of the best and runner-up and the error bound only steer the choice
    // of shifts to re-score and the reported gap: the hardware square root
    // (1 ulp) is ample there
    const double d1 = (double)__builtin_amdgcn_sqrtf(bv), d2 = (double)__builtin_amdgcn_sqrtf(fmaxf(cv, 0.0f));
    const double epsD = (double)((float)(kErrScale * err_u * (double)ilog2_ceil(N) * N * N) *
                                 __builtin_amdgcn_sqrtf((float)(n1 * n2)));
    const bool two = d1 - d2 < 2.0 * epsD;

    // candidate list (team-uniform order: by register, then by lane)
    int cnt = 0;
    bool capped = false, pruned = false;
    Pick pk;
    if (rescore == CA_RESCORE_WINDOW) {
        const double thr = d1 - 2.0 * epsD;
        float thr2 = thr > 0.0 ? (float)(thr * thr) : 0.0f;
        auto count_at = [&](float th) {
            int loc = 0;
#pragma unroll
            for (int q = 0; q < R; ++q) loc += (m2[q] >= th) ? 1 : 0;
            return team_sum<T>(loc);
        };
        if (count_at(thr2) > kCandCap) {
            // window wider than the cap: keep (about) the kCandCap largest
            // values, found by bisection on the threshold
            capped = true;
            float lo = thr2, hi = bv;
            for (int it = 0; it < 32 && lo < hi; ++it) {
                const float mid = lo + 0.5f * (hi - lo);
                if (mid <= lo || mid >= hi) break;
                if (count_at(mid) > kCandCap) lo = mid; else hi = mid;
            }
            thr2 = hi;
        }
        int skip0 = -1, skip1 = -1, skip2 = -1;
        if constexpr (PRUNE) {
            // The argmax and its two neighbours in one FP64 pass, then only
            // the window shifts whose bound |D| + epsD can still reach the
            // best n |C| found (less the near-tie gap) are re-scored: a shift
            // left out is strictly below the final best and cannot be within
            // the near-tie gap of it, so the choice is the full window's.
            const int cm = (bi + N - 1) & (N - 1), cp = (bi + 1) & (N - 1);
            double r0 = 0.0, j0 = 0.0, r1 = 0.0, j1 = 0.0, r2 = 0.0, j2 = 0.0;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const cf u = zat(cm, q), w = zat(bi, q), x = zat(cp, q);
                const double ax = a0[q].x, ay = a0[q].y;
                const double ux = u.x, uy = u.y, wx = w.x, wy = w.y, xx = x.x, xy = x.y;
                r0 = fma(ax, ux, fma(ay, uy, r0));
                j0 = fma(ay, ux, fma(-ax, uy, j0));
                r1 = fma(ax, wx, fma(ay, wy, r1));
                j1 = fma(ay, wx, fma(-ax, wy, j1));
                r2 = fma(ax, xx, fma(ay, xy, r2));
                j2 = fma(ay, xx, fma(-ax, xy, j2));
            }
            r0 = team_sum<T>(r0);
            j0 = team_sum<T>(j0);
            r1 = team_sum<T>(r1);
            j1 = team_sum<T>(j1);
            r2 = team_sum<T>(r2);
            j2 = team_sum<T>(j2);
            pk.offer(cm, r0, j0);
            pk.offer(bi, r1, j1);
            pk.offer(cp, r2, j2);
            const double tD = (double)N * sqrt(pk.best) * (1.0 - 2.0 * kNearTie) - epsD;
            if (tD > 0.0) thr2 = fmaxf(thr2, (float)(tD * tD));
            skip0 = cm;
            skip1 = bi;
            skip2 = cp;
            pruned = true;
        }
        {
            const int lane = threadIdx.x & 63;
            const int base = lane - t;
            const uint64_t tmask = (T == 64) ? ~0ull : (((1ull << T) - 1ull) << base);
            const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int sq = t + T * q;
                const bool hit = m2[q] >= thr2 && sq != skip0 && sq != skip1 && sq != skip2;
                const uint64_t msk = __ballot(hit) & tmask;
                if (hit) cand[cnt + __popcll(msk & below)] = sq;
                cnt += __popcll(msk);
            }
        }
    }
    if ((rescore != CA_RESCORE_WINDOW || cnt == 0) && !pruned) {
        // top two: the best shift, and the runner-up when the two are within
        // the bound; both are team-uniform, so no candidate list is needed
        double re, im;
        dot64(bi, re, im);
        pk.offer(bi, re, im);
        if (two) {
            const int ci = runner_up();
            dot64(ci, re, im);
            pk.offer(ci, re, im);
        }
        finish(res, pk, N, n1, n2, d1, d2, epsD, capped, theta_of(pk), theta64);
        return res;
    }
    wave_lds_sync();
    int k = 0;
    // with FUSE2 the candidates are re-scored two per pass: curve 1's nodes
    // are converted once per pass and the two dependency chains (candidate
    // read, node reads, products, team sums) overlap; each candidate's terms
    // are summed in the same order as alone
    for (; FUSE2 && k + 1 < cnt; k += 2) {
        const int c0 = cand[k], c1 = cand[k + 1];
        double re0 = 0.0, im0 = 0.0, re1 = 0.0, im1 = 0.0;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const cf u = zat(c0, q), w = zat(c1, q);
            const double ax = a0[q].x, ay = a0[q].y;
            const double ux = u.x, uy = u.y, wx = w.x, wy = w.y;
            re0 = fma(ax, ux, fma(ay, uy, re0));
            im0 = fma(ay, ux, fma(-ax, uy, im0));
            re1 = fma(ax, wx, fma(ay, wy, re1));
            im1 = fma(ay, wx, fma(-ax, wy, im1));
        }
        re0 = team_sum<T>(re0);
        im0 = team_sum<T>(im0);
        re1 = team_sum<T>(re1);
        im1 = team_sum<T>(im1);
        pk.offer(c0, re0, im0);
        pk.offer(c1, re1, im1);
    }
    for (; k < cnt; ++k) {
        const int c = cand[k];
        double re, im;
        dot64(c, re, im);
        pk.offer(c, re, im);
    }
    wave_lds_sync();
    finish(res, pk, N, n1, n2, d1, d2, epsD, capped, theta_of(pk), theta64);
    return res;
}

}  // namespace ca
