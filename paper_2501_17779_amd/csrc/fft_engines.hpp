// Two FFT engines for the correlation of section 2 (the DFT steps of
// Algorithm 2).  Both are Stockham auto-sort, decimation in time:
//
//   pass p with radix R and stride Ns (product of the earlier radices):
//     for butterfly j in [0, N/R), k = j mod Ns:
//       b[r] = x[j + r N/R] * w_{Ns R}^{r k},  r = 0..R-1
//       b    = DFT_R(b)
//       y[(j - k) R + k + r Ns] = b[r]
//
// which leaves the output in natural order.
//
// * Block engine (any n with factors 2, 3, 5, 7; n <= 4096): one pair per
//   workgroup, the signal lives in LDS, every pass reads, synchronises and
//   writes in place.  Twiddles w_n^m come from a per-n table.
// * Team engine (powers of two, FP32): a team of T lanes (T <= 64, inside one
//   wave) owns one signal, lane t holding x[t + T q] for q = 0..R-1 in
//   registers (R = n / T).  With butterflies j = t + u T every pass reads
//   exactly those elements, so each pass is: butterflies on registers, a
//   scatter of the outputs to a per-team LDS buffer, and a gather of
//   x[t + T q] back into registers; the last pass needs no exchange and
//   leaves lane t holding X[t + T q] again.  The LDS buffer is padded with one
//   element per 16 so the stride-R scatter of the first pass is free of bank
//   conflicts.
#pragma once

#include "dft_small.hpp"

namespace ca {

// ------------------------------------------------------------------ block engine
struct Plan {
    int32_t n;
    int32_t npass;
    int32_t radix[16];
    int64_t tw_off;      // offset of the plan's per-pass twiddles in the arena
};
// Per-pass twiddle layout of a plan: pass i (radix R, stride ns = product of
// the earlier radices) owns the (R - 1) ns entries w_{ns R}^{r k}, r = 1..R-1,
// k = 0..ns-1, at (r - 1) ns + k after the entries of the earlier passes (n - 1
// entries in all).  Lanes with consecutive k read consecutive entries.

// j mod ns for 0 <= j < 2^13 and ns >= 1 through a float reciprocal and one
// correction step (the quotient estimate is off by at most one).
__device__ __forceinline__ int mod_small(int j, int ns, float inv_ns) {
    int q = (int)((float)j * inv_ns);
    int r = j - q * ns;
    if (r < 0) r += ns;
    else if (r >= ns) r -= ns;
    return r;
}

// A pass first requests its twiddles (global memory for the large classes),
// then waits at the barrier that publishes the previous pass's output, so the
// loads are in flight during the wait and the LDS reads.  It ends after its
// writes without a barrier: the next pass, or the caller, synchronises.
template <int R, int NT, int NMAX, typename T>
__device__ __forceinline__ void blk_pass(cpx<T>* buf, int n, int ns, const cpx<T>* __restrict__ tw) {
    constexpr int UM = (NMAX / R + NT - 1) / NT;
    const int nb = n / R;
    const float inv_ns = 1.0f / (float)ns;
    int kk[UM];
    cpx<T> f[UM][R - 1];
#pragma unroll
    for (int u = 0; u < UM; ++u) {
        const int j = threadIdx.x + u * NT;
        kk[u] = 0;
        if (j < nb && ns > 1) {
            kk[u] = mod_small(j, ns, inv_ns);
#pragma unroll
            for (int r = 1; r < R; ++r) f[u][r - 1] = tw[(r - 1) * ns + kk[u]];
        }
    }
    __syncthreads();
    cpx<T> v[UM][R];
#pragma unroll
    for (int u = 0; u < UM; ++u) {
        const int j = threadIdx.x + u * NT;
        if (j < nb) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[u][r] = buf[j + r * nb];
            if (ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) v[u][r] = mul(v[u][r], f[u][r - 1]);
            }
            dft<R>(v[u]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < UM; ++u) {
        const int j = threadIdx.x + u * NT;
        if (j < nb) {
            const int k = kk[u];
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[base + r * ns] = v[u][r];
        }
    }
}

// The first pass of a transform (stride 1: no twiddles) with its inputs
// taken from load(k) instead of the buffer.  load is called for every
// 0 <= k < UM NT + (R - 1) n / R, branch-free and before any value is used (so
// all the loads are in flight together); it must accept any such k and return
// the input x_k for k < n (values for larger k are not used).  Returns the
// FP64 sum of |x_k|^2 over k < nsum.  Its barrier orders its writes after
// every earlier read of buf.
template <int R, int NT, int NMAX, typename T, typename Load>
__device__ __forceinline__ double blk_pass_first(cpx<T>* buf, int n, int nsum, Load load) {
    constexpr int UM = (NMAX / R + NT - 1) / NT;
    const int nb = n / R;
    cpx<T> v[UM][R];
#pragma unroll
    for (int u = 0; u < UM; ++u)
#pragma unroll
        for (int r = 0; r < R; ++r) v[u][r] = load((int)threadIdx.x + u * NT + r * nb);
    double q = 0.0;
#pragma unroll
    for (int u = 0; u < UM; ++u) {
        const int j = threadIdx.x + u * NT;
        if (j < nb) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double x = v[u][r].x, y = v[u][r].y;
                const double s = fma(x, x, y * y);
                q += (j + r * nb < nsum) ? s : 0.0;
            }
            dft<R>(v[u]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < UM; ++u) {
        const int j = threadIdx.x + u * NT;
        if (j < nb) {
#pragma unroll
            for (int r = 0; r < R; ++r) buf[j * R + r] = v[u][r];
        }
    }
    return q;
}

// Radix 16 is compiled only into the kernels of the large size classes (it
// needs more registers than the others can spare); plans use it only for
// transform sizes above kBlkR16Min / 2.
constexpr int kBlkR16Min = 4096;

// Passes first..npass-1 of a plan, the earlier passes having left stride ns
// and used the twiddles before tw; ends with a barrier.
template <int NT, int NMAX, typename T>
__device__ __forceinline__ void blk_fft_passes(cpx<T>* buf, const Plan& p, const cpx<T>* __restrict__ tw,
                                               int first, int ns) {
    for (int i = first; i < p.npass; ++i) {
        const int r = p.radix[i];
        switch (r) {
            case 2: blk_pass<2, NT, NMAX>(buf, p.n, ns, tw); break;
            case 3: blk_pass<3, NT, NMAX>(buf, p.n, ns, tw); break;
            case 4: blk_pass<4, NT, NMAX>(buf, p.n, ns, tw); break;
            case 5: blk_pass<5, NT, NMAX>(buf, p.n, ns, tw); break;
            case 7: blk_pass<7, NT, NMAX>(buf, p.n, ns, tw); break;
            case 16:
                if constexpr (NMAX >= kBlkR16Min) {
                    blk_pass<16, NT, NMAX>(buf, p.n, ns, tw);
                    break;
                }
                [[fallthrough]];
            default: blk_pass<8, NT, NMAX>(buf, p.n, ns, tw); break;
        }
        tw += (r - 1) * ns;
        ns *= r;
    }
    __syncthreads();
}

// The transform of the signal in buf, in place; ends with a barrier.
template <int NT, int NMAX, typename T>
__device__ __forceinline__ void blk_fft(cpx<T>* buf, const Plan& p, const cpx<T>* __restrict__ tw) {
    blk_fft_passes<NT, NMAX>(buf, p, tw, 0, 1);
}

// The transform of the signal load(k), 0 <= k < p.n, into buf: the first
// pass reads its inputs through load, the others work in place.  Returns the
// FP64 sum of |x_k|^2 over k < nsum; ends with a barrier.
template <int NT, int NMAX, typename T, typename Load>
__device__ __forceinline__ double blk_fft_load(cpx<T>* buf, const Plan& p, const cpx<T>* __restrict__ tw,
                                               int nsum, Load load) {
    const int r = p.radix[0];
    double q;
    switch (r) {
        case 2: q = blk_pass_first<2, NT, NMAX, T>(buf, p.n, nsum, load); break;
        case 3: q = blk_pass_first<3, NT, NMAX, T>(buf, p.n, nsum, load); break;
        case 4: q = blk_pass_first<4, NT, NMAX, T>(buf, p.n, nsum, load); break;
        case 5: q = blk_pass_first<5, NT, NMAX, T>(buf, p.n, nsum, load); break;
        case 7: q = blk_pass_first<7, NT, NMAX, T>(buf, p.n, nsum, load); break;
        case 16:
            if constexpr (NMAX >= kBlkR16Min) {
                q = blk_pass_first<16, NT, NMAX, T>(buf, p.n, nsum, load);
                break;
            }
            [[fallthrough]];
        default: q = blk_pass_first<8, NT, NMAX, T>(buf, p.n, nsum, load); break;
    }
    blk_fft_passes<NT, NMAX>(buf, p, tw + (r - 1), 1, r);
    return q;
}

// ------------------------------------------------------------------- team engine
// LDS exchange layout: element i lives at i + (i >> PS), one pad slot per 2^PS.
template <int PS> __device__ __forceinline__ int lpadp(int i) { return i + (i >> PS); }

// Radix schedules: N = T * R (T lanes, R values per lane); every radix
// divides R.  Passes after the first multiply by w_{NS RP}^{r k}; those
// twiddles are stored per pass as tw[TWO + (r - 1) NS + k], so a lane's
// twiddles are one base address plus compile-time offsets.  PS is the pad
// shift of the exchange layout (exchanging passes need NS = 1 or a multiple
// of 2^PS, which makes every LDS address a lane base plus a constant).  AW is
// the minimum number of waves per SIMD the all-pairs kernel is compiled for.
template <int N> struct TeamCfg;
template <> struct TeamCfg<64> { static constexpr int T = 8, TW = 56, PS = 4, AW = 2; };      // 8 x 8
template <> struct TeamCfg<128> { static constexpr int T = 8, TW = 112, PS = 4, AW = 2; };    // 16 x 8
template <> struct TeamCfg<256> { static constexpr int T = 16, TW = 240, PS = 4, AW = 2; };   // 16 x 16
template <> struct TeamCfg<512> { static constexpr int T = 32, TW = 496, PS = 4, AW = 2; };   // 16 x 16 x 2
template <> struct TeamCfg<1024> { static constexpr int T = 64, TW = 1008, PS = 4, AW = 2; }; // 16 x 16 x 4
template <int N> __device__ __forceinline__ int lpad(int i) { return lpadp<TeamCfg<N>::PS>(i); }
template <int N> constexpr int team_padn() { return N + (N >> TeamCfg<N>::PS); }

// One Stockham pass on the team's registers.  Non-final passes scatter the
// outputs to LDS and gather x[t + T q] back; all LDS addresses are a lane base
// plus compile-time offsets (the pad function is additive on the pieces).
template <int N, int T, int RP, int NS, bool LAST, int TWO>
__device__ __forceinline__ void team_pass(cf (&v)[N / T], cf* lds, const cf* tws, int t) {
    constexpr int R = N / T;
    constexpr int U = R / RP;
    constexpr int PS = TeamCfg<N>::PS;
    static_assert(R % RP == 0, "radix must divide the per-lane count");
    static_assert(LAST || U == 1, "exchanging passes hold one butterfly per lane");
    static_assert(NS == 1 || NS % (1 << PS) == 0 || LAST, "exchange layout needs NS = 1 or a multiple of 2^PS");
    static_assert(RP <= (1 << PS), "first-pass radix must fit a pad group");
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = t + u * T;
        const int k = j & (NS - 1);
        cf b[RP];
#pragma unroll
        for (int r = 0; r < RP; ++r) b[r] = v[u + r * U];
        if constexpr (NS > 1) {
#pragma unroll
            for (int r = 1; r < RP; ++r) b[r] = mul(b[r], tws[TWO + (r - 1) * NS + k]);
        }
        dft<RP>(b);
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < RP; ++r) v[u + r * U] = b[r];
        } else if constexpr (NS == 1) {
            cf* wp = lds + (RP * j + ((RP * j) >> PS));
#pragma unroll
            for (int r = 0; r < RP; ++r) wp[r] = b[r];
        } else {
            const int i0 = (j - k) * RP + k;
            cf* wp = lds + lpadp<PS>(i0);
#pragma unroll
            for (int r = 0; r < RP; ++r) wp[r * (NS + (NS >> PS))] = b[r];
        }
    }
    if constexpr (!LAST) {
        wave_lds_sync();
        const cf* rp = lds + (t + (t >> PS));
#pragma unroll
        for (int q = 0; q < R; ++q) v[q] = rp[T * q + ((T * q) >> PS)];
        wave_lds_sync();
    }
}

// The same pass on two signals with shared twiddle loads.
template <int N, int T, int RP, int NS, bool LAST, int TWO>
__device__ __forceinline__ void team_pass2(cf (&v)[N / T], cf (&w)[N / T], cf* lds, const cf* tws, int t) {
    constexpr int R = N / T;
    constexpr int U = R / RP;
    static_assert(LAST || U == 1, "exchanging passes hold one butterfly per lane");
    cf bo[LAST ? 1 : RP], co[LAST ? 1 : RP];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = t + u * T;
        const int k = j & (NS - 1);
        cf b[RP], c[RP];
#pragma unroll
        for (int r = 0; r < RP; ++r) { b[r] = v[u + r * U]; c[r] = w[u + r * U]; }
        if constexpr (NS > 1) {
#pragma unroll
            for (int r = 1; r < RP; ++r) {
                const cf f = tws[TWO + (r - 1) * NS + k];
                b[r] = mul(b[r], f);
                c[r] = mul(c[r], f);
            }
        }
        dft<RP>(b);
        dft<RP>(c);
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < RP; ++r) { v[u + r * U] = b[r]; w[u + r * U] = c[r]; }
        } else {
#pragma unroll
            for (int r = 0; r < RP; ++r) { bo[r] = b[r]; co[r] = c[r]; }
        }
    }
    if constexpr (!LAST) {
        constexpr int PS = TeamCfg<N>::PS;
        const int j = t;
        const int k = j & (NS - 1);
        cf* wp;
        int stride;
        if constexpr (NS == 1) { wp = lds + (RP * j + ((RP * j) >> PS)); stride = 1; }
        else { wp = lds + lpadp<PS>((j - k) * RP + k); stride = NS + (NS >> PS); }
        const cf* rp = lds + (t + (t >> PS));
#pragma unroll
        for (int r = 0; r < RP; ++r) wp[r * stride] = bo[r];
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < R; ++q) v[q] = rp[T * q + ((T * q) >> PS)];
        wave_lds_sync();
#pragma unroll
        for (int r = 0; r < RP; ++r) wp[r * stride] = co[r];
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < R; ++q) w[q] = rp[T * q + ((T * q) >> PS)];
        wave_lds_sync();
    }
}

template <int N, int T>
__device__ __forceinline__ void team_fft(cf (&v)[N / T], cf* lds, const cf* tws, int t) {
    if constexpr (N == 64) {
        team_pass<64, T, 8, 1, false, 0>(v, lds, tws, t);
        team_pass<64, T, 8, 8, true, 0>(v, lds, tws, t);
    } else if constexpr (N == 128) {
        team_pass<128, T, 16, 1, false, 0>(v, lds, tws, t);
        team_pass<128, T, 8, 16, true, 0>(v, lds, tws, t);
    } else if constexpr (N == 256) {
        team_pass<256, T, 16, 1, false, 0>(v, lds, tws, t);
        team_pass<256, T, 16, 16, true, 0>(v, lds, tws, t);
    } else if constexpr (N == 512) {
        team_pass<512, T, 16, 1, false, 0>(v, lds, tws, t);
        team_pass<512, T, 16, 16, false, 0>(v, lds, tws, t);
        team_pass<512, T, 2, 256, true, 240>(v, lds, tws, t);
    } else {
        static_assert(N == 1024, "team engine sizes: 64..1024");
        team_pass<1024, T, 16, 1, false, 0>(v, lds, tws, t);
        team_pass<1024, T, 16, 16, false, 0>(v, lds, tws, t);
        team_pass<1024, T, 4, 256, true, 240>(v, lds, tws, t);
    }
}

template <int N, int T>
__device__ __forceinline__ void team_fft2(cf (&v)[N / T], cf (&w)[N / T], cf* lds, const cf* tws, int t) {
    if constexpr (N == 64) {
        team_pass2<64, T, 8, 1, false, 0>(v, w, lds, tws, t);
        team_pass2<64, T, 8, 8, true, 0>(v, w, lds, tws, t);
    } else if constexpr (N == 128) {
        team_pass2<128, T, 16, 1, false, 0>(v, w, lds, tws, t);
        team_pass2<128, T, 8, 16, true, 0>(v, w, lds, tws, t);
    } else if constexpr (N == 256) {
        team_pass2<256, T, 16, 1, false, 0>(v, w, lds, tws, t);
        team_pass2<256, T, 16, 16, true, 0>(v, w, lds, tws, t);
    } else if constexpr (N == 512) {
        team_pass2<512, T, 16, 1, false, 0>(v, w, lds, tws, t);
        team_pass2<512, T, 16, 16, false, 0>(v, w, lds, tws, t);
        team_pass2<512, T, 2, 256, true, 240>(v, w, lds, tws, t);
    } else {
        team_pass2<1024, T, 16, 1, false, 0>(v, w, lds, tws, t);
        team_pass2<1024, T, 16, 16, false, 0>(v, w, lds, tws, t);
        team_pass2<1024, T, 4, 256, true, 240>(v, w, lds, tws, t);
    }
}

}  // namespace ca
