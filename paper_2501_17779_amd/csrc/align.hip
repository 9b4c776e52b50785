// Alignment kernels: Algorithm 2 of section 2 as
//   FFT(z1), FFT(z2) -> P = conj(Z1) Z2 -> D = FFT(P) = n conj(C)
//   -> argmax |D|^2 -> FP64 re-scoring of the candidate shifts -> theta, e0.
// (Forward-transforming conj(Z1) Z2 gives n conj(C(s)) with
//  C(s) = sum_k z1[k] conj(z2[k - s]); |C| and arg C follow without a
//  separate inverse transform.)
#include <math.h>

#include "epilogue.hpp"
#include "launch.hpp"

namespace ca {

template <int TW>
__device__ __forceinline__ void load_twiddles(cf* tws, const cf* __restrict__ tw) {
    for (int i = threadIdx.x; i < TW; i += blockDim.x) tws[i] = tw[i];
    __syncthreads();
}

// Persistent batch kernel: each team loops over pairs.
template <int N>
__global__ __launch_bounds__(256, 2) void k_align_team(const cf* __restrict__ z1, const cf* __restrict__ z2,
                                                    int64_t num_pairs, ca_result_t* __restrict__ out,
                                                    const cf* __restrict__ tw, int rescore, int theta64) {
    constexpr int T = TeamCfg<N>::T;
    constexpr int R = N / T;
    constexpr int TEAMS = 256 / T;
    constexpr int PADN = team_padn<N>();
    // per team: the FFT exchange area, later two copies of curve 2's nodes;
    // with several teams in a wave the areas are 8 entries (16 banks) apart
    // beyond their size, so the teams of a half-wave do not meet on the same
    // LDS banks (every area size here is a multiple of the bank count)
    constexpr int BUF = (PADN > 2 * N ? PADN : 2 * N) + (T < 64 ? 8 : 0);
    __shared__ cf tws[TeamCfg<N>::TW];
    __shared__ cf lds_all[TEAMS * BUF];
    __shared__ int cand_all[TEAMS * kCandCap];
    load_twiddles<TeamCfg<N>::TW>(tws, tw);
    // a team of 64 is one wave: its pair index is wave-uniform, which keeps
    // the pair's base addresses in scalar registers
    const int team = T == 64 ? __builtin_amdgcn_readfirstlane(threadIdx.x / T) : threadIdx.x / T;
    const int t = threadIdx.x % T;
    cf* lds = lds_all + team * BUF;
    int* cand = cand_all + team * kCandCap;
    const int64_t stride = (int64_t)gridDim.x * TEAMS;
    for (int64_t pair = (int64_t)blockIdx.x * TEAMS + team; pair < num_pairs; pair += stride) {
        const cf* pa = z1 + pair * N;
        const cf* pb = z2 + pair * N;
        cf v[R], w[R], a0[R], b0[R];
#pragma unroll
        for (int q = 0; q < R; ++q) { v[q] = pa[t + T * q]; w[q] = pb[t + T * q]; }
        // both norms in the epilogue, which converts both curves' nodes anyway
#pragma unroll
        for (int q = 0; q < R; ++q) { a0[q] = v[q]; b0[q] = w[q]; }
        team_fft2<N, T>(v, w, lds, tws, t);
#pragma unroll
        for (int q = 0; q < R; ++q) v[q] = cjmul(v[q], w[q]);
        team_fft<N, T>(v, lds, tws, t);
        // z2 nodes, twice, for the shifted FP64 dot products
#pragma unroll
        for (int q = 0; q < R; ++q) {
            lds[t + T * q] = b0[q];
            lds[N + t + T * q] = b0[q];
        }
        wave_lds_sync();
        const ca_result_t res = team_epilogue<N, T, kZTwice, true, true>(v, a0, lds, cand, t, 0.0, 0.0, rescore, theta64);
        if (t == 0) out[pair] = res;
        wave_lds_sync();
    }
}

// ------------------------------------------------------------------ all pairs
// Per-curve spectra Z_i = FFT(z_i) in natural order and n_i = (1/n) sum |z_i|^2.
template <int N>
__global__ __launch_bounds__(256) void k_spectra(const cf* __restrict__ curves, int m, cf* __restrict__ spec,
                                                 double* __restrict__ norms, const cf* __restrict__ tw) {
    constexpr int T = TeamCfg<N>::T;
    constexpr int R = N / T;
    constexpr int TEAMS = 256 / T;
    constexpr int PADN = team_padn<N>();
    constexpr int BUF = PADN + (T < 64 ? 8 : 0);    // team areas 16 banks apart (see k_align_team)
    __shared__ cf tws[TeamCfg<N>::TW];
    __shared__ cf lds_all[TEAMS * BUF];
    load_twiddles<TeamCfg<N>::TW>(tws, tw);
    const int team = threadIdx.x / T;
    const int t = threadIdx.x % T;
    const int64_t i = (int64_t)blockIdx.x * TEAMS + team;
    if (i >= m) return;
    cf* lds = lds_all + team * BUF;
    const cf* z = curves + i * N;
    cf v[R];
    double q2 = 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        v[q] = z[t + T * q];
        q2 = fma((double)v[q].x, (double)v[q].x, fma((double)v[q].y, (double)v[q].y, q2));
    }
    team_fft<N, T>(v, lds, tws, t);
#pragma unroll
    for (int q = 0; q < R; ++q) spec[i * N + t + T * q] = v[q];
    q2 = team_sum<T>(q2);
    if (t == 0) norms[i] = q2 / N;
}

// Upper-triangle tiles of TEAMS rows i and `cols` columns j over a persistent
// grid of G blocks: block b takes the tiles t = b, b + G, b + 2 G, ... of the
// row-major tile grid (row tile t / tx_n, column tile t % tx_n; tx_n, the
// padded column-tile count, and G are multiples of 8, and G / 8 is odd) and
// skips at once the tiles without a pair j > i.  All blocks advance through
// the grid together, so the rows in use at any time are those of one or two
// row tiles (they stay in L2); workgroups are dealt to the 8 XCDs round-robin
// by block id, so column tile x is always aligned on XCD x mod 8 and its
// spectra and nodes are re-read from that XCD's L2; with G / 8 odd a block's
// column tiles run through every residue (the work of a column tile grows with
// its index, so a block held to a few column tiles would get an uneven share).
// Each row's spectrum and nodes stay in registers; every column's spectrum and nodes are
// staged once in LDS (double-buffered: the next column is loaded while the
// current one is aligned) and shared by the rows.
template <int N>
__global__ __launch_bounds__(256, TeamCfg<N>::AW) void k_allpairs(const cf* __restrict__ curves, const cf* __restrict__ spec,
                                                  const double* __restrict__ norms, int m, int cols,
                                                  int tx_n, int64_t tiles, ca_result_t* __restrict__ out,
                                                  const cf* __restrict__ tw, int rescore, int theta64) {
    constexpr int T = TeamCfg<N>::T;
    constexpr int R = N / T;
    constexpr int TEAMS = 256 / T;
    constexpr int PADN = team_padn<N>();
    constexpr int PER = (N + 255) / 256;
    __shared__ cf tws[TeamCfg<N>::TW];
    // column nodes: twice (shifted reads at constant offsets) where two
    // blocks per CU still fit in LDS, else once in the padded layout
    constexpr int ZL = N <= 512 ? kZTwice : kZPad;
    constexpr int ZS = ZL == kZTwice ? 2 * N : PADN;
    __shared__ cf sZ[2][N];
    __shared__ cf sz[2][ZS];
    constexpr int XB = PADN + (T < 64 ? 8 : 0);     // team areas 16 banks apart (see k_align_team)
    __shared__ cf xbuf[TEAMS * XB];
    __shared__ int cand_all[TEAMS * kCandCap];
    load_twiddles<TeamCfg<N>::TW>(tws, tw);
    const int team = threadIdx.x / T;
    const int t = threadIdx.x % T;
    cf* lds = xbuf + team * XB;
    int* cand = cand_all + team * kCandCap;
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int i0 = (int)(tile / tx_n) * TEAMS;
    const int j0 = (int)(tile % tx_n) * cols;
    if (j0 >= m || j0 + cols - 1 <= i0) continue;   // padding column tile, or no j > i in this tile
    const int i = i0 + team;
    const bool row_ok = i < m;
    cf Zi[R], zi[R];
    double ni = 0.0;
    if (row_ok) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            Zi[q] = spec[(int64_t)i * N + t + T * q];
            zi[q] = curves[(int64_t)i * N + t + T * q];
        }
        ni = norms[i];
    }
    const int jbeg = max(j0, i0 + 1);
    const int jend = min(j0 + cols, m);
    cf gZ[PER], gz[PER];
    auto fetch = [&](int j) {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int k = threadIdx.x + 256 * p;
            if (k < N) {
                gZ[p] = spec[(int64_t)j * N + k];
                gz[p] = curves[(int64_t)j * N + k];
            }
        }
    };
    auto stash = [&](int b) {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int k = threadIdx.x + 256 * p;
            if (k < N) {
                sZ[b][k] = gZ[p];
                if constexpr (ZL == kZTwice) {
                    sz[b][k] = gz[p];
                    sz[b][N + k] = gz[p];
                } else {
                    sz[b][lpad<N>(k)] = gz[p];
                }
            }
        }
    };
    if (jbeg < jend) {
        fetch(jbeg);
        stash(0);
    }
    __syncthreads();
    for (int j = jbeg; j < jend; ++j) {
        const int cur = (j - jbeg) & 1;
        if (j + 1 < jend) fetch(j + 1);
        if (row_ok && j > i) {
            cf v[R];
#pragma unroll
            for (int q = 0; q < R; ++q) v[q] = cjmul(Zi[q], sZ[cur][t + T * q]);
            team_fft<N, T>(v, lds, tws, t);
            const ca_result_t res =
                team_epilogue<N, T, ZL>(v, zi, sz[cur], cand, t, ni, norms[j], rescore, theta64);
            if (t == 0) {
                const int64_t k = (int64_t)i * m - (int64_t)i * (i + 1) / 2 + (j - i - 1);
                out[k] = res;
            }
        }
        if (j + 1 < jend) stash(cur ^ 1);
        __syncthreads();
    }
    }
}

bool team_supported(int n) { return n == 64 || n == 128 || n == 256 || n == 512 || n == 1024; }
bool allpairs_supported(int n) { return team_supported(n); }

template <int N>
static hipError_t launch_team_n(const void* z1, const void* z2, int64_t np, ca_result_t* out,
                                const void* tw, int rescore, int theta64, int max_blocks, hipStream_t s) {
    constexpr int TEAMS = 256 / TeamCfg<N>::T;
    int64_t blocks = (np + TEAMS - 1) / TEAMS;
    if (max_blocks > 0 && blocks > max_blocks) blocks = max_blocks;
    hipLaunchKernelGGL(k_align_team<N>, dim3((unsigned)blocks), dim3(256), 0, s, (const cf*)z1,
                       (const cf*)z2, np, out, (const cf*)tw, rescore, theta64);
    return hipGetLastError();
}

template <int N>
static int team_blocks_per_cu() {
    static int cached = -1;
    if (cached < 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_align_team<N>, 256, 0) != hipSuccess || nb < 1)
            nb = 1;
        cached = nb;
    }
    return cached;
}

hipError_t launch_align_team(const void* z1, const void* z2, int n, int64_t np, ca_result_t* out,
                             const void* tw, int rescore, int theta64, int num_cus, int grid_mult,
                             hipStream_t s) {
    if (grid_mult < 0) return hipErrorInvalidValue;
    switch (n) {
        case 64: return launch_team_n<64>(z1, z2, np, out, tw, rescore, theta64, num_cus * team_blocks_per_cu<64>() * grid_mult, s);
        case 128: return launch_team_n<128>(z1, z2, np, out, tw, rescore, theta64, num_cus * team_blocks_per_cu<128>() * grid_mult, s);
        case 256: return launch_team_n<256>(z1, z2, np, out, tw, rescore, theta64, num_cus * team_blocks_per_cu<256>() * grid_mult, s);
        case 512: return launch_team_n<512>(z1, z2, np, out, tw, rescore, theta64, num_cus * team_blocks_per_cu<512>() * grid_mult, s);
        case 1024: return launch_team_n<1024>(z1, z2, np, out, tw, rescore, theta64, num_cus * team_blocks_per_cu<1024>() * grid_mult, s);
        default: return hipErrorInvalidValue;
    }
}

int team_twiddle_count(int n) {
    switch (n) {
        case 64: return TeamCfg<64>::TW;
        case 128: return TeamCfg<128>::TW;
        case 256: return TeamCfg<256>::TW;
        case 512: return TeamCfg<512>::TW;
        case 1024: return TeamCfg<1024>::TW;
        default: return 0;
    }
}

template <int N>
static hipError_t launch_spectra_n(const void* curves, int m, void* spec, double* norms, const void* tw,
                                   hipStream_t s) {
    constexpr int TEAMS = 256 / TeamCfg<N>::T;
    hipLaunchKernelGGL(k_spectra<N>, dim3((unsigned)((m + TEAMS - 1) / TEAMS)), dim3(256), 0, s,
                       (const cf*)curves, m, (cf*)spec, norms, (const cf*)tw);
    return hipGetLastError();
}

template <int N>
static hipError_t launch_allpairs_n(const void* curves, const void* spec, const double* norms, int m,
                                    ca_result_t* out, const void* tw, int rescore, int theta64, int cols,
                                    int num_cus, hipStream_t s) {
    if (cols < 1) return hipErrorInvalidValue;
    // persistent grid: at most the occupancy limit on every CU, a multiple of
    // 8 with an odd multiplier (see the kernel)
    static int per_cu = -1;
    if (per_cu < 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_allpairs<N>, 256, 0) != hipSuccess || nb < 1)
            nb = 1;
        per_cu = nb;
    }
    constexpr int TEAMS = 256 / TeamCfg<N>::T;
    const int tx_n = ((m + cols - 1) / cols + 7) / 8 * 8;
    const int64_t tiles = (int64_t)tx_n * ((m + TEAMS - 1) / TEAMS);
    int64_t g8 = (int64_t)num_cus * per_cu / 8;
    if (g8 < 1) g8 = 1;
    if (g8 % 2 == 0) --g8;                 // odd: a block visits every column-tile residue
    int64_t grid = 8 * g8;
    if (grid > tiles) grid = tiles;
    hipLaunchKernelGGL((k_allpairs<N>), dim3((unsigned)grid), dim3(256), 0, s, (const cf*)curves, (const cf*)spec,
                       norms, m, cols, tx_n, tiles, out, (const cf*)tw, rescore, theta64);
    return hipGetLastError();
}

hipError_t launch_spectra(const void* curves, int m, int n, void* spec, double* norms, const void* tw,
                          hipStream_t s) {
    switch (n) {
        case 64: return launch_spectra_n<64>(curves, m, spec, norms, tw, s);
        case 128: return launch_spectra_n<128>(curves, m, spec, norms, tw, s);
        case 256: return launch_spectra_n<256>(curves, m, spec, norms, tw, s);
        case 512: return launch_spectra_n<512>(curves, m, spec, norms, tw, s);
        case 1024: return launch_spectra_n<1024>(curves, m, spec, norms, tw, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_allpairs(const void* curves, const void* spec, const double* norms, int m, int n,
                           ca_result_t* out, const void* tw, int rescore, int theta64, int cols,
                           int num_cus, hipStream_t s) {
    switch (n) {
        case 64: return launch_allpairs_n<64>(curves, spec, norms, m, out, tw, rescore, theta64, cols, num_cus, s);
        case 128: return launch_allpairs_n<128>(curves, spec, norms, m, out, tw, rescore, theta64, cols, num_cus, s);
        case 256: return launch_allpairs_n<256>(curves, spec, norms, m, out, tw, rescore, theta64, cols, num_cus, s);
        case 512: return launch_allpairs_n<512>(curves, spec, norms, m, out, tw, rescore, theta64, cols, num_cus, s);
        case 1024: return launch_allpairs_n<1024>(curves, spec, norms, m, out, tw, rescore, theta64, cols, num_cus, s);
        default: return hipErrorInvalidValue;
    }
}

// -------------------------------------------------------------- block engine
// Persistent kernels, one pair per workgroup at a time; each launch serves
// one size class of transform sizes with NT threads and LDS for one signal of
// MMAX values (the other spectrum waits in registers): a whole uniform batch,
// or the list that k_blk_bin built for the class in a ragged batch.
//
// A 7-smooth n is transformed at size M = n.  Any other n uses the plan's
// 7-smooth M >= 2n: with a = z1 followed by zeros and b = (z2, z2, zeros),
// the cyclic correlation of length M has no wrap-around at the lags
// M - n + s, 0 <= s < n, where it equals C(s) = sum_k z1[k] conj(z2[k - s])
// (indices mod n).  The forward transform of conj(A) B then gives
// D[M - n + s] = M conj(C(s)).
// Size class of a transform size (the launch order of launch_blk).
__device__ __forceinline__ int blk_class(int M) {
    return M <= 512 ? 0 : M <= 1024 ? 1 : M <= 2048 ? 2 : M <= 4096 ? 3 : 4;
}

__global__ void k_zero_ints(int* p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

// Ragged batches: every pair goes to the list of its size class (the order
// inside a list does not affect any result); pairs that no class can take get
// their CA_FLAG_UNSUPPORTED_N record here.  Positions are reserved per wave in
// LDS and per block with one global atomic per class; the class counters sit
// in separate cache lines, so the blocks' atomics on different classes do not
// queue on one line.
__global__ __launch_bounds__(256) void k_blk_bin(const int64_t* __restrict__ offsets, int64_t num_pairs,
                                                 const Plan* __restrict__ plans, int mcap, int* __restrict__ bins,
                                                 ca_result_t* __restrict__ out) {
    __shared__ int s_cnt[kBlkClasses], s_base[kBlkClasses];
    if (threadIdx.x < kBlkClasses) s_cnt[threadIdx.x] = 0;
    const int64_t pair = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int cls = -1;
    if (pair < num_pairs) {
        const int64_t len = offsets[pair + 1] - offsets[pair];
        const int n = (len >= 2 && len <= kMaxN) ? (int)len : 0;
        const int M = n ? plans[n].n : 0;
        if (M == 0 || M > mcap) {
            ca_result_t r;
            r.shift = 0; r.flags = CA_FLAG_UNSUPPORTED_N; r.theta = 0.0; r.err_est = 0.0f; r.gap = 0.0f;
            r.e0 = __builtin_nan("");
            out[pair] = r;
        } else {
            cls = blk_class(M);
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    int pos = 0;                                   // position inside the block's share of the list
    for (int c = 0; c < kBlkClasses; ++c) {
        const uint64_t mask = __ballot(cls == c);
        if (mask == 0ull) continue;
        const int leader = __ffsll((long long)mask) - 1;
        int wbase = 0;
        if (lane == leader) wbase = atomicAdd(&s_cnt[c], __popcll(mask));
        wbase = __shfl(wbase, leader, 64);
        if (cls == c) pos = wbase + __popcll(mask & below);
    }
    __syncthreads();
    if (threadIdx.x < kBlkClasses) {
        const int k = s_cnt[threadIdx.x];
        s_base[threadIdx.x] = k > 0 ? atomicAdd(&bins[threadIdx.x * kBinStride], k) : 0;
    }
    __syncthreads();
    if (cls >= 0) bins[kBlkClasses * kBinStride + cls * num_pairs + s_base[cls] + pos] = (int)pair;
}

// Largest value and runner-up of a block in one pair of barriers.  Each
// thread brings its own largest (b1 at i1) and second largest (b2 at i2),
// smallest index first on equal values.  Returns the block's largest (bv at
// bi) and the largest over every other index (cv at ci), both with the
// smallest index on equal values; scratch holds 4 * (blockDim / 64) doubles.
template <int NT, typename V>
__device__ __forceinline__ void block_top2(V b1, int i1, V b2, int i2, V& bv, int& bi, V& cv, int& ci,
                                           double* scratch) {
    // per wave: its largest, then the largest over its other indices (the
    // lane holding the wave's largest offers its second largest)
    V w1 = b1;
    int j1 = i1;
    team_argmax<64>(w1, j1);
    V w2 = i1 == j1 ? b2 : b1;
    int j2 = i1 == j1 ? i2 : i1;
    team_argmax<64>(w2, j2);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        scratch[4 * w] = (double)w1;
        scratch[4 * w + 1] = (double)j1;
        scratch[4 * w + 2] = (double)w2;
        scratch[4 * w + 3] = (double)j2;
    }
    __syncthreads();
    // the block's largest, and which wave holds it
    V v = (V)scratch[0];
    int iv = (int)scratch[1], kw = 0;
#pragma unroll
    for (int k = 1; k < NT / 64; ++k) {
        const V o = (V)scratch[4 * k];
        const int oi = (int)scratch[4 * k + 1];
        if (o > v || (o == v && oi < iv)) { v = o; iv = oi; kw = k; }
    }
    // runner-up: that wave's second, every other wave's first
    V c = (V)scratch[4 * kw + 2];
    int ic = (int)scratch[4 * kw + 3];
#pragma unroll
    for (int k = 0; k < NT / 64; ++k)
        if (k != kw) argmax_combine(c, ic, (V)scratch[4 * k], (int)scratch[4 * k + 1]);
    bv = v; bi = iv; cv = c; ci = ic;
}

// Waves per SIMD each block-engine kernel is compiled for: the most its
// registers allow without spilling.
template <typename T, int NT, int MMAX> constexpr int blk_waves() {
    if (sizeof(T) == 8) return MMAX >= 4096 ? 1 : 2;
    if (MMAX <= 2048) return 4;
    if (MMAX == 4096) return NT == 512 ? 4 : 3;
    return NT == 1024 ? 4 : NT == 512 ? 2 : 1;
}

template <typename T, int NT, int MMAX>
__global__ __launch_bounds__(NT, (blk_waves<T, NT, MMAX>())) void k_align_blk(const cpx<T>* __restrict__ z1, const cpx<T>* __restrict__ z2,
                                                  const int64_t* __restrict__ offsets, int n_uniform,
                                                  int64_t num_pairs, ca_result_t* __restrict__ out,
                                                  const Plan* __restrict__ plans,
                                                  const cpx<T>* __restrict__ arena, int rescore, int theta64,
                                                  const int* __restrict__ list_count, const int* __restrict__ list) {
    // the plan's twiddles are staged in LDS where the table is small, or
    // where the registers allow one block per CU anyway
    constexpr bool kTwLds = MMAX * sizeof(cpx<T>) <= 16384 || blk_waves<T, NT, MMAX>() * 256 / NT <= 1;
    constexpr int HN = MMAX / NT;        // spectrum values of curve 2 held per thread
    constexpr int kRsU = HN < 4 ? HN : 4;  // node pairs per thread in flight in the re-scoring
    // with at most four transform values per thread (the small-batch kernels
    // of classes 0 and 1) both curves' nodes are staged in LDS with the
    // twiddles: every input of a pair is requested at once, and the first
    // passes and the re-scoring read LDS (a pair's latency sees one global
    // round trip instead of four)
    constexpr bool kStageIn = HN <= 4;
    static_assert(!kStageIn || kTwLds, "staged inputs come with staged twiddles");
    __shared__ cpx<T> A[MMAX];
    __shared__ cpx<T> TWL[kTwLds ? MMAX : 1];
    __shared__ cpx<T> ZA[kStageIn ? MMAX : 1];
    __shared__ cpx<T> ZB[kStageIn ? MMAX : 1];
    __shared__ double red[4 * (NT / 64)];
    __shared__ int clist[kCandCap + 1];
    const int64_t todo = list ? (int64_t)*list_count : num_pairs;
    for (int64_t it = blockIdx.x; it < todo; it += gridDim.x) {
        const int64_t pair = list ? (int64_t)list[it] : it;
        int64_t off;
        int n;
        if (offsets) {
            off = offsets[pair];
            n = (int)(offsets[pair + 1] - off);
        } else {
            off = pair * (int64_t)n_uniform;
            n = n_uniform;
        }
        const int M = plans[n].n;
        const Plan& p = plans[n];
        const cpx<T>* tw = arena + p.tw_off;
        const cpx<T>* pa = z1 + off;
        const cpx<T>* pb = z2 + off;
        if constexpr (kStageIn) {
            // HN NT = MMAX covers the M - 1 twiddles and the n <= M nodes
            cpx<T> tv[HN], va[HN], vb[HN];
#pragma unroll
            for (int i = 0; i < HN; ++i) {
                const int k = threadIdx.x + i * NT;
                tv[i] = tw[k < M - 1 ? k : 0];
                va[i] = pa[k < n ? k : 0];
                vb[i] = pb[k < n ? k : 0];
            }
#pragma unroll
            for (int i = 0; i < HN; ++i) {
                const int k = threadIdx.x + i * NT;
                if (k < M - 1) TWL[k] = tv[i];
                if (k < n) {
                    ZA[k] = va[i];
                    ZB[k] = vb[i];
                }
            }
            tw = TWL;
            __syncthreads();                 // the first passes read ZA and ZB before their barriers
        } else if constexpr (kTwLds) {
            // four loads in flight per thread, then their stores
            for (int k0 = 0; k0 < M - 1; k0 += 4 * NT) {
                cpx<T> tv[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int k = k0 + threadIdx.x + i * NT;
                    tv[i] = tw[k < M - 1 ? k : 0];
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int k = k0 + threadIdx.x + i * NT;
                    if (k < M - 1) TWL[k] = tv[i];
                }
            }
            tw = TWL;                        // first read after the barrier of the first pass
        }
        // where the first passes and the re-scoring read the nodes
        const cpx<T>* sa = kStageIn ? ZA : pa;
        const cpx<T>* sb = kStageIn ? ZB : pb;
        const bool padded = M != n;
        const int base = M - n;              // D index of shift 0
        const int nb = padded ? 2 * n : n;   // extent of b
        const cpx<T> zero = {T(0), T(0)};

        // One signal buffer: the spectrum of b is computed first and held in
        // registers (thread t keeps entries t + NT i), then the spectrum of a
        // takes the buffer and is multiplied in place by conj(.) b, then that
        // product is transformed.  Both first passes read the nodes from
        // global memory (or their LDS copies).
        const double q2 = blk_fft_load<NT, MMAX>(A, p, tw, n, [&](int k) {
            const cpx<T> x = sb[k < nb ? (k < n ? k : k - n) : 0];
            return k < nb ? x : zero;
        });
        cpx<T> h[HN];
#pragma unroll
        for (int i = 0; i < HN; ++i) {
            const int k = threadIdx.x + i * NT;
            h[i] = k < M ? A[k] : zero;
        }
        const double q1 = blk_fft_load<NT, MMAX>(A, p, tw, n, [&](int k) {
            const cpx<T> x = sa[k < n ? k : 0];
            return k < n ? x : zero;
        });
#pragma unroll
        for (int i = 0; i < HN; ++i) {
            const int k = threadIdx.x + i * NT;
            if (k < M) A[k] = cjmul(A[k], h[i]);
        }
        __syncthreads();
        blk_fft<NT, MMAX>(A, p, tw);
        // largest |D|^2 and runner-up in one scan: per thread the two
        // largest (smallest shift first on equal values), then one reduction
        T b1 = T(-1), b2 = T(-1);
        int i1 = 0, i2 = 0;
        for (int k = threadIdx.x; k < n; k += NT) {
            const T m = norm2(A[base + k]);
            if (m > b1) {
                b2 = b1; i2 = i1; b1 = m; i1 = k;
            } else if (m > b2) {
                b2 = m; i2 = k;
            }
        }
        T bv, cv;
        int bi, ci;
        block_top2<NT>(b1, i1, b2, i2, bv, bi, cv, ci, red);

        // this thread's part of the FP64 C at shift c (times n): kRsU node
        // pairs in flight per thread before their products (indices past n
        // read node 0 and add zero); the terms are summed in the order
        // k = t, t + NT, ...
        auto dot_part = [&](int c, double& re, double& im) {
            re = 0.0;
            im = 0.0;
            for (int k0 = 0; k0 < n; k0 += kRsU * NT) {
                cpx<T> av[kRsU], bw[kRsU];
#pragma unroll
                for (int i = 0; i < kRsU; ++i) {
                    const int k = k0 + threadIdx.x + i * NT;
                    int idx = k - c;
                    if (idx < 0) idx += n;
                    av[i] = sa[k < n ? k : 0];
                    bw[i] = sb[k < n ? idx : 0];
                }
#pragma unroll
                for (int i = 0; i < kRsU; ++i) {
                    const bool in = k0 + threadIdx.x + i * NT < n;
                    const double ax = in ? (double)av[i].x : 0.0, ay = in ? (double)av[i].y : 0.0;
                    const double bx = bw[i].x, by = bw[i].y;
                    re = fma(ax, bx, fma(ay, by, re));
                    im = fma(ay, bx, fma(-ax, by, im));
                }
            }
        };
        // the argmax is re-scored first, its two sums reduced together with
        // the norms' (one pair of barriers for the four)
        double re0, im0, s1 = q1, s2 = q2;
        dot_part(bi, re0, im0);
        block_sum4<NT>(re0, im0, s1, s2, red);
        const double n1 = s1 / n, n2 = s2 / n;

        ca_result_t res;
        if (!special_case(res, n1, n2, (double)bv)) {
            const double d1 = sqrt((double)bv), d2 = sqrt(fmax((double)cv, 0.0));
            double lg = 0.0;
            for (int m = 1; m < M; m <<= 1) lg += 1.0;
            // |D| error bound: transform size M, |a| |b| = n sqrt(n1 n2) (times
            // sqrt 2 when curve 2 is repeated)
            const double epsD = kErrScale * num<T>::u * lg * (double)M * (double)n * sqrt(n1 * n2) *
                                (padded ? 1.4142135623730951 : 1.0);
            Pick pk;
            pk.offer(bi, re0, im0);
            auto rescore_one = [&](int c) {
                double re, im;
                dot_part(c, re, im);
                block_sum2<NT>(re, im, red);
                pk.offer(c, re, im);
            };
            bool capped = false;
            if (rescore == CA_RESCORE_WINDOW) {
                const double thr = d1 - 2.0 * epsD;
                const double thr2 = thr > 0.0 ? thr * thr : 0.0;
                if (threadIdx.x == 0) clist[0] = 0;
                __syncthreads();
                for (int k = threadIdx.x; k < n; k += NT) {
                    if (k != bi && (double)norm2(A[base + k]) >= thr2) {
                        const int pos = atomicAdd(&clist[0], 1);
                        if (pos < kCandCap) clist[1 + pos] = k;
                    }
                }
                __syncthreads();
                const int cnt = clist[0];
                if (thr > 0.0 && cnt < kCandCap) {
                    for (int c = 0; c < cnt; ++c) rescore_one(clist[1 + c]);
                } else {
                    capped = true;
                }
            }
            if ((rescore != CA_RESCORE_WINDOW || capped) && d1 - d2 < 2.0 * epsD) rescore_one(ci);
            // theta from the FP64 re-scored C at the chosen shift: an FP32 arc
            // tangent on the FP32 path, FP64 on the FP64 path
            double thp;
            if constexpr (sizeof(T) == 4) thp = (double)wrap_pi(atan2f((float)pk.im, (float)pk.re));
            else thp = wrap_pi(atan2_fp64(pk.im, pk.re));
            finish(res, pk, n, n1, n2, d1, d2, epsD, capped, thp, theta64);
        }
        if (threadIdx.x == 0) out[pair] = res;
        __syncthreads();
    }
}


template <typename T, int NT, int MMAX>
static hipError_t launch_blk_class(const BlkArgs& a, int cls, hipStream_t s) {
    static int per_cu = -1;
    if (per_cu < 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_align_blk<T, NT, MMAX>, NT, 0) != hipSuccess ||
            nb < 1)
            nb = 1;
        per_cu = nb;
    }
    const int g = a.grid_mult[cls];
    if (g < 0) return hipErrorInvalidValue;
    int64_t grid = g == 0 ? a.num_pairs : (int64_t)a.num_cus * per_cu * g;
    if (grid > a.num_pairs) grid = a.num_pairs;
    const int* count = a.offsets ? a.bins + cls * kBinStride : nullptr;
    const int* list = a.offsets ? a.bins + kBlkClasses * kBinStride + cls * a.num_pairs : nullptr;
    hipLaunchKernelGGL((k_align_blk<T, NT, MMAX>), dim3((unsigned)grid), dim3(NT), 0, s,
                       (const cpx<T>*)a.z1, (const cpx<T>*)a.z2, a.offsets, a.n_uniform, a.num_pairs, a.out,
                       a.plans, (const cpx<T>*)a.tw_arena, a.rescore, a.theta64, count, list);
    return hipGetLastError();
}

// Size classes by transform size: (64 threads, M <= 512), (128, <= 1024),
// both 256 for batches of at most one pair per CU,
// (256, <= 2048), (256 or, FP32, 512, <= 4096) and, FP32 only, (1024, 512
// or 256, <= 8192); the FP32 thread counts of the two large classes are
// tuning choices.  A uniform batch launches its one class; a ragged batch is
// binned on the device first.
template <typename T>
static hipError_t launch_blk(const BlkArgs& a, hipStream_t s) {
    const int lo = a.offsets ? 0 : a.m_uniform, hi = a.offsets ? a.m_cap : a.m_uniform;
    hipError_t e = hipSuccess;
    if (a.offsets) {
        hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(kBlkClasses * kBinStride), 0, s, a.bins,
                           kBlkClasses * kBinStride);
        hipLaunchKernelGGL(k_blk_bin, dim3((unsigned)((a.num_pairs + 255) / 256)), dim3(256), 0, s, a.offsets,
                           a.num_pairs, a.plans, a.m_cap, a.bins, a.out);
        e = hipGetLastError();
    }
    // a batch that cannot fill the chip runs the two small classes at 256
    // threads per pair: each pair's butterflies spread over four SIMDs
    // instead of one or two, which shortens the call (one pair: its latency)
    const bool few = a.num_pairs <= a.num_cus;
    if (lo <= 512 && e == hipSuccess)
        e = few ? launch_blk_class<T, 256, 512>(a, 0, s) : launch_blk_class<T, 64, 512>(a, 0, s);
    if (hi > 512 && lo <= 1024 && e == hipSuccess)
        e = few ? launch_blk_class<T, 256, 1024>(a, 1, s) : launch_blk_class<T, 128, 1024>(a, 1, s);
    if (hi > 1024 && lo <= 2048 && e == hipSuccess) e = launch_blk_class<T, 256, 2048>(a, 2, s);
    if constexpr (sizeof(T) == 4) {
        if (hi > 2048 && lo <= 4096 && e == hipSuccess)
            e = a.threads[3] == 512 ? launch_blk_class<T, 512, 4096>(a, 3, s) : launch_blk_class<T, 256, 4096>(a, 3, s);
        if (hi > 4096 && e == hipSuccess)
            e = a.threads[4] == 256   ? launch_blk_class<T, 256, 8192>(a, 4, s)
                : a.threads[4] == 512 ? launch_blk_class<T, 512, 8192>(a, 4, s)
                                      : launch_blk_class<T, 1024, 8192>(a, 4, s);
    } else {
        if (hi > 2048 && lo <= 4096 && e == hipSuccess) e = launch_blk_class<T, 256, 4096>(a, 3, s);
    }
    return e;
}

hipError_t launch_align_blk_f32(const BlkArgs& a, hipStream_t s) { return launch_blk<float>(a, s); }
hipError_t launch_align_blk_f64(const BlkArgs& a, hipStream_t s) { return launch_blk<double>(a, s); }

}  // namespace ca
