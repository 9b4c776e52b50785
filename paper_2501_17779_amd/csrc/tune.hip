// Launch tuning (ca_autotune, ca_tune_get/set/save/load): candidate sweeps
// timed with HIP events on a synthetic batch generated on the device, and a
// JSON cache keyed by architecture and CU count.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <ctype.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <utility>
#include <vector>

#include "common.hpp"
#include "context.hpp"

using namespace ca::host;

namespace ca {

// 32-bit mix of (a, b) (a murmur3-style finaliser over a combined word).
__device__ __forceinline__ uint32_t tune_hash(uint32_t a, uint32_t b) {
    uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u + (a << 6) + (a >> 2));
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}
__device__ __forceinline__ float tune_unit(uint32_t h) { return (float)(h >> 8) * (1.0f / 16777216.0f); }

// Smooth star-shaped curves r(t) = 1 + sum of three low modes, and templates:
// curve 1 rotated, cyclically shifted and perturbed by 1e-3 noise.  Node k of
// pair p (n nodes from index base) sits at index i.
__device__ __forceinline__ void tune_node(cf* __restrict__ z1, cf* __restrict__ z2, int64_t i, uint32_t p, int k,
                                          int n, uint32_t seed) {
    const float two_pi = 6.2831853f;
    const float ph1 = two_pi * tune_unit(tune_hash(p, seed + 1));
    const float ph2 = two_pi * tune_unit(tune_hash(p, seed + 2));
    const float ph3 = two_pi * tune_unit(tune_hash(p, seed + 3));
    const float rot = two_pi * tune_unit(tune_hash(p, seed + 4));
    const int shift = (int)(tune_hash(p, seed + 5) % (uint32_t)n);
    auto node = [&](int j) {
        const float t = two_pi * (float)j / (float)n;
        const float r = 1.0f + 0.1f * cosf(3.0f * t + ph1) + 0.05f * cosf(5.0f * t + ph2) +
                        0.03f * cosf(7.0f * t + ph3);
        return cf{r * cosf(t), r * sinf(t)};
    };
    z1[i] = node(k);
    if (z2) {
        int j = k + shift;
        if (j >= n) j -= n;
        const cf a = node(j);
        const float c = cosf(rot), s = sinf(rot);
        const uint32_t h = tune_hash((uint32_t)i, seed + 6);
        const float ex = 2e-3f * (tune_unit(h) - 0.5f), ey = 2e-3f * (tune_unit(h * 747796405u + 1u) - 0.5f);
        z2[i] = cf{c * a.x - s * a.y + ex, s * a.x + c * a.y + ey};
    }
}

// A uniform batch: one thread per node.
__global__ void k_tune_curves(cf* __restrict__ z1, cf* __restrict__ z2, int n, int64_t pairs, uint32_t seed) {
    const int64_t total = pairs * n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t p = (uint32_t)(i / n);
        tune_node(z1, z2, i, p, (int)(i - (int64_t)p * n), n, seed);
    }
}

// A ragged batch (pair p holds nodes offsets[p] .. offsets[p+1]-1): one block
// per pair, strided over the grid.
__global__ __launch_bounds__(256) void k_tune_curves_ragged(cf* __restrict__ z1, cf* __restrict__ z2,
                                                            const int64_t* __restrict__ offsets, int64_t pairs,
                                                            uint32_t seed) {
    for (int64_t p = blockIdx.x; p < pairs; p += gridDim.x) {
        const int64_t base = offsets[p];
        const int n = (int)(offsets[p + 1] - base);
        for (int k = threadIdx.x; k < n; k += blockDim.x) tune_node(z1, z2, base + k, (uint32_t)p, k, n, seed);
    }
}

}  // namespace ca

namespace {

constexpr int kKnobs = 5;
const char* const kKnobNames[kKnobs] = {"team_grid", "allpairs_cols", "block_plan", "block_grid", "block_threads"};
const int kDefaultThreads[ca::kBlkClasses] = {64, 128, 256, 256, 1024};
const int kTeamSizes[kTeamKeys] = {64, 128, 256, 512, 1024};
const int kClassMax[ca::kBlkClasses] = {512, 1024, 2048, 4096, 8192};

bool team_size(int n) { return ca::team_supported(n); }

// Checks (knob, key, values) against the rules of the header; the message
// names the first violation.
ca_status_t validate(int knob, int key, const std::vector<int>& v) {
    switch (knob) {
        case CA_TUNE_TEAM_GRID:
            if (!team_size(key)) return fail(CA_ERR_INVALID_ARG, "team_grid key must be n in {64, ..., 1024}");
            if (v.size() != 1 || v[0] < 0 || v[0] > 8)
                return fail(CA_ERR_INVALID_ARG, "team_grid takes one value in [0, 8]");
            return CA_OK;
        case CA_TUNE_ALLPAIRS_COLS:
            if (!team_size(key)) return fail(CA_ERR_INVALID_ARG, "allpairs_cols key must be n in {64, ..., 1024}");
            if (v.size() != 1 || v[0] < 1 || v[0] > 256)
                return fail(CA_ERR_INVALID_ARG, "allpairs_cols takes one value in [1, 256]");
            return CA_OK;
        case CA_TUNE_BLOCK_PLAN:
            if (key < 2 || key > kMaxM || !smooth7_size(key))
                return fail(CA_ERR_INVALID_ARG, "block_plan key must be a 7-smooth size in [2, 8192]");
            if (!valid_radices(key, v))
                return fail(CA_ERR_INVALID_ARG,
                            "block_plan takes 1..16 radices from {2, 3, 4, 5, 7, 8} (and 16 for keys above 2048) whose product is the key");
            return CA_OK;
        case CA_TUNE_BLOCK_GRID:
            if (key < 0 || key >= ca::kBlkClasses) return fail(CA_ERR_INVALID_ARG, "block_grid key must be 0..4");
            if (v.size() != 1 || v[0] < 0 || v[0] > 8)
                return fail(CA_ERR_INVALID_ARG, "block_grid takes one value in [0, 8]");
            return CA_OK;
        case CA_TUNE_BLOCK_THREADS:
            if (key != 3 && key != 4) return fail(CA_ERR_INVALID_ARG, "block_threads key must be class 3 or 4");
            if (v.size() != 1 || (v[0] != 256 && v[0] != 512 && (key != 4 || v[0] != 1024)))
                return fail(CA_ERR_INVALID_ARG, "block_threads takes one value: 256 or 512, or 1024 for class 4");
            return CA_OK;
        default:
            return fail(CA_ERR_INVALID_ARG, "unknown tuning knob");
    }
}

std::vector<int> current(const ca_context* c, int knob, int key) {
    switch (knob) {
        case CA_TUNE_TEAM_GRID: return {c->tune.team_grid[team_key(key)]};
        case CA_TUNE_ALLPAIRS_COLS: return {c->tune.allpairs_cols[team_key(key)]};
        case CA_TUNE_BLOCK_PLAN: return radices_for(c, key);
        case CA_TUNE_BLOCK_THREADS: return {c->tune.blk_threads[key]};
        default: return {c->tune.blk_grid[key]};
    }
}

bool is_default(int knob, int key, const std::vector<int>& v) {
    switch (knob) {
        case CA_TUNE_TEAM_GRID: return v[0] == 1;
        case CA_TUNE_ALLPAIRS_COLS: return v[0] == 64;
        case CA_TUNE_BLOCK_PLAN: return v == default_radices(key);
        case CA_TUNE_BLOCK_THREADS: return v[0] == kDefaultThreads[key];
        default: return v[0] == 1;
    }
}

// Installs validated values; a radix schedule also goes to the device tables
// unless `upload` is false (the caller then uploads a batch of sizes).
ca_status_t install(ca_context* c, int knob, int key, const std::vector<int>& v, float ms, bool upload = true) {
    switch (knob) {
        case CA_TUNE_TEAM_GRID: c->tune.team_grid[team_key(key)] = v[0]; break;
        case CA_TUNE_ALLPAIRS_COLS: c->tune.allpairs_cols[team_key(key)] = v[0]; break;
        case CA_TUNE_BLOCK_PLAN:
            if (v == default_radices(key)) c->tune.blk_plan.erase(key);
            else c->tune.blk_plan[key] = v;
            break;
        case CA_TUNE_BLOCK_THREADS: c->tune.blk_threads[key] = v[0]; break;
        default: c->tune.blk_grid[key] = v[0]; break;
    }
    const auto id = std::make_pair(knob, key);
    if (is_default(knob, key, v) && ms < 0.0f) c->tune.ms.erase(id);
    else c->tune.ms[id] = ms;
    if (knob == CA_TUNE_BLOCK_PLAN && upload) return upload_block_plans(c, {key});
    return CA_OK;
}

// Radix schedules tried for size m: the power-of-two part as eights (with a
// trailing four or two), as eights with the remainder first, as fours (with a
// trailing two), as eights and fours alternating, and (sizes of the large
// classes only) as sixteens with the remainder last or first; each with the
// odd radices last or first.  Duplicates removed, the default first.
std::vector<std::vector<int>> plan_candidates(int m) {
    int p2 = 0, rest = m;
    while (rest % 2 == 0) { rest /= 2; ++p2; }
    std::vector<int> odd;
    for (int p : {3, 5, 7})
        while (rest % p == 0) { odd.push_back(p); rest /= p; }
    std::vector<std::vector<int>> pow2;
    {
        std::vector<int> a;
        int e = p2;
        while (e >= 3) { a.push_back(8); e -= 3; }
        if (e == 2) a.push_back(4);
        if (e == 1) a.push_back(2);
        pow2.push_back(a);
        std::vector<int> b;
        if (e == 2) b.push_back(4);
        if (e == 1) b.push_back(2);
        for (int i = 0; i < p2 / 3; ++i) b.push_back(8);
        pow2.push_back(b);
    }
    {
        std::vector<int> a;
        int e = p2;
        while (e >= 2) { a.push_back(4); e -= 2; }
        if (e == 1) a.push_back(2);
        pow2.push_back(a);
    }
    {
        std::vector<int> a;
        int e = p2;
        bool eight = true;
        while (e > 0) {
            const int take = eight ? std::min(e, 3) : std::min(e, 2);
            a.push_back(1 << take);
            e -= take;
            eight = !eight;
        }
        pow2.push_back(a);
    }
    if (m > ca::kBlkR16Min / 2 && p2 >= 4) {
        std::vector<int> a, rem;
        int e = p2;
        while (e >= 4) { a.push_back(16); e -= 4; }
        if (e == 3) rem.push_back(8);
        if (e == 2) rem.push_back(4);
        if (e == 1) rem.push_back(2);
        std::vector<int> b = rem;
        b.insert(b.end(), a.begin(), a.end());
        a.insert(a.end(), rem.begin(), rem.end());
        pow2.push_back(a);
        pow2.push_back(b);
    }
    std::vector<std::vector<int>> out;
    out.push_back(default_radices(m));
    for (const auto& q : pow2) {
        for (int first = 0; first < 2; ++first) {
            std::vector<int> r;
            if (first) r.insert(r.end(), odd.begin(), odd.end());
            r.insert(r.end(), q.begin(), q.end());
            if (!first) r.insert(r.end(), odd.begin(), odd.end());
            if (r.empty() || !valid_radices(m, r)) continue;
            if (std::find(out.begin(), out.end(), r) == out.end()) out.push_back(r);
        }
    }
    return out;
}

// A curve size whose block-engine transform has size m (m itself when m is a
// valid n, else the largest zero-padded n that maps to m), or 0.
int representative_n(int m) {
    if (m <= CA_MAX_N) return m;
    for (int n = CA_MAX_N; n >= 2; --n)
        if (!smooth7(n) && transform_size(n) == m) return n;
    return 0;
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// One warm-up launch, then the mean of three launches between two events.
template <class F>
ca_status_t time_launch(F&& launch, hipStream_t s, Timer& t, float& ms) {
    hipError_t e = launch();
    if (e != hipSuccess) return hip_fail(e, "autotune launch");
    if ((e = hipEventRecord(t.a, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    for (int r = 0; r < 3; ++r)
        if ((e = launch()) != hipSuccess) return hip_fail(e, "autotune launch");
    if ((e = hipEventRecord(t.b, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if ((e = hipEventSynchronize(t.b)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float total = 0.0f;
    if ((e = hipEventElapsedTime(&total, t.a, t.b)) != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    ms = total / 3.0f;
    return CA_OK;
}

ca_status_t gen_curves(void* z1, void* z2, int n, int64_t pairs, hipStream_t s) {
    const int64_t total = pairs * n;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(ca::k_tune_curves, dim3((unsigned)blocks), dim3(256), 0, s, (ca::cf*)z1, (ca::cf*)z2, n,
                       pairs, 17779u);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? CA_OK : hip_fail(e, "curve generator launch");
}

ca_status_t alloc(DevBuf& b, size_t bytes) {
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
        b.p = nullptr;
        return fail(CA_ERR_OOM, "autotune buffers");
    }
    return CA_OK;
}

constexpr int64_t kTuneNodes = int64_t(1) << 25;   // nodes per side of a grid / radix sweep

// A uniform batch of size n, or (offsets non-NULL) a ragged batch whose
// transforms are at most m_cap, binned into the workspace `bins`.
ca::BlkArgs blk_args(ca_context* c, const void* z1, const void* z2, int n, int64_t pairs, ca_result_t* out,
                     const int64_t* offsets = nullptr, int m_cap = kMaxM, int* bins = nullptr) {
    ca::BlkArgs a;
    a.z1 = z1;
    a.z2 = z2;
    a.offsets = offsets;
    a.n_uniform = offsets ? 0 : n;
    a.m_uniform = offsets ? 0 : transform_size(n);
    a.m_cap = m_cap;
    a.num_pairs = pairs;
    a.out = out;
    a.plans = c->d_plans;
    a.tw_arena = c->d_tw32;
    a.rescore = CA_RESCORE_TOP2;
    a.theta64 = 0;
    a.num_cus = c->num_cus;
    for (int k = 0; k < ca::kBlkClasses; ++k) {
        a.grid_mult[k] = c->tune.blk_grid[k];
        a.threads[k] = c->tune.blk_threads[k];
    }
    a.bins = bins;
    return a;
}

// Pair sizes of a ragged batch for a size-class knob: every curve size whose
// block-engine transform falls in the class, drawn by a hash of the pair
// index, until each side holds about `nodes` nodes.
std::vector<int64_t> class_offsets(int cls, int64_t nodes) {
    std::vector<int> sizes;
    const int lo = cls > 0 ? kClassMax[cls - 1] : 0;
    for (int n = 2; n <= CA_MAX_N; ++n) {
        const int m = transform_size(n);
        if (m > lo && m <= kClassMax[cls]) sizes.push_back(n);
    }
    std::vector<int64_t> off(1, 0);
    if (sizes.empty()) return off;
    for (uint32_t p = 0; off.back() < nodes; ++p) {
        uint32_t h = (p + 1u) * 0x9E3779B1u;
        h ^= h >> 15;
        h *= 0x2C1B3C6Du;
        h ^= h >> 12;
        off.push_back(off.back() + sizes[h % (uint32_t)sizes.size()]);
    }
    return off;
}

ca_status_t autotune(ca_context* c, int knob, int key, hipStream_t s, float& best_ms) {
    ca_status_t st = ensure_tables(c, false);
    if (st != CA_OK) return st;
    st = ensure_team_tables(c);
    if (st != CA_OK) return st;
    Timer t;
    hipError_t e;
    if ((e = hipEventCreate(&t.a)) != hipSuccess || (e = hipEventCreate(&t.b)) != hipSuccess)
        return hip_fail(e, "hipEventCreate");

    std::vector<std::vector<int>> cands;
    int n = 0;
    switch (knob) {
        case CA_TUNE_TEAM_GRID:
        case CA_TUNE_BLOCK_GRID:
            cands = {{1}, {2}, {4}, {0}};
            break;
        case CA_TUNE_BLOCK_THREADS:
            if (key == 4) cands = {{256}, {512}, {1024}};
            else cands = {{256}, {512}};
            break;
        case CA_TUNE_ALLPAIRS_COLS:
            cands = {{2}, {4}, {8}, {16}, {32}, {64}};
            break;
        default:
            cands = plan_candidates(key);
            break;
    }
    // a size-class knob is timed on a ragged batch spread over the class
    const bool by_class = knob == CA_TUNE_BLOCK_GRID || knob == CA_TUNE_BLOCK_THREADS;
    if (knob == CA_TUNE_TEAM_GRID || knob == CA_TUNE_ALLPAIRS_COLS) n = key;
    else if (knob == CA_TUNE_BLOCK_PLAN) n = representative_n(key);
    else n = representative_n(kClassMax[key]);
    if (n == 0) return fail(CA_ERR_UNSUPPORTED_N, "no curve size in [2, 4096] uses this transform size");

    DevBuf z1, z2, out, spec, norms, offs, bins;
    int64_t pairs = 0;
    int m = 0;
    if (knob == CA_TUNE_ALLPAIRS_COLS) {
        m = n <= 512 ? 2048 : 1024;
        const int64_t np = (int64_t)m * (m - 1) / 2;
        if ((st = alloc(z1, (size_t)m * n * sizeof(ca::cf))) != CA_OK) return st;
        if ((st = alloc(spec, (size_t)m * n * sizeof(ca::cf))) != CA_OK) return st;
        if ((st = alloc(norms, (size_t)m * sizeof(double))) != CA_OK) return st;
        if ((st = alloc(out, (size_t)np * sizeof(ca_result_t))) != CA_OK) return st;
        if ((st = gen_curves(z1.p, nullptr, n, m, s)) != CA_OK) return st;
        e = ca::launch_spectra(z1.p, m, n, spec.p, (double*)norms.p, team_tw_for(c, n), s);
        if (e != hipSuccess) return hip_fail(e, "spectra kernel launch");
    } else if (by_class) {
        const std::vector<int64_t> h_off = class_offsets(key, kTuneNodes / 2);
        pairs = (int64_t)h_off.size() - 1;
        if (pairs < 1) return fail(CA_ERR_UNSUPPORTED_N, "no curve size in [2, 4096] falls in this size class");
        const size_t nodes = (size_t)h_off.back();
        if ((st = alloc(z1, nodes * sizeof(ca::cf))) != CA_OK) return st;
        if ((st = alloc(z2, nodes * sizeof(ca::cf))) != CA_OK) return st;
        if ((st = alloc(out, (size_t)pairs * sizeof(ca_result_t))) != CA_OK) return st;
        if ((st = alloc(offs, h_off.size() * sizeof(int64_t))) != CA_OK) return st;
        if ((st = alloc(bins, (size_t)ca::blk_bin_ints(pairs) * sizeof(int))) != CA_OK) return st;
        if ((e = hipMemcpyAsync(offs.p, h_off.data(), h_off.size() * sizeof(int64_t), hipMemcpyHostToDevice, s)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return hip_fail(e, "autotune offsets upload");
        const int64_t blocks = std::min<int64_t>(pairs, 65536);
        hipLaunchKernelGGL(ca::k_tune_curves_ragged, dim3((unsigned)blocks), dim3(256), 0, s, (ca::cf*)z1.p,
                           (ca::cf*)z2.p, (const int64_t*)offs.p, pairs, 17779u);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "curve generator launch");
    } else {
        pairs = std::max<int64_t>(1, (knob == CA_TUNE_TEAM_GRID ? kTuneNodes : kTuneNodes / 2) / n);
        if ((st = alloc(z1, (size_t)pairs * n * sizeof(ca::cf))) != CA_OK) return st;
        if ((st = alloc(z2, (size_t)pairs * n * sizeof(ca::cf))) != CA_OK) return st;
        if ((st = alloc(out, (size_t)pairs * sizeof(ca_result_t))) != CA_OK) return st;
        if ((st = gen_curves(z1.p, z2.p, n, pairs, s)) != CA_OK) return st;
    }

    const std::vector<int> before = current(c, knob, key);
    // One candidate: install it where it lives in tables, then time it.
    auto run = [&](size_t i, float& ms) -> ca_status_t {
        const std::vector<int>& v = cands[i];
        if (knob == CA_TUNE_TEAM_GRID) {
            auto launch = [&]() {
                return ca::launch_align_team(z1.p, z2.p, n, pairs, (ca_result_t*)out.p, team_tw_for(c, n),
                                             CA_RESCORE_TOP2, 0, c->num_cus, v[0], s);
            };
            return time_launch(launch, s, t, ms);
        }
        if (knob == CA_TUNE_ALLPAIRS_COLS) {
            auto launch = [&]() {
                return ca::launch_allpairs(z1.p, spec.p, (const double*)norms.p, m, n, (ca_result_t*)out.p,
                                           team_tw_for(c, n), CA_RESCORE_TOP2, 0, v[0], c->num_cus, s);
            };
            return time_launch(launch, s, t, ms);
        }
        if (knob == CA_TUNE_BLOCK_PLAN) {
            if (v == default_radices(key)) c->tune.blk_plan.erase(key);
            else c->tune.blk_plan[key] = v;
            const ca_status_t us = upload_block_plans(c, {key});
            if (us != CA_OK) return us;
        }
        ca::BlkArgs a = by_class ? blk_args(c, z1.p, z2.p, 0, pairs, (ca_result_t*)out.p, (const int64_t*)offs.p,
                                            kClassMax[key], (int*)bins.p)
                                 : blk_args(c, z1.p, z2.p, n, pairs, (ca_result_t*)out.p);
        if (knob == CA_TUNE_BLOCK_GRID) a.grid_mult[key] = v[0];
        if (knob == CA_TUNE_BLOCK_THREADS) a.threads[key] = v[0];
        auto launch = [&]() { return ca::launch_align_blk_f32(a, s); };
        return time_launch(launch, s, t, ms);
    };
    // The GPU clock needs tens of milliseconds of load to settle: run the
    // first candidate for at least ~20 ms before timing, then time every
    // candidate in each of three rounds and keep its best time.
    float warm = 0.0f;
    if ((st = run(0, warm)) != CA_OK) {
        (void)install(c, knob, key, before, -1.0f);
        return st;
    }
    for (int r = 0, reps = (int)(20.0f / fmaxf(4.0f * warm, 0.05f)); r < reps && r < 400; ++r)
        if ((st = run(0, warm)) != CA_OK) break;
    std::vector<float> best_of(cands.size(), 3.0e38f);
    for (int round = 0; round < 3 && st == CA_OK; ++round) {
        for (size_t i = 0; i < cands.size(); ++i) {
            float ms = 0.0f;
            if ((st = run(i, ms)) != CA_OK) break;
            best_of[i] = fminf(best_of[i], ms);
        }
    }
    int best = 0;
    for (size_t i = 1; i < cands.size(); ++i)
        if (best_of[i] < best_of[best]) best = (int)i;
    best_ms = best_of[best];
    if (st != CA_OK) {
        (void)install(c, knob, key, before, -1.0f);   // leave the previous choice in place
        return st;
    }
    return install(c, knob, key, cands[best], best_ms);
}

// ------------------------------------------------------------------ JSON
// A small reader for the cache format (objects, arrays, strings without
// escapes other than \" and \\, numbers, true/false/null).
struct JVal {
    enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
    double num = 0.0;
    std::string str;
    std::vector<JVal> arr;
    std::vector<std::pair<std::string, JVal>> obj;
    const JVal* get(const char* k) const {
        for (const auto& kv : obj)
            if (kv.first == k) return &kv.second;
        return nullptr;
    }
};

struct JParser {
    const char* p;
    const char* end;
    int depth = 0;
    void ws() {
        while (p < end && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
    }
    bool lit(const char* s) {
        const size_t k = strlen(s);
        if ((size_t)(end - p) < k || strncmp(p, s, k) != 0) return false;
        p += k;
        return true;
    }
    bool string(std::string& out) {
        if (p >= end || *p != '"') return false;
        ++p;
        out.clear();
        while (p < end && *p != '"') {
            if (*p == '\\') {
                ++p;
                if (p >= end || (*p != '"' && *p != '\\')) return false;
            }
            out.push_back(*p++);
        }
        if (p >= end) return false;
        ++p;
        return true;
    }
    bool value(JVal& v) {
        if (++depth > 16) return false;
        ws();
        bool ok = false;
        if (p >= end) {
            ok = false;
        } else if (*p == '{') {
            v.kind = JVal::OBJ;
            ++p;
            ws();
            if (p < end && *p == '}') {
                ++p;
                ok = true;
            } else {
                for (;;) {
                    ws();
                    std::pair<std::string, JVal> kv;
                    if (!string(kv.first)) break;
                    ws();
                    if (p >= end || *p != ':') break;
                    ++p;
                    if (!value(kv.second)) break;
                    v.obj.push_back(std::move(kv));
                    ws();
                    if (p < end && *p == ',') { ++p; continue; }
                    if (p < end && *p == '}') { ++p; ok = true; }
                    break;
                }
            }
        } else if (*p == '[') {
            v.kind = JVal::ARR;
            ++p;
            ws();
            if (p < end && *p == ']') {
                ++p;
                ok = true;
            } else {
                for (;;) {
                    JVal x;
                    if (!value(x)) break;
                    v.arr.push_back(std::move(x));
                    ws();
                    if (p < end && *p == ',') { ++p; continue; }
                    if (p < end && *p == ']') { ++p; ok = true; }
                    break;
                }
            }
        } else if (*p == '"') {
            v.kind = JVal::STR;
            ok = string(v.str);
        } else if (lit("true") || lit("false")) {
            v.kind = JVal::BOOL;
            ok = true;
        } else if (lit("null")) {
            v.kind = JVal::NUL;
            ok = true;
        } else {
            std::string num;
            while (p < end && (isdigit((unsigned char)*p) || *p == '-' || *p == '+' || *p == '.' || *p == 'e' ||
                               *p == 'E'))
                num.push_back(*p++);
            char* stop = nullptr;
            v.kind = JVal::NUM;
            v.num = num.empty() ? 0.0 : strtod(num.c_str(), &stop);
            ok = !num.empty() && stop && *stop == '\0' && isfinite(v.num);
        }
        --depth;
        return ok;
    }
};

bool as_int(const JVal* v, int& out) {
    if (!v || v->kind != JVal::NUM || v->num != floor(v->num) || fabs(v->num) > 1e9) return false;
    out = (int)v->num;
    return true;
}

int knob_of(const std::string& s) {
    for (int k = 0; k < kKnobs; ++k)
        if (s == kKnobNames[k]) return k;
    return -1;
}

struct Entry {
    int knob, key;
    std::vector<int> values;
    float ms;
};

ca_status_t parse_cache(const std::string& text, std::string& arch, int& cus, std::vector<Entry>& entries) {
    JParser jp{text.data(), text.data() + text.size()};
    JVal root;
    if (!jp.value(root)) return fail(CA_ERR_INVALID_ARG, "tuning file is not valid JSON");
    jp.ws();
    if (jp.p != jp.end) return fail(CA_ERR_INVALID_ARG, "tuning file has trailing characters");
    if (root.kind != JVal::OBJ) return fail(CA_ERR_INVALID_ARG, "tuning file must hold a JSON object");
    const JVal* fmt = root.get("format");
    if (!fmt || fmt->kind != JVal::STR || fmt->str != "curvealign-tune/1")
        return fail(CA_ERR_INVALID_ARG, "tuning file format must be \"curvealign-tune/1\"");
    const JVal* a = root.get("arch");
    if (!a || a->kind != JVal::STR) return fail(CA_ERR_INVALID_ARG, "tuning file lacks \"arch\"");
    arch = a->str;
    if (!as_int(root.get("num_cus"), cus)) return fail(CA_ERR_INVALID_ARG, "tuning file lacks \"num_cus\"");
    const JVal* es = root.get("entries");
    if (!es || es->kind != JVal::ARR) return fail(CA_ERR_INVALID_ARG, "tuning file lacks \"entries\"");
    for (const JVal& e : es->arr) {
        Entry en;
        const JVal* kn = e.kind == JVal::OBJ ? e.get("knob") : nullptr;
        if (!kn || kn->kind != JVal::STR || (en.knob = knob_of(kn->str)) < 0)
            return fail(CA_ERR_INVALID_ARG, "tuning entry with an unknown knob");
        if (!as_int(e.get("key"), en.key)) return fail(CA_ERR_INVALID_ARG, "tuning entry without an integer key");
        const JVal* vs = e.get("values");
        if (!vs || vs->kind != JVal::ARR || vs->arr.size() > 16)
            return fail(CA_ERR_INVALID_ARG, "tuning entry without a values array");
        for (const JVal& x : vs->arr) {
            int iv = 0;
            if (!as_int(&x, iv)) return fail(CA_ERR_INVALID_ARG, "tuning entry values must be integers");
            en.values.push_back(iv);
        }
        const JVal* ms = e.get("ms");
        en.ms = (ms && ms->kind == JVal::NUM) ? (float)ms->num : -1.0f;
        const ca_status_t st = validate(en.knob, en.key, en.values);
        if (st != CA_OK) return st;
        entries.push_back(std::move(en));
    }
    return CA_OK;
}

}  // namespace

extern "C" {

ca_status_t ca_autotune(ca_context_t c, int32_t knob, int32_t key, float* best_ms, void* stream) {
    if (!c) return fail(CA_ERR_INVALID_ARG, "context is NULL");
    if (knob < 0 || knob >= kKnobs) return fail(CA_ERR_INVALID_ARG, "unknown tuning knob");
    if (knob == CA_TUNE_TEAM_GRID || knob == CA_TUNE_ALLPAIRS_COLS) {
        if (!team_size(key)) return fail(CA_ERR_UNSUPPORTED_N, "key must be n in {64, 128, 256, 512, 1024}");
    } else if (knob == CA_TUNE_BLOCK_PLAN) {
        if (key < 2 || key > kMaxM || !smooth7_size(key))
            return fail(CA_ERR_UNSUPPORTED_N, "block_plan key must be a 7-smooth size in [2, 8192]");
    } else if (knob == CA_TUNE_BLOCK_THREADS) {
        if (key != 3 && key != 4) return fail(CA_ERR_INVALID_ARG, "block_threads key must be class 3 or 4");
    } else if (key < 0 || key >= ca::kBlkClasses) {
        return fail(CA_ERR_INVALID_ARG, "block_grid key must be 0..4");
    }
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    float ms = 0.0f;
    const ca_status_t st = autotune(c, knob, key, (hipStream_t)stream, ms);
    if (st == CA_OK && best_ms) *best_ms = ms;
    return st;
}

ca_status_t ca_tune_get(ca_context_t c, int32_t knob, int32_t key, int32_t* values, int32_t* count) {
    if (!c) return fail(CA_ERR_INVALID_ARG, "context is NULL");
    if (!values || !count) return fail(CA_ERR_INVALID_ARG, "values and count must be non-NULL");
    if (knob < 0 || knob >= kKnobs) return fail(CA_ERR_INVALID_ARG, "unknown tuning knob");
    if (knob == CA_TUNE_BLOCK_PLAN && (key < 2 || key > kMaxM || !smooth7_size(key)))
        return fail(CA_ERR_INVALID_ARG, "block_plan key must be a 7-smooth size in [2, 8192]");
    std::vector<int> probe = knob == CA_TUNE_BLOCK_PLAN ? default_radices(key) : std::vector<int>{1};
    if (knob == CA_TUNE_ALLPAIRS_COLS) probe = {64};
    if (knob == CA_TUNE_BLOCK_THREADS) probe = {256};
    ca_status_t st = validate(knob, key, probe);        // key check only
    if (st != CA_OK) return st;
    std::lock_guard<std::mutex> lk(c->mu);
    const std::vector<int> v = current(c, knob, key);
    if (*count < (int32_t)v.size()) return fail(CA_ERR_INVALID_ARG, "values capacity too small");
    for (size_t i = 0; i < v.size(); ++i) values[i] = v[i];
    *count = (int32_t)v.size();
    return CA_OK;
}

ca_status_t ca_tune_set(ca_context_t c, int32_t knob, int32_t key, const int32_t* values, int32_t count) {
    if (!c) return fail(CA_ERR_INVALID_ARG, "context is NULL");
    if (!values || count < 1 || count > 16) return fail(CA_ERR_INVALID_ARG, "values must hold 1..16 entries");
    const std::vector<int> v(values, values + count);
    ca_status_t st = validate(knob, key, v);
    if (st != CA_OK) return st;
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    return install(c, knob, key, v, -1.0f);
}

ca_status_t ca_tune_save(ca_context_t c, const char* path) {
    if (!c) return fail(CA_ERR_INVALID_ARG, "context is NULL");
    if (!path) return fail(CA_ERR_INVALID_ARG, "path is NULL");
    std::lock_guard<std::mutex> lk(c->mu);
    std::vector<std::pair<int, int>> ids;
    for (int i = 0; i < kTeamKeys; ++i) {
        ids.push_back({CA_TUNE_TEAM_GRID, kTeamSizes[i]});
        ids.push_back({CA_TUNE_ALLPAIRS_COLS, kTeamSizes[i]});
    }
    for (const auto& kv : c->tune.blk_plan) ids.push_back({CA_TUNE_BLOCK_PLAN, kv.first});
    for (int k = 0; k < ca::kBlkClasses; ++k) ids.push_back({CA_TUNE_BLOCK_GRID, k});
    for (int k = 3; k < ca::kBlkClasses; ++k) ids.push_back({CA_TUNE_BLOCK_THREADS, k});
    for (const auto& kv : c->tune.ms)   // measured defaults are kept too (they record the sweep)
        if (std::find(ids.begin(), ids.end(), kv.first) == ids.end()) ids.push_back(kv.first);
    std::sort(ids.begin(), ids.end());
    std::string s = "{\"format\": \"curvealign-tune/1\", \"arch\": \"" + c->arch +
                    "\", \"num_cus\": " + std::to_string(c->num_cus) + ",\n \"entries\": [";
    bool first = true;
    for (const auto& id : ids) {
        const std::vector<int> v = current(c, id.first, id.second);
        auto it = c->tune.ms.find(id);
        if (is_default(id.first, id.second, v) && it == c->tune.ms.end()) continue;
        char ms[32];
        snprintf(ms, sizeof(ms), "%.6g", it == c->tune.ms.end() ? -1.0 : (double)it->second);
        s += first ? "\n  " : ",\n  ";
        first = false;
        s += "{\"knob\": \"" + std::string(kKnobNames[id.first]) + "\", \"key\": " + std::to_string(id.second) +
             ", \"values\": [";
        for (size_t i = 0; i < v.size(); ++i) s += (i ? ", " : "") + std::to_string(v[i]);
        s += "], \"ms\": " + std::string(ms) + "}";
    }
    s += "\n ]}\n";
    FILE* f = fopen(path, "wb");
    if (!f) return fail(CA_ERR_INVALID_ARG, std::string("cannot write ") + path);
    const bool ok = fwrite(s.data(), 1, s.size(), f) == s.size();
    if (fclose(f) != 0 || !ok) return fail(CA_ERR_INVALID_ARG, std::string("write failed: ") + path);
    return CA_OK;
}

ca_status_t ca_tune_load(ca_context_t c, const char* path, int32_t* applied) {
    if (!c) return fail(CA_ERR_INVALID_ARG, "context is NULL");
    if (!path) return fail(CA_ERR_INVALID_ARG, "path is NULL");
    if (applied) *applied = 0;
    FILE* f = fopen(path, "rb");
    if (!f) return fail(CA_ERR_INVALID_ARG, std::string("cannot read ") + path);
    std::string text;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof(buf), f)) > 0 && text.size() < (1u << 22)) text.append(buf, k);
    fclose(f);
    std::string arch;
    int cus = 0;
    std::vector<Entry> entries;
    ca_status_t st = parse_cache(text, arch, cus, entries);
    if (st != CA_OK) return st;
    std::lock_guard<std::mutex> lk(c->mu);
    if (arch != c->arch || cus != c->num_cus) return CA_OK;
    DeviceGuard g(c->device);
    int32_t n = 0;
    std::vector<int> plans;
    for (const Entry& e : entries) {
        if ((st = install(c, e.knob, e.key, e.values, e.ms, false)) != CA_OK) return st;
        if (e.knob == CA_TUNE_BLOCK_PLAN) plans.push_back(e.key);
        ++n;
    }
    if ((st = upload_block_plans(c, plans)) != CA_OK) return st;
    if (applied) *applied = n;
    return CA_OK;
}

}  // extern "C"
