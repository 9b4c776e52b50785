// Library context and the host helpers shared by the C ABI (capi.cpp) and
// the autotuner (tune.hip).  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/curvealign.h"
#include "fft_engines.hpp"
#include "launch.hpp"

namespace ca {
namespace host {

constexpr int kMaxM = 2 * CA_MAX_N;    // largest block-engine transform (zero-padded n = 4096)
constexpr int kFp64MaxM = CA_MAX_N;    // LDS of the FP64 block engine
constexpr int kTeamKeys = 5;           // team / all-pairs sizes 64, 128, 256, 512, 1024

// Runtime launch choices of one context.  Every field has a default that
// needs no tuning; ca_autotune measures the candidates and ca_tune_set /
// ca_tune_load install choices.
struct Tuning {
    int team_grid[kTeamKeys] = {1, 1, 1, 1, 1};       // per log2(n) - 6: occupancy multiples, 0 = one block per group
    int allpairs_cols[kTeamKeys] = {64, 64, 64, 64, 64};
    int blk_grid[kBlkClasses] = {1, 1, 1, 1, 1};
    int blk_threads[kBlkClasses] = {64, 128, 256, 256, 1024};   // classes 3 and 4 (FP32) are tunable
    std::map<int, std::vector<int>> blk_plan;           // transform size -> radices (absent: default)
    std::map<std::pair<int, int>, float> ms;            // (knob, key) -> measured time of the choice
};

}  // namespace host
}  // namespace ca

struct ca_context {
    int device = 0;
    int num_cus = 0;
    size_t lds_per_block = 0;
    std::string arch;
    std::mutex mu;
    // block-engine plans for every n in [0, CA_MAX_N] and the twiddle arenas
    ca::Plan* d_plans = nullptr;
    std::vector<ca::Plan> h_plans;
    std::vector<int64_t> tw_off;   // per transform size M: offset of its twiddles in the arenas (-1: none)
    void* d_tw32 = nullptr;   // float2 arena
    void* d_tw64 = nullptr;   // double2 arena
    void* d_team_tw[11] = {};  // per-pass team-engine twiddles, index log2(n)
    void* d_bf16 = nullptr;    // split-BF16 per-lane constants, n = 128 (64 x 128 bytes)
    void* d_bf16_1k = nullptr; // split-BF16 constants and twiddles, n = 1024
    // resampler scratch and the list of curves for the general kernel
    void* d_rs = nullptr;
    int64_t rs_slots = 0;
    int* d_slow = nullptr;          // [0] = count, [1..] = curve indices
    size_t slow_bytes = 0;
    // block-engine size-class lists of ragged batches
    int* d_bins = nullptr;
    size_t bins_bytes = 0;
    // all-pairs spectra workspace
    void* d_spec = nullptr;
    size_t spec_bytes = 0;
    double* d_norms = nullptr;
    size_t norms_bytes = 0;
    // library-owned capture stream of ca_graph_begin / ca_graph_end
    hipStream_t cap_stream = nullptr;
    bool capturing = false;
    bool capture_failed = false;
    // device address of the allocation-free entry point's static scratch on
    // this context's device (looked up by ca_create)
    void* noalloc_scratch = nullptr;
    // workspace buffers the context has outgrown: kept until ca_destroy,
    // since graphs captured before the growth still address them
    std::vector<void*> retired;
    ca::host::Tuning tune;
};

// A HIP graph recorded by ca_graph_begin / ca_graph_end.
struct ca_graph {
    int device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace ca {
namespace host {

ca_status_t fail(ca_status_t st, const std::string& msg);
ca_status_t hip_fail(hipError_t e, const char* what);

bool smooth7_size(int m);
bool smooth7(int n);
int transform_size(int n);

// Radix schedules of the block engine: the default one, and a plan from a
// radix list (radices 2, 3, 4, 5, 7, 8 whose product is the size).
std::vector<int> default_radices(int m);
bool valid_radices(int m, const std::vector<int>& r);
Plan plan_from(int m, const std::vector<int>& r);
std::vector<int> radices_for(const ca_context* c, int m);

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

ca_status_t ensure_tables(ca_context* c, bool need64);
ca_status_t ensure_team_tables(ca_context* c);
const void* team_tw_for(ca_context* c, int n);
// Installs the current radix schedules of the given transform sizes in the
// device plan table and both twiddle arenas (synchronises the device first).
ca_status_t upload_block_plans(ca_context* c, const std::vector<int>& sizes);

inline int team_key(int n) {
    int lg = 0;
    while ((1 << lg) < n) ++lg;
    return lg - 6;
}

}  // namespace host
}  // namespace ca
