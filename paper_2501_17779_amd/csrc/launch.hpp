// Host-side launch wrappers for the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/curvealign.h"

namespace ca {

struct Plan;

struct BlkArgs {
    const void* z1;
    const void* z2;
    const int64_t* offsets;   // device, or nullptr for a uniform batch
    int n_uniform;
    int n_max;                // largest n the launch must hold in LDS
    int64_t num_pairs;
    ca_result_t* out;
    const Plan* plans;        // device table indexed by n
    const void* tw_arena;     // device twiddle arena (float2 or double2)
    int rescore;
    int theta64;
};

// One pair per workgroup, LDS-resident Stockham FFT, any supported n.
// Dynamic LDS bytes of one launch (the caller checks it against the device).
size_t blk_dynamic_lds(int n_max, size_t elem);
hipError_t launch_align_blk_f32(const BlkArgs& a, hipStream_t s);
hipError_t launch_align_blk_f64(const BlkArgs& a, hipStream_t s);

// Register-resident team FFT for n in {64, 128, 256, 512, 1024}, FP32.
bool team_supported(int n);
hipError_t launch_align_team(const void* z1, const void* z2, int n, int64_t num_pairs,
                             ca_result_t* out, const void* tw, int rescore, int theta64,
                             hipStream_t s);

// All-pairs: per-curve spectra, then the upper-triangle tile kernel.
hipError_t launch_spectra(const void* curves, int m, int n, void* spectra, double* norms,
                          const void* tw, hipStream_t s);
hipError_t launch_allpairs(const void* curves, const void* spectra, const double* norms, int m,
                           int n, ca_result_t* out, const void* tw, int rescore, int theta64,
                           hipStream_t s);
bool allpairs_supported(int n);

// Arc-length resampling, one workgroup per curve.
hipError_t launch_resample(const void* raw, const int64_t* raw_off, int64_t num_curves,
                           const int64_t* out_off, void* out, double* norms, uint32_t* flags,
                           int mode, void* scratch, int64_t scratch_per_curve_bytes,
                           int64_t curves_per_launch, hipStream_t s);

}  // namespace ca
