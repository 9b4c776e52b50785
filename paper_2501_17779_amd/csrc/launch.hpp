// Host-side launch wrappers for the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/curvealign.h"

namespace ca {

struct Plan;

constexpr int kBlkClasses = 5;

struct BlkArgs {
    const void* z1;
    const void* z2;
    const int64_t* offsets;   // device, or nullptr for a uniform batch
    int n_uniform;
    int m_uniform;            // transform size of a uniform batch (n, or the padded size)
    int m_cap;                // largest transform size this precision supports
    int64_t num_pairs;
    ca_result_t* out;
    const Plan* plans;        // device table indexed by n: the plan of n's transform
    const void* tw_arena;     // device twiddle arena (float2 or double2)
    int rescore;
    int theta64;
    int num_cus;
    // persistent blocks per CU of each size class, in multiples of the
    // kernel's occupancy limit; 0 = one block per pair
    int grid_mult[kBlkClasses];
    // threads per block of the FP32 classes 3 and 4 (256 or 512, or 1024 for class 4; other
    // classes and FP64 use their fixed sizes)
    int threads[kBlkClasses];
    // ragged batches: device workspace of kBlkClasses counters (kBinStride
    // ints apart, one cache line each) followed by kBlkClasses lists of
    // num_pairs pair indices (blk_bin_ints(num_pairs) ints)
    int* bins;
};

constexpr int kBinStride = 32;
inline int64_t blk_bin_ints(int64_t num_pairs) { return kBlkClasses * kBinStride + kBlkClasses * num_pairs; }

// Persistent size-class kernels, one pair per workgroup at a time,
// LDS-resident Stockham FFT.  A 7-smooth n is transformed at size n; any
// other n uses the zero-padded correlation at the 7-smooth size M >= 2n of
// its plan (curve 1 padded with zeros, curve 2 repeated twice).
hipError_t launch_align_blk_f32(const BlkArgs& a, hipStream_t s);
hipError_t launch_align_blk_f64(const BlkArgs& a, hipStream_t s);

// Register-resident team FFT for n in {64, 128, 256, 512, 1024}, FP32.
// `tw` is the per-pass twiddle table of team_twiddle_count(n) entries
// (see TeamCfg): entry TWO + (r - 1) NS + k = w_{NS RP}^{r k}.
bool team_supported(int n);
int team_twiddle_count(int n);
// The persistent grid is grid_mult times the occupancy limit per CU
// (grid_mult = 0: one block per group of pairs).
hipError_t launch_align_team(const void* z1, const void* z2, int n, int64_t num_pairs,
                             ca_result_t* out, const void* tw, int rescore, int theta64,
                             int num_cus, int grid_mult, hipStream_t s);

// Split-BF16 MFMA path, n = 128, two pairs per wave.  lane_consts: 64
// per-lane blocks of 192 bytes (the 16-point DFT matrix and the
// pair-block-diagonal 8-point one as BF16 hi/lo operands of the 16x16x32
// MFMA, and the twiddles of both transform kinds).
hipError_t launch_align_bf16(const void* z1, const void* z2, int64_t num_pairs, ca_result_t* out,
                             const void* lane_consts, int theta64, int num_cus, hipStream_t s);
// Split-BF16 MFMA path, n = 1024 (four-step 32 x 32 DFTs on the 32x32x16
// MFMA).  tables: 64 per-lane blocks of 192 bytes (the 32-point DFT matrix
// Re, Im and -Im parts as BF16 hi/lo operands) followed by the per-lane
// twiddles w_1024^{row c} as 8 x 64 float4.
constexpr int kBf16Tables1kBytes = 64 * 192 + 8 * 64 * 16;
hipError_t launch_align_bf16_1k(const void* z1, const void* z2, int64_t num_pairs, ca_result_t* out,
                                const void* tables, int theta64, int num_cus, hipStream_t s);

// All-pairs: per-curve spectra, then the upper-triangle tile kernel with
// tiles of (pairs per block) rows x `cols` columns over a persistent grid
// (the occupancy limit on every CU).
hipError_t launch_spectra(const void* curves, int m, int n, void* spectra, double* norms,
                          const void* tw, hipStream_t s);
hipError_t launch_allpairs(const void* curves, const void* spectra, const double* norms, int m,
                           int n, ca_result_t* out, const void* tw, int rescore, int theta64,
                           int cols, int num_cus, hipStream_t s);
bool allpairs_supported(int n);

// Hand-off records -> (t0*, R*) in the paper's notation.
hipError_t launch_initializer(const ca_result_t* res, int n, const int64_t* offsets, int64_t count,
                              double* t0, double* rot, hipStream_t s);

// Square-root-velocity transform (section 3), one wave per curve.
hipError_t launch_srv(const void* z, const int64_t* offsets, int n, int64_t count, void* q, int num_cus,
                      hipStream_t s);

// Arc-length resampling, one workgroup per curve.
// A wave-per-curve fast kernel handles every curve it can; the others (fewer
// than 3 vertices, duplicates, non-finite values, above the vertex cap) are
// listed in slow_list (count in *slow_count, device) and resampled by the
// general workgroup-per-curve kernel with `slots` scratch slots.
hipError_t launch_resample(const void* raw, const int64_t* raw_off, int64_t num_curves,
                           const int64_t* out_off, void* out, double* norms, uint32_t* flags,
                           int mode, void* scratch, int64_t slot_bytes, int64_t slots,
                           int* slow_count, int* slow_list, hipStream_t s);

}  // namespace ca
