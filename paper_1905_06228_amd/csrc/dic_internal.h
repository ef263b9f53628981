// Internal types shared by the host API and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dic.h"

namespace dic {

constexpr int kMaxM = 20;
constexpr int kMaxS = 32;
constexpr int kWave = 64;
constexpr int kMaxRefineSlack = 16;  // largest tuning icgn_slack
// Particle swarm search (Sec. 2.1, Eqs. 2-4; settings of Sec. 5.2)
constexpr int kPsoParticles = 50;
constexpr int kPsoGenerations = 5;
constexpr int kPsoStar = 5;            // positions per particle and generation, modified form
constexpr double kPsoC1 = 2.0, kPsoC2 = 2.0;
constexpr double kPsoStopCC = 0.995;

// Interpolation of the deformed image in the FP32 refinements.
enum Interp : int {
  kInterpBicubic = 0,     // Keys taps from the LDS patch (or the image)
  kInterpBilinear = 1,    // Eq. (5), 2x2 taps from the LDS patch (or the image)
  kInterpBicubicLut = 2,  // Keys interpolant from the per-cell coefficient table
  kInterpBSpline = 3,     // cubic B-spline, 4x4 taps of the spline coefficient image
};
__host__ __device__ constexpr int interp_taps(int im) { return im == kInterpBilinear ? 2 : 4; }

// Device copy of a pair description plus derived offsets.
struct DevPair {
  int32_t width, height, M, S;
  int64_t ref_off, def_off;
  int64_t poi_off, poi_count;
  int64_t grad_off;  // float offset of this pair's [2, H, W] gradient block
  int64_t tmpl_off;  // float offset of this pair's templates
  int32_t tmpl_pitch;  // template row pitch: 2M+1 rounded up to a multiple of 8,
                       // zero-filled beyond the subset, (2M+1) rows per POI
  int32_t pad_;
  int64_t box_off;   // double offset of this pair's five [H, W] box-sum planes:
                     // column sums of g and g^2, subset sums of g and g^2, and
                     // float pairs (subset mean, 1/sqrt(sum (g - mean)^2))
  int64_t lut_off;   // float4 offset of this pair's [H, W, 4] bicubic coefficient
                     // table (DIC_FLAG_BICUBIC_LUT) or of its [H, W] B-spline
                     // coefficient image followed by an [H, W] scratch image
                     // (DIC_FLAG_INTERP_BSPLINE)
};

__host__ __device__ __forceinline__ int template_pitch(int M) { return (2 * M + 1 + 7) / 8 * 8; }

// Per-POI reference-side record.  Everything the search and IC-GN need from
// the reference subset, computed once.
struct RefRec {
  double fbar;       // subset mean
  double df;         // sqrt(sum (f - fbar)^2)
  double sd_sum[6];  // sum_i SD_i
  double sdf_sum[6]; // sum_i SD_i (f_i - fbar)
  double L[21];      // Cholesky factor of the centred Hessian, packed rows
  double rdiag[6];   // 1 / L_kk
  float tsum;        // sum of the float search template (f_i - fbar)
  int32_t status;    // DIC_POI_*
};

// Device-visible state of a bound plan.
struct DevState {
  const DevPair* pairs;
  const int32_t* poi_pair;  // pair index of every POI
  const int32_t* work;      // POI indices, decreasing subset size
  int32_t* counters;        // persistent-launch work counters
  float* grads;             // gradient arena
  RefRec* recs;             // [N]
  float* tmpl;              // template arena (written for the vector-ALU search form)
  double* box;              // box-sum arena (deformed images)
  float* lut;               // bicubic coefficient tables (16 floats per pixel) or B-spline
                            // coefficient images (1 float per pixel, then 1 of scratch) of
                            // the deformed images
  int32_t* bsp_flags;       // per pair: the deformed image has a non-finite pixel (B-spline)
  int64_t N;
  int32_t num_pairs;
  int32_t maxM, maxS;
  int32_t max_width, max_height;
  int32_t max_iters;
  double conv_tol;
};

// Persistent-launch work counters: one per search group, then one per
// refinement group.
enum Counter { kCtrSearch = 0, kMaxSearchGroups = 16, kCtrIcgn = 16, kNumCounters = 32 };

// A run of the work list whose subsets share the search kernel's template
// row length NP (the work list is ordered by decreasing subset size).
struct SearchGroup {
  int np;
  int64_t begin, count;
};

// Refinement kernels (IC-GN, Newton-Raphson) come in sizes of 4, 8, 12, 16,
// 20 and 28 sample slots per lane (64 samples per slot); subsets of 29 and 31
// columns (M = 14, 15) use the 16-slot kernel with two subset rows per slot.
// A plan refines its work list (ordered by decreasing M) in runs of POIs that
// share a kernel, one persistent launch each, so a small subset never runs in
// a kernel sized (registers, LDS patch) for the plan's largest one.
__host__ __device__ constexpr int refine_slots(int M) {
  return ((2 * M + 1) * (2 * M + 1) + 63) / 64 <= 4    ? 4
         : ((2 * M + 1) * (2 * M + 1) + 63) / 64 <= 8  ? 8
         : ((2 * M + 1) * (2 * M + 1) + 63) / 64 <= 12 ? 12
         : ((2 * M + 1) * (2 * M + 1) + 63) / 64 <= 16 ? 16
         : ((2 * M + 1) * (2 * M + 1) + 63) / 64 <= 20 ? 20
                                                       : 28;
}
// The two-rows layout serves M = kR2MinM and kR2MinM + 1.
constexpr int kR2MinM = 14;
__host__ __device__ constexpr bool refine_two_rows(int M) { return M == kR2MinM || M == kR2MinM + 1; }
// The fewest slots a subset of the maxs-slot class fills: one more than the
// next smaller class holds.  Slots below it need no per-slot test.
__host__ __device__ constexpr int refine_min_slots(int maxs) {
  return maxs <= 4 ? 1 : maxs <= 8 ? 5 : maxs <= 12 ? 9 : maxs <= 16 ? 13 : maxs <= 20 ? 17 : 21;
}
// the refinement kernel a radius runs in (slots and layout)
__host__ __device__ constexpr int refine_class(int M) {
  return 2 * refine_slots(M) + (refine_two_rows(M) ? 1 : 0);
}
struct RefineGroup {
  int64_t begin, count;  // a run of the work list
  int maxM;              // its largest subset radius (the first in the run)
};
constexpr int kMaxRefineGroups = 16;

// Kernel launchers (defined in the .hip files).  All asynchronous on `s`.
hipError_t launch_reset_counters(const DevState& st, hipStream_t s);
hipError_t launch_gradients(const DevState& st, const float* ref, hipStream_t s);
hipError_t launch_box_sums(const DevState& st, const float* def, hipStream_t s);
hipError_t launch_bicubic_lut(const DevState& st, const float* def, hipStream_t s);
hipError_t launch_bspline_coeffs(const DevState& st, const float* def, hipStream_t s);
hipError_t launch_pso(const DevState& st, bool modified, const float* ref, const float* def,
                      const int32_t* poi, const int32_t* seed, const float* rand, int32_t* uv,
                      float* zn, int32_t* status, int32_t* gens, int32_t* evals, int num_cu,
                      hipStream_t s);
// write_tmpl: also store the FP32 search template (read by the vector-ALU
// search form only).  groups: the plan's refinement runs of the work list
// (the statistics kernel is sized per run).
hipError_t launch_ref_prep_f32(const DevState& st, const RefineGroup* groups, int ngroups,
                               const float* ref, const int32_t* poi, bool write_tmpl,
                               hipStream_t s);
// The two halves of launch_ref_prep_f32: the statistics the search reads
// (mean, norm, template sum, status), then the steepest-descent sums,
// Hessian and factor IC-GN reads (after the gradients).
hipError_t launch_ref_prep_stats(const DevState& st, const RefineGroup* groups, int ngroups,
                                 const float* ref, const int32_t* poi, bool write_tmpl,
                                 hipStream_t s);
hipError_t launch_ref_prep_hessian(const DevState& st, const float* ref, const int32_t* poi,
                                   hipStream_t s);
hipError_t launch_ref_prep_f64(const DevState& st, const DevPair* host_pairs,
                               const float* ref, const int32_t* poi, hipStream_t s);
hipError_t launch_search_f32(const DevState& st, const dic_tuning_t& tu,
                             const SearchGroup* groups, int ngroups, const float* ref,
                             const float* def, const int32_t* poi, const int32_t* seed,
                             int32_t* uv, float* zncc, int32_t* status, int num_cu,
                             hipStream_t s);
// Matrix-core search (tuning search_block == kMfmaBlock): windows up to
// +-kMfmaMaxS, grouped by the number of 16-wide K blocks a template row of
// 2M+1 plus the 32 Toeplitz shifts spans.
constexpr int kMfmaBlock = 32;
constexpr int kMfmaMaxS = 16;       // one tile, or two for a 33 x 33 window
constexpr int kMfmaWideMaxS = 31;   // 2 x 2 tiles of 32 x 32 candidates
__host__ __device__ __forceinline__ int mfma_kb(int M) { return (2 * M + 48) / 16; }
hipError_t launch_search_mfma(const DevState& st, const dic_tuning_t& tu,
                              const SearchGroup* groups, int ngroups, const float* ref,
                              const float* def, const int32_t* poi, const int32_t* seed,
                              int32_t* uv, float* zncc, int32_t* status, int num_cu,
                              hipStream_t s);
// LDS bytes of one matrix-core search wave (one wave per workgroup); `wide`
// for windows beyond +-kMfmaMaxS.
size_t search_mfma_wave_lds(int kb, int maxM, bool wide);
// Template row length the search kernel with tile width `block` uses.
__host__ __device__ __forceinline__ int search_np(int M, int block) {
  return (2 * M + 1 + block - 1) / block * block;
}
hipError_t launch_search_f64(const DevState& st, const DevPair* host_pairs, const float* ref,
                             const float* def, const int32_t* poi, const int32_t* seed,
                             int32_t* uv, float* zncc, int32_t* status, hipStream_t s);
hipError_t launch_icgn_f32(const DevState& st, const dic_tuning_t& tu,
                           const RefineGroup* groups, int ngroups, const float* ref,
                           const float* def, const int32_t* poi, const int32_t* uv_init,
                           const int32_t* status_in, const double* p_init, double* p_out,
                           float* zncc, int32_t* iters, int32_t* status, int num_cu,
                           hipStream_t s, int interp);
hipError_t launch_nr_f32(const DevState& st, const dic_tuning_t& tu, const RefineGroup* groups,
                         int ngroups, const float* ref, const float* def, const int32_t* poi,
                         const int32_t* uv_init, const int32_t* status_in,
                         const double* p_init, double* p_out, float* zncc, int32_t* iters,
                         int32_t* status, int num_cu, hipStream_t s, int interp);
hipError_t launch_nr_f64(const DevState& st, const DevPair* host_pairs, const float* ref,
                         const float* def, const int32_t* poi, const int32_t* uv_init,
                         const int32_t* status_in, const double* p_init, double* p_out,
                         float* zncc, int32_t* iters, int32_t* status, hipStream_t s);
hipError_t launch_icgn_f64(const DevState& st, const DevPair* host_pairs, const float* ref,
                           const float* def, const int32_t* poi, const int32_t* uv_init,
                           const int32_t* status_in, const double* p_init, double* p_out,
                           float* zncc, int32_t* iters, int32_t* status, hipStream_t s);
hipError_t launch_znssd(const DevState& st, const float* ref, const float* def,
                        const int32_t* poi, const double* p, const float* grad_c,
                        float* c_out, double* grad_p, float* grad_def,
                        unsigned long long* fix_acc, const int64_t* fix_off,
                        const int32_t* fix_owner, int num_regions, int64_t fix_count,
                        int num_cu, hipStream_t s);
hipError_t launch_seed_update(int64_t N, const double* p, const int32_t* status,
                              int32_t* seed_uv, double* p_seed, hipStream_t s);

// Search LDS bytes per workgroup for the given radii and tile.
size_t search_lds_bytes(int maxM, int maxS, int block);
// Threads per search workgroup (one lane per candidate tile of the widest window).
int search_threads(int maxS, int block);
// Largest search workgroup the kernels are compiled for.
int search_max_threads();

}  // namespace dic
