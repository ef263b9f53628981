// Internal types shared by the host API and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dic.h"

namespace dic {

constexpr int kMaxM = 20;
constexpr int kMaxS = 32;
constexpr int kWave = 64;

// Device copy of a pair description plus derived offsets.
struct DevPair {
  int32_t width, height, M, S;
  int64_t ref_off, def_off;
  int64_t poi_off, poi_count;
  int64_t grad_off;  // float offset of this pair's [2, H, W] gradient block
  int64_t tmpl_off;  // float offset of this pair's templates, n floats per POI
};

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
  float* tmpl;              // template arena
  int64_t N;
  int32_t num_pairs;
  int32_t maxM, maxS;
  int32_t max_width, max_height;
  int32_t max_iters;
  double conv_tol;
};

enum Counter { kCtrSearch = 0, kCtrIcgn = 1, kCtrZnssd = 2, kNumCounters = 8 };

// Kernel launchers (defined in the .hip files).  All asynchronous on `s`.
hipError_t launch_reset_counters(const DevState& st, hipStream_t s);
hipError_t launch_gradients(const DevState& st, const float* ref, hipStream_t s);
hipError_t launch_ref_prep_f32(const DevState& st, const float* ref, const int32_t* poi,
                               hipStream_t s);
hipError_t launch_ref_prep_f64(const DevState& st, const DevPair* host_pairs,
                               const float* ref, const int32_t* poi, hipStream_t s);
hipError_t launch_search_f32(const DevState& st, const dic_tuning_t& tu, const float* ref,
                             const float* def, const int32_t* poi, const int32_t* seed,
                             int32_t* uv, float* zncc, int32_t* status, int num_cu,
                             hipStream_t s);
hipError_t launch_search_f64(const DevState& st, const DevPair* host_pairs, const float* ref,
                             const float* def, const int32_t* poi, const int32_t* seed,
                             int32_t* uv, float* zncc, int32_t* status, hipStream_t s);
hipError_t launch_icgn_f32(const DevState& st, const dic_tuning_t& tu, const float* ref,
                           const float* def, const int32_t* poi, const int32_t* uv_init,
                           const int32_t* status_in, const double* p_init, double* p_out,
                           float* zncc, int32_t* iters, int32_t* status, int num_cu,
                           hipStream_t s);
hipError_t launch_icgn_f64(const DevState& st, const DevPair* host_pairs, const float* ref,
                           const float* def, const int32_t* poi, const int32_t* uv_init,
                           const int32_t* status_in, const double* p_init, double* p_out,
                           float* zncc, int32_t* iters, int32_t* status, hipStream_t s);
hipError_t launch_znssd(const DevState& st, const float* ref, const float* def,
                        const int32_t* poi, const double* p, const float* grad_c,
                        float* c_out, double* grad_p, float* grad_def,
                        unsigned long long* fix_acc, const int64_t* fix_off, int64_t fix_count,
                        int num_cu, hipStream_t s);
hipError_t launch_seed_update(int64_t N, const double* p, const int32_t* status,
                              int32_t* seed_uv, double* p_seed, hipStream_t s);

// Search LDS bytes per workgroup for the given radii and tile.
size_t search_lds_bytes(int maxM, int maxS, int block);
// IC-GN LDS bytes per workgroup.
size_t icgn_lds_bytes(int maxM, int slack, int waves);

}  // namespace dic
