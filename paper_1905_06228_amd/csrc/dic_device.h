// Device helpers: wave reductions, Keys cubic weights,
// 6x6 Cholesky and the affine warp algebra.
#pragma once

#include <math.h>

#include <type_traits>

#include "dic_internal.h"

namespace dic {

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// A record's status, which the reference preparation's Hessian kernel may
// turn from OK to SINGULAR_HESSIAN while a search reads it: relaxed atomic
// accesses (a search takes the two alike).
__device__ __forceinline__ int load_status(const RefRec* R) {
  return __hip_atomic_load(const_cast<int32_t*>(&R->status), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_status(RefRec* R, int v) {
  __hip_atomic_store(&R->status, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The lane index as a value the compiler cannot hoist out of a loop: the
// lane-dependent quantities derived from it inside a persistent loop are
// recomputed per item instead of being held (and spilled) across the loop.
__device__ __forceinline__ int opaque_lane() {
  int l = lane_id();
  __asm__ volatile("" : "+v"(l));
  return l;
}

// Next item of a work counter shared by persistent waves, the same in every
// lane.  Every lane takes part in one atomic (lane 0 adds 1, the others 0) and
// the wave reads lane 0's result, so no lane-dependent branch surrounds the
// fetch: a branch there would let the compiler route the other lanes back to
// the cross-lane read without lane 0.  All lanes must be active.
__device__ __forceinline__ int wave_next_item(int* counter) {
  const int old = atomicAdd(counter, lane_id() == 0 ? 1 : 0);
  return __builtin_amdgcn_readlane(old, 0);
}

// Makes LDS writes of one wave visible to its other lanes (no block barrier:
// waves of a workgroup work on different POIs).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// DPP move of a 64-bit value (both halves), every source lane valid.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave, identical bits in every lane: within rows
// of 16 by DPP (quad xor 1, quad xor 2, half-row mirror, row mirror: every
// step adds a lane pair symmetrically), then the four row sums read from
// lanes 0, 16, 32, 48 and added in a fixed order.  All lanes must be active.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// DPP move of a 32-bit float inside rows of 16 lanes, every source lane valid.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}

__device__ __forceinline__ float readlane_f32(float v, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

// Sums over the 64 lanes of N per-lane FP32 values, each returned as FP64
// with identical bits in every lane; FP32 additions in a fixed order.  Inside
// each row of 16 lanes the DPP butterfly of wave_sum_dpp leaves the row sum
// in every lane.  Then two values share a register: a permlane32 swap (lanes
// 32-63 of the first with lanes 0-31 of the second) and an add put rows 0+2
// and 1+3 of value 2j in lanes 0-31 and of value 2j+1 in lanes 32-63; a
// permlane16 swap (odd rows of the first with even rows of the second) and an
// add of two such registers leave the totals of values 4i, 4i+2, 4i+1, 4i+3
// in rows 0, 1, 2, 3, read from lanes 0, 16, 32, 48.  All lanes must be
// active.
template <int N>
__device__ __forceinline__ void wave_sums_f32(const float* v, double* out) {
  constexpr int N2 = (N + 1) / 2, N4 = (N2 + 1) / 2;
  float r[2 * N2], h[2 * N4];
#pragma unroll
  for (int a = 0; a < N; ++a) {
    float x = v[a];
    x += dpp_f32<0xB1>(x);   // quad_perm [1,0,3,2]
    x += dpp_f32<0x4E>(x);   // quad_perm [2,3,0,1]
    x += dpp_f32<0x141>(x);  // row_half_mirror
    x += dpp_f32<0x140>(x);  // row_mirror
    r[a] = x;
  }
  if constexpr ((N & 1) != 0) r[N] = 0.f;
#pragma unroll
  for (int j = 0; j < N2; ++j) {
    const auto q = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, r[2 * j]),
                                                    __builtin_bit_cast(unsigned, r[2 * j + 1]),
                                                    false, false);
    h[j] = __builtin_bit_cast(float, (unsigned)q[0]) + __builtin_bit_cast(float, (unsigned)q[1]);
  }
  if constexpr ((N2 & 1) != 0) h[N2] = 0.f;
#pragma unroll
  for (int i = 0; i < N4; ++i) {
    const auto q = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, h[2 * i]),
                                                    __builtin_bit_cast(unsigned, h[2 * i + 1]),
                                                    false, false);
    const float t =
        __builtin_bit_cast(float, (unsigned)q[0]) + __builtin_bit_cast(float, (unsigned)q[1]);
    constexpr int kLane[4] = {0, 32, 16, 48};
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (4 * i + u < N) out[4 * i + u] = (double)readlane_f32(t, kLane[u]);
  }
}

// Maximum over the 64 lanes of a wave by DPP within rows of 16, then the
// four row maxima; every lane returns the same value.  All lanes active.
__device__ __forceinline__ float wave_max_dpp(float v) {
  const auto mv = [](float x, auto ctrl) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), decltype(ctrl)::value, 0xF,
                                        0xF, true));
  };
  v = fmaxf(v, mv(v, std::integral_constant<int, 0xB1>{}));
  v = fmaxf(v, mv(v, std::integral_constant<int, 0x4E>{}));
  v = fmaxf(v, mv(v, std::integral_constant<int, 0x141>{}));
  v = fmaxf(v, mv(v, std::integral_constant<int, 0x140>{}));
  const auto rl = [](float x, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
  };
  return fmaxf(fmaxf(rl(v, 0), rl(v, 16)), fmaxf(rl(v, 32), rl(v, 48)));
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

__device__ __forceinline__ int wave_min_int(int v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
  return v;
}

__device__ __forceinline__ int wave_or_int(int v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v |= __shfl_xor(v, o, kWave);
  return v;
}

// Keys cubic-convolution weights (a = -1/2) for taps -1, 0, 1, 2 around
// floor(x), t = x - floor(x).  Horner forms of
//   w-1 = (-t^3 + 2t^2 - t)/2, w0 = (3t^3 - 5t^2 + 2)/2,
//   w1 = (-3t^3 + 4t^2 + t)/2, w2 = (t^3 - t^2)/2.
template <typename T>
__device__ __forceinline__ void cubic_weights(T t, T w[4]) {
  const T tm = t - T(1);
  w[0] = T(-0.5) * t * tm * tm;
  w[1] = fma(t * t, fma(T(1.5), t, T(-2.5)), T(1));
  w[2] = t * fma(t, fma(T(-1.5), t, T(2)), T(0.5));
  w[3] = T(0.5) * t * t * tm;
}

// d/dt of the weights above.
template <typename T>
__device__ __forceinline__ void cubic_dweights(T t, T w[4]) {
  w[0] = T(-0.5) * fma(T(3), t, T(-1)) * (t - T(1));
  w[1] = t * fma(T(4.5), t, T(-5));
  w[2] = fma(t, fma(T(-4.5), t, T(4)), T(0.5));
  w[3] = t * fma(T(1.5), t, T(-1));
}

__device__ __forceinline__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// Cholesky H = L L^T of a packed symmetric 6x6 (lower triangle, row order).
// Fails when a pivot d_k does not exceed 1e-10 * H_kk (also for NaN).
__device__ __forceinline__ bool cholesky6(const double* H, double* L, double* rdiag) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double d = H[tri(k, k)];
#pragma unroll
    for (int j = 0; j < k; ++j) d -= L[tri(k, j)] * L[tri(k, j)];
    if (!(d > 1e-10 * H[tri(k, k)])) return false;
    const double lkk = sqrt(d);
    L[tri(k, k)] = lkk;
    rdiag[k] = 1.0 / lkk;
#pragma unroll
    for (int i = k + 1; i < 6; ++i) {
      double a = H[tri(i, k)];
#pragma unroll
      for (int j = 0; j < k; ++j) a -= L[tri(i, j)] * L[tri(k, j)];
      L[tri(i, k)] = a * rdiag[k];
    }
  }
  return true;
}

// Solve L L^T x = b.
__device__ __forceinline__ void cholesky6_solve(const double* L, const double* rdiag,
                                                const double* b, double* x) {
  double z[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double a = b[i];
#pragma unroll
    for (int j = 0; j < i; ++j) a -= L[tri(i, j)] * z[j];
    z[i] = a * rdiag[i];
  }
#pragma unroll
  for (int i = 5; i >= 0; --i) {
    double a = z[i];
#pragma unroll
    for (int j = i + 1; j < 6; ++j) a -= L[tri(j, i)] * x[j];
    x[i] = a * rdiag[i];
  }
}

// Inverse-compositional update W(p) <- W(p) W(dp)^-1 for the first-order
// warp, p = (u, ux, uy, v, vx, vy).
__device__ __forceinline__ void compose_inverse(double* p, const double* dp) {
  const double a00 = 1.0 + dp[1], a01 = dp[2], a10 = dp[4], a11 = 1.0 + dp[5];
  const double rdet = 1.0 / (a00 * a11 - a01 * a10);
  const double i00 = a11 * rdet, i01 = -a01 * rdet, i10 = -a10 * rdet, i11 = a00 * rdet;
  const double it0 = -(i00 * dp[0] + i01 * dp[3]);
  const double it1 = -(i10 * dp[0] + i11 * dp[3]);
  const double b00 = 1.0 + p[1], b01 = p[2], b10 = p[4], b11 = 1.0 + p[5];
  const double n00 = b00 * i00 + b01 * i10, n01 = b00 * i01 + b01 * i11;
  const double n10 = b10 * i00 + b11 * i10, n11 = b10 * i01 + b11 * i11;
  const double t0 = b00 * it0 + b01 * it1 + p[0];
  const double t1 = b10 * it0 + b11 * it1 + p[3];
  p[0] = t0;
  p[1] = n00 - 1.0;
  p[2] = n01;
  p[3] = t1;
  p[4] = n10;
  p[5] = n11 - 1.0;
}

// Stop-rule norm: displacement change at the subset edge.
__device__ __forceinline__ double update_norm(const double* dp, int M) {
  const double m2 = (double)M * (double)M;
  return sqrt(dp[0] * dp[0] + dp[3] * dp[3] +
              m2 * (dp[1] * dp[1] + dp[2] * dp[2] + dp[4] * dp[4] + dp[5] * dp[5]));
}

// Flat-subset rule shared by search, refinement and their FP64 forms:
// sum (s - mean)^2 must exceed 1e-6 * sum s^2.
__device__ __forceinline__ bool not_flat(double var_sum, double sq_sum) {
  return var_sum > 1e-6 * sq_sum;
}

// A POI is usable when its subset plus the one-pixel gradient border is
// inside the reference image.
__device__ __forceinline__ bool poi_inside(int x0, int y0, int M, int W, int H) {
  return x0 - M >= 1 && x0 + M <= W - 2 && y0 - M >= 1 && y0 + M <= H - 2;
}

}  // namespace dic
