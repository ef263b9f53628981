// Reference-side precomputation: gradients of the reference images and the
// per-POI record IC-GN precomputes (Sec. 2.2), plus small utility kernels.
#include "dic_device.h"

namespace dic {

__global__ void reset_counters_kernel(int32_t* counters) {
  if (threadIdx.x < kNumCounters) counters[threadIdx.x] = 0;
}

hipError_t launch_reset_counters(const DevState& st, hipStream_t s) {
  hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, s, st.counters);
  return hipGetLastError();
}

// Central-difference gradients, fx = (f[x+1] - f[x-1]) / 2, zero on the
// one-pixel border.  Grid: (column blocks, rows, pairs).
__global__ void __launch_bounds__(256) gradients_kernel(const DevPair* __restrict__ pairs,
                                                        const float* __restrict__ ref,
                                                        float* __restrict__ grads) {
  const DevPair P = pairs[blockIdx.z];
  const int y = blockIdx.y;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= P.height || x >= P.width) return;
  const int W = P.width, H = P.height;
  const float* f = ref + P.ref_off;
  const int64_t i = (int64_t)y * W + x;
  float gx = 0.f, gy = 0.f;
  if (x > 0 && x < W - 1) gx = 0.5f * (f[i + 1] - f[i - 1]);
  if (y > 0 && y < H - 1) gy = 0.5f * (f[i + W] - f[i - W]);
  float* out = grads + P.grad_off;
  out[i] = gx;
  out[i + (int64_t)W * H] = gy;
}

hipError_t launch_gradients(const DevState& st, const float* ref, hipStream_t s) {
  dim3 grid((st.max_width + 255) / 256, st.max_height, st.num_pairs);
  hipLaunchKernelGGL(gradients_kernel, grid, dim3(256), 0, s, st.pairs, ref, st.grads);
  return hipGetLastError();
}

// Subset sums of every deformed image, for every subset centre, in FP64
// (sums of these float grey levels are exact in FP64 for images of ordinary
// range, and the fixed evaluation order keeps them deterministic anyway):
// S1[y][x] = sum g, S2[y][x] = sum g^2 over the (2M+1)^2 subset centred on
// (x, y).  A centre whose subset leaves the image or holds a non-finite
// pixel gets S2 = -1.  Two passes: column sums (running down 64-row
// segments, one term in and one out per step), then row sums of those
// (direct, 2M+1 terms from an LDS tile); the order is fixed, so the results
// are deterministic.  The second pass
// also stores per centre the float pair (mean, 1/sqrt(sum (g - mean)^2)) that
// the matrix-core search scores with, (0, 0) where the subset is inadmissible
// or flat by the FP64 rule.
constexpr int kBoxSeg = 64;

__global__ void __launch_bounds__(256) box_cols_kernel(const DevPair* __restrict__ pairs,
                                                       const float* __restrict__ def,
                                                       double* __restrict__ box) {
  const DevPair P = pairs[blockIdx.z];
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y0 = blockIdx.y * kBoxSeg;
  const int W = P.width, H = P.height, M = P.M;
  if (x >= W || y0 >= H) return;
  const float* col = def + P.def_off + x;
  const int64_t plane = (int64_t)W * H;
  double* v1 = box + P.box_off;
  double* v2 = v1 + plane;
  const int y1 = min(y0 + kBoxSeg, H);
  // centres whose subset rows lie in the image: M <= y <= H - 1 - M
  const int ya = max(y0, M), yb = max(ya, min(y1, H - M));
  for (int y = y0; y < y1; ++y)
    if (y < ya || y >= yb) {
      v1[(int64_t)y * W + x] = 0.0;
      v2[(int64_t)y * W + x] = -1.0;
    }
  if (ya >= yb) return;
  double s1 = 0.0, s2 = 0.0;
  int bad = 0;
  auto take = [&](float v, int sign) {
    if (isfinite(v)) {
      s1 += sign * (double)v;
      s2 += sign * (double)v * (double)v;
    } else {
      bad += sign;
    }
  };
  auto put = [&](int y) {
    v1[(int64_t)y * W + x] = s1;
    v2[(int64_t)y * W + x] = bad ? -1.0 : s2;
  };
  auto at = [&](int y) { return col[(int64_t)y * W]; };
  // The first centre's 2M+1 rows, then per centre y the row y + M in and
  // the row y - M - 1 out, in that order; the rows are requested eight
  // centres at a time (one memory round trip per eight), the sums run in
  // the same order as one row at a time.
  constexpr int kB = 8;
  int i = ya - M;
  for (; i + kB <= ya + M + 1; i += kB) {
    float v[kB];
#pragma unroll
    for (int j = 0; j < kB; ++j) v[j] = at(i + j);
#pragma unroll
    for (int j = 0; j < kB; ++j) take(v[j], 1);
  }
  for (; i <= ya + M; ++i) take(at(i), 1);
  put(ya);
  int y = ya + 1;
  for (; y + kB <= yb; y += kB) {
    float vi[kB], vo[kB];
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      vi[j] = at(y + j + M);
      vo[j] = at(y + j - M - 1);
    }
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      take(vi[j], 1);
      take(vo[j], -1);
      put(y + j);
    }
  }
  for (; y < yb; ++y) {
    take(at(y + M), 1);
    take(at(y - M - 1), -1);
    put(y);
  }
}

// Row pass: a workgroup stages one row segment of the column sums (with the
// 2M-column halo) in LDS; each thread then sums its 2M+1 columns directly.
constexpr int kBoxRowTile = 256;

__global__ void __launch_bounds__(kBoxRowTile) box_rows_kernel(const DevPair* __restrict__ pairs,
                                                               double* __restrict__ box) {
  __shared__ double l1[kBoxRowTile + 2 * kMaxM];
  __shared__ double l2[kBoxRowTile + 2 * kMaxM];
  const DevPair P = pairs[blockIdx.z];
  const int x0 = blockIdx.x * kBoxRowTile, y = blockIdx.y;
  const int W = P.width, H = P.height, M = P.M;
  if (x0 >= W || y >= H) return;   // uniform over the workgroup
  const int64_t plane = (int64_t)W * H;
  const double* v1 = box + P.box_off + (int64_t)y * W;
  const double* v2 = v1 + plane;
  for (int i = threadIdx.x; i < kBoxRowTile + 2 * M; i += kBoxRowTile) {
    const int j = x0 - M + i;
    const bool in = j >= 0 && j < W;
    l1[i] = in ? v1[j] : 0.0;
    l2[i] = in ? v2[j] : -1.0;
  }
  __syncthreads();
  const int x = x0 + threadIdx.x;
  if (x >= W) return;
  double* o1 = box + P.box_off + 2 * plane + (int64_t)y * W;
  double* o2 = o1 + plane;
  float2* o3 = reinterpret_cast<float2*>(o2 + plane);
  double s1 = 0.0, s2 = 0.0;
  bool bad = x - M < 0 || x + M > W - 1;
  const int t0 = threadIdx.x;
  for (int i = t0; i <= t0 + 2 * M; ++i) {
    const double q = l2[i];
    bad |= q < 0.0;
    s1 += l1[i];
    s2 += q;
  }
  o1[x] = bad ? 0.0 : s1;
  o2[x] = bad ? -1.0 : s2;
  const double n = (double)(2 * M + 1) * (double)(2 * M + 1);
  const double var = s2 - s1 * s1 / n;
  o3[x] = !bad && not_flat(var, s2) ? make_float2((float)(s1 / n), (float)(1.0 / sqrt(var)))
                                    : make_float2(0.f, 0.f);
}

hipError_t launch_box_sums(const DevState& st, const float* def, hipStream_t s) {
  const dim3 gc((st.max_width + 255) / 256, (st.max_height + kBoxSeg - 1) / kBoxSeg,
                st.num_pairs);
  hipLaunchKernelGGL(box_cols_kernel, gc, dim3(256), 0, s, st.pairs, def, st.box);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 gr((st.max_width + kBoxRowTile - 1) / kBoxRowTile, st.max_height, st.num_pairs);
  hipLaunchKernelGGL(box_rows_kernel, gr, dim3(kBoxRowTile), 0, s, st.pairs, st.box);
  return hipGetLastError();
}

// Bicubic coefficient table of every deformed image (the look-up table of
// interpolation coefficients): per cell (x, y) with 1 <= x <= W - 3 and
// 1 <= y <= H - 3, the 16 coefficients C[b][a] of the Keys interpolant on
// [x, x+1) x [y, y+1) written as sum C[b][a] t^a s^b.  With Keys' weights
// expanded in powers of t, the taps g-1..g2 of a row give
//   t^0: g0,  t^1: (g1 - g-1)/2,  t^2: g-1 - 5/2 g0 + 2 g1 - 1/2 g2,
//   t^3: -1/2 g-1 + 3/2 g0 - 3/2 g1 + 1/2 g2,
// applied along x to the four rows, then along y to those row coefficients.
// Formed in FP64 and rounded once; cells outside that range hold zeros (the
// refinements' bounds test never reads them).  Grid: (column blocks, rows,
// pairs); each thread writes its cell's four float4 rows (64 contiguous bytes).
__device__ __forceinline__ void keys_powers(double gm, double g0, double g1, double g2,
                                            double* c) {
  c[0] = g0;
  c[1] = 0.5 * (g1 - gm);
  c[2] = gm - 2.5 * g0 + 2.0 * g1 - 0.5 * g2;
  c[3] = -0.5 * gm + 1.5 * g0 - 1.5 * g1 + 0.5 * g2;
}

__global__ void __launch_bounds__(256) bicubic_lut_kernel(const DevPair* __restrict__ pairs,
                                                          const float* __restrict__ def,
                                                          float4* __restrict__ lut) {
  const DevPair P = pairs[blockIdx.z];
  const int y = blockIdx.y;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= P.height || x >= P.width) return;
  const int W = P.width, H = P.height;
  float4* out = lut + P.lut_off + ((int64_t)y * W + x) * 4;
  if (x < 1 || x > W - 3 || y < 1 || y > H - 3) {
#pragma unroll
    for (int b = 0; b < 4; ++b) out[b] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  const float* g = def + P.def_off + (int64_t)(y - 1) * W + (x - 1);
  double rc[4][4];  // [row][power of t]
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    const float* row = g + (int64_t)l * W;
    keys_powers(row[0], row[1], row[2], row[3], rc[l]);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double cb[4];
    keys_powers(rc[0][a], rc[1][a], rc[2][a], rc[3][a], cb);
    // cb[b] = C[b][a]; row b of the output holds powers a = 0..3
    rc[0][a] = cb[0];
    rc[1][a] = cb[1];
    rc[2][a] = cb[2];
    rc[3][a] = cb[3];
  }
#pragma unroll
  for (int b = 0; b < 4; ++b)
    out[b] = make_float4((float)rc[b][0], (float)rc[b][1], (float)rc[b][2], (float)rc[b][3]);
}

// Cubic B-spline coefficients of every deformed image (the spline
// interpolation of Sec. 2.2): c with (c[k-1] + 4 c[k] + c[k+1]) / 6 = g[k]
// along each axis, the image extended symmetrically about its end samples.
// The inverse of that three-tap filter has the impulse response
// sqrt(3) z^|j| with z = sqrt(3) - 2, so along one axis
//   c[k] = sqrt(3) (g[k] + sum_{j=1..16} z^j (g[k - j] + g[k + j]))
// over the symmetric extension (index reflected into one period of 2n - 2
// samples), truncated at |j| <= 16: the terms dropped sum to below 1e-9 of
// the largest pixel, under FP32 rounding.  Every output is independent.  A
// rows pass writes a scratch image, a columns pass reads it and writes the
// coefficient image, FP64 sums rounded once per pass.  The rows pass stages
// a row tile in LDS (reflected indices resolved while staging) and each
// thread forms four outputs from one run of staged values held in
// registers; the columns pass does the same down a column from direct
// loads.  A non-finite pixel has no spline through it: the rows pass sets
// its pair's flag and the columns pass then writes NaN over the whole image
// (the recursive form's result, whose recursions carry such a value along
// every row and column).
constexpr int kBsplineHalf = 16;
constexpr int kBsplineRowTile = 1024;   // rows pass: outputs per block, 4 per thread
static_assert(256 * 4 == kBsplineRowTile, "rows pass: 4 outputs per thread");

__device__ __forceinline__ int bspline_mirror(int i, int n) {
  if (i >= 0 && i < n) return i;
  const int per = 2 * n - 2;
  i %= per;
  if (i < 0) i += per;
  return i < n ? i : per - i;
}

// sqrt(3) (v[16 + u] + sum_j z^j (v[16 + u - j] + v[16 + u + j])) for the
// outputs u = 0..NOUT-1 of a run v of NOUT + 32 staged values
template <int NOUT>
__device__ __forceinline__ void bspline_run(const double* v, double* c) {
  constexpr double z = -0.2679491924311227;  // sqrt(3) - 2
#pragma unroll
  for (int u = 0; u < NOUT; ++u) {
    double acc = v[kBsplineHalf + u], w = 1.0;
#pragma unroll
    for (int j = 1; j <= kBsplineHalf; ++j) {
      w *= z;
      acc = fma(w, v[kBsplineHalf + u - j] + v[kBsplineHalf + u + j], acc);
    }
    c[u] = 1.7320508075688772 * acc;  // sqrt(3)
  }
}

__global__ void __launch_bounds__(256) bspline_flags_kernel(int32_t* __restrict__ flags, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flags[i] = 0;
}

// Grid (row tiles of 1024, rows, pairs).  Thread t forms outputs
// x0 + 4t .. x0 + 4t + 3 from staged values 4t .. 4t + 35 (nine 16-byte
// LDS reads).
__global__ void __launch_bounds__(256) bspline_rows_kernel(const DevPair* __restrict__ pairs,
                                                           const float* __restrict__ def,
                                                           float* __restrict__ coef,
                                                           int32_t* __restrict__ flags) {
  __shared__ __attribute__((aligned(16))) float s[kBsplineRowTile + 2 * kBsplineHalf];
  const DevPair P = pairs[blockIdx.z];
  const int W = P.width, H = P.height, y = blockIdx.y;
  const int x0 = blockIdx.x * kBsplineRowTile;
  if (y >= H || x0 >= W) return;  // whole block
  const float* row = def + P.def_off + (int64_t)y * W;
  for (int t = threadIdx.x; t < kBsplineRowTile + 2 * kBsplineHalf; t += blockDim.x) {
    const int x = x0 - kBsplineHalf + t;
    s[t] = x < W + kBsplineHalf ? row[bspline_mirror(x, W)] : 0.f;
  }
  __syncthreads();
  const int xo = x0 + 4 * (int)threadIdx.x;
  bool bad = false;
  if (xo < W) {
    double v[4 + 2 * kBsplineHalf], c[4];
    const float4* q = reinterpret_cast<const float4*>(s) + threadIdx.x;
#pragma unroll
    for (int a = 0; a < (4 + 2 * kBsplineHalf) / 4; ++a) {
      const float4 f4 = q[a];
      v[4 * a] = f4.x;
      v[4 * a + 1] = f4.y;
      v[4 * a + 2] = f4.z;
      v[4 * a + 3] = f4.w;
    }
    bspline_run<4>(v, c);
    // scratch image: the second half of the pair's region
    float* o = coef + 4 * P.lut_off + (int64_t)W * H + (int64_t)y * W + xo;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (xo + u < W) {
        o[u] = (float)c[u];
        bad |= !isfinite(c[u]);
      }
  }
  const unsigned long long m = __ballot(bad);
  if (m && lane_id() == __ffsll((long long)m) - 1) atomicOr(&flags[blockIdx.z], 1);
}

// Grid (column blocks of 256, row groups of 4, pairs): a thread forms the
// outputs of 4 consecutive rows of one column from the 36 values around
// them, read straight from the scratch image (coalesced across the wave;
// the reflected indices only for the groups within 16 rows of an edge).
__global__ void __launch_bounds__(256) bspline_cols_kernel(const DevPair* __restrict__ pairs,
                                                           float* __restrict__ coef,
                                                           const int32_t* __restrict__ flags) {
  const DevPair P = pairs[blockIdx.z];
  const int W = P.width, H = P.height, y0 = 4 * blockIdx.y;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (y0 >= H || x >= W) return;
  float* out = coef + 4 * P.lut_off;
  const float* col = out + (int64_t)W * H + x;
  double v[4 + 2 * kBsplineHalf], c[4];
  if (y0 >= kBsplineHalf && y0 + 3 + kBsplineHalf < H) {
#pragma unroll
    for (int i = 0; i < 4 + 2 * kBsplineHalf; ++i)
      v[i] = col[(int64_t)(y0 - kBsplineHalf + i) * W];
  } else {
#pragma unroll
    for (int i = 0; i < 4 + 2 * kBsplineHalf; ++i)
      v[i] = col[(int64_t)bspline_mirror(y0 - kBsplineHalf + i, H) * W];
  }
  bspline_run<4>(v, c);
  const bool poisoned = flags[blockIdx.z] != 0;
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (y0 + u < H) out[(int64_t)(y0 + u) * W + x] = poisoned ? nanf("") : (float)c[u];
}

hipError_t launch_bspline_coeffs(const DevState& st, const float* def, hipStream_t s) {
  hipLaunchKernelGGL(bspline_flags_kernel, dim3((st.num_pairs + 255) / 256), dim3(256), 0, s,
                     st.bsp_flags, st.num_pairs);
  hipLaunchKernelGGL(bspline_rows_kernel,
                     dim3((st.max_width + kBsplineRowTile - 1) / kBsplineRowTile, st.max_height,
                          st.num_pairs),
                     dim3(256), 0, s, st.pairs, def, st.lut, st.bsp_flags);
  hipLaunchKernelGGL(bspline_cols_kernel, dim3((st.max_width + 255) / 256,
                                                 (st.max_height + 3) / 4, st.num_pairs),
                     dim3(256), 0, s, st.pairs, st.lut, st.bsp_flags);
  return hipGetLastError();
}

hipError_t launch_bicubic_lut(const DevState& st, const float* def, hipStream_t s) {
  dim3 grid((st.max_width + 255) / 256, st.max_height, st.num_pairs);
  hipLaunchKernelGGL(bicubic_lut_kernel, grid, dim3(256), 0, s, st.pairs, def,
                     reinterpret_cast<float4*>(st.lut));
  return hipGetLastError();
}

// Writes the record of a POI that cannot be processed.
__device__ __forceinline__ void write_bad_record(RefRec* R, int status, int lane) {
  if (lane == 0) {
    R->fbar = nan("");
    R->df = nan("");
    R->tsum = 0.f;
    R->status = status;
  }
}

// FP32 form, in two kernels: the statistics the search needs, then (beside
// the search, in a correlate with a side stream) the steepest-descent sums,
// the Hessian and its factor that only IC-GN reads.  One wave per POI
// (pixel k on lane k mod 64, its row and column stepped without division).
//
// Statistics.  Pass 1, in FP64: sum f (the mean decides ZERO_VARIANCE exactly
// as the FP64 definition does).  Pass 2, in FP64: sum (f - fbar)^2, sum f^2
// and the sum of the float template f - (float)fbar.  Writes fbar, df, tsum
// and the status; with write_tmpl also stores the float search template,
// which only the vector-ALU search reads (the other kernels form those values
// from f).  One launch per run of the work list that shares a refinement
// kernel class; NS: pixels kept per lane, at least the run's largest subset
// over 64 (fewer registers for small subsets, more waves in flight).
template <int NS>
__global__ void __launch_bounds__(256) ref_prep_stats_kernel(DevState st,
                                                             const int32_t* __restrict__ work,
                                                             int64_t count,
                                                             const float* __restrict__ ref,
                                                             const int32_t* __restrict__ poi,
                                                             int write_tmpl) {
  // the POI of this wave, wave-uniform: its pointers stay in scalar registers
  const int64_t item = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (item >= count) return;
  const int g = uniform(work[item]);
  const int lane = lane_id();
  const DevPair P = st.pairs[uniform(st.poi_pair[g])];
  RefRec* R = st.recs + g;
  const int x0 = uniform(poi[2 * g]), y0 = uniform(poi[2 * g + 1]);
  const int M = P.M, n1 = 2 * M + 1, n = n1 * n1, W = P.width;
  if (!poi_inside(x0, y0, M, P.width, P.height)) {
    write_bad_record(R, DIC_POI_OUT_OF_BOUNDS, lane);
    return;
  }
  const float* f = ref + P.ref_off + (int64_t)(y0 - M) * W + (x0 - M);
  const int tp = P.tmpl_pitch;
  float* tmpl = st.tmpl + P.tmpl_off + (g - P.poi_off) * (int64_t)(n1 * tp);
  if (write_tmpl)
    for (int k = lane; k < n1 * (tp - n1); k += kWave) {
      const int r = k / (tp - n1);
      tmpl[r * tp + n1 + (k - r * (tp - n1))] = 0.f;   // zero padding of every row
    }
  const int dr = kWave / n1, dc = kWave - dr * n1;
  auto step = [&](int& r, int& c) {
    c += dc;
    r += dr;
    if (c >= n1) {
      c -= n1;
      ++r;
    }
  };

  // the lane's pixels, all requested at once and kept for both passes (one
  // memory round trip); slot j is pixel lane + 64 j
  constexpr int kSlots = NS;
  float fv[kSlots];
  {
    int r = lane / n1, c = lane - r * n1;
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
      fv[j] = 0.f;
      if (lane + kWave * j < n) fv[j] = f[(unsigned)(r * W + c)];   // 32-bit offset from a scalar base
      step(r, c);
    }
  }
  double s1 = 0.0;
  int bad = 0;
#pragma unroll
  for (int j = 0; j < kSlots; ++j)
    if (lane + kWave * j < n) {
      bad |= !isfinite(fv[j]);
      s1 += (double)fv[j];
    }
  s1 = wave_sum_dpp(s1);
  bad = wave_or_int(bad);
  if (bad) {
    write_bad_record(R, DIC_POI_NAN_INPUT, lane);
    return;
  }
  const double fbar = s1 / (double)n;
  const float fbar_f = (float)fbar;

  double q = 0.0, sq = 0.0, ts = 0.0;
#pragma unroll
  for (int j = 0; j < kSlots; ++j)
    if (lane + kWave * j < n) {
      const float v = fv[j];
      const double d = (double)v - fbar;
      q += d * d;
      sq += (double)v * (double)v;
      ts += (double)(v - fbar_f);
    }
  if (write_tmpl) {
    int r = lane / n1, c = lane - r * n1;
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
      if (lane + kWave * j < n) tmpl[r * tp + c] = fv[j] - fbar_f;
      step(r, c);
    }
  }
  q = wave_sum_dpp(q);
  sq = wave_sum_dpp(sq);
  ts = wave_sum_dpp(ts);
  if (lane == 0) {
    R->fbar = fbar;
    R->df = sqrt(q);
    R->tsum = (float)ts;
    R->status = not_flat(q, sq) ? DIC_POI_OK : DIC_POI_ZERO_VARIANCE;
  }
}

// Steepest-descent sums, Hessian and factor, for the POIs the statistics
// kernel left OK or flat (it has written the record of the others).  One
// pass: the six sums sum SD in FP64 (they enter IC-GN's right-hand side, so
// they decide its fixed point), the six sum SD (f - fbar) and the 21 products
// of the shifted steepest-descent images in FP32 per lane with fused
// multiply-adds (at most a few tens of terms), added across lanes in a fixed
// FP32 tree (six levels).  Removal of the shifted mean, factorisation and
// singularity test in FP64.  A singular Hessian turns the
// status to SINGULAR_HESSIAN with an atomic store: a search may read the
// status meanwhile, and takes OK and SINGULAR_HESSIAN alike.
__global__ void __launch_bounds__(256) ref_prep_hessian_kernel(DevState st,
                                                               const float* __restrict__ ref,
                                                               const int32_t* __restrict__ poi) {
  const int g = uniform((int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave));
  if (g >= st.N) return;
  const int lane = lane_id();
  const DevPair P = st.pairs[uniform(st.poi_pair[g])];
  RefRec* R = st.recs + g;
  const int status0 = uniform(load_status(R));
  if (status0 != DIC_POI_OK && status0 != DIC_POI_ZERO_VARIANCE) return;
  const int x0 = uniform(poi[2 * g]), y0 = uniform(poi[2 * g + 1]);
  const int M = P.M, n1 = 2 * M + 1, n = n1 * n1, W = P.width;
  const float* f = ref + P.ref_off + (int64_t)(y0 - M) * W + (x0 - M);
  const float* gxi = st.grads + P.grad_off + (int64_t)(y0 - M) * W + (x0 - M);
  const float* gyi = gxi + (int64_t)P.width * P.height;
  const int dr = kWave / n1, dc = kWave - dr * n1;
  auto step = [&](int& r, int& c) {
    c += dc;
    r += dr;
    if (c >= n1) {
      c -= n1;
      ++r;
    }
  };
  auto sd_of = [&](float fx, float fy, int r, int c, float* sd) {
    const float dx = (float)(c - M), dy = (float)(r - M);
    sd[0] = fx;
    sd[1] = fx * dx;
    sd[2] = fx * dy;
    sd[3] = fy;
    sd[4] = fy * dx;
    sd[5] = fy * dy;
  };

  // One pass.  The steepest-descent images enter the Hessian shifted by
  // their value at the subset centre, K = (gx, 0, 0, gy, 0, 0) there, and
  // the shifted mean m' is removed in FP64 afterwards: sum (s - K)(s - K)^T
  // - n m' m'^T.  K follows the gradients' level (a ramp's constant gradient
  // cancels exactly; the offset-weighted terms have mean ~0 over the
  // symmetric subset), so the removal cancels little.
  const unsigned oc = (unsigned)(M * W + M);
  const float kx = gxi[oc], ky = gyi[oc];
  double ks[6] = {0, 0, 0, 0, 0, 0};
  float ksdf[6] = {0, 0, 0, 0, 0, 0}, kh[21];
#pragma unroll
  for (int a = 0; a < 21; ++a) kh[a] = 0.f;
  const float fbar_f = (float)R->fbar;
  {
    int r = lane / n1, c = lane - r * n1;
#pragma unroll 4
    for (int k = lane; k < n; k += kWave) {
      const unsigned o = (unsigned)(r * W + c);   // 32-bit offset from a scalar base
      const float t = f[o] - fbar_f;
      float sd[6];
      sd_of(gxi[o], gyi[o], r, c, sd);
#pragma unroll
      for (int a = 0; a < 6; ++a) ksdf[a] = fmaf(sd[a], t, ksdf[a]);
      sd[0] -= kx;
      sd[3] -= ky;
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        ks[a] += (double)sd[a];
#pragma unroll
        for (int b = 0; b <= a; ++b) kh[tri(a, b)] = fmaf(sd[a], sd[b], kh[tri(a, b)]);
      }
      step(r, c);
    }
  }
  double shs[6], sdfsum[6], h[21], sdsum[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) shs[a] = wave_sum_dpp(ks[a]);
  wave_sums_f32<6>(ksdf, sdfsum);
  wave_sums_f32<21>(kh, h);
#pragma unroll
  for (int a = 0; a < 6; ++a) sdsum[a] = shs[a];
  sdsum[0] += (double)n * (double)kx;
  sdsum[3] += (double)n * (double)ky;

  int status = status0;
  double L[21], rd[6];
  if (status == DIC_POI_OK) {
    double m[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) m[a] = shs[a] / (double)n;
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b) h[tri(a, b)] -= (double)n * m[a] * m[b];
    if (!cholesky6(h, L, rd)) status = DIC_POI_SINGULAR_HESSIAN;
  }
  if (lane == 0) {
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      R->sd_sum[a] = sdsum[a];
      R->sdf_sum[a] = sdfsum[a];
      R->rdiag[a] = status == DIC_POI_OK ? rd[a] : 0.0;
    }
#pragma unroll
    for (int a = 0; a < 21; ++a) R->L[a] = status == DIC_POI_OK ? L[a] : 0.0;
    if (status != status0) store_status(R, status);
  }
}

hipError_t launch_ref_prep_stats(const DevState& st, const RefineGroup* groups, int ngroups,
                                 const float* ref, const int32_t* poi, bool write_tmpl,
                                 hipStream_t s) {
  const int wt = write_tmpl ? 1 : 0;
  for (int i = 0; i < ngroups; ++i) {
    const RefineGroup& gr = groups[i];
    if (gr.count == 0) continue;
    const dim3 grid((unsigned)((gr.count + 3) / 4)), block(256);
    const int32_t* w = st.work + gr.begin;
    switch (refine_slots(gr.maxM)) {
#define DIC_STATS(NS)                                                                       \
  case NS:                                                                                  \
    hipLaunchKernelGGL(ref_prep_stats_kernel<NS>, grid, block, 0, s, st, w, gr.count, ref, \
                       poi, wt);                                                            \
    break;
      DIC_STATS(4)
      DIC_STATS(8)
      DIC_STATS(12)
      DIC_STATS(16)
      DIC_STATS(20)
      DIC_STATS(28)
#undef DIC_STATS
      default: return hipErrorInvalidValue;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_ref_prep_hessian(const DevState& st, const float* ref, const int32_t* poi,
                                   hipStream_t s) {
  if (st.N == 0) return hipSuccess;
  const int64_t blocks = (st.N + 3) / 4;
  hipLaunchKernelGGL(ref_prep_hessian_kernel, dim3((unsigned)blocks), dim3(256), 0, s, st, ref,
                     poi);
  return hipGetLastError();
}

hipError_t launch_ref_prep_f32(const DevState& st, const RefineGroup* groups, int ngroups,
                               const float* ref, const int32_t* poi, bool write_tmpl,
                               hipStream_t s) {
  hipError_t e = launch_ref_prep_stats(st, groups, ngroups, ref, poi, write_tmpl, s);
  if (e != hipSuccess) return e;
  return launch_ref_prep_hessian(st, ref, poi, s);
}

// FP64 plain form: one 64-thread workgroup per POI of one pair, everything
// in FP64, gradients straight from the reference image.
__global__ void __launch_bounds__(64) ref_prep_f64_kernel(DevState st, DevPair P, int pair,
                                                          const float* __restrict__ ref,
                                                          const int32_t* __restrict__ poi) {
  const int64_t g = P.poi_off + blockIdx.x;
  const int lane = threadIdx.x;
  RefRec* R = st.recs + g;
  const int x0 = poi[2 * g], y0 = poi[2 * g + 1];
  const int M = P.M, n1 = 2 * M + 1, n = n1 * n1, W = P.width;
  if (!poi_inside(x0, y0, M, P.width, P.height)) {
    write_bad_record(R, DIC_POI_OUT_OF_BOUNDS, lane);
    return;
  }
  const float* f = ref + P.ref_off;
  double s1 = 0.0;
  int bad = 0;
  for (int k = lane; k < n; k += kWave) {
    const int r = k / n1, c = k - r * n1;
    const float v = f[(int64_t)(y0 - M + r) * W + (x0 - M + c)];
    bad |= !isfinite(v);
    s1 += (double)v;
  }
  s1 = wave_sum(s1);
  bad = wave_or_int(bad);
  if (bad) {
    write_bad_record(R, DIC_POI_NAN_INPUT, lane);
    return;
  }
  const double fbar = s1 / (double)n;
  double q = 0.0, sq = 0.0, sd_s[6] = {0}, sdf_s[6] = {0}, h[21] = {0};
  for (int k = lane; k < n; k += kWave) {
    const int r = k / n1, c = k - r * n1;
    const int64_t idx = (int64_t)(y0 - M + r) * W + (x0 - M + c);
    const double v = (double)f[idx];
    const double d = v - fbar;
    q += d * d;
    sq += v * v;
    const double fx = ((double)f[idx + 1] - (double)f[idx - 1]) / 2.0;
    const double fy = ((double)f[idx + W] - (double)f[idx - W]) / 2.0;
    const double dx = (double)(c - M), dy = (double)(r - M);
    const double sd[6] = {fx, fx * dx, fx * dy, fy, fy * dx, fy * dy};
    for (int a = 0; a < 6; ++a) {
      sd_s[a] += sd[a];
      sdf_s[a] += sd[a] * d;
      for (int b = 0; b <= a; ++b) h[tri(a, b)] += sd[a] * sd[b];
    }
  }
  q = wave_sum(q);
  sq = wave_sum(sq);
  for (int a = 0; a < 6; ++a) {
    sd_s[a] = wave_sum(sd_s[a]);
    sdf_s[a] = wave_sum(sdf_s[a]);
  }
  for (int a = 0; a < 21; ++a) h[a] = wave_sum(h[a]);
  int status = DIC_POI_OK;
  double L[21], rd[6];
  if (!not_flat(q, sq)) {
    status = DIC_POI_ZERO_VARIANCE;
  } else {
    for (int a = 0; a < 6; ++a)
      for (int b = 0; b <= a; ++b) h[tri(a, b)] -= sd_s[a] * sd_s[b] / (double)n;
    if (!cholesky6(h, L, rd)) status = DIC_POI_SINGULAR_HESSIAN;
  }
  if (lane == 0) {
    R->fbar = fbar;
    R->df = sqrt(q);
    R->tsum = 0.f;
    R->status = status;
    for (int a = 0; a < 6; ++a) {
      R->sd_sum[a] = sd_s[a];
      R->sdf_sum[a] = sdf_s[a];
      R->rdiag[a] = status == DIC_POI_OK ? rd[a] : 0.0;
    }
    for (int a = 0; a < 21; ++a) R->L[a] = status == DIC_POI_OK ? L[a] : 0.0;
  }
}

hipError_t launch_ref_prep_f64(const DevState& st, const DevPair* host_pairs, const float* ref,
                               const int32_t* poi, hipStream_t s) {
  for (int k = 0; k < st.num_pairs; ++k) {
    const DevPair& P = host_pairs[k];
    if (P.poi_count == 0) continue;
    hipLaunchKernelGGL(ref_prep_f64_kernel, dim3((unsigned)P.poi_count), dim3(64), 0, s, st, P,
                       k, ref, poi);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Sequence seeding: the last frame with status OK supplies the next seed.
__global__ void seed_update_kernel(int64_t N, const double* __restrict__ p,
                                   const int32_t* __restrict__ status, int32_t* __restrict__ seed,
                                   double* __restrict__ p_seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N || status[i] != DIC_POI_OK) return;
#pragma unroll
  for (int a = 0; a < 6; ++a) p_seed[6 * i + a] = p[6 * i + a];
  seed[2 * i] = (int32_t)rint(p[6 * i]);
  seed[2 * i + 1] = (int32_t)rint(p[6 * i + 3]);
}

hipError_t launch_seed_update(int64_t N, const double* p, const int32_t* status, int32_t* seed,
                              double* p_seed, hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(seed_update_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, p,
                     status, seed, p_seed);
  return hipGetLastError();
}

}  // namespace dic
