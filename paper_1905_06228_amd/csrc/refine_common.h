// Pieces shared by the sub-pixel refinements of Sec. 2.2 (IC-GN and
// Newton-Raphson, FP32 batched forms): the first-order warp in FP32 local
// form, the bounding box of the taps it touches, the centring constant of
// the deformed samples, the per-wave LDS patch of the deformed image,
// interpolation from that patch or from the image (Keys bicubic, NT = 4
// taps per direction; Eq. (5)'s bilinear, NT = 2; or the cubic B-spline,
// NT = 4 taps of the image's spline coefficients), or
// bicubic from a per-cell table of polynomial coefficients, and the final
// pass that evaluates Eq. (1) at the converged warp.
//
// Sample layout: lane l holds samples s = l + 64 k (slot k) of the subset in
// row-major order; slots below n / 64 are full, the next one is partial and
// the rest are empty and skipped.  The empty samples of the partial slot have
// offsets (0, 0) and zero reference data, so only their interpolated value
// has to be masked for every sum to ignore them.
#pragma once

#include "dic_device.h"

namespace dic {

__host__ __device__ __forceinline__ int icgn_patch_side(int maxM, int slack) {
  return 2 * maxM + 4 + 2 * slack;
}

// Largest subset radius M with (2M + 1)^2 <= 64 * maxs samples.
__host__ __device__ constexpr int refine_max_radius(int maxs) {
  int m = 0;
  while ((2 * m + 3) * (2 * m + 3) <= kWave * maxs) ++m;
  return m;
}

// Largest patch slack of the maxs-slot kernel: the tuning's, except in the
// 28-slot kernel, whose patch is sized for a slack of at most 6 so that three
// waves' patches per SIMD fit a CU's LDS (a larger tuned slack is clamped:
// the slack changes when the patch is restaged, not the results).
__host__ __device__ constexpr int refine_max_slack(int maxs) {
  return maxs >= 28 ? 6 : kMaxRefineSlack;
}

// Row pitch (floats) of the LDS patch of a kernel built for at most 64 * maxs
// samples per subset: odd, and at least the widest patch side such a subset
// can need.  A compile-time pitch lets the 16 taps of a sample be read from
// one address with immediate offsets (at most 3 * pitch + 3 dwords).
__host__ __device__ constexpr int refine_patch_pitch(int maxs) {
  return (2 * refine_max_radius(maxs) + 4 + 2 * refine_max_slack(maxs)) | 1;
}
static_assert(3 * refine_patch_pitch(28) + 3 <= 255, "tap offsets exceed the LDS read2 range");
static_assert(refine_max_radius(28) >= kMaxM, "largest kernel does not cover kMaxM");

// LDS bytes of a refinement workgroup: one patch of `side` rows per wave.
__host__ __device__ constexpr size_t refine_lds_bytes(int pitch, int side, int waves) {
  return (size_t)waves * side * pitch * sizeof(float);
}

// A sample's subset offsets (dx, dy): small integers, exact in fp16.
typedef _Float16 half2v __attribute__((ext_vector_type(2)));

// Warp W(p) in local FP32 form around an integer base:
//   x = bx + ax dx + uy dy + uf,  y = by + vx dx + ay dy + vf,
// ax = 1 + du/dx and ay = 1 + dv/dy rounded once to FP32, (uf, vf) the
// translation minus its rounded integer part (bx - x0, by - y0).
struct Warp32 {
  int bx, by;
  float ax, uy, uf, vx, ay, vf;
};

__device__ __forceinline__ Warp32 make_warp32(const double* p, int x0, int y0) {
  Warp32 w;
  const double ur = rint(p[0]), vr = rint(p[3]);
  w.bx = x0 + (int)ur;
  w.by = y0 + (int)vr;
  w.uf = (float)(p[0] - ur);
  w.vf = (float)(p[3] - vr);
  w.ax = (float)(1.0 + p[1]);
  w.uy = (float)p[2];
  w.vx = (float)p[4];
  w.ay = (float)(1.0 + p[5]);
  return w;
}

// Centring constant of a refinement's deformed samples: the deformed image
// (or its spline coefficients) at the integer base of the starting warp, one
// of the first iteration's taps.  Samples are handled as g - c0 in FP32, so
// c0 has to lie among the grey levels the subset meets whatever offset the
// deformed image has against the reference (ZNCC ignores a change g = a f +
// b): the reference mean would leave that offset in every FP32 sum and lose
// the variance sum g^2 - n gbar^2 to cancellation.  0 when the base is
// outside the image (the first iteration then stops with OUT_OF_BOUNDS); a
// non-finite value makes the first iteration's sums non-finite, as the tap
// it is would (NAN_INPUT).
__device__ __forceinline__ float deformed_centre(const float* __restrict__ gimg, int W, int H,
                                                 const double* p, int x0, int y0) {
  const int bx = x0 + (int)rint(p[0]), by = y0 + (int)rint(p[3]);
  if (bx < 0 || bx >= W || by < 0 || by >= H) return 0.f;
  return gimg[(int64_t)by * W + bx];
}

__device__ __forceinline__ float warp_x(const Warp32& w, float dx, float dy) {
  return fmaf(w.ax, dx, fmaf(w.uy, dy, w.uf));
}
__device__ __forceinline__ float warp_y(const Warp32& w, float dx, float dy) {
  return fmaf(w.vx, dx, fmaf(w.ay, dy, w.vf));
}

// Bounding box (absolute pixel indices) of every NT x NT neighbourhood the
// warped subset touches (bicubic: floor - 1 .. floor + 2, bilinear: floor ..
// floor + 1); extremes of an affine map over a square are at its corners.
template <int NT>
__device__ __forceinline__ void tap_box(const Warp32& w, int M, int& x_lo, int& x_hi, int& y_lo,
                                        int& y_hi) {
  float xmn = INFINITY, xmx = -INFINITY, ymn = INFINITY, ymx = -INFINITY;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const float dx = a ? (float)M : -(float)M, dy = b ? (float)M : -(float)M;
      const float xs = warp_x(w, dx, dy), ys = warp_y(w, dx, dy);
      xmn = fminf(xmn, xs);
      xmx = fmaxf(xmx, xs);
      ymn = fminf(ymn, ys);
      ymx = fmaxf(ymx, ys);
    }
  constexpr int lo = NT == 4 ? 1 : 0, hi = NT == 4 ? 2 : 1;
  x_lo = w.bx + (int)floorf(xmn) - lo;
  x_hi = w.bx + (int)floorf(xmx) + hi;
  y_lo = w.by + (int)floorf(ymn) - lo;
  y_hi = w.by + (int)floorf(ymx) + hi;
}

// Keys weights (a = -1/2) of taps -1, 0, 1, 2 at fractional offset t; with
// s = 1 - t: w-1 = -t s^2 / 2, w2 = -s t^2 / 2, w0 = 1 + t^2 (3t - 5) / 2 and
// w1 = 1 - w-1 - w0 - w2 (the four sum to one and w-1 + w2 = -t s / 2).
__device__ __forceinline__ void keys_weights32(float t, float* w) {
  const float s = 1.f - t;
  const float q = -0.5f * (t * s);
  w[0] = q * s;
  w[3] = q * t;
  w[1] = fmaf(t * t, fmaf(1.5f, t, -2.5f), 1.f);
  w[2] = (1.f - q) - w[1];
}

// d/dt of the weights above: w-1' = -s (s - 2t) / 2, w0' = t (9t - 10) / 2,
// w2' = -t (2s - t) / 2 and w1' = -(w-1' + w0' + w2').
__device__ __forceinline__ void keys_dweights32(float t, float* w) {
  const float s = 1.f - t;
  w[0] = (-0.5f * s) * fmaf(-2.f, t, s);
  w[3] = (-0.5f * t) * fmaf(2.f, s, -t);
  w[1] = t * fmaf(4.5f, t, -5.f);
  w[2] = -((w[0] + w[1]) + w[3]);
}

// Cubic B-spline basis at taps -1, 0, 1, 2 for fractional offset t; with
// s = 1 - t: w-1 = s^3 / 6, w2 = t^3 / 6, w0 = 2/3 + t^2 (t / 2 - 1) and
// w1 = 1 - w-1 - w0 - w2.
__device__ __forceinline__ void bspline_weights32(float t, float* w) {
  const float s = 1.f - t;
  w[0] = (s * s) * (s * (1.f / 6.f));
  w[3] = (t * t) * (t * (1.f / 6.f));
  w[1] = fmaf(t * t, fmaf(0.5f, t, -1.f), 2.f / 3.f);
  w[2] = ((1.f - w[0]) - w[1]) - w[3];
}

// d/dt of the basis: w-1' = -s^2 / 2, w2' = t^2 / 2, w0' = t (3t / 2 - 2)
// and w1' = -(w-1' + w0' + w2').
__device__ __forceinline__ void bspline_dweights32(float t, float* w) {
  const float s = 1.f - t;
  w[0] = -0.5f * (s * s);
  w[3] = 0.5f * (t * t);
  w[1] = t * fmaf(1.5f, t, -2.f);
  w[2] = -((w[0] + w[1]) + w[3]);
}

// Interpolation weights of the taps at fractional offset t: Keys (taps
// -1..2), Eq. (5)'s bilinear (taps 0, 1: G = a00 + a10 x' + ... is the
// weighted sum (1 - x') g0 + x' g1 along each direction) or the cubic
// B-spline basis (taps -1..2, applied to spline coefficients).
template <int IM>
__device__ __forceinline__ void interp_weights(float t, float* w) {
  if constexpr (IM == kInterpBilinear) {
    w[0] = 1.f - t;
    w[1] = t;
  } else if constexpr (IM == kInterpBSpline) {
    bspline_weights32(t, w);
  } else {
    keys_weights32(t, w);
  }
}
template <int IM>
__device__ __forceinline__ void interp_dweights(float t, float* w) {
  if constexpr (IM == kInterpBilinear) {
    w[0] = -1.f;
    w[1] = 1.f;
  } else if constexpr (IM == kInterpBSpline) {
    bspline_dweights32(t, w);
  } else {
    keys_dweights32(t, w);
  }
}

// Interpolation of one sample at local offset (xs, ys) from the integer
// base.  PatchSampler reads a wave's LDS patch, which holds g - c0 (or the
// spline coefficients minus c0: the basis sums to one, so that is the
// interpolant minus c0 too); q0 addresses its element at offset (-1, -1)
// from the base.
template <int P, int IM>
struct PatchSampler {
  static constexpr int NT = interp_taps(IM);
  const float* q0;

  __device__ __forceinline__ const float* taps(float xs, float ys, float* wx, float* wy,
                                               float& tx, float& ty) const {
    const float fx = floorf(xs), fy = floorf(ys);
    tx = xs - fx;
    ty = ys - fy;
    interp_weights<IM>(tx, wx);
    interp_weights<IM>(ty, wy);
    constexpr int first = NT == 4 ? 0 : P + 1;   // the 2x2 neighbourhood starts at (0, 0)
    // fy P + fx is a small integer, exact in FP32: one multiply-add and one
    // conversion instead of two conversions and an integer multiply-add
    return q0 + (first + (int)fmaf(fy, (float)P, fx));
  }
  static constexpr int pitch() { return P; }
  static constexpr int ntaps() { return NT; }
  static constexpr int kIm = IM;
  static constexpr bool kLut = false;
  __device__ __forceinline__ float tap(const float* q) const { return *q; }
};

// The same from the deformed image itself (row pitch W), each tap centred as
// the patch stores it (g - c0 in FP32), so both paths give the same bits; the
// NT x NT neighbourhood origin is clamped to [0, W - NT] x [0, H - NT]: the
// tap box test already keeps it there, the clamp only guards the reads of a
// degenerate warp.
template <int IM>
struct ImageSampler {
  static constexpr int NT = interp_taps(IM);
  const float* img;
  int W, H, bx, by;
  float c0;

  __device__ __forceinline__ const float* taps(float xs, float ys, float* wx, float* wy,
                                               float& tx, float& ty) const {
    const float fx = floorf(xs), fy = floorf(ys);
    tx = xs - fx;
    ty = ys - fy;
    interp_weights<IM>(tx, wx);
    interp_weights<IM>(ty, wy);
    constexpr int lo = NT == 4 ? 1 : 0;
    const int c = min(max(bx + (int)fx - lo, 0), W - NT);
    const int r = min(max(by + (int)fy - lo, 0), H - NT);
    return img + (int64_t)r * W + c;
  }
  __device__ __forceinline__ int pitch() const { return W; }
  static constexpr int ntaps() { return NT; }
  static constexpr int kIm = IM;
  static constexpr bool kLut = false;
  __device__ __forceinline__ float tap(const float* q) const { return *q - c0; }
};

// Keys bicubic from the coefficient table: cell (c, r) holds the interpolant
// on [c, c+1) x [r, r+1) as sum_{a,b} C[b][a] t^a s^b (t, s the fractional
// offsets), four float4 rows b = 0..3 of powers a = 0..3.  The value is
// Horner in t per row, then in s, with c0 taken off C[0][0] first so the
// sums run on g - c0 like the tap samplers'.  The cell is clamped to
// [1, W - 3] x [1, H - 3]: the tap box test keeps it there, the clamp only
// guards the reads of a degenerate warp.
struct LutSampler {
  const float4* lut;
  int W, H, bx, by;
  float c0;
  static constexpr int ntaps() { return 4; }
  static constexpr bool kLut = true;

  __device__ __forceinline__ const float4* cell(float xs, float ys, float& t, float& s) const {
    const float fx = floorf(xs), fy = floorf(ys);
    t = xs - fx;
    s = ys - fy;
    const int c = min(max(bx + (int)fx, 1), W - 3);
    const int r = min(max(by + (int)fy, 1), H - 3);
    return lut + ((int64_t)r * W + c) * 4;
  }
  static __device__ __forceinline__ float horner(const float4& c, float t) {
    return fmaf(fmaf(fmaf(c.w, t, c.z), t, c.y), t, c.x);
  }
  __device__ __forceinline__ float value(float xs, float ys) const {
    float t, s;
    const float4* q = cell(xs, ys, t, s);
    float4 c[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) c[b] = q[b];
    c[0].x -= c0;
    float r[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) r[b] = horner(c[b], t);
    return fmaf(fmaf(fmaf(r[3], s, r[2]), s, r[1]), s, r[0]);
  }
  __device__ __forceinline__ void value_grad(float xs, float ys, float& v, float& gx,
                                             float& gy) const {
    float t, s;
    const float4* q = cell(xs, ys, t, s);
    float4 c[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) c[b] = q[b];
    c[0].x -= c0;
    float r[4], d[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      r[b] = horner(c[b], t);
      d[b] = fmaf(fmaf(3.f * c[b].w, t, 2.f * c[b].z), t, c[b].y);
    }
    v = fmaf(fmaf(fmaf(r[3], s, r[2]), s, r[1]), s, r[0]);
    gx = fmaf(fmaf(fmaf(d[3], s, d[2]), s, d[1]), s, d[0]);
    gy = fmaf(fmaf(3.f * r[3], s, 2.f * r[2]), s, r[1]);
  }
};

// g - c0 at local offset (xs, ys).
template <class Smp>
__device__ __forceinline__ float sample_value(const Smp& smp, float xs, float ys) {
  if constexpr (Smp::kLut) {
    return smp.value(xs, ys);
  } else {
    constexpr int NT = Smp::ntaps();
    float wx[NT], wy[NT], tx, ty;
    const float* q = smp.taps(xs, ys, wx, wy, tx, ty);
    const int P = smp.pitch();
    float acc = 0.f;
#pragma unroll
    for (int l = 0; l < NT; ++l) {
      const float* row = q + l * P;
      float r = wx[0] * smp.tap(row);
#pragma unroll
      for (int k = 1; k < NT; ++k) r = fmaf(wx[k], smp.tap(row + k), r);
      acc = l == 0 ? wy[0] * r : fmaf(wy[l], r, acc);
    }
    return acc;
  }
}

// sample_value split in two for software pipelining: the taps and weights of
// one sample fetched ahead, and their combination later (the same
// arithmetic in the same order).
template <int NT>
struct TapSet {
  float t[NT * NT];
  float wx[NT], wy[NT];
};

template <class Smp>
__device__ __forceinline__ TapSet<Smp::ntaps()> taps_fetch(const Smp& smp, float xs, float ys) {
  constexpr int NT = Smp::ntaps();
  TapSet<NT> s;
  float tx, ty;
  const float* q = smp.taps(xs, ys, s.wx, s.wy, tx, ty);
  const int P = smp.pitch();
#pragma unroll
  for (int l = 0; l < NT; ++l)
#pragma unroll
    for (int c = 0; c < NT; ++c) s.t[l * NT + c] = smp.tap(q + l * P + c);
  return s;
}

template <int NT>
__device__ __forceinline__ float taps_combine(const TapSet<NT>& s) {
  float acc = 0.f;
#pragma unroll
  for (int l = 0; l < NT; ++l) {
    float r = s.wx[0] * s.t[l * NT];
#pragma unroll
    for (int k = 1; k < NT; ++k) r = fmaf(s.wx[k], s.t[l * NT + k], r);
    acc = l == 0 ? s.wy[0] * r : fmaf(s.wy[l], r, acc);
  }
  return acc;
}

// g - c0 and the interpolant's gradient (d/dx, d/dy) at local offset (xs, ys).
template <class Smp>
__device__ __forceinline__ void sample_value_grad(const Smp& smp, float xs, float ys, float& v,
                                                  float& gx, float& gy) {
  if constexpr (Smp::kLut) {
    smp.value_grad(xs, ys, v, gx, gy);
  } else {
    constexpr int NT = Smp::ntaps();
    float wx[NT], wy[NT], tx, ty, dwx[NT], dwy[NT];
    const float* q = smp.taps(xs, ys, wx, wy, tx, ty);
    interp_dweights<Smp::kIm>(tx, dwx);
    interp_dweights<Smp::kIm>(ty, dwy);
    const int P = smp.pitch();
#pragma unroll
    for (int l = 0; l < NT; ++l) {
      const float* row = q + l * P;
      float t[NT];
#pragma unroll
      for (int c = 0; c < NT; ++c) t[c] = smp.tap(row + c);
      float r = wx[0] * t[0], rd = dwx[0] * t[0];
#pragma unroll
      for (int c = 1; c < NT; ++c) {
        r = fmaf(wx[c], t[c], r);
        rd = fmaf(dwx[c], t[c], rd);
      }
      v = l == 0 ? wy[0] * r : fmaf(wy[l], r, v);
      gx = l == 0 ? wy[0] * rd : fmaf(wy[l], rd, gx);
      gy = l == 0 ? dwy[0] * r : fmaf(dwy[l], r, gy);
    }
  }
}

// Offsets and one or (TWO) two per-sample reference values of every slot of
// this lane, stepping (row, column) of the subset by 64 samples per slot.
// ref0 / ref1 address the subset's top-left sample with row pitch `pitch`.
// (The second array is chosen at compile time: a run-time null test of its
// pointer keeps the array in scratch memory, a private address of zero being
// valid.)
template <int MAXS, bool TWO>
__device__ __forceinline__ void load_slots(int M, int n, const float* __restrict__ ref0,
                                           const float* __restrict__ ref1, int pitch,
                                           half2v* dxy, float* v0, float* v1) {
  const int n1 = 2 * M + 1, lane = lane_id();
  const int dr = kWave / n1, dc = kWave - dr * n1;
  int r = lane / n1, c = lane - r * n1;
#pragma unroll
  for (int k = 0; k < MAXS; ++k) {
    dxy[k] = half2v{(_Float16)0.f, (_Float16)0.f};
    v0[k] = 0.f;
    if constexpr (TWO) v1[k] = 0.f;
    if (lane + kWave * k < n) {
      const int o = __umul24(r, pitch) + c;
      v0[k] = ref0[o];
      if constexpr (TWO) v1[k] = ref1[o];
      dxy[k] = half2v{(_Float16)(c - M), (_Float16)(r - M)};
    }
    c += dc;
    r += dr;
    if (c >= n1) {
      c -= n1;
      ++r;
    }
  }
}

// Slot bookkeeping of one pass: whether slot k holds samples, and the mask
// for the missing samples of the partial slot.  The sample count is made
// opaque at the start of every pass so the per-slot tests stay scalar
// compares inside the pass instead of masks kept live across the solve.
struct Slots {
  int n;
  bool tail_valid;
  __device__ __forceinline__ explicit Slots(int n_) : n(__builtin_amdgcn_readfirstlane(n_)) {
    tail_valid = lane_id() < n % kWave;
  }
  __device__ __forceinline__ bool used(int k) const { return kWave * k < n; }
  // v, or 0 for a missing sample of slot k
  __device__ __forceinline__ float mask(int k, float v) const {
    return (kWave * (k + 1) > n && !tail_valid) ? 0.f : v;
  }
};

// Subset offsets (dx, dy) of a lane's sample in slot k.  Kept per slot as
// exact fp16 pairs, or, where registers decide the occupancy, recomputed from the sample index k' = lane + 64 k: row trunc((k' + 1/2) /
// n1) in FP32 (exact for k' < 4096: the rounding error is far inside the
// distance 1 / (2 n1) to an integer), column k' - row n1.  A lane past the
// subset takes its last sample (its values are masked either way).
struct OffsetsKept {
  const half2v* dxy;
  __device__ __forceinline__ void operator()(int k, float& dx, float& dy) const {
    dx = (float)dxy[k].x;
    dy = (float)dxy[k].y;
  }
};
struct OffsetsComputed {
  int lane, M, n1, last;
  float inv, hinv;
  __device__ __forceinline__ explicit OffsetsComputed(int M_) {
    lane = lane_id();
    M = M_;
    n1 = 2 * M_ + 1;
    last = n1 * n1 - 1;
    inv = 1.0f / (float)n1;
    hinv = 0.5f * inv;
  }
  __device__ __forceinline__ void operator()(int k, float& dx, float& dy) const {
    // opaque per use, so the offsets are not hoisted out of the iteration
    // loop into registers again
    int l = lane;
    __asm__ volatile("" : "+v"(l));
    const int t = min(l + kWave * k, last);
    const int r = (int)fmaf((float)t, inv, hinv);
    dx = (float)(t - (int)__umul24((uint32_t)r, (uint32_t)n1) - M);
    dy = (float)(r - M);
  }
};

// Sums over this lane's samples at the final warp: sum (g - c0),
// sum (g - c0)^2 and sum (f - fbar)(g - c0), with f - fbar of slot k at
// offsets (dx, dy) given by tval(k, dx, dy).
// The template values are all requested before the sampling (one memory
// round trip), and the slots every subset of the class fills run without a
// per-slot test, so their reads can overlap.
template <int MAXS, class Smp, class OF, class TV>
__device__ __forceinline__ void final_pass(const Smp& smp, int n, const Warp32& w,
                                           const OF& offs, const TV& tval, float* K) {
  constexpr int MINS = refine_min_slots(MAXS);
  const Slots sl(n);
  float tv[MAXS];
#pragma unroll
  for (int k = 0; k < MAXS; ++k) {
    tv[k] = 0.f;
    if (k < MINS || sl.used(k)) {
      float dx, dy;
      offs(k, dx, dy);
      tv[k] = tval(k, dx, dy);
    }
  }
  K[0] = K[1] = K[2] = 0.f;
#pragma unroll
  for (int k = 0; k < MAXS; ++k) {
    if (k >= MINS && !sl.used(k)) continue;
    float dx, dy;
    offs(k, dx, dy);
    const float v = sample_value(smp, warp_x(w, dx, dy), warp_y(w, dx, dy));
    const float gs = k + 1 >= MINS ? sl.mask(k, v) : v;
    K[0] += gs;
    K[1] = fmaf(gs, gs, K[1]);
    K[2] = fmaf(tv[k], gs, K[2]);
  }
}

// Two-rows-per-slot layout, for subsets of at most 31 columns: lane l holds
// column c = l mod 32 (clamped to the subset; lanes past it carry zero
// gradients and have their two value sums cleared after the pass) of row
// 2k + l / 32 in slot k < M, and slot M holds the last row 2M in the lower
// half-wave (the upper half repeats it, masked).  A lane's column offset dx
// is then fixed, so its x position advances by 2 uy per slot from one base,
// sum SD g dx is dx times sum SD g, and the dy-weighted sums take the slot's
// even row offset 2k as a constant plus (l / 32 - M) times the plain sum:
// fewer operations per sample than the general layout and no per-slot
// offsets in registers.  The two-rows kernels' LDS patch pitch is sized for
// radius 15 and a slack of at most kR2MaxSlack pixels (a larger tuned slack
// is clamped: the slack changes when the patch is restaged, not the
// results), so that four waves' patches fit a CU's LDS.
constexpr int kR2MaxSlack = 6;
constexpr int kR2Pitch = (2 * 15 + 4 + 2 * kR2MaxSlack) | 1;
static_assert(3 * kR2Pitch + 3 <= 255, "tap offsets exceed the LDS read2 range");

struct R2Lane {
  float dx;      // column offset of this lane (clamped into the subset)
  float hm;      // l / 32 - M: the row offset of slot 0
  bool colok;    // the column lies in the subset
  bool upper;    // l / 32 == 1
};

__device__ __forceinline__ R2Lane r2_lane(int M) {
  const int lane = lane_id(), c = lane & 31, h = lane >> 5, n1 = 2 * M + 1;
  R2Lane L;
  L.colok = c < n1;
  L.dx = (float)((L.colok ? c : n1 - 1) - M);
  L.hm = (float)(h - M);
  L.upper = h != 0;
  return L;
}

// Per-sample reference values of the lane in the two-rows layout: slots
// k < M, then the last row's value (zero for the upper half and for columns
// outside the subset).  `a` (and `b`, nullable) address the subset's
// top-left sample with row pitch `pitch`.
template <int MAXS>
__device__ __forceinline__ void load_slots_r2(int M, const R2Lane& L, const float* __restrict__ a,
                                              const float* __restrict__ b, int pitch, float* va,
                                              float* vb, float& pa, float& pb) {
  const int c = (int)L.dx + M, h = L.upper ? 1 : 0;
#pragma unroll
  for (int k = 0; k < MAXS - 1; ++k) {
    va[k] = 0.f;
    if (b) vb[k] = 0.f;
    if (k < M && L.colok) {
      const int o = __umul24(2 * k + h, pitch) + c;
      va[k] = a[o];
      if (b) vb[k] = b[o];
    }
  }
  pa = pb = 0.f;
  if (L.colok && !L.upper) {
    const int o = __umul24(2 * M, pitch) + c;
    pa = a[o];
    if (b) pb = b[o];
  }
}

// final_pass in the two-rows layout: sum (g - c0), sum (g - c0)^2 and
// sum (f - fbar)(g - c0), the template value at (dx, dy) from tval.
template <int MAXS, class Smp, class TV>
__device__ __forceinline__ void final_pass_r2(const Smp& smp, int M, const R2Lane& L,
                                              const Warp32& w, const TV& tval, float* K) {
  const int Mu = __builtin_amdgcn_readfirstlane(M);
  const float bx = fmaf(w.ax, L.dx, fmaf(w.uy, L.hm, w.uf));
  const float by = fmaf(w.vx, L.dx, fmaf(w.ay, L.hm, w.vf));
  // the template values first (one memory round trip); slots below kR2MinM
  // hold samples for every subset of the layout, so they need no test
  float tv[MAXS - 1];
#pragma unroll
  for (int k = 0; k < MAXS - 1; ++k) {
    tv[k] = 0.f;
    if (k < kR2MinM || k < Mu) tv[k] = tval(0, L.dx, (float)(2 * k) + L.hm);
  }
  const float dm = (float)Mu;
  const float tvm = tval(0, L.dx, dm);
  float k0 = 0.f, k1 = 0.f, k2 = 0.f;
#pragma unroll
  for (int k = 0; k < MAXS - 1; ++k) {
    if (k >= kR2MinM && k >= Mu) continue;
    const float dk = (float)(2 * k);
    const float gs = sample_value(smp, fmaf(w.uy, dk, bx), fmaf(w.ay, dk, by));
    k0 += gs;
    k1 = fmaf(gs, gs, k1);
    k2 = fmaf(tv[k], gs, k2);
  }
  {
    const float v = sample_value(smp, fmaf(w.ax, L.dx, fmaf(w.uy, dm, w.uf)),
                                 fmaf(w.vx, L.dx, fmaf(w.ay, dm, w.vf)));
    const float gs = L.upper ? 0.f : v;
    k0 += gs;
    k1 = fmaf(gs, gs, k1);
    k2 = fmaf(tvm, gs, k2);
  }
  K[0] = L.colok ? k0 : 0.f;
  K[1] = L.colok ? k1 : 0.f;
  K[2] = L.colok ? k2 : 0.f;
}

// Per-wave LDS patch of the deformed image: `side` rows of pitch P holding
// g - c0 (zero outside the image).
template <int P>
struct LdsPatch {
  float* buf;
  int side;
  int x0 = INT_MIN, y0 = INT_MIN;

  // Makes [x_lo, x_hi] x [y_lo, y_hi] resident, centred in the patch; false
  // when it cannot fit.  One column per lane (two passes when the side
  // exceeds 64).  A patch inside the image is read in batches of 16 rows; one
  // that is not reads clamped, always valid addresses in batches of eight, so
  // a batch is issued back to back, and replaces the pixels outside the image
  // by zero afterwards.
  __device__ __forceinline__ bool ensure(const float* __restrict__ img, int W, int H, int x_lo,
                                         int x_hi, int y_lo, int y_hi, float c0) {
    if (x_lo >= x0 && x_hi < x0 + side && y_lo >= y0 && y_hi < y0 + side) return true;
    const int bw = x_hi - x_lo + 1, bh = y_hi - y_lo + 1;
    if (bw > side || bh > side) return false;
    x0 = x_lo - (side - bw) / 2;
    y0 = y_lo - (side - bh) / 2;
    wave_lds_sync();
    if (x0 >= 0 && x0 + side <= W && y0 >= 0 && y0 + side <= H) {
      // the whole patch lies in the image: no clamping, 16 rows per batch
      for (int c = lane_id(); c < side; c += kWave) {
        const float* col = img + (int64_t)y0 * W + x0 + c;
        for (int r0 = 0; r0 < side; r0 += 16) {
          float v[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) v[u] = col[(int64_t)min(r0 + u, side - 1) * W];
#pragma unroll
          for (int u = 0; u < 16; ++u)
            if (r0 + u < side) buf[(r0 + u) * P + c] = v[u] - c0;
        }
      }
    } else {
      for (int c = lane_id(); c < side; c += kWave) {
        const int X = x0 + c;
        const bool col_in = X >= 0 && X < W;
        const float* col = img + min(max(X, 0), W - 1);
        for (int r0 = 0; r0 < side; r0 += 8) {
          float v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) v[u] = col[(int64_t)min(max(y0 + r0 + u, 0), H - 1) * W];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int Y = y0 + r0 + u;
            if (r0 + u < side)
              buf[(r0 + u) * P + c] = (col_in && Y >= 0 && Y < H) ? v[u] - c0 : 0.f;
          }
        }
      }
    }
    wave_lds_sync();
    return true;
  }

  // Sampler for a warp whose integer base is (bx, by).
  template <int IM>
  __device__ __forceinline__ PatchSampler<P, IM> sampler(int bx, int by) const {
    return PatchSampler<P, IM>{buf + (by - y0 - 1) * P + (bx - x0 - 1)};
  }
};

}  // namespace dic
