// Pieces shared by the sub-pixel refinements of Sec. 2.2 (IC-GN and
// Newton-Raphson, FP32 batched forms): the first-order warp in FP32 local
// form, the bounding box of the taps it touches, Keys bicubic interpolation
// from an image or a per-wave LDS patch, and the final pass that evaluates
// Eq. (1) at the converged warp.
#pragma once

#include "dic_device.h"

namespace dic {

__host__ __device__ __forceinline__ int icgn_patch_side(int maxM, int slack) {
  return 2 * maxM + 4 + 2 * slack;
}


// A sample's subset offsets (dx, dy): small integers, exact in fp16, one
// register per sample.
typedef _Float16 half2v __attribute__((ext_vector_type(2)));

struct Warp32 {
  int bx, by;                  // integer base of the sample positions
  float uf, vf, ux, uy, vx, vy;  // local offsets: x = bx + dx + ux dx + uy dy + uf
};

__device__ __forceinline__ Warp32 make_warp32(const double* p, int x0, int y0) {
  Warp32 w;
  const double ur = rint(p[0]), vr = rint(p[3]);
  w.bx = x0 + (int)ur;
  w.by = y0 + (int)vr;
  w.uf = (float)(p[0] - ur);
  w.vf = (float)(p[3] - vr);
  w.ux = (float)p[1];
  w.uy = (float)p[2];
  w.vx = (float)p[4];
  w.vy = (float)p[5];
  return w;
}

__device__ __forceinline__ float warp_x(const Warp32& w, float dx, float dy) {
  return dx + fmaf(w.ux, dx, fmaf(w.uy, dy, w.uf));
}
__device__ __forceinline__ float warp_y(const Warp32& w, float dx, float dy) {
  return dy + fmaf(w.vx, dx, fmaf(w.vy, dy, w.vf));
}

// Bounding box (absolute pixel indices) of every 4x4 neighbourhood the
// warped subset touches; extremes of an affine map over a square are at its
// corners.
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
  x_lo = w.bx + (int)floorf(xmn) - 1;
  x_hi = w.bx + (int)floorf(xmx) + 2;
  y_lo = w.by + (int)floorf(ymn) - 1;
  y_hi = w.by + (int)floorf(ymx) + 2;
}

// Interpolated grey level at local offset (xs, ys).  `src` holds the image
// (or the staged patch) with row pitch `pitch`; (ox, oy) is the position of
// the integer base inside it.  With kClamp the 4x4 neighbourhood origin is
// clamped to [0, maxc] x [0, maxr]: the tap box test already keeps it there,
// the clamp only guarantees in-bounds reads for a degenerate warp.
template <bool kClamp>
__device__ __forceinline__ float interp32(const float* src, int pitch, int ox, int oy, float xs,
                                          float ys, int maxc, int maxr) {
  const float fx = floorf(xs), fy = floorf(ys);
  float wx[4], wy[4];
  cubic_weights(xs - fx, wx);
  cubic_weights(ys - fy, wy);
  int c0 = (int)fx - 1 + ox, r0 = (int)fy - 1 + oy;
  if (kClamp) {
    c0 = min(max(c0, 0), maxc);
    r0 = min(max(r0, 0), maxr);
  }
  // patch offsets fit 24 bits: a full-rate multiply
  const float* q = kClamp ? src + (int64_t)r0 * pitch + c0 : src + (__umul24(r0, pitch) + c0);
  float acc = 0.f;
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    const float* row = q + l * pitch;
    const float r = fmaf(wx[3], row[3], fmaf(wx[2], row[2], fmaf(wx[1], row[1], wx[0] * row[0])));
    acc = fmaf(wy[l], r, acc);
  }
  return acc;
}

template <int MAXS, bool kClamp>
__device__ __forceinline__ void final_pass(const float* src, int pitch, int ox, int oy, int maxc,
                                           int maxr, int n, const Warp32& w, float c0,
                                           const half2v* dxy, const float* __restrict__ tm,
                                           int tp, int M, float* K) {
  const int lane = lane_id();
#pragma unroll
  for (int k = 0; k < MAXS; ++k) {
    if (lane + kWave * k < n) {
      const float dx = (float)dxy[k].x, dy = (float)dxy[k].y;
      const float gs =
          interp32<kClamp>(src, pitch, ox, oy, warp_x(w, dx, dy), warp_y(w, dx, dy), maxc, maxr) -
          c0;
      K[0] += gs;
      K[1] = fmaf(gs, gs, K[1]);
      K[2] = fmaf(tm[((int)dy + M) * tp + (int)dx + M], gs, K[2]);
    }
  }
}

// Per-wave LDS patch of the deformed image.
struct Patch {
  float* buf;
  int side;
  int x0 = INT_MIN, y0 = INT_MIN;
  // Makes [x_lo, x_hi] x [y_lo, y_hi] resident; false when it cannot fit.
  __device__ __forceinline__ bool ensure(const float* __restrict__ img, int W, int H, int x_lo,
                                         int x_hi, int y_lo, int y_hi) {
    if (x_lo >= x0 && x_hi < x0 + side && y_lo >= y0 && y_hi < y0 + side) return true;
    const int bw = x_hi - x_lo + 1, bh = y_hi - y_lo + 1;
    if (bw > side || bh > side) return false;
    x0 = x_lo - (side - bw) / 2;
    y0 = y_lo - (side - bh) / 2;
    const int lane = lane_id();
    wave_lds_sync();
    for (int idx = lane; idx < side * side; idx += kWave) {
      const int r = idx / side, c = idx - r * side;
      const int X = x0 + c, Y = y0 + r;
      buf[idx] = (X >= 0 && X < W && Y >= 0 && Y < H) ? img[(int64_t)Y * W + X] : 0.f;
    }
    wave_lds_sync();
    return true;
  }
};

}  // namespace dic
