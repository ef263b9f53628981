// Pieces shared by the integer-search kernels (Sec. 2.1, Eq. (1)): the FP64
// re-score that decides the winner and the capacity of the near-tie list.
//
// Every search form first scores all candidates approximately, then keeps
// the few whose approximate score could still be the maximum and evaluates
// Eq. (1) for them in FP64 with this one routine, so the winner and its
// coefficient do not depend on the form or its launch shape.
#pragma once

#include "dic_device.h"

namespace dic {

constexpr int kNearCap = 64;   // re-scored candidates kept per POI (a second sweep covers more)

// Eq. (1) in FP64 for up to B candidates (cnt of them, cnt uniform, 1 <= cnt
// <= B) whose subsets are centred at (xg[b], yg[b]), in one pass over the
// subset: per candidate the window mean is its FP64 box sum (s1 plane) over
// n, and each lane accumulates sum (f - fbar)(g - gbar) and sum (g - gbar)^2
// over pixels k = lane, lane + 64, ... in that order; one DPP reduction per
// sum adds the lanes in a fixed order.  The flatness test takes sum g^2 as
// sum (g - gbar)^2 + gbar sum g.  The arithmetic of a candidate does not
// depend on B, cnt or the other candidates.  Loads are issued sixteen rounds
// of 64 pixels at a time, the last (partial) round's with the first batch,
// so their latencies overlap; only that round masks its lanes.  All 64 lanes
// of the wave must call it together; z[b] (b < cnt) is the same on every
// lane, -inf for a flat window.  `lane` is the lane index.
template <int B>
__device__ __forceinline__ void rescore_wave(const float* __restrict__ f,
                                             const float* __restrict__ gimg, int W, int x0,
                                             int y0, const int* xg, const int* yg, int cnt,
                                             int M, double fbar, double df,
                                             const double* __restrict__ s1plane, double* z,
                                             int lane) {
  const int n1 = 2 * M + 1, n = n1 * n1;
  const char* fb = reinterpret_cast<const char*>(f + (int64_t)(y0 - M) * W + (x0 - M));
  const char* gb[B];
  double s1[B], gbar[B], num[B], q[B];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int k = b < cnt ? b : 0;
    gb[b] = reinterpret_cast<const char*>(gimg + (int64_t)(yg[k] - M) * W + (xg[k] - M));
    s1[b] = s1plane[(int64_t)yg[k] * W + xg[k]];
    gbar[b] = s1[b] / (double)n;
    num[b] = q[b] = 0.0;
  }
  // Pixel k of the subset (row k / n1, column k % n1) lies k + (k / n1)(W - n1)
  // pixels past the subset's corner.  k / n1 is taken as trunc((k + 1/2) / n1)
  // in FP32: for k < 4096 the rounding error (below 1e-4) is far inside the
  // distance, at least 1 / (2 n1), of (k + 1/2) / n1 from an integer.
  const float inv = 1.0f / (float)n1, hinv = 0.5f * inv;
  const uint32_t wstep4 = 4u * (uint32_t)(W - n1);
  const float lanef = (float)lane;
  const uint32_t lane4 = 4u * (uint32_t)lane;
  // byte offset of pixel 64 rr + lane (rr uniform)
  auto offset = [&](int rr) -> uint32_t {
    const uint32_t r = (uint32_t)fmaf(lanef + (float)(rr * kWave), inv, hinv);
    return __umul24(r, wstep4) + lane4 + (uint32_t)(4 * kWave * rr);
  };
  auto ld = [](const char* p, uint32_t o) { return *reinterpret_cast<const float*>(p + o); };
  const int nfull = n / kWave;   // rounds with every lane's pixel in the subset
  const bool tail = nfull * kWave < n;
  float ft = 0.f, gt[B];
#pragma unroll
  for (int b = 0; b < B; ++b) gt[b] = 0.f;
  if (tail) {
    // lanes past the subset's last pixel read that pixel
    const int k = min(nfull * kWave + lane, n - 1);
    const uint32_t o = 4u * (__umul24((uint32_t)fmaf((float)k, inv, hinv), wstep4 >> 2) + (uint32_t)k);
    ft = ld(fb, o);
#pragma unroll
    for (int b = 0; b < B; ++b)
      if (b < cnt) gt[b] = ld(gb[b], o);
  }
  constexpr int U = 16;
  for (int r0 = 0; r0 < nfull; r0 += U) {
    // rounds r0 .. r0 + nr - 1 in slots s0 .. U - 1
    const int nr = min(U, nfull - r0), s0 = U - nr;
    float fv[U], gv[B][U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      fv[u] = 0.f;
#pragma unroll
      for (int b = 0; b < B; ++b) gv[b][u] = 0.f;
      if (u >= s0) {
        const uint32_t o = offset(r0 + u - s0);
        fv[u] = ld(fb, o);
#pragma unroll
        for (int b = 0; b < B; ++b)
          if (b < cnt) gv[b][u] = ld(gb[b], o);
      }
    }
    // slots s0 .. U - 1 in order, entered at s0 and falling through (no
    // per-slot condition the compiler could turn into selects); one copy for
    // each candidate count
    auto run = [&](auto nb_c) {
      constexpr int NB = decltype(nb_c)::value;
      auto acc = [&](int u) {
        const double e = (double)fv[u] - fbar;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const double d = (double)gv[b][u] - gbar[b];
          num[b] += e * d;
          q[b] += d * d;
        }
      };
      switch (s0) {
        case 0: acc(0); [[fallthrough]];
        case 1: acc(1); [[fallthrough]];
        case 2: acc(2); [[fallthrough]];
        case 3: acc(3); [[fallthrough]];
        case 4: acc(4); [[fallthrough]];
        case 5: acc(5); [[fallthrough]];
        case 6: acc(6); [[fallthrough]];
        case 7: acc(7); [[fallthrough]];
        case 8: acc(8); [[fallthrough]];
        case 9: acc(9); [[fallthrough]];
        case 10: acc(10); [[fallthrough]];
        case 11: acc(11); [[fallthrough]];
        case 12: acc(12); [[fallthrough]];
        case 13: acc(13); [[fallthrough]];
        case 14: acc(14); [[fallthrough]];
        default: acc(15);
      }
    };
    if (B > 1 && cnt < B)
      run(std::integral_constant<int, 1>{});
    else
      run(std::integral_constant<int, B>{});
  }
  if (tail) {
    const bool in = nfull * kWave + lane < n;
    const double e = in ? (double)ft - fbar : 0.0;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      if (b >= cnt) continue;
      const double d = in ? (double)gt[b] - gbar[b] : 0.0;
      num[b] += e * d;
      q[b] += d * d;
    }
  }
#pragma unroll
  for (int b = 0; b < B; ++b) {
    if (b < cnt) {
      const double nu = wave_sum_dpp(num[b]), qq = wave_sum_dpp(q[b]);
      z[b] = not_flat(qq, qq + gbar[b] * s1[b]) ? nu / (df * sqrt(qq)) : -INFINITY;
    }
  }
}

}  // namespace dic
