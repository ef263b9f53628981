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

// Eq. (1) in FP64 for up to B candidates (cnt of them, cnt uniform and at
// least 1) whose subsets are centred at (xg[b], yg[b]), in one pass over the
// subset: per candidate the window mean is its FP64 box sum (s1 plane) over
// n, and each lane accumulates sum (f - fbar)(g - gbar), sum (g - gbar)^2 and
// sum g^2 over pixels k = lane, lane + 64, ...; one DPP reduction per sum adds
// the lanes in a fixed order.  The arithmetic of a candidate does not depend
// on B or on the other candidates.  Loads are issued sixteen rounds at a time
// (a subset of up to 1024 pixels in one batch) from clamped, always valid
// addresses so their latencies overlap.  All 64
// lanes of the wave must call it together; z[b] is the same on every lane,
// -inf for a flat window.
template <int B>
__device__ __forceinline__ void rescore_wave(const float* __restrict__ f,
                                             const float* __restrict__ gimg, int W, int x0,
                                             int y0, const int* xg, const int* yg, int cnt,
                                             int M, double fbar, double df,
                                             const double* __restrict__ s1plane, double* z) {
  const int n1 = 2 * M + 1, n = n1 * n1, lane = lane_id();
  const float* fb = f + (int64_t)(y0 - M) * W + (x0 - M);
  const float* gb[B];
  double sum_g[B], num[B], q[B], sq[B];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int k = b < cnt ? b : 0;
    gb[b] = gimg + (int64_t)(yg[k] - M) * W + (xg[k] - M);
    sum_g[b] = s1plane[(int64_t)yg[k] * W + xg[k]];
    num[b] = q[b] = sq[b] = 0.0;
  }
  // pixel k = (r, c) of this lane, advanced by 64 pixels per round
  const int dr = kWave / n1, dc = kWave - dr * n1;
  int r = lane / n1, c = lane - r * n1;
  constexpr int U = 16;
  for (int k0 = 0; k0 < n; k0 += U * kWave) {
    float fv[U], gv[B][U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool in = k0 + u * kWave + lane < n;
      const int o = in ? r * W + c : (n1 - 1) * (W + 1);
      fv[u] = fb[o];
#pragma unroll
      for (int b = 0; b < B; ++b) gv[b][u] = gb[b][o];
      c += dc;
      r += dr;
      if (c >= n1) {
        c -= n1;
        ++r;
      }
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const double gbar = sum_g[b] / (double)n;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool in = k0 + u * kWave + lane < n;
        const double d = in ? (double)gv[b][u] - gbar : 0.0;
        const double e = in ? (double)fv[u] - fbar : 0.0;
        const double gg = in ? (double)gv[b][u] : 0.0;
        num[b] += e * d;
        q[b] += d * d;
        sq[b] += gg * gg;
      }
    }
  }
#pragma unroll
  for (int b = 0; b < B; ++b) {
    if (b < cnt) {
      const double nu = wave_sum_dpp(num[b]), qq = wave_sum_dpp(q[b]), ss = wave_sum_dpp(sq[b]);
      z[b] = not_flat(qq, ss) ? nu / (df * sqrt(qq)) : -INFINITY;
    }
  }
}

}  // namespace dic
