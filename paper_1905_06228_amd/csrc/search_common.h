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

// Eq. (1) in FP64 for the candidate whose subset is centred at (xg, yg):
// the window mean is the FP64 box sum *s1 over n, then one pass over the
// subset accumulates sum (f - fbar)(g - gbar), sum (g - gbar)^2 and sum g^2
// per lane (pixel k on lane k mod 64) and one DPP reduction adds the lanes in
// a fixed order.  Loads are issued eight rounds at a time from clamped,
// always valid addresses so their latencies overlap.  All 64 lanes of the
// wave must call it together; every lane returns the same value.  `ok` is
// false for a flat window.
__device__ __forceinline__ double rescore_wave(const float* __restrict__ f,
                                               const float* __restrict__ gimg, int W, int x0,
                                               int y0, int xg, int yg, int M, double fbar,
                                               double df, const double* s1, bool* ok) {
  const int n1 = 2 * M + 1, n = n1 * n1, lane = lane_id();
  const float* fb = f + (int64_t)(y0 - M) * W + (x0 - M);
  const float* gb = gimg + (int64_t)(yg - M) * W + (xg - M);
  const double sum_g = *s1;
  double num = 0.0, q = 0.0, sq = 0.0;
  for (int k0 = 0; k0 < n; k0 += 8 * kWave) {
    float gv[8], fv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = min(k0 + u * kWave + lane, n - 1);
      const int r = k / n1, c = k - r * n1;
      gv[u] = gb[(int64_t)r * W + c];
      fv[u] = fb[(int64_t)r * W + c];
    }
    const double gbar = sum_g / (double)n;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool in = k0 + u * kWave + lane < n;
      const double d = in ? (double)gv[u] - gbar : 0.0;
      const double e = in ? (double)fv[u] - fbar : 0.0;
      const double gg = in ? (double)gv[u] : 0.0;
      num += e * d;
      q += d * d;
      sq += gg * gg;
    }
  }
  num = wave_sum_dpp(num);
  q = wave_sum_dpp(q);
  sq = wave_sum_dpp(sq);
  *ok = not_flat(q, sq);
  return num / (df * sqrt(q));
}

}  // namespace dic
