// Brute-force integer search (Sec. 2.1): Eq. (1) at every candidate of a
// (2S+1)^2 window per POI.
//
// FP32 batched form.  One workgroup per POI at a time, persistent over a
// shared work counter.  The deformed window (2S+2M+1 square, shifted by the
// subset mean so sums stay small) is staged in LDS once.  Per candidate the
// window sums sum(g) and sum(g^2) come from running box sums (Kahan), and the
// cross term sum(t_i g_i) with the mean-free template t from a register-
// blocked loop: a lane owns L horizontally adjacent candidates, keeps a
// sliding window of L grey levels in registers and reads each template value
// once from scalar memory, so one LDS read feeds L FMAs.  Per template row
// the L partial sums are added to Kahan totals.  The FP32 maximum selects the
// candidates within 2e-5 of it, which one wave re-scores two-pass in FP64
// before the tie rule picks the winner.
#include "dic_device.h"

namespace dic {

namespace {

struct SearchGeom {
  int M, S, n1, n, side, L, NB, n1p, Wn, P;
};

__host__ __device__ __forceinline__ SearchGeom search_geom(int M, int S, int L) {
  SearchGeom G;
  G.M = M;
  G.S = S;
  G.n1 = 2 * M + 1;
  G.n = G.n1 * G.n1;
  G.side = 2 * S + 1;
  G.L = L;
  G.NB = (G.side + L - 1) / L;
  G.n1p = (G.n1 + L - 1) / L * L;
  G.Wn = G.side + G.n1 - 1;
  const int pc = G.NB * L + G.n1p - 1;
  G.P = pc | 1;
  return G;
}

__host__ __device__ __forceinline__ size_t search_lds_floats(const SearchGeom& G) {
  return (size_t)G.Wn * G.P + 2 * (size_t)G.side * G.Wn + 3 * (size_t)G.side * G.side;
}

}  // namespace

size_t search_lds_bytes(int maxM, int maxS, int block) {
  // The layout depends on M and S jointly; take the largest over the plan's
  // range (monotone in both).
  return search_lds_floats(search_geom(maxM, maxS, block)) * sizeof(float) + 64;
}

// FP64 two-pass coefficient of one candidate, computed by a whole wave
// exactly as Eq. (1) defines it.
__device__ double rescore_f64(const float* __restrict__ f, const float* __restrict__ gimg, int W,
                              int x0, int y0, int xg, int yg, int M, double fbar, double df,
                              bool* valid) {
  const int lane = lane_id(), n1 = 2 * M + 1, n = n1 * n1;
  double sg = 0.0;
  int bad = 0;
  for (int k = lane; k < n; k += kWave) {
    const int r = k / n1, c = k - r * n1;
    const float v = gimg[(int64_t)(yg - M + r) * W + (xg - M + c)];
    bad |= !isfinite(v);
    sg += (double)v;
  }
  sg = wave_sum(sg);
  bad = wave_or_int(bad);
  if (bad) {
    *valid = false;
    return 0.0;
  }
  const double gbar = sg / (double)n;
  double num = 0.0, q = 0.0, sq = 0.0;
  for (int k = lane; k < n; k += kWave) {
    const int r = k / n1, c = k - r * n1;
    const double gv = (double)gimg[(int64_t)(yg - M + r) * W + (xg - M + c)];
    const double fv = (double)f[(int64_t)(y0 - M + r) * W + (x0 - M + c)];
    const double d = gv - gbar;
    num += (fv - fbar) * d;
    q += d * d;
    sq += gv * gv;
  }
  num = wave_sum(num);
  q = wave_sum(q);
  sq = wave_sum(sq);
  *valid = not_flat(q, sq);
  return num / (df * sqrt(q));
}

template <int L>
__global__ void __launch_bounds__(1024) search_f32_kernel(
    DevState st, const float* __restrict__ ref, const float* __restrict__ def,
    const int32_t* __restrict__ poi, const int32_t* __restrict__ seed,
    int32_t* __restrict__ uv_out, float* __restrict__ zncc_out, int32_t* __restrict__ status_out) {
  extern __shared__ float lds[];
  __shared__ int s_item;
  __shared__ float s_wmax[16];
  __shared__ int s_pick[2];
  __shared__ float s_zncc;
  const int tid = threadIdx.x, nthr = blockDim.x, lane = lane_id(), wid = tid / kWave;
  const float kNegInf = -INFINITY;

  for (;;) {
    if (tid == 0) s_item = atomicAdd(&st.counters[kCtrSearch], 1);
    __syncthreads();
    const int item = uniform(s_item);
    if (item >= st.N) break;
    const int g = uniform(st.work[item]);
    const DevPair P = st.pairs[uniform(st.poi_pair[g])];
    const RefRec* R = st.recs + g;
    const int x0 = uniform(poi[2 * g]), y0 = uniform(poi[2 * g + 1]);
    const int cu = seed ? uniform(seed[2 * g]) : 0;
    const int cv = seed ? uniform(seed[2 * g + 1]) : 0;
    const int rstat = uniform(R->status);
    if (rstat != DIC_POI_OK) {
      if (tid == 0) {
        uv_out[2 * g] = 0;
        uv_out[2 * g + 1] = 0;
        zncc_out[g] = nanf("");
        status_out[g] = rstat == DIC_POI_SINGULAR_HESSIAN ? DIC_POI_OK : rstat;
      }
      // A singular Hessian does not stop the search; fall through below.
      if (rstat != DIC_POI_SINGULAR_HESSIAN) {
        __syncthreads();
        continue;
      }
    }
    const SearchGeom G = search_geom(P.M, P.S, L);
    const int W = P.width, H = P.height;
    const float* gimg = def + P.def_off;
    const float c0 = (float)R->fbar;
    const int wx0 = x0 + cu - G.S - G.M, wy0 = y0 + cv - G.S - G.M;

    float* win = lds;
    float* colS = win + G.Wn * G.P;
    float* colQ = colS + G.side * G.Wn;
    float* boxS = colQ + G.side * G.Wn;
    float* boxQ = boxS + G.side * G.side;
    float* scores = boxQ + G.side * G.side;

    // 1. stage the window; non-finite pixels become 0 and are counted.
    int nonfinite = 0;
    for (int idx = tid; idx < G.Wn * G.P; idx += nthr) {
      const int r = idx / G.P, c = idx - r * G.P;
      const int X = wx0 + c, Y = wy0 + r;
      float v = 0.f;
      if (c < G.Wn && X >= 0 && X < W && Y >= 0 && Y < H) {
        v = gimg[(int64_t)Y * W + X];
        if (!isfinite(v)) {
          nonfinite = 1;
          v = 0.f;
        } else {
          v -= c0;
        }
      }
      win[idx] = v;
    }
    const int has_bad = __syncthreads_or(nonfinite);

    int* boxN = reinterpret_cast<int*>(scores);
    if (has_bad) {
      // Exact integer box counts of non-finite pixels (rare path).
      int* colN = reinterpret_cast<int*>(colS);
      for (int c = tid; c < G.Wn; c += nthr) {
        int cnt = 0;
        for (int r = 0; r < G.Wn; ++r) {
          const int X = wx0 + c, Y = wy0 + r;
          int b = 0;
          if (X >= 0 && X < W && Y >= 0 && Y < H) b = !isfinite(gimg[(int64_t)Y * W + X]);
          cnt += b;
          if (r >= G.n1) {
            const int Xo = X, Yo = wy0 + r - G.n1;
            if (Xo >= 0 && Xo < W && Yo >= 0 && Yo < H) cnt -= !isfinite(gimg[(int64_t)Yo * W + Xo]);
          }
          if (r >= G.n1 - 1) colN[(r - G.n1 + 1) * G.Wn + c] = cnt;
        }
      }
      __syncthreads();
      for (int r = tid; r < G.side; r += nthr) {
        int cnt = 0;
        for (int c = 0; c < G.Wn; ++c) {
          cnt += colN[r * G.Wn + c];
          if (c >= G.n1) cnt -= colN[r * G.Wn + c - G.n1];
          if (c >= G.n1 - 1) boxN[r * G.side + c - G.n1 + 1] = cnt;
        }
      }
      __syncthreads();
    }

    // 2. column sums over n1 rows, then row sums over n1 columns (running,
    //    compensated).
    for (int c = tid; c < G.Wn; c += nthr) {
      Kahan s, q;
      for (int r = 0; r < G.n1; ++r) {
        const float v = win[r * G.P + c];
        s.add(v);
        q.add(v * v);
      }
      colS[c] = s.s - s.c;
      colQ[c] = q.s - q.c;
      for (int r = 1; r < G.side; ++r) {
        const float vin = win[(r + G.n1 - 1) * G.P + c];
        const float vout = win[(r - 1) * G.P + c];
        s.add(vin);
        s.add(-vout);
        q.add(vin * vin);
        q.add(-(vout * vout));
        colS[r * G.Wn + c] = s.s - s.c;
        colQ[r * G.Wn + c] = q.s - q.c;
      }
    }
    __syncthreads();
    for (int r = tid; r < G.side; r += nthr) {
      Kahan s, q;
      for (int c = 0; c < G.n1; ++c) {
        s.add(colS[r * G.Wn + c]);
        q.add(colQ[r * G.Wn + c]);
      }
      boxS[r * G.side] = s.s - s.c;
      boxQ[r * G.side] = (has_bad && boxN[r * G.side] > 0) ? -1.f : q.s - q.c;
      for (int c = 1; c < G.side; ++c) {
        s.add(colS[r * G.Wn + c + G.n1 - 1]);
        s.add(-colS[r * G.Wn + c - 1]);
        q.add(colQ[r * G.Wn + c + G.n1 - 1]);
        q.add(-colQ[r * G.Wn + c - 1]);
        boxS[r * G.side + c] = s.s - s.c;
        boxQ[r * G.side + c] = (has_bad && boxN[r * G.side + c] > 0) ? -1.f : q.s - q.c;
      }
    }
    __syncthreads();

    // 3. cross terms, register-blocked along du.
    const float* tm = st.tmpl + P.tmpl_off + (int64_t)(g - P.poi_off) * G.n;
    const double dfd = R->df;
    const float df = (float)dfd;
    const float rn = 1.0f / (float)G.n;
    const float tsum = R->tsum;
    const int items = G.side * G.NB;
    for (int it = tid; it < items; it += nthr) {
      const int r = it % G.side, b = it / G.side;
      float tot[L];
      float cmp[L];
#pragma unroll
      for (int k = 0; k < L; ++k) tot[k] = cmp[k] = 0.f;
      const float* wrow = win + r * G.P + b * L;
      for (int i = 0; i < G.n1; ++i) {
        const float* trow = tm + i * G.n1;
        const float* gw = wrow + i * G.P;
        float w[L];
        float part[L];
#pragma unroll
        for (int k = 0; k < L; ++k) part[k] = 0.f;
#pragma unroll
        for (int k = 0; k < L - 1; ++k) w[k] = gw[k];
        for (int j = 0; j < G.n1p; j += L) {
#pragma unroll
          for (int u = 0; u < L; ++u) {
            w[(u + L - 1) % L] = gw[j + u + L - 1];
            const int jj = j + u;
            float t = trow[jj < G.n1 ? jj : G.n1 - 1];
            t = jj < G.n1 ? t : 0.f;
#pragma unroll
            for (int k = 0; k < L; ++k) part[k] = fmaf(t, w[(u + k) % L], part[k]);
          }
        }
#pragma unroll
        for (int k = 0; k < L; ++k) {
          const float y = part[k] - cmp[k];
          const float tt = tot[k] + y;
          cmp[k] = (tt - tot[k]) - y;
          tot[k] = tt;
        }
      }
#pragma unroll
      for (int k = 0; k < L; ++k) {
        const int c = b * L + k;
        if (c >= G.side) break;
        const int du = cu - G.S + c, dv = cv - G.S + r;
        const bool adm = x0 + du - G.M >= 0 && x0 + du + G.M <= W - 1 && y0 + dv - G.M >= 0 &&
                         y0 + dv + G.M <= H - 1;
        const float sg = boxS[r * G.side + c];
        const float sq = boxQ[r * G.side + c];
        const float var = sq - sg * sg * rn;
        const float sumg2 = sq + 2.f * c0 * sg + (float)G.n * c0 * c0;
        float sc = kNegInf;
        if (adm && sq >= 0.f && var > 1e-6f * sumg2) {
          const float num = (tot[k] - cmp[k]) - sg * rn * tsum;
          sc = num / (df * sqrtf(var));
          if (!isfinite(sc)) sc = kNegInf;
        }
        scores[r * G.side + c] = sc;
      }
    }
    __syncthreads();

    // 4. block maximum.
    const int K = G.side * G.side;
    float m = kNegInf;
    for (int c = tid; c < K; c += nthr) m = fmaxf(m, scores[c]);
    m = wave_max(m);
    if (lane == 0) s_wmax[wid] = m;
    __syncthreads();
    if (wid == 0) {
      float mm = lane < (nthr / kWave) ? s_wmax[lane] : kNegInf;
      mm = wave_max(mm);
      int pick = -1;
      double best = -INFINITY;
      if (mm > kNegInf) {
        // 5. FP64 re-score of the near ties, then the tie rule.
        const float thr = mm - 2e-5f;
        const float* fimg = ref + P.ref_off;
        double cbest = -INFINITY;
        for (int base = 0; base < K; base += kWave) {
          const int c = base + lane;
          const bool hit = c < K && scores[c] >= thr;
          uint64_t bits = __ballot(hit);
          while (bits) {
            const int bit = __builtin_ctzll(bits);
            bits &= bits - 1;
            const int cand = base + bit;
            const int rr = cand / G.side, cc = cand - rr * G.side;
            bool ok;
            const double z = rescore_f64(fimg, gimg, W, x0, y0, x0 + cu - G.S + cc,
                                         y0 + cv - G.S + rr, G.M, R->fbar, dfd, &ok);
            if (ok && z > cbest) cbest = z;
          }
        }
        if (cbest > -INFINITY) {
          for (int base = 0; base < K && pick < 0; base += kWave) {
            const int c = base + lane;
            const bool hit = c < K && scores[c] >= thr;
            uint64_t bits = __ballot(hit);
            while (bits && pick < 0) {
              const int bit = __builtin_ctzll(bits);
              bits &= bits - 1;
              const int cand = base + bit;
              const int rr = cand / G.side, cc = cand - rr * G.side;
              bool ok;
              const double z = rescore_f64(fimg, gimg, W, x0, y0, x0 + cu - G.S + cc,
                                           y0 + cv - G.S + rr, G.M, R->fbar, dfd, &ok);
              if (ok && z >= cbest - 1e-12) {
                pick = cand;
                best = z;
              }
            }
          }
        }
      }
      if (lane == 0) {
        s_pick[0] = pick;
        s_zncc = (float)best;
      }
    }
    __syncthreads();
    if (tid == 0) {
      const int pick = s_pick[0];
      if (pick < 0) {
        uv_out[2 * g] = 0;
        uv_out[2 * g + 1] = 0;
        zncc_out[g] = nanf("");
        status_out[g] = DIC_POI_NO_VALID_CANDIDATE;
      } else {
        const int rr = pick / G.side, cc = pick - rr * G.side;
        uv_out[2 * g] = cu - G.S + cc;
        uv_out[2 * g + 1] = cv - G.S + rr;
        zncc_out[g] = s_zncc;
        status_out[g] = DIC_POI_OK;
      }
    }
    __syncthreads();
  }
}

template <int L>
static hipError_t launch_search_f32_t(const DevState& st, int threads, const float* ref,
                                      const float* def, const int32_t* poi, const int32_t* seed,
                                      int32_t* uv, float* zncc, int32_t* status, int num_cu,
                                      hipStream_t s) {
  const size_t lds = search_lds_bytes(st.maxM, st.maxS, L);
  if (lds > 65536) {
    hipError_t ea = hipFuncSetAttribute(reinterpret_cast<const void*>(&search_f32_kernel<L>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (ea != hipSuccess) return ea;
  }
  int occ = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, search_f32_kernel<L>, threads,
                                                              lds);
  if (e != hipSuccess) return e;
  if (occ < 1) return hipErrorInvalidConfiguration;
  int64_t blocks = (int64_t)occ * num_cu;
  if (blocks > st.N) blocks = st.N;
  hipLaunchKernelGGL(search_f32_kernel<L>, dim3((unsigned)blocks), dim3(threads), lds, s, st, ref,
                     def, poi, seed, uv, zncc, status);
  return hipGetLastError();
}

hipError_t launch_search_f32(const DevState& st, const dic_tuning_t& tu, const float* ref,
                             const float* def, const int32_t* poi, const int32_t* seed,
                             int32_t* uv, float* zncc, int32_t* status, int num_cu,
                             hipStream_t s) {
  if (st.N == 0) return hipSuccess;
  switch (tu.search_block) {
    case 4:
      return launch_search_f32_t<4>(st, tu.search_threads, ref, def, poi, seed, uv, zncc, status,
                                    num_cu, s);
    case 6:
      return launch_search_f32_t<6>(st, tu.search_threads, ref, def, poi, seed, uv, zncc, status,
                                    num_cu, s);
    case 8:
      return launch_search_f32_t<8>(st, tu.search_threads, ref, def, poi, seed, uv, zncc, status,
                                    num_cu, s);
    case 11:
      return launch_search_f32_t<11>(st, tu.search_threads, ref, def, poi, seed, uv, zncc, status,
                                     num_cu, s);
    default:
      return hipErrorInvalidValue;
  }
}

// FP64 plain form: one 64-thread workgroup per POI of one pair; each lane
// walks its candidates and evaluates Eq. (1) two-pass in FP64 straight from
// global memory.  Scores go to LDS for the tie rule.
__global__ void __launch_bounds__(64) search_f64_kernel(DevState st, DevPair P,
                                                        const float* __restrict__ ref,
                                                        const float* __restrict__ def,
                                                        const int32_t* __restrict__ poi,
                                                        const int32_t* __restrict__ seed,
                                                        int32_t* __restrict__ uv_out,
                                                        float* __restrict__ zncc_out,
                                                        int32_t* __restrict__ status_out) {
  extern __shared__ double dscores[];
  const int64_t g = P.poi_off + blockIdx.x;
  const int lane = threadIdx.x;
  const RefRec* R = st.recs + g;
  const int rstat = R->status;
  if (rstat != DIC_POI_OK && rstat != DIC_POI_SINGULAR_HESSIAN) {
    if (lane == 0) {
      uv_out[2 * g] = 0;
      uv_out[2 * g + 1] = 0;
      zncc_out[g] = nanf("");
      status_out[g] = rstat;
    }
    return;
  }
  const int x0 = poi[2 * g], y0 = poi[2 * g + 1];
  const int cu = seed ? seed[2 * g] : 0, cv = seed ? seed[2 * g + 1] : 0;
  const int M = P.M, S = P.S, n1 = 2 * M + 1, n = n1 * n1, side = 2 * S + 1, K = side * side;
  const int W = P.width, H = P.height;
  const float* f = ref + P.ref_off;
  const float* gi = def + P.def_off;
  const double fbar = R->fbar, df = R->df;
  double best = -INFINITY;
  for (int c = lane; c < K; c += kWave) {
    const int r = c / side, cc = c - r * side;
    const int du = cu - S + cc, dv = cv - S + r;
    double sc = -INFINITY;
    if (x0 + du - M >= 0 && x0 + du + M <= W - 1 && y0 + dv - M >= 0 && y0 + dv + M <= H - 1) {
      const float* gs = gi + (int64_t)(y0 + dv - M) * W + (x0 + du - M);
      double s = 0.0;
      for (int a = 0; a < n1; ++a)
        for (int b = 0; b < n1; ++b) s += (double)gs[(int64_t)a * W + b];
      const double gbar = s / (double)n;
      double num = 0.0, q = 0.0, sq = 0.0;
      const float* fs = f + (int64_t)(y0 - M) * W + (x0 - M);
      for (int a = 0; a < n1; ++a)
        for (int b = 0; b < n1; ++b) {
          const double gv = (double)gs[(int64_t)a * W + b];
          const double d = gv - gbar;
          num += ((double)fs[(int64_t)a * W + b] - fbar) * d;
          q += d * d;
          sq += gv * gv;
        }
      if (isfinite(s) && isfinite(sq) && not_flat(q, sq)) {
        sc = num / (df * sqrt(q));
        if (!isfinite(sc)) sc = -INFINITY;
      }
    }
    dscores[c] = sc;
    best = fmax(best, sc);
  }
  best = wave_max(best);
  __syncthreads();
  int pick = 0x7fffffff;
  if (best > -INFINITY)
    for (int c = lane; c < K; c += kWave)
      if (dscores[c] >= best - 1e-12 && c < pick) pick = c;
  pick = wave_min_int(pick);
  if (lane == 0) {
    if (best == -INFINITY) {
      uv_out[2 * g] = 0;
      uv_out[2 * g + 1] = 0;
      zncc_out[g] = nanf("");
      status_out[g] = DIC_POI_NO_VALID_CANDIDATE;
    } else {
      const int r = pick / side, cc = pick - r * side;
      uv_out[2 * g] = cu - S + cc;
      uv_out[2 * g + 1] = cv - S + r;
      zncc_out[g] = (float)dscores[pick];
      status_out[g] = DIC_POI_OK;
    }
  }
}

hipError_t launch_search_f64(const DevState& st, const DevPair* host_pairs, const float* ref,
                             const float* def, const int32_t* poi, const int32_t* seed,
                             int32_t* uv, float* zncc, int32_t* status, hipStream_t s) {
  for (int k = 0; k < st.num_pairs; ++k) {
    const DevPair& P = host_pairs[k];
    if (P.poi_count == 0) continue;
    const size_t lds = sizeof(double) * (size_t)(2 * P.S + 1) * (2 * P.S + 1);
    hipLaunchKernelGGL(search_f64_kernel, dim3((unsigned)P.poi_count), dim3(64), lds, s, st, P,
                       ref, def, poi, seed, uv, zncc, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace dic
