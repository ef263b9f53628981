// Brute-force integer search (Sec. 2.1): Eq. (1) at every candidate of a
// (2S+1)^2 window per POI.
//
// FP32 batched form on the vector ALUs.  One workgroup per POI at a time,
// persistent over a shared work counter.  The deformed window (2S+2M+1
// square, shifted by the mean of its centre subset so sums stay small) is
// staged in LDS once.  Per candidate the window sums sum(g) and sum(g^2) come from the
// FP64 box-sum images, and the cross term sum(t_i g_i) with the mean-free
// template t from a register-blocked loop: a lane owns L horizontally
// adjacent candidates, keeps a sliding window of grey levels in registers and
// reads each template value once from scalar memory, so one LDS read feeds L
// FMAs.  Row partial sums accumulate in FP64.  Each FP32 score s_c comes
// with a bound E_c on its distance from Eq. (1) (search_f32_error); the
// candidates whose s_c + E_c reaches max_k (s_k - E_k) may hold the maximum,
// and one wave re-scores them in FP64 (always at least the winner); the tie
// rule then picks the smallest row-major index within 1e-12 of the FP64
// maximum.
#include "search_common.h"

namespace dic {

namespace {

constexpr int kSearchMaxThreads = 640;  // lanes of the widest search workgroup

struct SearchGeom {
  int M, S, n1, n, side, L, NB, NP, Wn, P;
};

// NP: template row length the cross-term loop runs over (2M+1 rounded up to
// a multiple of L; the stored template is zero beyond 2M+1).
__host__ __device__ __forceinline__ SearchGeom search_geom(int M, int S, int L) {
  SearchGeom G;
  G.M = M;
  G.S = S;
  G.n1 = 2 * M + 1;
  G.n = G.n1 * G.n1;
  G.side = 2 * S + 1;
  G.L = L;
  G.NB = (G.side + L - 1) / L;
  G.NP = (G.n1 + L - 1) / L * L;
  G.Wn = G.side + G.n1 - 1;
  const int pc = G.NB * L + G.NP + L - 2;  // columns the cross-term loop touches
  G.P = pc | 1;
  return G;
}

// Window and the candidate scores.
__host__ __device__ __forceinline__ size_t search_lds_floats(const SearchGeom& G) {
  return (size_t)G.Wn * G.P + (size_t)G.side * G.side;
}

__host__ __device__ __forceinline__ int search_items(int S, int L) {
  const int side = 2 * S + 1;
  return side * ((side + L - 1) / L);
}

// Cross terms sum_i t_i g_i of L horizontally adjacent candidates.  Every
// template row is fully unrolled: its NP values are wave-uniform (scalar
// loads into SGPRs) and the NP + L - 1 window values it needs are read from
// LDS once, so each LDS value feeds up to L FMAs.  Row partial sums (FP32,
// at most 48 terms) are accumulated in FP64, which on this GPU costs no more
// than an FP32 add.  The order of every candidate's sum (row by row, left to
// right, trailing zero-template terms adding exactly 0) does not depend on L.
template <int N>
__device__ __forceinline__ void load_vals(const float* __restrict__ src, float* dst) {
#pragma unroll
  for (int j = 0; j < N; ++j) dst[j] = src[j];
}

// part[k] += sum_{j < N} t[j] * g[j + k] for the L candidates of a lane.
template <int L, int N>
__device__ __forceinline__ void fma_block(const float* t, const float* g, float* part) {
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int k = 0; k < L; ++k) part[k] = fmaf(t[j], g[j + k], part[k]);
}

// One template row against the window row in g, with the next row's loads
// interleaved: the second half of this row's template and, once the first
// half has been used, the first half of the next row's template (SGPRs) and
// the next window row (the other VGPR buffer) are requested before the FMAs
// that do not need them.
template <int L, int NP>
__device__ __forceinline__ void row_pipelined(const float* __restrict__ trow,
                                              const float* __restrict__ tnext,
                                              const float* gnext_src, float* th0, float* th1,
                                              const float* g, float* gnext, double* tot) {
  constexpr int NH = NP / 2;
  load_vals<NH>(trow + NH, th1);
  float part[L];
#pragma unroll
  for (int k = 0; k < L; ++k) part[k] = 0.f;
  fma_block<L, NH>(th0, g, part);
  load_vals<NH>(tnext, th0);
  load_vals<NP + L - 1>(gnext_src, gnext);
  fma_block<L, NH>(th1, g + NH, part);
#pragma unroll
  for (int k = 0; k < L; ++k) tot[k] += (double)part[k];
}

// Cross terms sum_i t_i g_i of L horizontally adjacent candidates.  Every
// template row is fully unrolled: its NP values are wave-uniform (scalar
// loads into SGPRs) and the NP + L - 1 window values it needs are read from
// LDS once, so each LDS value feeds up to L FMAs.  Loads of the next row are
// issued ahead of the FMAs of the current one (see row_pipelined) so their
// latency hides behind them.  Row partial sums (FP32, at most 48 terms)
// accumulate in FP64, which on this GPU costs no more than an FP32 add.  The
// order of every candidate's sum (row by row, left to right, trailing
// zero-template terms adding exactly 0) does not depend on L.
template <int L, int NP>
__device__ __forceinline__ void cross_terms(const float* __restrict__ tm, int tp, int n1,
                                            const float* wrow, int P, double* tot) {
  constexpr int NH = NP / 2;
#pragma unroll
  for (int k = 0; k < L; ++k) tot[k] = 0.0;
  float th0[NH], th1[NH], ga[NP + L - 1], gb[NP + L - 1];
  load_vals<NH>(tm, th0);
  load_vals<NP + L - 1>(wrow, ga);
  for (int i = 0; i < n1; i += 2) {
    // rows past the last are clamped to it: loaded, never used
    const int i1 = min(i + 1, n1 - 1), i2 = min(i + 2, n1 - 1);
    row_pipelined<L, NP>(tm + i * tp, tm + i1 * tp, wrow + i1 * P, th0, th1, ga, gb, tot);
    if (i + 1 >= n1) break;
    row_pipelined<L, NP>(tm + i1 * tp, tm + i2 * tp, wrow + i2 * P, th0, th1, gb, ga, tot);
  }
}

// Bound on |s_c - Eq. (1)| for the FP32 score of a candidate whose
// template rows run over NP terms.  The cross term sum t_i (g_i - c0) is
// formed from FP32 inputs rounded once (t and g - c0) by FP32 multiply-adds
// over at most NP terms per row, the rows added in FP64, so its error is at
// most (NP + 2) 2^-24 sum |t_i| |g_i - c0|, and by Cauchy-Schwarz at most
// (NP + 2) 2^-24 df sqrt(sum (g_i - c0)^2); divided by df sqrt(var), the
// score's scale, that is (NP + 2) 2^-24 R with R = sqrt(sum (g - c0)^2 /
// var), which grows with the window's offset from c0.  The final FP32
// division, square root and conversions add at most 6 2^-24 to a score of
// magnitude at most 1.  Margins: NP + 4 and 8 in place of NP + 2 and 6, and
// 1 %.
__device__ __forceinline__ float search_f32_error(int np, double sgc2, double var) {
  const float R = sqrtf(fmaxf((float)(sgc2 / var), 1.f));
  return 1.01f * fmaf((float)(np + 4), R, 8.f) * 5.9604645e-8f;
}

}  // namespace

size_t search_lds_bytes(int maxM, int maxS, int block) {
  // The layout grows with M and S; the plan's maxima bound every pair.
  return search_lds_floats(search_geom(maxM, maxS, block)) * sizeof(float) +
         kNearCap * (sizeof(int) + sizeof(double)) + 64;
}

int search_threads(int maxS, int block) {
  const int items = search_items(maxS, block);
  return (items + kWave - 1) / kWave * kWave;  // one lane per candidate tile
}

int search_max_threads() { return kSearchMaxThreads; }

template <int L, int NP>
__global__ void __launch_bounds__(kSearchMaxThreads) search_f32_kernel(
    DevState st, const int32_t* __restrict__ work, int64_t count, int ctr,
    const float* __restrict__ tmpl_arena, const double* __restrict__ box,
    const float* __restrict__ ref,
    const float* __restrict__ def, const int32_t* __restrict__ poi,
    const int32_t* __restrict__ seed, int32_t* __restrict__ uv_out, float* __restrict__ zncc_out,
    int32_t* __restrict__ status_out) {
  extern __shared__ float lds[];
  __shared__ int s_item;
  __shared__ float s_wmax[16];
  __shared__ int s_cnt;
  const int tid = threadIdx.x, nthr = blockDim.x, lane = lane_id(), wid = tid / kWave;
  const float kNegInf = -INFINITY;

  for (;;) {
    if (tid == 0) s_item = atomicAdd(&st.counters[ctr], 1);
    __syncthreads();
    const int item = uniform(s_item);
    if (item >= count) break;
    const int g = uniform(work[item]);
    const DevPair P = st.pairs[uniform(st.poi_pair[g])];
    const RefRec* R = st.recs + g;
    const int x0 = uniform(poi[2 * g]), y0 = uniform(poi[2 * g + 1]);
    const int cu = seed ? uniform(seed[2 * g]) : 0;
    const int cv = seed ? uniform(seed[2 * g + 1]) : 0;
    const int rstat = uniform(load_status(R));
    // A singular Hessian does not stop the search; every other record status does.
    if (rstat != DIC_POI_OK && rstat != DIC_POI_SINGULAR_HESSIAN) {
      if (tid == 0) {
        uv_out[2 * g] = 0;
        uv_out[2 * g + 1] = 0;
        zncc_out[g] = nanf("");
        status_out[g] = rstat;
      }
      __syncthreads();
      continue;
    }
    const SearchGeom G = search_geom(P.M, P.S, L);
    const int W = P.width, H = P.height;
    const float* gimg = def + P.def_off;
    const int64_t plane = (int64_t)W * H;
    const double* s1img = box + P.box_off + 2 * plane;
    const double* s2img = s1img + plane;
    const double rnd = 1.0 / (double)G.n;
    // The window is staged as g - c0: c0 is the exact mean of the subset at
    // the window centre (clamped into the image) when that subset is
    // admissible, so the staged values stay within the grey levels the window
    // holds whatever its offset against the reference; else the reference mean.
    float c0 = (float)R->fbar;
    {
      const int64_t oc = (int64_t)min(max(y0 + cv, 0), H - 1) * W + min(max(x0 + cu, 0), W - 1);
      if (s2img[oc] >= 0.0) c0 = (float)(s1img[oc] * rnd);
    }
    const int wx0 = x0 + cu - G.S - G.M, wy0 = y0 + cv - G.S - G.M;

    float* win = lds;
    float* scores = win + G.Wn * G.P;
    int* near_idx = reinterpret_cast<int*>(scores + G.side * G.side);
    double* near_val = reinterpret_cast<double*>(
        (reinterpret_cast<uintptr_t>(near_idx + kNearCap) + 7) & ~uintptr_t(7));
    const int items = G.side * G.NB;
    const bool mine = tid < items;   // one candidate tile per lane
    const int r = mine ? tid % G.side : 0, b = mine ? tid / G.side : 0;

    // 1. stage the window (shifted by the subset mean; non-finite pixels
    //    become 0, the box-sum images mark their candidates invalid).
    //    Thread t walks rows t / P0 + k * (nthr / P0) of columns t % P0 with
    //    P0 = min(P, nthr), no per-element division.
    {
      const int P0 = G.P < nthr ? G.P : nthr;
      const int rstep = nthr / P0;
      const int c1 = tid % P0;
      for (int rr = tid / P0; rr < G.Wn && tid < rstep * P0; rr += rstep) {
        const int Y = wy0 + rr;
        const bool rowin = Y >= 0 && Y < H;
        const float* grow = gimg + (int64_t)Y * W;
        for (int c = c1; c < G.P; c += P0) {
          const int X = wx0 + c;
          float v = 0.f;
          if (c < G.Wn && rowin && X >= 0 && X < W) {
            v = grow[X];
            v = isfinite(v) ? v - c0 : 0.f;
          }
          win[rr * G.P + c] = v;
        }
      }
    }
    __syncthreads();

    // 2. cross terms; window sums from the box-sum images; scores.
    const int tp = P.tmpl_pitch;
    const float* tm = tmpl_arena + P.tmpl_off + (int64_t)(g - P.poi_off) * G.n1 * tp;
    const double dfd = R->df;
    const float df = (float)dfd;
    const double tsum = R->tsum;
    float lmax = kNegInf;   // this lane's largest s_c - E_c
    if (mine) {
      double tot[L];
      const float* wrow = win + r * G.P + b * L;
      cross_terms<L, NP>(tm, tp, G.n1, wrow, G.P, tot);   // G.NP == NP for this group
#pragma unroll
      for (int k = 0; k < L; ++k) {
        const int c = b * L + k;
        if (c >= G.side) break;
        const int du = cu - G.S + c, dv = cv - G.S + r;
        const bool adm = x0 + du - G.M >= 0 && x0 + du + G.M <= W - 1 && y0 + dv - G.M >= 0 &&
                         y0 + dv + G.M <= H - 1;
        float sc = kNegInf;
        if (adm) {
          const int64_t o = (int64_t)(y0 + dv) * W + (x0 + du);
          const double sg = s1img[o], sq = s2img[o];   // exact sums of g and g^2
          const double var = sq - sg * sg * rnd;
          if (sq >= 0.0 && not_flat(var, sq)) {
            // sum t (g - gbar) = sum t (g - c0) - (gbar - c0) sum t
            const double num = tot[k] - (sg * rnd - (double)c0) * tsum;
            sc = (float)num / (df * sqrtf((float)var));
            if (isfinite(sc)) {
              // sum (g - c0)^2 from the exact sums
              const double sgc2 = sq - 2.0 * (double)c0 * sg + (double)G.n * (double)c0 * c0;
              const float e = search_f32_error(NP, sgc2, var);
              lmax = fmaxf(lmax, sc - e);
              sc += e;
            } else {
              sc = kNegInf;
            }
          }
        }
        scores[r * G.side + c] = sc;   // the upper bound s_c + E_c
      }
    }
    if (tid == 0) s_cnt = 0;
    __syncthreads();

    // 4. block maximum of the lower bounds s_c - E_c.
    const int K = G.side * G.side;
    float m = wave_max(lmax);
    if (lane == 0) s_wmax[wid] = m;
    __syncthreads();
    float mm = kNegInf;
    for (int k = 0; k < nthr / kWave; ++k) mm = fmaxf(mm, s_wmax[k]);

    // 5. Candidates whose upper bound reaches the largest lower bound go to
    //    a list (the FP64 maximum is among them); wave 0 re-scores them in
    //    FP64 and applies the tie rule: the smallest row-major index within
    //    1e-12 of the FP64 maximum.  A list that overflows is swept twice in
    //    index order instead.
    if (mm > kNegInf) {
      const float thr = mm;
      for (int c = tid; c < K; c += nthr)
        if (scores[c] >= thr) {
          const int slot = atomicAdd(&s_cnt, 1);
          if (slot < kNearCap) near_idx[slot] = c;
        }
    }
    __syncthreads();
    if (wid == 0) {
      const float* fimg = ref + P.ref_off;
      auto rescore = [&](int cand) -> double {
        const int rr = cand / G.side, cc = cand - rr * G.side;
        const int xg = x0 + cu - G.S + cc, yg = y0 + cv - G.S + rr;
        double z;
        rescore_wave<1>(fimg, gimg, W, x0, y0, &xg, &yg, 1, G.M, R->fbar, dfd, s1img, &z,
                        lane_id());
        return z;
      };
      int pick = -1;
      double best = -INFINITY;
      const int cnt = mm > kNegInf ? uniform(s_cnt) : 0;
      if (cnt <= kNearCap) {
        double cmax = -INFINITY;
        for (int e = 0; e < cnt; ++e) {
          const double z = rescore(uniform(near_idx[e]));
          if (lane == 0) near_val[e] = z;
          cmax = fmax(cmax, z);
        }
        wave_lds_sync();
        if (cmax > -INFINITY)
          for (int e = 0; e < cnt; ++e) {
            const int cand = near_idx[e];
            if (near_val[e] >= cmax - 1e-12 && (pick < 0 || cand < pick)) {
              pick = cand;
              best = near_val[e];
            }
          }
      } else {
        const float thr = mm;
        double cmax = -INFINITY;
        for (int cand = 0; cand < K; ++cand)
          if (scores[cand] >= thr) cmax = fmax(cmax, rescore(cand));
        for (int cand = 0; cand < K && pick < 0 && cmax > -INFINITY; ++cand) {
          if (!(scores[cand] >= thr)) continue;
          const double z = rescore(cand);
          if (z >= cmax - 1e-12) {
            pick = cand;
            best = z;
          }
        }
      }
      if (lane == 0) {
        if (pick < 0) {
          uv_out[2 * g] = 0;
          uv_out[2 * g + 1] = 0;
          zncc_out[g] = nanf("");
          status_out[g] = DIC_POI_NO_VALID_CANDIDATE;
        } else {
          const int rr = pick / G.side, cc = pick - rr * G.side;
          uv_out[2 * g] = cu - G.S + cc;
          uv_out[2 * g + 1] = cv - G.S + rr;
          zncc_out[g] = (float)best;
          status_out[g] = DIC_POI_OK;
        }
      }
    }
    __syncthreads();
  }
}

template <int L, int NP>
static hipError_t launch_search_group(const DevState& st, const SearchGroup& gr, int ctr,
                                      int occ_cap, const float* ref, const float* def,
                                      const int32_t* poi, const int32_t* seed, int32_t* uv,
                                      float* zncc, int32_t* status, int num_cu, hipStream_t s) {
  const int threads = search_threads(st.maxS, L);
  if (threads > kSearchMaxThreads) return hipErrorInvalidConfiguration;
  const size_t lds = search_lds_bytes(st.maxM, st.maxS, L);
  const void* fn = reinterpret_cast<const void*>(&search_f32_kernel<L, NP>);
  if (lds > 65536) {
    hipError_t ea = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (ea != hipSuccess) return ea;
  }
  int occ = 0;
  hipError_t e =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, search_f32_kernel<L, NP>, threads, lds);
  if (e != hipSuccess) return e;
  if (occ < 1) return hipErrorInvalidConfiguration;
  if (occ_cap > 0 && occ > occ_cap) occ = occ_cap;
  int64_t blocks = (int64_t)occ * num_cu;
  if (blocks > gr.count) blocks = gr.count;
  hipLaunchKernelGGL((search_f32_kernel<L, NP>), dim3((unsigned)blocks), dim3(threads), lds, s, st,
                     st.work + gr.begin, gr.count, ctr, st.tmpl, st.box, ref, def, poi, seed, uv,
                     zncc, status);
  return hipGetLastError();
}

template <int L, int NP0, int... NPs>
static hipError_t launch_search_np(const DevState& st, const SearchGroup& gr, int ctr, int occ,
                                   const float* ref, const float* def, const int32_t* poi,
                                   const int32_t* seed, int32_t* uv, float* zncc, int32_t* status,
                                   int num_cu, hipStream_t s) {
  if (gr.np == NP0)
    return launch_search_group<L, NP0>(st, gr, ctr, occ, ref, def, poi, seed, uv, zncc, status,
                                       num_cu, s);
  if constexpr (sizeof...(NPs) > 0)
    return launch_search_np<L, NPs...>(st, gr, ctr, occ, ref, def, poi, seed, uv, zncc, status,
                                       num_cu, s);
  return hipErrorInvalidValue;
}

hipError_t launch_search_f32(const DevState& st, const dic_tuning_t& tu,
                             const SearchGroup* groups, int ngroups, const float* ref,
                             const float* def, const int32_t* poi, const int32_t* seed,
                             int32_t* uv, float* zncc, int32_t* status, int num_cu,
                             hipStream_t s) {
  if (ngroups > kMaxSearchGroups) return hipErrorInvalidValue;
  for (int k = 0; k < ngroups; ++k) {
    const SearchGroup& gr = groups[k];
    if (gr.count == 0) continue;
    hipError_t e = hipErrorInvalidValue;
    if (tu.search_block == 4)
      e = launch_search_np<4, 4, 8, 12, 16, 20, 24, 28, 32, 36, 40, 44>(
          st, gr, kCtrSearch + k, tu.search_occupancy, ref, def, poi, seed, uv, zncc, status,
          num_cu, s);
    else if (tu.search_block == 8)
      e = launch_search_np<8, 8, 16, 24, 32, 40, 48>(st, gr, kCtrSearch + k, tu.search_occupancy,
                                                     ref, def, poi, seed, uv, zncc, status, num_cu,
                                                     s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
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
