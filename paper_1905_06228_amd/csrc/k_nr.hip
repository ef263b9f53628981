// Newton-Raphson sub-pixel refinement (Sec. 2.2: the method whose quantities
// are recomputed at every iteration, where IC-GN precomputes them) on the
// ZNSSD criterion C(p) = sum (fhat_i - ghat_i)^2 with the first-order warp
// applied forward, x_i = x0 + W(p) xi_i, and updated additively.
//
// Per iteration, with g and its gradient (gx, gy) interpolated at the warped
// samples, J_i = [gx, gx dx, gx dy, gy, gy dx, gy dy] and Jc = J - mean(J):
//   dp = Hc^-1 sum Jc_i [ (dg/df)(f_i - fbar) - ZNCC (g_i - gbar) ],
//   Hc = sum Jc_i^T Jc_i,
// which is p <- p - H^-1 dC/dp with dC/dp exact and the Gauss-Newton Hessian
// H = (2/dg^2) Hc; the fixed point is a stationary point of ZNSSD itself.
//
// FP32 batched form: one wave per POI, persistent; the lane's template values
// f_i - fbar and sample offsets stay in registers; the deformed patch is
// staged per wave in LDS as for IC-GN.  One pass per iteration accumulates
// sum g, sum g^2, sum (f - fbar) g, sum J, sum J J^T, sum J (f - fbar) and
// sum J g (42 sums, g taken relative to c0, a deformed grey level at the
// subset's centre) in FP32 per lane and in a fixed
// FP32 tree across lanes; the centring by the means is applied to the sums in
// FP64.  Hessian, solve and update in FP64.
#include "refine_common.h"

namespace dic {

namespace {

// Per-lane partial sums of one iteration (g taken relative to c0), in the
// order they are reduced.
struct NrSums {
  float g, gg, fg;
  float J[6], Jf[6], Jg[6], JJ[21];
};

template <int MAXS, class Smp>
__device__ __forceinline__ void nr_pass(const Smp& smp, int n, const Warp32& w, const float* tv,
                                        const half2v* dxy, NrSums& A) {
  const Slots sl(n);
  A.g = A.gg = A.fg = 0.f;
#pragma unroll
  for (int a = 0; a < 6; ++a) A.J[a] = A.Jf[a] = A.Jg[a] = 0.f;
#pragma unroll
  for (int a = 0; a < 21; ++a) A.JJ[a] = 0.f;
#pragma unroll
  for (int k = 0; k < MAXS; ++k) {
    if (!sl.used(k)) continue;
    const float dx = (float)dxy[k].x, dy = (float)dxy[k].y;
    float v, gx, gy;
    sample_value_grad(smp, warp_x(w, dx, dy), warp_y(w, dx, dy), v, gx, gy);
    // a missing sample of the partial slot has zero template value and
    // offsets; zeroing its value and gradient removes it from every sum
    const float gs = sl.mask(k, v);
    gx = sl.mask(k, gx);
    gy = sl.mask(k, gy);
    const float t = tv[k];
    const float J[6] = {gx, gx * dx, gx * dy, gy, gy * dx, gy * dy};
    A.g += gs;
    A.gg = fmaf(gs, gs, A.gg);
    A.fg = fmaf(t, gs, A.fg);
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      A.J[a] += J[a];
      A.Jf[a] = fmaf(J[a], t, A.Jf[a]);
      A.Jg[a] = fmaf(J[a], gs, A.Jg[a]);
#pragma unroll
      for (int b = 0; b <= a; ++b) A.JJ[tri(a, b)] = fmaf(J[a], J[b], A.JJ[tri(a, b)]);
    }
  }
}

}  // namespace

template <int MAXS, int IM>
__global__ void __launch_bounds__(512) nr_f32_kernel(
    DevState st, int slack, const float* __restrict__ def, const int32_t* __restrict__ poi,
    const int32_t* __restrict__ uv_init, const int32_t* __restrict__ status_in,
    const double* __restrict__ p_init, double* __restrict__ p_out, float* __restrict__ zncc_out,
    int32_t* __restrict__ iters_out, int32_t* __restrict__ status_out) {
  constexpr int PP = refine_patch_pitch(MAXS);
  constexpr int NT = interp_taps(IM);
  extern __shared__ float lds[];
  const int wid = threadIdx.x / kWave;
  const int pside = icgn_patch_side(st.maxM, slack);
  LdsPatch<PP> patch;
  patch.buf = lds + (size_t)wid * pside * PP;
  patch.side = pside;

  for (;;) {
    const int item = wave_next_item(&st.counters[kCtrIcgn]);
    if (item >= st.N) break;
    const int g = uniform(st.work[item]);
    const DevPair P = st.pairs[uniform(st.poi_pair[g])];
    const RefRec* R = st.recs + g;
    const int x0 = uniform(poi[2 * g]), y0 = uniform(poi[2 * g + 1]);
    double p[6] = {(double)uv_init[2 * g], 0.0, 0.0, (double)uv_init[2 * g + 1], 0.0, 0.0};
    if (p_init) {
      p[1] = p_init[6 * g + 1];
      p[2] = p_init[6 * g + 2];
      p[4] = p_init[6 * g + 4];
      p[5] = p_init[6 * g + 5];
    }
    int status = uniform(R->status);
    // the reference-side Hessian is IC-GN's; Newton-Raphson forms its own
    if (status == DIC_POI_SINGULAR_HESSIAN) status = DIC_POI_OK;
    if (status_in && status == DIC_POI_OK) status = uniform(status_in[g]);
    int it = 0;
    float zn = nanf("");
    if (status == DIC_POI_OK) {
      const int M = P.M, n1 = 2 * M + 1, n = n1 * n1, W = P.width, H = P.height;
      // the taps: the image's pixels, or its cubic B-spline coefficients
      const float* gimg =
          IM == kInterpBSpline ? st.lut + 4 * P.lut_off : def + P.def_off;
      const float4* glut = reinterpret_cast<const float4*>(st.lut) + P.lut_off;
      const int tp = P.tmpl_pitch;
      const float* tm = st.tmpl + P.tmpl_off + (int64_t)(g - P.poi_off) * n1 * tp;
      float tv[MAXS];
      half2v dxy[MAXS];
      load_slots<MAXS>(M, n, tm, nullptr, tp, dxy, tv, nullptr);
      const float c0 = deformed_centre(gimg, W, H, p, x0, y0);
      const double df = R->df, tsum = (double)R->tsum;
      const double nn = (double)n;
      patch.x0 = patch.y0 = INT_MIN;
      status = DIC_POI_NOT_CONVERGED;
      while (it < st.max_iters) {
        ++it;
        const Warp32 w = make_warp32(p, x0, y0);
        int xl, xh, yl, yh;
        tap_box<NT>(w, M, xl, xh, yl, yh);
        if (xl < 0 || xh > W - 1 || yl < 0 || yh > H - 1) {
          status = DIC_POI_OUT_OF_BOUNDS;
          break;
        }
        NrSums A;
        if constexpr (IM == kInterpBicubicLut)
          nr_pass<MAXS>(LutSampler{glut, W, H, w.bx, w.by, c0}, n, w, tv, dxy, A);
        else if (patch.ensure(gimg, W, H, xl, xh, yl, yh, c0))
          nr_pass<MAXS>(patch.template sampler<IM>(w.bx, w.by), n, w, tv, dxy, A);
        else
          nr_pass<MAXS>(ImageSampler<IM>{gimg, W, H, w.bx, w.by, c0}, n, w, tv, dxy, A);
        // all 42 sums in one reduction, in struct order
        static_assert(sizeof(NrSums) == 42 * sizeof(float), "NrSums layout");
        double S[42];
        wave_sums_f32<42>(&A.g, S);
        const double sg = S[0], sgg = S[1], sfg = S[2];
        const double* sJ = S + 3;
        const double* sJf = S + 9;
        const double* sJg = S + 15;
        double hc[21];
#pragma unroll
        for (int a = 0; a < 21; ++a) hc[a] = S[21 + a];
        bool fin = isfinite(sg) && isfinite(sgg);
#pragma unroll
        for (int a = 0; a < 6; ++a) fin = fin && isfinite(sJ[a]);
        if (!fin) {
          status = DIC_POI_NAN_INPUT;
          break;
        }
        const double ms = sg / nn;
        const double var = sgg - sg * ms;
        const double sumg2 = sgg + 2.0 * (double)c0 * sg + nn * (double)c0 * (double)c0;
        if (!not_flat(var, sumg2)) {
          status = DIC_POI_ZERO_VARIANCE;
          break;
        }
        const double dg = sqrt(var);
        const double zc = (sfg - ms * tsum) / (df * dg);
        double rhs[6];
#pragma unroll
        for (int a = 0; a < 6; ++a) {
          // sum Jc (f - fbar) = sum J t - mean(J) sum t;  sum Jc (g - gbar) = sum J g - gbar sum J
          rhs[a] = dg / df * (sJf[a] - sJ[a] / nn * tsum) - zc * (sJg[a] - ms * sJ[a]);
#pragma unroll
          for (int b = 0; b <= a; ++b) hc[tri(a, b)] -= sJ[a] * sJ[b] / nn;
        }
        double L[21], rd[6], dp[6];
        if (!cholesky6(hc, L, rd)) {
          status = DIC_POI_SINGULAR_HESSIAN;
          break;
        }
        cholesky6_solve(L, rd, rhs, dp);
#pragma unroll
        for (int a = 0; a < 6; ++a) p[a] += dp[a];
        if (update_norm(dp, M) < st.conv_tol) {
          status = DIC_POI_OK;
          break;
        }
      }
      if (status == DIC_POI_OK || status == DIC_POI_NOT_CONVERGED) {
        const Warp32 w = make_warp32(p, x0, y0);
        int xl, xh, yl, yh;
        tap_box<NT>(w, M, xl, xh, yl, yh);
        if (xl < 0 || xh > W - 1 || yl < 0 || yh > H - 1) {
          status = DIC_POI_OUT_OF_BOUNDS;
        } else {
          const auto tval = [&](int k, float, float) { return tv[k]; };
          float K[3];
          if constexpr (IM == kInterpBicubicLut)
            final_pass<MAXS>(LutSampler{glut, W, H, w.bx, w.by, c0}, n, w, dxy, tval, K);
          else if (patch.ensure(gimg, W, H, xl, xh, yl, yh, c0))
            final_pass<MAXS>(patch.template sampler<IM>(w.bx, w.by), n, w, dxy, tval, K);
          else
            final_pass<MAXS>(ImageSampler<IM>{gimg, W, H, w.bx, w.by, c0}, n, w, dxy,
                             tval, K);
          double S[3];
          wave_sums_f32<3>(K, S);
          if (!isfinite(S[0]) || !isfinite(S[1])) {
            status = DIC_POI_NAN_INPUT;
          } else {
            const double ms = S[0] / nn;
            const double var = S[1] - S[0] * ms;
            const double sumg2 = S[1] + 2.0 * (double)c0 * S[0] + nn * (double)c0 * (double)c0;
            if (!not_flat(var, sumg2))
              status = DIC_POI_ZERO_VARIANCE;
            else
              zn = (float)((S[2] - ms * tsum) / (df * sqrt(var)));
          }
        }
      }
    }
    // every lane stores the same (wave-uniform) results: no lane-dependent
    // branch at the end of the persistent loop either
#pragma unroll
    for (int a = 0; a < 6; ++a) p_out[6 * g + a] = p[a];
    zncc_out[g] = (status == DIC_POI_OK || status == DIC_POI_NOT_CONVERGED) ? zn : nanf("");
    iters_out[g] = it;
    status_out[g] = status;
  }
}

template <int MAXS, int IM>
static hipError_t launch_nr_f32_t(const DevState& st, const dic_tuning_t& tu, const float* def,
                                  const int32_t* poi, const int32_t* uv_init,
                                  const int32_t* status_in, const double* p_init, double* p_out,
                                  float* zncc, int32_t* iters, int32_t* status, int num_cu,
                                  hipStream_t s) {
  const int threads = tu.icgn_waves * kWave;
  // the table form reads no LDS patch
  const size_t lds = IM == kInterpBicubicLut
                         ? 0
                         : refine_lds_bytes(refine_patch_pitch(MAXS),
                                            icgn_patch_side(st.maxM, tu.icgn_slack), tu.icgn_waves);
  if (lds > 65536) {
    hipError_t ea = hipFuncSetAttribute(reinterpret_cast<const void*>(&nr_f32_kernel<MAXS, IM>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (ea != hipSuccess) return ea;
  }
  int occ = 0;
  hipError_t e =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, nr_f32_kernel<MAXS, IM>, threads, lds);
  if (e != hipSuccess) return e;
  if (occ < 1) return hipErrorInvalidConfiguration;
  int64_t blocks = (int64_t)occ * num_cu;
  const int64_t need = (st.N + tu.icgn_waves - 1) / tu.icgn_waves;
  if (blocks > need) blocks = need;
  hipLaunchKernelGGL((nr_f32_kernel<MAXS, IM>), dim3((unsigned)blocks), dim3(threads), lds, s, st,
                     tu.icgn_slack, def, poi, uv_init, status_in, p_init, p_out, zncc, iters,
                     status);
  return hipGetLastError();
}

hipError_t launch_nr_f32(const DevState& st, const dic_tuning_t& tu, const float* def,
                         const int32_t* poi, const int32_t* uv_init, const int32_t* status_in,
                         const double* p_init, double* p_out, float* zncc, int32_t* iters,
                         int32_t* status, int num_cu, hipStream_t s, int interp) {
  if (st.N == 0) return hipSuccess;
  const int n = (2 * st.maxM + 1) * (2 * st.maxM + 1);
  const int need = (n + kWave - 1) / kWave;
#define DIC_NR_CASE(S_)                                                                       \
  if (need <= S_) {                                                                           \
    if (interp == kInterpBilinear)                                                            \
      return launch_nr_f32_t<S_, kInterpBilinear>(st, tu, def, poi, uv_init, status_in, p_init,  \
                                                  p_out, zncc, iters, status, num_cu, s);      \
    if (interp == kInterpBSpline)                                                             \
      return launch_nr_f32_t<S_, kInterpBSpline>(st, tu, def, poi, uv_init, status_in,        \
                                                  p_init, p_out, zncc, iters, status, num_cu, s);\
    if (interp == kInterpBicubicLut)                                                          \
      return launch_nr_f32_t<S_, kInterpBicubicLut>(st, tu, def, poi, uv_init, status_in,     \
                                                    p_init, p_out, zncc, iters, status, num_cu, \
                                                    s);                                       \
    return launch_nr_f32_t<S_, kInterpBicubic>(st, tu, def, poi, uv_init, status_in, p_init,   \
                                               p_out, zncc, iters, status, num_cu, s);         \
  }
  DIC_NR_CASE(4)
  DIC_NR_CASE(8)
  DIC_NR_CASE(12)
  DIC_NR_CASE(16)
  DIC_NR_CASE(20)
  DIC_NR_CASE(28)
#undef DIC_NR_CASE
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// FP64 plain form: one 64-thread workgroup per POI of one pair, FP64
// throughout, taps read from global memory, two-pass statistics (means of g
// and of J first, then the centred sums).
// ---------------------------------------------------------------------------

template <int MAXS>
__global__ void __launch_bounds__(64) nr_f64_kernel(
    DevState st, DevPair P, const float* __restrict__ ref, const float* __restrict__ def,
    const int32_t* __restrict__ poi, const int32_t* __restrict__ uv_init,
    const int32_t* __restrict__ status_in, const double* __restrict__ p_init,
    double* __restrict__ p_out, float* __restrict__ zncc_out, int32_t* __restrict__ iters_out,
    int32_t* __restrict__ status_out) {
  const int64_t g = P.poi_off + blockIdx.x;
  const int lane = threadIdx.x;
  const RefRec* R = st.recs + g;
  const int x0 = poi[2 * g], y0 = poi[2 * g + 1];
  double p[6] = {(double)uv_init[2 * g], 0.0, 0.0, (double)uv_init[2 * g + 1], 0.0, 0.0};
  if (p_init) {
    p[1] = p_init[6 * g + 1];
    p[2] = p_init[6 * g + 2];
    p[4] = p_init[6 * g + 4];
    p[5] = p_init[6 * g + 5];
  }
  int status = R->status;
  if (status == DIC_POI_SINGULAR_HESSIAN) status = DIC_POI_OK;
  if (status_in && status == DIC_POI_OK) status = status_in[g];
  int it = 0;
  double zn = nan("");
  const int M = P.M, n1 = 2 * M + 1, n = n1 * n1, W = P.width, H = P.height;
  const float* f = ref + P.ref_off;
  const float* gi = def + P.def_off;
  const double fbar = R->fbar, df = R->df;
  double gl[MAXS], gxl[MAXS], gyl[MAXS];

  // Interpolates value and gradient of every sample at p; returns 1 if any
  // tap leaves the image, 2 if a value is non-finite, 3 if the subset is
  // flat, else 0 with its mean and norm.
  auto sample = [&](double* mean, double* dg) -> int {
    int oob = 0;
#pragma unroll
    for (int k = 0; k < MAXS; ++k) {
      const int s = lane + kWave * k;
      if (s >= n) continue;
      const double dx = (double)(s % n1 - M), dy = (double)(s / n1 - M);
      const double xs = x0 + (1.0 + p[1]) * dx + p[2] * dy + p[0];
      const double ys = y0 + p[4] * dx + (1.0 + p[5]) * dy + p[3];
      const double fx = floor(xs), fy = floor(ys);
      if (fx < 1.0 || fx + 2.0 > W - 1 || fy < 1.0 || fy + 2.0 > H - 1) oob = 1;
    }
    if (wave_or_int(oob)) return 1;
    double s1 = 0.0;
    int bad = 0;
#pragma unroll
    for (int k = 0; k < MAXS; ++k) {
      const int s = lane + kWave * k;
      gl[k] = gxl[k] = gyl[k] = 0.0;
      if (s >= n) continue;
      const double dx = (double)(s % n1 - M), dy = (double)(s / n1 - M);
      const double xs = x0 + (1.0 + p[1]) * dx + p[2] * dy + p[0];
      const double ys = y0 + p[4] * dx + (1.0 + p[5]) * dy + p[3];
      const double fx = floor(xs), fy = floor(ys);
      double wx[4], wy[4], dwx[4], dwy[4];
      cubic_weights(xs - fx, wx);
      cubic_weights(ys - fy, wy);
      cubic_dweights(xs - fx, dwx);
      cubic_dweights(ys - fy, dwy);
      const float* q = gi + (int64_t)((int)fy - 1) * W + ((int)fx - 1);
      double v = 0.0, vx = 0.0, vy = 0.0;
      for (int l = 0; l < 4; ++l)
        for (int c = 0; c < 4; ++c) {
          const double t = (double)q[(int64_t)l * W + c];
          v += wy[l] * wx[c] * t;
          vx += wy[l] * dwx[c] * t;
          vy += dwy[l] * wx[c] * t;
        }
      gl[k] = v;
      gxl[k] = vx;
      gyl[k] = vy;
      bad |= !(isfinite(v) && isfinite(vx) && isfinite(vy));
      s1 += v;
    }
    if (wave_or_int(bad)) return 2;
    s1 = wave_sum(s1);
    *mean = s1 / (double)n;
    double q2 = 0.0, sq = 0.0;
#pragma unroll
    for (int k = 0; k < MAXS; ++k) {
      const int s = lane + kWave * k;
      if (s >= n) continue;
      const double d = gl[k] - *mean;
      q2 += d * d;
      sq += gl[k] * gl[k];
    }
    q2 = wave_sum(q2);
    sq = wave_sum(sq);
    if (!not_flat(q2, sq)) return 3;
    *dg = sqrt(q2);
    return 0;
  };

  if (status == DIC_POI_OK) {
    status = DIC_POI_NOT_CONVERGED;
    while (it < st.max_iters) {
      ++it;
      double gbar, dg;
      const int r = sample(&gbar, &dg);
      if (r) {
        status = r == 1 ? DIC_POI_OUT_OF_BOUNDS : r == 2 ? DIC_POI_NAN_INPUT : DIC_POI_ZERO_VARIANCE;
        break;
      }
      // pass 1: mean of J and the coefficient
      double jm[6] = {0, 0, 0, 0, 0, 0}, num = 0.0;
#pragma unroll
      for (int k = 0; k < MAXS; ++k) {
        const int s = lane + kWave * k;
        if (s >= n) continue;
        const int dxi = s % n1 - M, dyi = s / n1 - M;
        const double dx = dxi, dy = dyi;
        const double J[6] = {gxl[k], gxl[k] * dx, gxl[k] * dy, gyl[k], gyl[k] * dx, gyl[k] * dy};
        for (int a = 0; a < 6; ++a) jm[a] += J[a];
        num += ((double)f[(int64_t)(y0 + dyi) * W + (x0 + dxi)] - fbar) * (gl[k] - gbar);
      }
      for (int a = 0; a < 6; ++a) jm[a] = wave_sum(jm[a]) / (double)n;
      const double zc = wave_sum(num) / (df * dg);
      // pass 2: centred Hessian and right-hand side
      double hc[21] = {0}, rhs[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int k = 0; k < MAXS; ++k) {
        const int s = lane + kWave * k;
        if (s >= n) continue;
        const int dxi = s % n1 - M, dyi = s / n1 - M;
        const double dx = dxi, dy = dyi;
        const double Jc[6] = {gxl[k] - jm[0], gxl[k] * dx - jm[1], gxl[k] * dy - jm[2],
                              gyl[k] - jm[3], gyl[k] * dx - jm[4], gyl[k] * dy - jm[5]};
        const double e = dg / df * ((double)f[(int64_t)(y0 + dyi) * W + (x0 + dxi)] - fbar) -
                         zc * (gl[k] - gbar);
        for (int a = 0; a < 6; ++a) {
          rhs[a] += Jc[a] * e;
          for (int b = 0; b <= a; ++b) hc[tri(a, b)] += Jc[a] * Jc[b];
        }
      }
      for (int a = 0; a < 6; ++a) rhs[a] = wave_sum(rhs[a]);
      for (int a = 0; a < 21; ++a) hc[a] = wave_sum(hc[a]);
      double L[21], rd[6], dp[6];
      if (!cholesky6(hc, L, rd)) {
        status = DIC_POI_SINGULAR_HESSIAN;
        break;
      }
      cholesky6_solve(L, rd, rhs, dp);
      for (int a = 0; a < 6; ++a) p[a] += dp[a];
      if (update_norm(dp, M) < st.conv_tol) {
        status = DIC_POI_OK;
        break;
      }
    }
    if (status == DIC_POI_OK || status == DIC_POI_NOT_CONVERGED) {
      double gbar, dg;
      const int r = sample(&gbar, &dg);
      if (r) {
        status = r == 1 ? DIC_POI_OUT_OF_BOUNDS : r == 2 ? DIC_POI_NAN_INPUT : DIC_POI_ZERO_VARIANCE;
      } else {
        double num = 0.0;
#pragma unroll
        for (int k = 0; k < MAXS; ++k) {
          const int s = lane + kWave * k;
          if (s >= n) continue;
          const int64_t idx = (int64_t)(y0 + s / n1 - M) * W + (x0 + s % n1 - M);
          num += ((double)f[idx] - fbar) * (gl[k] - gbar);
        }
        zn = wave_sum(num) / (df * dg);
      }
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int a = 0; a < 6; ++a) p_out[6 * g + a] = p[a];
    zncc_out[g] = (status == DIC_POI_OK || status == DIC_POI_NOT_CONVERGED) ? (float)zn : nanf("");
    iters_out[g] = it;
    status_out[g] = status;
  }
}

hipError_t launch_nr_f64(const DevState& st, const DevPair* host_pairs, const float* ref,
                         const float* def, const int32_t* poi, const int32_t* uv_init,
                         const int32_t* status_in, const double* p_init, double* p_out,
                         float* zncc, int32_t* iters, int32_t* status, hipStream_t s) {
  for (int k = 0; k < st.num_pairs; ++k) {
    const DevPair& P = host_pairs[k];
    if (P.poi_count == 0) continue;
    const int need = ((2 * P.M + 1) * (2 * P.M + 1) + kWave - 1) / kWave;
    const dim3 grid((unsigned)P.poi_count), block(64);
#define DIC_NR64_CASE(S_)                                                                     \
  if (need <= S_) {                                                                           \
    hipLaunchKernelGGL(nr_f64_kernel<S_>, grid, block, 0, s, st, P, ref, def, poi, uv_init,   \
                       status_in, p_init, p_out, zncc, iters, status);                        \
    hipError_t e = hipGetLastError();                                                         \
    if (e != hipSuccess) return e;                                                            \
    continue;                                                                                 \
  }
    DIC_NR64_CASE(4)
    DIC_NR64_CASE(8)
    DIC_NR64_CASE(12)
    DIC_NR64_CASE(16)
    DIC_NR64_CASE(20)
    DIC_NR64_CASE(28)
#undef DIC_NR64_CASE
    return hipErrorInvalidValue;
  }
  return hipSuccess;
}

}  // namespace dic
