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
    // slots every subset of the class fills run without a test
    if (k >= refine_min_slots(MAXS) && !sl.used(k)) continue;
    const float dx = (float)dxy[k].x, dy = (float)dxy[k].y;
    float v, gx, gy;
    sample_value_grad(smp, warp_x(w, dx, dy), warp_y(w, dx, dy), v, gx, gy);
    // a missing sample of the partial slot has zero template value and
    // offsets; zeroing its value and gradient removes it from every sum
    const bool may_miss = k + 1 >= refine_min_slots(MAXS);   // the partial slot or later
    const float gs = may_miss ? sl.mask(k, v) : v;
    if (may_miss) {
      gx = sl.mask(k, gx);
      gy = sl.mask(k, gy);
    }
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

// nr_pass in the two-rows layout of IC-GN (subsets of 29 and 31 columns):
// with the lane's column offset dx fixed and the row offset dy = 2k + (l /
// 32 - M), every sum over J = (gx, gx dx, gx dy, gy, gy dx, gy dy) is a
// lane constant times one of 24 sums over gx, gy and their products weighted
// by 1, 2k and (2k)^2; they are expanded into the 42 sums of nr_pass per
// lane before the cross-lane reduction.  `tv` holds the lane's template
// values in the same layout (slot M: the last row, zero in the upper half).
template <int MAXS, class Smp>
__device__ __forceinline__ void nr_pass_r2(const Smp& smp, int M, const R2Lane& L, const Warp32& w,
                                           const float* tv, float tvp, NrSums& A) {
  const int Mu = __builtin_amdgcn_readfirstlane(M);
  const float bx = fmaf(w.ax, L.dx, fmaf(w.uy, L.hm, w.uf));
  const float by = fmaf(w.vx, L.dx, fmaf(w.ay, L.hm, w.vf));
  float sg = 0.f, sgg = 0.f, sfg = 0.f;
  float ax0 = 0.f, ax1 = 0.f, ay0 = 0.f, ay1 = 0.f;       // gx, gy (x 1, 2k)
  float fx0 = 0.f, fx1 = 0.f, fy0 = 0.f, fy1 = 0.f;       // gx t, gy t
  float gx0 = 0.f, gx1 = 0.f, gy0 = 0.f, gy1 = 0.f;       // gx g, gy g
  float xx0 = 0.f, xx1 = 0.f, xx2 = 0.f;                  // gx^2 (x 1, 2k, 4k^2)
  float xy0 = 0.f, xy1 = 0.f, xy2 = 0.f;                  // gx gy
  float yy0 = 0.f, yy1 = 0.f, yy2 = 0.f;                  // gy^2
  const auto add = [&](float gs, float gx, float gy, float t, float dk) {
    const float dk2 = dk * dk;
    sg += gs;
    sgg = fmaf(gs, gs, sgg);
    sfg = fmaf(t, gs, sfg);
    ax0 += gx;
    ax1 = fmaf(gx, dk, ax1);
    ay0 += gy;
    ay1 = fmaf(gy, dk, ay1);
    const float xt = gx * t, yt = gy * t, xg = gx * gs, yg = gy * gs;
    fx0 += xt;
    fx1 = fmaf(xt, dk, fx1);
    fy0 += yt;
    fy1 = fmaf(yt, dk, fy1);
    gx0 += xg;
    gx1 = fmaf(xg, dk, gx1);
    gy0 += yg;
    gy1 = fmaf(yg, dk, gy1);
    const float qx = gx * gx, qxy = gx * gy, qy = gy * gy;
    xx0 += qx;
    xx1 = fmaf(qx, dk, xx1);
    xx2 = fmaf(qx, dk2, xx2);
    xy0 += qxy;
    xy1 = fmaf(qxy, dk, xy1);
    xy2 = fmaf(qxy, dk2, xy2);
    yy0 += qy;
    yy1 = fmaf(qy, dk, yy1);
    yy2 = fmaf(qy, dk2, yy2);
  };
#pragma unroll
  for (int k = 0; k < MAXS - 1; ++k) {
    if (k >= kR2MinM && k >= Mu) continue;   // slots below kR2MinM always hold samples
    const float dk = (float)(2 * k);
    float v, gx, gy;
    sample_value_grad(smp, fmaf(w.uy, dk, bx), fmaf(w.ay, dk, by), v, gx, gy);
    add(v, gx, gy, tv[k], dk);
  }
  {
    // the last row, read by both half-waves at the lower one's positions and
    // counted once (the upper half's value and gradient are zeroed)
    const float dm = (float)Mu;
    float v, gx, gy;
    sample_value_grad(smp, fmaf(w.ax, L.dx, fmaf(w.uy, dm, w.uf)),
                      fmaf(w.vx, L.dx, fmaf(w.ay, dm, w.vf)), v, gx, gy);
    const bool on = !L.upper;
    add(on ? v : 0.f, on ? gx : 0.f, on ? gy : 0.f, tvp, 2.f * dm);
  }
  // columns outside the subset: their value sums are cleared (their
  // template values are zero, and gradients below are zeroed with them)
  const float cm = L.colok ? 1.f : 0.f;
  sg *= cm;
  sgg *= cm;
  ax0 *= cm; ax1 *= cm; ay0 *= cm; ay1 *= cm;
  gx0 *= cm; gx1 *= cm; gy0 *= cm; gy1 *= cm;
  xx0 *= cm; xx1 *= cm; xx2 *= cm;
  xy0 *= cm; xy1 *= cm; xy2 *= cm;
  yy0 *= cm; yy1 *= cm; yy2 *= cm;
  // sums weighted by dy = 2k + hm and dy^2
  const float h = L.hm, h2 = L.hm * L.hm, d = L.dx, d2 = L.dx * L.dx;
  const float AX1 = fmaf(h, ax0, ax1), AY1 = fmaf(h, ay0, ay1);
  const float FX1 = fmaf(h, fx0, fx1), FY1 = fmaf(h, fy0, fy1);
  const float GX1 = fmaf(h, gx0, gx1), GY1 = fmaf(h, gy0, gy1);
  const float X1 = fmaf(h, xx0, xx1), X2 = fmaf(h2, xx0, fmaf(2.f * h, xx1, xx2));
  const float XY1 = fmaf(h, xy0, xy1), XY2 = fmaf(h2, xy0, fmaf(2.f * h, xy1, xy2));
  const float Y1 = fmaf(h, yy0, yy1), Y2 = fmaf(h2, yy0, fmaf(2.f * h, yy1, yy2));
  A.g = sg;
  A.gg = sgg;
  A.fg = sfg;
  const float J[6] = {ax0, d * ax0, AX1, ay0, d * ay0, AY1};
  const float Jf[6] = {fx0, d * fx0, FX1, fy0, d * fy0, FY1};
  const float Jg[6] = {gx0, d * gx0, GX1, gy0, d * gy0, GY1};
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    A.J[a] = J[a];
    A.Jf[a] = Jf[a];
    A.Jg[a] = Jg[a];
  }
  // J J^T, packed rows (a >= b)
  const float JJ[21] = {xx0,                                          // (0,0)
                        d * xx0, d2 * xx0,                            // (1,0) (1,1)
                        X1, d * X1, X2,                               // (2,0..2)
                        xy0, d * xy0, XY1, yy0,                       // (3,0..3)
                        d * xy0, d2 * xy0, d * XY1, d * yy0, d2 * yy0,  // (4,0..4)
                        XY1, d * XY1, XY2, Y1, d * Y1, Y2};           // (5,0..5)
#pragma unroll
  for (int a = 0; a < 21; ++a) A.JJ[a] = JJ[a];
}

}  // namespace

// The two-rows kernels run at three waves per SIMD.
template <int MAXS, int IM, bool R2>
__global__ void __launch_bounds__(512)
__attribute__((amdgpu_waves_per_eu(R2 ? 3 : 1))) nr_f32_kernel(
    DevState st, const int32_t* __restrict__ work, int64_t count, int ctr, int gmaxM, int slack,
    const float* __restrict__ ref, const float* __restrict__ def, const int32_t* __restrict__ poi,
    const int32_t* __restrict__ uv_init, const int32_t* __restrict__ status_in,
    const double* __restrict__ p_init, double* __restrict__ p_out, float* __restrict__ zncc_out,
    int32_t* __restrict__ iters_out, int32_t* __restrict__ status_out) {
  constexpr int PP = R2 ? kR2Pitch : refine_patch_pitch(MAXS);
  constexpr int NT = interp_taps(IM);
  extern __shared__ float lds[];
  const int wid = threadIdx.x / kWave;
  const int pside = icgn_patch_side(gmaxM, slack);
  LdsPatch<PP> patch;
  patch.buf = lds + (size_t)wid * pside * PP;
  patch.side = pside;

  for (;;) {
    const int item = wave_next_item(&st.counters[ctr]);
    if (item >= count) break;
    const int g = uniform(work[item]);
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
      // the template values f - fbar of the lane's samples (rounded as the
      // record's tsum counts them), zero for missing samples
      const float* fsub = ref + P.ref_off + (int64_t)(y0 - M) * W + (x0 - M);
      const float fb = (float)R->fbar;
      float tv[MAXS], tvp = 0.f, unused = 0.f;
      half2v dxy[R2 ? 1 : MAXS];
      R2Lane L2{};
      if constexpr (R2) {
        L2 = r2_lane(M);
        load_slots_r2<MAXS>(M, L2, fsub, nullptr, W, tv, nullptr, tvp, unused);
#pragma unroll
        for (int k = 0; k < MAXS - 1; ++k) tv[k] = (k < M && L2.colok) ? tv[k] - fb : 0.f;
        tvp = (L2.colok && !L2.upper) ? tvp - fb : 0.f;
      } else {
        load_slots<MAXS, false>(M, n, fsub, nullptr, W, dxy, tv, nullptr);
#pragma unroll
        for (int k = 0; k < MAXS; ++k) tv[k] = (lane_id() + kWave * k < n) ? tv[k] - fb : 0.f;
      }
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
        const auto pass = [&](const auto& smp) {
          if constexpr (R2)
            nr_pass_r2<MAXS>(smp, M, L2, w, tv, tvp, A);
          else
            nr_pass<MAXS>(smp, n, w, tv, dxy, A);
        };
        if constexpr (IM == kInterpBicubicLut)
          pass(LutSampler{glut, W, H, w.bx, w.by, c0});
        else if (patch.ensure(gimg, W, H, xl, xh, yl, yh, c0))
          pass(patch.template sampler<IM>(w.bx, w.by));
        else
          pass(ImageSampler<IM>{gimg, W, H, w.bx, w.by, c0});
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
          float K[3];
          const auto fpass = [&](const auto& smp) {
            if constexpr (R2) {
              // the template value at offset (dx, dy) from the subset centre
              const float* fc = fsub + (int64_t)M * W + M;
              const auto tval = [&](int, float dx, float dy) {
                return fc[(int)dy * W + (int)dx] - fb;
              };
              final_pass_r2<MAXS>(smp, M, L2, w, tval, K);
            } else {
              const auto tval = [&](int k, float, float) { return tv[k]; };
              final_pass<MAXS>(smp, n, w, OffsetsKept{dxy}, tval, K);
            }
          };
          if constexpr (IM == kInterpBicubicLut)
            fpass(LutSampler{glut, W, H, w.bx, w.by, c0});
          else if (patch.ensure(gimg, W, H, xl, xh, yl, yh, c0))
            fpass(patch.template sampler<IM>(w.bx, w.by));
          else
            fpass(ImageSampler<IM>{gimg, W, H, w.bx, w.by, c0});
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

template <int MAXS, int IM, bool R2 = false>
static hipError_t launch_nr_f32_t(const DevState& st, const dic_tuning_t& tu,
                                  const RefineGroup& gr, int ctr, const float* ref,
                                  const float* def,
                                  const int32_t* poi, const int32_t* uv_init,
                                  const int32_t* status_in, const double* p_init, double* p_out,
                                  float* zncc, int32_t* iters, int32_t* status, int num_cu,
                                  hipStream_t s) {
  const int threads = tu.icgn_waves * kWave;
  const int slack = min(tu.icgn_slack, R2 ? kR2MaxSlack : refine_max_slack(MAXS));
  // the table form reads no LDS patch
  const size_t lds = IM == kInterpBicubicLut
                         ? 0
                         : refine_lds_bytes(R2 ? kR2Pitch : refine_patch_pitch(MAXS),
                                            icgn_patch_side(gr.maxM, slack), tu.icgn_waves);
  const void* fn = reinterpret_cast<const void*>(&nr_f32_kernel<MAXS, IM, R2>);
  if (lds > 65536) {
    hipError_t ea = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (ea != hipSuccess) return ea;
  }
  int occ = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, nr_f32_kernel<MAXS, IM, R2>,
                                                              threads, lds);
  if (e != hipSuccess) return e;
  if (occ < 1) return hipErrorInvalidConfiguration;
  int64_t blocks = (int64_t)occ * num_cu;
  const int64_t need = (gr.count + tu.icgn_waves - 1) / tu.icgn_waves;
  if (blocks > need) blocks = need;
  hipLaunchKernelGGL((nr_f32_kernel<MAXS, IM, R2>), dim3((unsigned)blocks), dim3(threads), lds,
                     s, st, st.work + gr.begin, gr.count, ctr, gr.maxM, slack, ref, def, poi, uv_init,
                     status_in, p_init, p_out, zncc, iters, status);
  return hipGetLastError();
}

// One group: the kernel its subset size runs in.
template <int IM>
static hipError_t launch_nr_f32_group(const DevState& st, const dic_tuning_t& tu,
                                     const RefineGroup& gr, int ctr, const float* ref,
                                    const float* def,
                                     const int32_t* poi, const int32_t* uv_init,
                                     const int32_t* status_in, const double* p_init,
                                     double* p_out, float* zncc, int32_t* iters,
                                     int32_t* status, int num_cu, hipStream_t s) {
#define DIC_REFINE_ARGS st, tu, gr, ctr, ref, def, poi, uv_init, status_in, p_init, p_out, zncc, iters, \
                        status, num_cu, s
  if (refine_two_rows(gr.maxM)) return launch_nr_f32_t<16, IM, true>(DIC_REFINE_ARGS);
  switch (refine_slots(gr.maxM)) {
    case 4: return launch_nr_f32_t<4, IM>(DIC_REFINE_ARGS);
    case 8: return launch_nr_f32_t<8, IM>(DIC_REFINE_ARGS);
    case 12: return launch_nr_f32_t<12, IM>(DIC_REFINE_ARGS);
    case 16: return launch_nr_f32_t<16, IM>(DIC_REFINE_ARGS);
    case 20: return launch_nr_f32_t<20, IM>(DIC_REFINE_ARGS);
    case 28: return launch_nr_f32_t<28, IM>(DIC_REFINE_ARGS);
    default: return hipErrorInvalidValue;
  }
#undef DIC_REFINE_ARGS
}

hipError_t launch_nr_f32(const DevState& st, const dic_tuning_t& tu, const RefineGroup* groups,
                         int ngroups, const float* ref, const float* def, const int32_t* poi,
                         const int32_t* uv_init, const int32_t* status_in,
                         const double* p_init, double* p_out, float* zncc, int32_t* iters,
                         int32_t* status, int num_cu, hipStream_t s, int interp) {
  if (ngroups > kMaxRefineGroups) return hipErrorInvalidValue;
  for (int k = 0; k < ngroups; ++k) {
    const RefineGroup& gr = groups[k];
    if (gr.count == 0) continue;
    const int ctr = kCtrIcgn + k;
    hipError_t e;
    if (interp == kInterpBilinear)
      e = launch_nr_f32_group<kInterpBilinear>(st, tu, gr, ctr, ref, def, poi, uv_init, status_in,
                                               p_init, p_out, zncc, iters, status, num_cu, s);
    else if (interp == kInterpBSpline)
      e = launch_nr_f32_group<kInterpBSpline>(st, tu, gr, ctr, ref, def, poi, uv_init, status_in,
                                              p_init, p_out, zncc, iters, status, num_cu, s);
    else if (interp == kInterpBicubicLut)
      e = launch_nr_f32_group<kInterpBicubicLut>(st, tu, gr, ctr, ref, def, poi, uv_init,
                                                 status_in, p_init, p_out, zncc, iters, status,
                                                 num_cu, s);
    else
      e = launch_nr_f32_group<kInterpBicubic>(st, tu, gr, ctr, ref, def, poi, uv_init, status_in,
                                              p_init, p_out, zncc, iters, status, num_cu, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
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
