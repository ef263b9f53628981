// IC-GN sub-pixel refinement (Sec. 2.2) with a first-order warp and Keys
// bicubic interpolation of the deformed image.
//
// FP32 batched form.  One wave per POI, persistent over a shared work counter
// (several waves per workgroup, each independent).  Per lane: the reference
// gradients of its samples stay in registers for the whole solve, so an
// iteration reads only the deformed image, from a per-wave LDS patch (holding
// g - c0, c0 a deformed grey level at the subset's centre, compile-time row
// pitch) that is restaged only when the warped subset leaves it.  Sample
// positions are an integer base (POI + rounded translation) plus an FP32
// local offset below ~M+slack pixels.  Eight sums per iteration (sum g,
// sum g^2 and the six steepest-descent products, g taken relative to c0)
// are blocked: each lane sums its at most MAXS samples in FP32 (fused
// multiply-adds) and the 64 lane partials are added in
// FP32 in a fixed tree of six levels, so the relative error stays near
// (MAXS + 6) * 2^-24 of the sum of magnitudes; with the precomputed
// sum SD_i (f_i - fbar) and sum SD_i the right-hand side needs no second pass:
//   sum SD_i e_i = sum SD_i (f_i - fbar) - (df/dg) (sum SD_i g_i - gbar sum SD_i).
// The 6x6 solve and the warp composition run in FP64.
#include "refine_common.h"

namespace dic {

namespace {

template <int MAXS, class Smp, class OF>
__device__ __forceinline__ void iter_pass(const Smp& smp, int n, const Warp32& w,
                                          const float* fxs, const float* fys, const OF& offs,
                                          float* K) {
  constexpr int MINS = refine_min_slots(MAXS);
  const Slots sl(n);
#pragma unroll
  for (int a = 0; a < 8; ++a) K[a] = 0.f;
#pragma unroll
  for (int k = 0; k < MAXS; ++k) {
    // slots every subset of the class fills run without a test, so the
    // reads of consecutive slots can overlap
    if (k >= MINS && !sl.used(k)) continue;
    float dx, dy;
    offs(k, dx, dy);
    const float v = sample_value(smp, warp_x(w, dx, dy), warp_y(w, dx, dy));
    const float gs = k + 1 >= MINS ? sl.mask(k, v) : v;
    const float fg = fxs[k] * gs, hg = fys[k] * gs;
    K[0] += gs;
    K[1] = fmaf(gs, gs, K[1]);
    K[2] += fg;
    K[3] = fmaf(fg, dx, K[3]);
    K[4] = fmaf(fg, dy, K[4]);
    K[5] += hg;
    K[6] = fmaf(hg, dx, K[6]);
    K[7] = fmaf(hg, dy, K[7]);
  }
}

// The pass of iter_pass in the two-rows layout (same eight sums).
template <int MAXS, class Smp>
__device__ __forceinline__ void iter_pass_r2(const Smp& smp, int M, const R2Lane& L,
                                             const Warp32& w, const float* fxs, const float* fys,
                                             float fxp, float fyp, float* K) {
  const int Mu = __builtin_amdgcn_readfirstlane(M);
  const float bx = fmaf(w.ax, L.dx, fmaf(w.uy, L.hm, w.uf));
  const float by = fmaf(w.vx, L.dx, fmaf(w.ay, L.hm, w.vf));
  float k0 = 0.f, k1 = 0.f, k2 = 0.f, k4 = 0.f, k5 = 0.f, k7 = 0.f;
  const auto add = [&](int k, float gs) {
    const float dk = (float)(2 * k);
    const float fg = fxs[k] * gs, hg = fys[k] * gs;
    k0 += gs;
    k1 = fmaf(gs, gs, k1);
    k2 += fg;
    k4 = fmaf(fg, dk, k4);
    k5 += hg;
    k7 = fmaf(hg, dk, k7);
  };
  const auto pos_x = [&](int k) { return fmaf(w.uy, (float)(2 * k), bx); };
  const auto pos_y = [&](int k) { return fmaf(w.ay, (float)(2 * k), by); };
  if constexpr (!Smp::kLut) {
    // slots below kR2MinM always hold samples: software-pipelined, the taps
    // of slot k + 1 requested before slot k's are combined (the scheduling
    // barrier keeps that order, so the reads' latency overlaps the work)
    using TS = TapSet<Smp::ntaps()>;
    TS ta = taps_fetch(smp, pos_x(0), pos_y(0)), tb;
#pragma unroll
    for (int k = 0; k < kR2MinM; ++k) {
      TS& cur = (k & 1) ? tb : ta;
      TS& nxt = (k & 1) ? ta : tb;
      if (k + 1 < kR2MinM) nxt = taps_fetch(smp, pos_x(k + 1), pos_y(k + 1));
      __builtin_amdgcn_sched_barrier(0);
      add(k, taps_combine(cur));
    }
#pragma unroll
    for (int k = kR2MinM; k < MAXS - 1; ++k)
      if (k < Mu) add(k, sample_value(smp, pos_x(k), pos_y(k)));
  } else {
#pragma unroll
    for (int k = 0; k < MAXS - 1; ++k)
      if (k < kR2MinM || k < Mu) add(k, sample_value(smp, pos_x(k), pos_y(k)));
  }
  {
    // the last row (offset M), read by both half-waves at the lower one's
    // positions, counted once
    const float dm = (float)Mu;
    const float x = fmaf(w.ax, L.dx, fmaf(w.uy, dm, w.uf));
    const float y = fmaf(w.vx, L.dx, fmaf(w.ay, dm, w.vf));
    const float v = sample_value(smp, x, y);
    const float gs = L.upper ? 0.f : v;
    const float fg = fxp * gs, hg = fyp * gs;
    const float d2 = 2.f * dm;
    k0 += gs;
    k1 = fmaf(gs, gs, k1);
    k2 += fg;
    k4 = fmaf(fg, d2, k4);
    k5 += hg;
    k7 = fmaf(hg, d2, k7);
  }
  K[0] = L.colok ? k0 : 0.f;
  K[1] = L.colok ? k1 : 0.f;
  K[2] = k2;
  K[3] = L.dx * k2;
  K[4] = fmaf(L.hm, k2, k4);
  K[5] = k5;
  K[6] = L.dx * k5;
  K[7] = fmaf(L.hm, k5, k7);
}

}  // namespace

// Three waves per SIMD; the two-rows kernels fit four, which measured slower
// (0.54 against 0.52 ms on the 1024^2 benchmark pair).
template <int MAXS, int IM, bool R2>
__global__ void __launch_bounds__(512)
__attribute__((amdgpu_waves_per_eu(3))) icgn_f32_kernel(
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
    if (status_in && status == DIC_POI_OK) status = uniform(status_in[g]);
    int it = 0;
    float zn = nanf("");
    if (status == DIC_POI_OK) {
      const int M = P.M, n1 = 2 * M + 1, n = n1 * n1, W = P.width, H = P.height;
      // the taps: the image's pixels, or its cubic B-spline coefficients
      const float* gimg =
          IM == kInterpBSpline ? st.lut + 4 * P.lut_off : def + P.def_off;
      const float4* glut = reinterpret_cast<const float4*>(st.lut) + P.lut_off;
      const int64_t corner = (int64_t)(y0 - M) * W + (x0 - M);
      const float* gx = st.grads + P.grad_off + corner;
      const float* gy = gx + (int64_t)W * H;
      float fxs[MAXS], fys[MAXS], fxp = 0.f, fyp = 0.f;
      half2v dxy[R2 ? 1 : MAXS];
      // the 20- and 28-slot kernels recompute the offsets, which leaves them
      // registers for 3 waves per SIMD instead of 2
      const auto offs = [&] {
        if constexpr (MAXS >= 20)
          return OffsetsComputed(M);
        else
          return OffsetsKept{dxy};
      }();
      R2Lane L2{};
      if constexpr (R2) {
        L2 = r2_lane(M);
        load_slots_r2<MAXS>(M, L2, gx, gy, W, fxs, fys, fxp, fyp);
      } else {
        load_slots<MAXS, true>(M, n, gx, gy, W, dxy, fxs, fys);
      }
      const float c0 = deformed_centre(gimg, W, H, p, x0, y0);
      const double df = R->df;
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
        float K[8];
        const auto pass = [&](const auto& smp) {
          if constexpr (R2)
            iter_pass_r2<MAXS>(smp, M, L2, w, fxs, fys, fxp, fyp, K);
          else
            iter_pass<MAXS>(smp, n, w, fxs, fys, offs, K);
        };
        if constexpr (IM == kInterpBicubicLut)
          pass(LutSampler{glut, W, H, w.bx, w.by, c0});
        else if (patch.ensure(gimg, W, H, xl, xh, yl, yh, c0))
          pass(patch.template sampler<IM>(w.bx, w.by));
        else
          pass(ImageSampler<IM>{gimg, W, H, w.bx, w.by, c0});
        double S[8];
        wave_sums_f32<8>(K, S);
        if (!isfinite(S[0]) || !isfinite(S[1])) {
          status = DIC_POI_NAN_INPUT;
          break;
        }
        const double ms = S[0] / nn;
        const double var = S[1] - S[0] * ms;
        const double sumg2 = S[1] + 2.0 * (double)c0 * S[0] + nn * (double)c0 * (double)c0;
        if (!not_flat(var, sumg2)) {
          status = DIC_POI_ZERO_VARIANCE;
          break;
        }
        const double ratio = df / sqrt(var);
        double b[6], dp[6];
#pragma unroll
        for (int a = 0; a < 6; ++a) b[a] = -(R->sdf_sum[a] - ratio * (S[2 + a] - ms * R->sd_sum[a]));
        cholesky6_solve(R->L, R->rdiag, b, dp);
        compose_inverse(p, dp);
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
          // the template value f - fbar at offset (dx, dy), rounded as the
          // record's tsum counts it
          const float* fc = ref + P.ref_off + (int64_t)y0 * W + x0;
          const float fb = (float)R->fbar;
          const auto tval = [&](int, float dx, float dy) {
            return fc[(int)dy * W + (int)dx] - fb;
          };
          float K[3];
          const auto fpass = [&](const auto& smp) {
            if constexpr (R2)
              final_pass_r2<MAXS>(smp, M, L2, w, tval, K);
            else
              final_pass<MAXS>(smp, n, w, offs, tval, K);
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
              zn = (float)((S[2] - ms * (double)R->tsum) / (df * sqrt(var)));
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
static hipError_t launch_icgn_f32_t(const DevState& st, const dic_tuning_t& tu,
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
  const void* fn = reinterpret_cast<const void*>(&icgn_f32_kernel<MAXS, IM, R2>);
  if (lds > 65536) {
    hipError_t ea = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (ea != hipSuccess) return ea;
  }
  int occ = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, icgn_f32_kernel<MAXS, IM, R2>,
                                                              threads, lds);
  if (e != hipSuccess) return e;
  if (occ < 1) return hipErrorInvalidConfiguration;
  int64_t blocks = (int64_t)occ * num_cu;
  const int64_t need = (gr.count + tu.icgn_waves - 1) / tu.icgn_waves;
  if (blocks > need) blocks = need;
  hipLaunchKernelGGL((icgn_f32_kernel<MAXS, IM, R2>), dim3((unsigned)blocks), dim3(threads), lds,
                     s, st, st.work + gr.begin, gr.count, ctr, gr.maxM, slack, ref, def, poi, uv_init,
                     status_in, p_init, p_out, zncc, iters, status);
  return hipGetLastError();
}

// One group: the kernel its subset size runs in.
template <int IM>
static hipError_t launch_icgn_f32_group(const DevState& st, const dic_tuning_t& tu,
                                     const RefineGroup& gr, int ctr, const float* ref,
                                    const float* def,
                                     const int32_t* poi, const int32_t* uv_init,
                                     const int32_t* status_in, const double* p_init,
                                     double* p_out, float* zncc, int32_t* iters,
                                     int32_t* status, int num_cu, hipStream_t s) {
#define DIC_REFINE_ARGS st, tu, gr, ctr, ref, def, poi, uv_init, status_in, p_init, p_out, zncc, iters, \
                        status, num_cu, s
  if (refine_two_rows(gr.maxM)) return launch_icgn_f32_t<16, IM, true>(DIC_REFINE_ARGS);
  switch (refine_slots(gr.maxM)) {
    case 4: return launch_icgn_f32_t<4, IM>(DIC_REFINE_ARGS);
    case 8: return launch_icgn_f32_t<8, IM>(DIC_REFINE_ARGS);
    case 12: return launch_icgn_f32_t<12, IM>(DIC_REFINE_ARGS);
    case 16: return launch_icgn_f32_t<16, IM>(DIC_REFINE_ARGS);
    case 20: return launch_icgn_f32_t<20, IM>(DIC_REFINE_ARGS);
    case 28: return launch_icgn_f32_t<28, IM>(DIC_REFINE_ARGS);
    default: return hipErrorInvalidValue;
  }
#undef DIC_REFINE_ARGS
}

hipError_t launch_icgn_f32(const DevState& st, const dic_tuning_t& tu, const RefineGroup* groups,
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
      e = launch_icgn_f32_group<kInterpBilinear>(st, tu, gr, ctr, ref, def, poi, uv_init, status_in,
                                               p_init, p_out, zncc, iters, status, num_cu, s);
    else if (interp == kInterpBSpline)
      e = launch_icgn_f32_group<kInterpBSpline>(st, tu, gr, ctr, ref, def, poi, uv_init, status_in,
                                              p_init, p_out, zncc, iters, status, num_cu, s);
    else if (interp == kInterpBicubicLut)
      e = launch_icgn_f32_group<kInterpBicubicLut>(st, tu, gr, ctr, ref, def, poi, uv_init,
                                                 status_in, p_init, p_out, zncc, iters, status,
                                                 num_cu, s);
    else
      e = launch_icgn_f32_group<kInterpBicubic>(st, tu, gr, ctr, ref, def, poi, uv_init, status_in,
                                              p_init, p_out, zncc, iters, status, num_cu, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// FP64 plain form: one 64-thread workgroup per POI of one pair; FP64
// positions, weights and sums, taps and reference gradients read from global
// memory every iteration, two-pass statistics, residual formed per sample.
// ---------------------------------------------------------------------------

template <int MAXS>
__global__ void __launch_bounds__(64) icgn_f64_kernel(
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
  if (status_in && status == DIC_POI_OK) status = status_in[g];
  int it = 0;
  double zn = nan("");
  const int M = P.M, n1 = 2 * M + 1, n = n1 * n1, W = P.width, H = P.height;
  const float* f = ref + P.ref_off;
  const float* gi = def + P.def_off;
  const double fbar = R->fbar, df = R->df;
  double gl[MAXS];

  // Interpolates every sample at p into gl; returns 1 if any tap leaves the
  // image (checked per sample), 2 if any value is non-finite.
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
#pragma unroll
    for (int k = 0; k < MAXS; ++k) {
      const int s = lane + kWave * k;
      gl[k] = 0.0;
      if (s >= n) continue;
      const double dx = (double)(s % n1 - M), dy = (double)(s / n1 - M);
      const double xs = x0 + (1.0 + p[1]) * dx + p[2] * dy + p[0];
      const double ys = y0 + p[4] * dx + (1.0 + p[5]) * dy + p[3];
      const double fx = floor(xs), fy = floor(ys);
      double wx[4], wy[4];
      cubic_weights(xs - fx, wx);
      cubic_weights(ys - fy, wy);
      const float* q = gi + (int64_t)((int)fy - 1) * W + ((int)fx - 1);
      double v = 0.0;
      for (int l = 0; l < 4; ++l)
        for (int c = 0; c < 4; ++c) v += wy[l] * wx[c] * (double)q[(int64_t)l * W + c];
      gl[k] = v;
      s1 += v;
    }
    s1 = wave_sum(s1);
    if (!isfinite(s1)) return 2;
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
      double b[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int k = 0; k < MAXS; ++k) {
        const int s = lane + kWave * k;
        if (s >= n) continue;
        const int dxi = s % n1 - M, dyi = s / n1 - M;
        const int64_t idx = (int64_t)(y0 + dyi) * W + (x0 + dxi);
        const double fx = ((double)f[idx + 1] - (double)f[idx - 1]) / 2.0;
        const double fy = ((double)f[idx + W] - (double)f[idx - W]) / 2.0;
        const double e = ((double)f[idx] - fbar) - df / dg * (gl[k] - gbar);
        const double dx = dxi, dy = dyi;
        b[0] += fx * e;
        b[1] += fx * dx * e;
        b[2] += fx * dy * e;
        b[3] += fy * e;
        b[4] += fy * dx * e;
        b[5] += fy * dy * e;
      }
      double dp[6];
      for (int a = 0; a < 6; ++a) b[a] = -wave_sum(b[a]);
      cholesky6_solve(R->L, R->rdiag, b, dp);
      compose_inverse(p, dp);
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

hipError_t launch_icgn_f64(const DevState& st, const DevPair* host_pairs, const float* ref,
                           const float* def, const int32_t* poi, const int32_t* uv_init,
                           const int32_t* status_in, const double* p_init, double* p_out,
                           float* zncc, int32_t* iters, int32_t* status, hipStream_t s) {
  for (int k = 0; k < st.num_pairs; ++k) {
    const DevPair& P = host_pairs[k];
    if (P.poi_count == 0) continue;
    const int need = ((2 * P.M + 1) * (2 * P.M + 1) + kWave - 1) / kWave;
    const dim3 grid((unsigned)P.poi_count), block(64);
#define DIC_ICGN64_CASE(S_)                                                                    \
  if (need <= S_) {                                                                            \
    hipLaunchKernelGGL(icgn_f64_kernel<S_>, grid, block, 0, s, st, P, ref, def, poi, uv_init,  \
                       status_in, p_init, p_out, zncc, iters, status);                         \
    hipError_t e = hipGetLastError();                                                          \
    if (e != hipSuccess) return e;                                                             \
    continue;                                                                                  \
  }
    DIC_ICGN64_CASE(4)
    DIC_ICGN64_CASE(8)
    DIC_ICGN64_CASE(12)
    DIC_ICGN64_CASE(16)
    DIC_ICGN64_CASE(20)
    DIC_ICGN64_CASE(28)
#undef DIC_ICGN64_CASE
    return hipErrorInvalidValue;
  }
  return hipSuccess;
}

}  // namespace dic
