// ZNSSD criterion C = sum (fhat - ghat)^2 = 2 - 2 ZNCC and its adjoint with
// respect to the forward-additive warp parameters and to every deformed-image
// grey level the bicubic interpolation touches.
//
// One wave per POI.  Each lane interpolates its samples once (value and the
// analytic gradient of the interpolant from the derivative weights), keeps
// them in registers, reduces four sums (per-lane FP64, DPP across the wave),
// and then scatters
//   dC/dg_i = (2/dg) (ZNCC ghat_i - fhat_i)
// through the 16 bicubic weights.  The scatter goes first into a per-wave
// LDS patch covering the POI's tap box, as 2^-40 fixed-point int64 LDS
// atomics (neighbouring samples share taps; the integer adds measured four
// times faster than float LDS atomics here), and the patch is then added to
// the image gradient once per pixel: about (2M + 4)^2 global atomics per POI
// instead of 16 n.  Float atomics into grad_def, or in deterministic mode
// int64 atomics into a fixed-point accumulator (integer addition is order
// independent) that a second kernel converts to float.  A warp whose tap box
// does not fit the patch scatters straight to global memory.
#include "dic_device.h"

namespace dic {

namespace {

constexpr double kFixScale = 1099511627776.0;  // 2^40

struct Samp {
  float g, gx, gy;
};

__device__ __forceinline__ Samp interp_grad(const float* __restrict__ img, int W, int H, int bx,
                                            int by, float xs, float ys) {
  const float fx = floorf(xs), fy = floorf(ys);
  const float tx = xs - fx, ty = ys - fy;
  float wx[4], wy[4], dwx[4], dwy[4];
  cubic_weights(tx, wx);
  cubic_weights(ty, wy);
  cubic_dweights(tx, dwx);
  cubic_dweights(ty, dwy);
  // The corner test keeps the neighbourhood inside; the clamp only guarantees
  // in-bounds reads for a degenerate warp.
  const int c0 = min(max(bx + (int)fx - 1, 0), W - 4);
  const int r0 = min(max(by + (int)fy - 1, 0), H - 4);
  const float* q = img + (int64_t)r0 * W + c0;
  Samp s{0.f, 0.f, 0.f};
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    const float* row = q + (int64_t)l * W;
    const float r = fmaf(wx[3], row[3], fmaf(wx[2], row[2], fmaf(wx[1], row[1], wx[0] * row[0])));
    const float rd =
        fmaf(dwx[3], row[3], fmaf(dwx[2], row[2], fmaf(dwx[1], row[1], dwx[0] * row[0])));
    s.g = fmaf(wy[l], r, s.g);
    s.gy = fmaf(dwy[l], r, s.gy);
    s.gx = fmaf(wy[l], rd, s.gx);
  }
  return s;
}

}  // namespace

template <int MAXS>
__global__ void __launch_bounds__(256) znssd_kernel(
    DevState st, const float* __restrict__ ref, const float* __restrict__ def,
    const int32_t* __restrict__ poi,
    const double* __restrict__ pw, const float* __restrict__ grad_c, float* __restrict__ c_out,
    double* __restrict__ grad_p, float* __restrict__ grad_def,
    unsigned long long* __restrict__ fix_acc, const int64_t* __restrict__ fix_off, int pside) {
  extern __shared__ __attribute__((aligned(8))) unsigned char zlds[];
  const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (g >= st.N) return;
  const int lane = lane_id();
  // this wave's accumulation patch: pside^2 int64 in 2^-40 fixed point
  unsigned long long* acci =
      reinterpret_cast<unsigned long long*>(zlds) + (size_t)(threadIdx.x / kWave) * pside * pside;
  const DevPair P = st.pairs[uniform(st.poi_pair[g])];
  const RefRec* R = st.recs + g;
  const int x0 = uniform(poi[2 * g]), y0 = uniform(poi[2 * g + 1]);
  const int M = P.M, n1 = 2 * M + 1, n = n1 * n1, W = P.width, H = P.height;
  const int rs = uniform(R->status);
  double p[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) p[a] = pw[6 * g + a];
  const double ur = rint(p[0]), vr = rint(p[3]);
  const int bx = x0 + (int)ur, by = y0 + (int)vr;
  const float uf = (float)(p[0] - ur), vf = (float)(p[3] - vr);
  const float ux = (float)p[1], uy = (float)p[2], vx = (float)p[4], vy = (float)p[5];
  bool ok = rs == DIC_POI_OK || rs == DIC_POI_SINGULAR_HESSIAN;
  // the tap box [xl, xh] x [yl, yh] (absolute pixels)
  int xl = INT_MAX, xh = INT_MIN, yl = INT_MAX, yh = INT_MIN;
  if (ok) {
    // every tap inside the image (corners bound an affine map of a square)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const float dx = a ? (float)M : -(float)M, dy = b ? (float)M : -(float)M;
        const int ix = bx + (int)floorf(dx + fmaf(ux, dx, fmaf(uy, dy, uf)));
        const int iy = by + (int)floorf(dy + fmaf(vx, dx, fmaf(vy, dy, vf)));
        if (ix < 1 || ix + 2 > W - 1 || iy < 1 || iy + 2 > H - 1) ok = false;
        xl = min(xl, ix - 1);
        xh = max(xh, ix + 2);
        yl = min(yl, iy - 1);
        yh = max(yh, iy + 2);
      }
  }
  const float* gimg = def + P.def_off;
  const float* fimg = ref + P.ref_off;
  Samp sm[MAXS];
  float tv[MAXS];
  double K[4] = {0, 0, 0, 0};
  if (ok) {
    const float c0 = (float)R->fbar;
#pragma unroll
    for (int k = 0; k < MAXS; ++k) {
      const int s = lane + kWave * k;
      sm[k] = Samp{0.f, 0.f, 0.f};
      tv[k] = 0.f;
      if (s < n) {
        const float dx = (float)(s % n1 - M), dy = (float)(s / n1 - M);
        sm[k] = interp_grad(gimg, W, H, bx, by, dx + fmaf(ux, dx, fmaf(uy, dy, uf)),
                            dy + fmaf(vx, dx, fmaf(vy, dy, vf)));
        sm[k].g -= c0;
        tv[k] = fimg[(int64_t)(y0 + s / n1 - M) * W + (x0 + s % n1 - M)] - c0;
        K[0] += (double)sm[k].g;
        K[1] += (double)(sm[k].g * sm[k].g);
        K[2] += (double)(tv[k] * sm[k].g);
        K[3] += (double)tv[k];
      }
    }
  }
  const double s0 = wave_sum_dpp(K[0]), s1 = wave_sum_dpp(K[1]), s2 = wave_sum_dpp(K[2]),
               s3 = wave_sum_dpp(K[3]);
  const double nn = (double)n;
  const double ms = s0 / nn, var = s1 - s0 * ms;
  const double df = R->df, dg = sqrt(var);
  if (ok && !(isfinite(s0) && isfinite(s1) && var > 0.0)) ok = false;
  const double zn = (s2 - ms * s3) / (df * dg);
  const double up = grad_c ? (double)grad_c[g] : 1.0;
  double gp[6] = {0, 0, 0, 0, 0, 0};
  const bool scatter = ok && (grad_def || fix_acc);
  // the LDS patch holds the tap box when it fits (wave-uniform decision)
  const int pw_ = scatter ? xh - xl + 1 : 0, ph_ = scatter ? yh - yl + 1 : 0;
  const bool use_lds = scatter && pw_ <= pside && ph_ <= pside;
  if (use_lds) {
    for (int e = lane; e < pw_ * ph_; e += kWave) {
      const int r = e / pw_, c = e - r * pw_;
      acci[r * pside + c] = 0ull;
    }
    wave_lds_sync();
  }
  if (ok) {
    const double scale = up * 2.0 / dg;
#pragma unroll
    for (int k = 0; k < MAXS; ++k) {
      const int s = lane + kWave * k;
      if (s < n) {
        const double gh = ((double)sm[k].g - ms) / dg;
        const double fh = (double)tv[k] / df;
        const double dcdg = scale * (zn * gh - fh);
        const double dx = (double)(s % n1 - M), dy = (double)(s / n1 - M);
        const double gxv = (double)sm[k].gx, gyv = (double)sm[k].gy;
        gp[0] += dcdg * gxv;
        gp[1] += dcdg * gxv * dx;
        gp[2] += dcdg * gxv * dy;
        gp[3] += dcdg * gyv;
        gp[4] += dcdg * gyv * dx;
        gp[5] += dcdg * gyv * dy;
        if (grad_def || fix_acc) {
          const float xs = (float)dx + fmaf(ux, (float)dx, fmaf(uy, (float)dy, uf));
          const float ys = (float)dy + fmaf(vx, (float)dx, fmaf(vy, (float)dy, vf));
          const float fx = floorf(xs), fy = floorf(ys);
          float wx[4], wy[4];
          cubic_weights(xs - fx, wx);
          cubic_weights(ys - fy, wy);
          const int64_t base = (int64_t)min(max(by + (int)fy - 1, 0), H - 4) * W +
                               min(max(bx + (int)fx - 1, 0), W - 4);
          const float dcf = (float)dcdg;
          if (use_lds) {
            // the same neighbourhood origin, relative to the tap box
            const int lo = (by + (int)fy - 1 - yl) * pside + (bx + (int)fx - 1 - xl);
#pragma unroll
            for (int l = 0; l < 4; ++l)
#pragma unroll
              for (int c = 0; c < 4; ++c) {
                const double v = dcdg * (double)wy[l] * (double)wx[c];
                atomicAdd(acci + lo + l * pside + c,
                          (unsigned long long)(long long)llrint(v * kFixScale));
              }
          } else {
#pragma unroll
            for (int l = 0; l < 4; ++l)
#pragma unroll
              for (int c = 0; c < 4; ++c) {
                const int64_t idx = base + (int64_t)l * W + c;
                if (fix_acc) {
                  const double v = dcdg * (double)wy[l] * (double)wx[c];
                  atomicAdd(fix_acc + fix_off[uniform(st.poi_pair[g])] + idx,
                            (unsigned long long)(long long)llrint(v * kFixScale));
                } else {
                  atomicAdd(grad_def + P.def_off + idx, dcf * wy[l] * wx[c]);
                }
              }
          }
        }
      }
    }
  }
  if (use_lds) {
    // the patch, once per pixel, into grad_def (or the fixed-point
    // accumulator); pixels no sample touched stay zero and are skipped
    wave_lds_sync();
    const int64_t gbase = (int64_t)yl * W + xl;
    unsigned long long* facc = fix_acc ? fix_acc + fix_off[uniform(st.poi_pair[g])] : nullptr;
    for (int e = lane; e < pw_ * ph_; e += kWave) {
      const int r = e / pw_, c = e - r * pw_;
      const int64_t idx = gbase + (int64_t)r * W + c;
      const unsigned long long v = acci[r * pside + c];
      if (v == 0ull) continue;
      if (facc)
        atomicAdd(facc + idx, v);
      else
        atomicAdd(grad_def + P.def_off + idx, (float)((double)(long long)v / kFixScale));
    }
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) gp[a] = wave_sum_dpp(gp[a]);
  if (lane == 0) {
    if (c_out) c_out[g] = ok ? (float)(2.0 - 2.0 * zn) : nanf("");
    if (grad_p)
#pragma unroll
      for (int a = 0; a < 6; ++a) grad_p[6 * g + a] = ok ? gp[a] : 0.0;
  }
}

__global__ void fix_clear_kernel(unsigned long long* acc, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    acc[i] = 0ull;
}

// grad_def[image] += fixed-point accumulator, once per distinct deformed
// image (grid row y: the pair owner[y] that owns it; pairs on the same image
// accumulated into the same block, and no two owners overlap).
__global__ void fix_flush_kernel(const DevPair* __restrict__ pairs,
                                 const int64_t* __restrict__ fix_off,
                                 const int32_t* __restrict__ owner,
                                 const unsigned long long* __restrict__ acc,
                                 float* __restrict__ grad_def) {
  const int k = owner[blockIdx.y];
  const DevPair P = pairs[k];
  const int64_t count = (int64_t)P.width * P.height;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const long long v = (long long)acc[fix_off[k] + i];
    if (v != 0) grad_def[P.def_off + i] += (float)((double)v / kFixScale);
  }
}

hipError_t launch_znssd(const DevState& st, const float* ref, const float* def,
                        const int32_t* poi, const double* p, const float* grad_c, float* c_out,
                        double* grad_p, float* grad_def, unsigned long long* fix_acc,
                        const int64_t* fix_off, const int32_t* fix_owner, int num_regions,
                        int64_t fix_count, int /*num_cu*/, hipStream_t s) {
  if (st.N == 0) return hipSuccess;
  const bool det = fix_acc != nullptr && grad_def != nullptr;
  if (det) {
    hipLaunchKernelGGL(fix_clear_kernel, dim3(1024), dim3(256), 0, s, fix_acc, fix_count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int n = (2 * st.maxM + 1) * (2 * st.maxM + 1);
  const int need = (n + kWave - 1) / kWave;
  const dim3 grid((unsigned)((st.N + 3) / 4)), block(256);
  unsigned long long* acc = det ? fix_acc : nullptr;
  // accumulation patch per wave: the tap box of the subset (2M + 4) plus 6
  // pixels for the warp's gradient terms (|ux| + |uy| <= 3 / M, likewise for
  // v); only when image gradients are asked for
  const int pside = (grad_def != nullptr) ? 2 * st.maxM + 10 : 0;
  const size_t lds = (size_t)4 * pside * pside * sizeof(unsigned long long);
#define DIC_ZN_CASE(S_)                                                                       \
  if (need <= S_) {                                                                           \
    if (lds > 65536) {                                                                        \
      hipError_t ea = hipFuncSetAttribute(reinterpret_cast<const void*>(&znssd_kernel<S_>),   \
                                          hipFuncAttributeMaxDynamicSharedMemorySize,          \
                                          (int)lds);                                          \
      if (ea != hipSuccess) return ea;                                                        \
    }                                                                                         \
    hipLaunchKernelGGL(znssd_kernel<S_>, grid, block, lds, s, st, ref, def, poi, p, grad_c,   \
                       c_out, grad_p, det ? nullptr : grad_def, acc, fix_off, pside);         \
  } else
  DIC_ZN_CASE(4)
  DIC_ZN_CASE(8)
  DIC_ZN_CASE(12)
  DIC_ZN_CASE(16)
  DIC_ZN_CASE(20)
  DIC_ZN_CASE(28) { return hipErrorInvalidValue; }
#undef DIC_ZN_CASE
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (det && num_regions > 0) {
    hipLaunchKernelGGL(fix_flush_kernel, dim3(256, num_regions), dim3(256), 0, s, st.pairs,
                       fix_off, fix_owner, fix_acc, grad_def);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace dic
