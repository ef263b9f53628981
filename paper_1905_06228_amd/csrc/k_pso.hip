// Particle swarm integer search (Sec. 2.1, Eqs. 2-4) and its modified form
// with a star step (each particle also evaluates its four neighbours and
// moves to the best of the five), the paper's alternatives to the
// brute-force search (Sec. 5.2: 50 particles, at most 5 generations, stop at
// a coefficient of 0.995, at most 250 / 1250 evaluations).
//
// One wave per POI, persistent over a work counter; particle i on lane i.
// The swarm's random numbers are an input (float uniforms, [G, P, 4] per
// POI).  Per wave in LDS (about 10 KB at radius 16, so many waves share a
// CU): the coefficient of every window position already computed (the
// look-up table of Sec. 5.2), a claim bit per position and the list of
// positions to compute in the current generation.  Each generation the
// particles claim the positions they need that are not in the table (one
// claim per position), and the claimed positions are computed four at a
// time by the whole wave: lane l holds the FP64 deviations e = f - fbar of
// subset samples l + 64 k in registers, reads the four candidates' pixels at
// those samples (consecutive lanes, consecutive columns), and the lane sums
// are added by DPP.  A coefficient is Eq. (1) in
// FP64: sum e_i g_i minus gbar sum e_i, over df sqrt(sum g^2 - (sum g)^2 / n)
// from the FP64 box sums, the same admissibility and flatness rule as the
// brute-force forms.  Personal and
// swarm bests follow the brute-force tie rule (larger by more than 1e-12,
// else the smaller row-major index), the swarm best folded over the particles
// in index order; the velocity and position updates are evaluated in the
// order the equations are written, without fused multiply-adds.
#include "dic_device.h"

namespace dic {

namespace {

constexpr double kTieEps = 1e-12;
constexpr int kBatch = 4;   // positions computed together

__device__ __forceinline__ bool pso_better(double ca, int ia, double cb, int ib) {
  if (!(ca > -INFINITY)) return false;
  if (!(cb > -INFINITY)) return true;
  if (ca > cb + kTieEps) return true;
  return ca >= cb - kTieEps && ia < ib;
}

struct PsoLds {
  double* lut;
  uint32_t* claim;   // one bit per window position
  int* list;
};

__host__ __device__ __forceinline__ size_t pso_align(size_t b) { return (b + 15) / 16 * 16; }

__host__ __device__ __forceinline__ size_t pso_wave_lds(int maxS, int /*maxM*/) {
  const size_t side = 2 * (size_t)maxS + 1;
  return pso_align(side * side * 8) + pso_align((side * side + 31) / 32 * 4) +
         pso_align((size_t)kPsoStar * kPsoParticles * 4);
}

__device__ __forceinline__ PsoLds pso_carve(unsigned char* base, int maxS, int /*maxM*/) {
  const size_t side = 2 * (size_t)maxS + 1;
  PsoLds L;
  L.lut = reinterpret_cast<double*>(base);
  base += pso_align(side * side * 8);
  L.claim = reinterpret_cast<uint32_t*>(base);
  base += pso_align((side * side + 31) / 32 * 4);
  L.list = reinterpret_cast<int*>(base);
  return L;
}

// The velocity and position update of one direction, Eqs. (2)-(3), with a
// term whose best does not exist yet taken as zero; no contraction, so the
// result is the one the equations give in this order.
__device__ __forceinline__ void pso_update(double& q, double& v, double w, double r1, double r2,
                                           double pbest, bool has_p, double gbest, bool has_g,
                                           double S) {
#pragma clang fp contract(off)
  const double a = w * v;
  const double b = (kPsoC1 * r1) * ((has_p ? pbest : q) - q);
  const double c = (kPsoC2 * r2) * ((has_g ? gbest : q) - q);
  v = fmin(fmax((a + b) + c, -S), S);
  q = fmin(fmax(q + v, -S), S);
}

__device__ __forceinline__ double pso_init(float u, double S) {
#pragma clang fp contract(off)
  return (2.0 * S) * (double)u - S;
}

__device__ __forceinline__ double wave_max_f64(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

}  // namespace

template <bool MOD, int MAXS>
__global__ void __launch_bounds__(256) pso_kernel(
    DevState st, size_t wave_lds, const float* __restrict__ ref, const float* __restrict__ def,
    const int32_t* __restrict__ poi, const int32_t* __restrict__ seed_uv,
    const float* __restrict__ rand, int32_t* __restrict__ uv_out, float* __restrict__ zncc_out,
    int32_t* __restrict__ status_out, int32_t* __restrict__ gens_out,
    int32_t* __restrict__ evals_out) {
  extern __shared__ unsigned char lds_raw[];
  const int lane = lane_id(), wid = threadIdx.x / kWave;
  const PsoLds L = pso_carve(lds_raw + (size_t)wid * wave_lds, st.maxS, st.maxM);
  const bool part = lane < kPsoParticles;

  for (;;) {
    const int item = wave_next_item(&st.counters[kCtrSearch]);
    if (item >= st.N) break;
    const int g = uniform(st.work[item]);
    const DevPair P = st.pairs[uniform(st.poi_pair[g])];
    const RefRec* R = st.recs + g;
    const int x0 = uniform(poi[2 * g]), y0 = uniform(poi[2 * g + 1]);
    const int cu = seed_uv ? uniform(seed_uv[2 * g]) : 0;
    const int cv = seed_uv ? uniform(seed_uv[2 * g + 1]) : 0;
    int status = uniform(R->status);
    if (status == DIC_POI_SINGULAR_HESSIAN) status = DIC_POI_OK;   // the search still runs
    int gens = 0, evals = 0, gbx = 0, gby = 0;
    double gbc = -INFINITY;
    if (status == DIC_POI_OK) {
      const int M = P.M, S = P.S, n1 = 2 * M + 1, n = n1 * n1, side = 2 * S + 1;
      const int W = P.width, H = P.height;
      const double Sd = (double)S, fbar = R->fbar, df = R->df, rnd = 1.0 / (double)n;
      const float* fimg = ref + P.ref_off + (int64_t)(y0 - M) * W + (x0 - M);
      const float* gimg = def + P.def_off;
      const int64_t plane = (int64_t)W * H;
      const double* s1img = st.box + P.box_off + 2 * plane;
      const double* s2img = s1img + plane;
      // this lane's subset samples: FP64 deviations and image offsets from the
      // subset's top-left pixel (missing samples of the last slot: zero
      // weight, offset 0)
      double ev[MAXS];
      int off[MAXS];
      double es = 0.0;
      {
        const int dr = kWave / n1, dc = kWave - dr * n1;
        int r = lane / n1, c = lane - r * n1;
#pragma unroll
        for (int k = 0; k < MAXS; ++k) {
          const bool in = lane + kWave * k < n;
          const float fv = fimg[in ? r * W + c : 0];
          ev[k] = in ? (double)fv - fbar : 0.0;
          off[k] = in ? r * W + c : 0;
          es += ev[k];
          c += dc;
          r += dr;
          if (c >= n1) {
            c -= n1;
            ++r;
          }
        }
      }
      es = wave_sum_dpp(es);
      for (int k = lane; k < (side * side + 31) / 32; k += kWave) L.claim[k] = 0u;
      // the swarm's random numbers for this lane, all generations
      float4 ur[kPsoGenerations];
      {
        const float* up = rand + (int64_t)g * (kPsoGenerations * kPsoParticles * 4) +
                          (part ? lane : 0) * 4;
#pragma unroll
        for (int t = 0; t < kPsoGenerations; ++t)
          ur[t] = *reinterpret_cast<const float4*>(up + t * kPsoParticles * 4);
      }
      wave_lds_sync();

      // Eq. (1) at the cnt (1..4) listed window positions, by the whole wave;
      // -inf where the subset leaves the image, is not finite or is flat
      const auto coeff_batch = [&](const int* idx, int cnt, double* z) {
        const float* base[kBatch];
        bool adm[kBatch];
        double sg[kBatch], var[kBatch], acc[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
          const int id = idx[b < cnt ? b : 0];
          const int ky = id / side - S, kx = id - (ky + S) * side - S;
          const int cx = x0 + cu + kx, cy = y0 + cv + ky;
          adm[b] = cx - M >= 0 && cx + M <= W - 1 && cy - M >= 0 && cy + M <= H - 1;
          const int64_t o = adm[b] ? (int64_t)cy * W + cx : 0;
          sg[b] = s1img[o];
          const double sq = s2img[o];
          var[b] = sq - sg[b] * sg[b] * rnd;
          adm[b] = adm[b] && sq >= 0.0 && not_flat(var[b], sq);
          // an inadmissible position reads the POI's own subset instead (its
          // result is discarded), so every read stays inside the image
          base[b] = gimg + (adm[b] ? (int64_t)(cy - M) * W + (cx - M)
                                    : (int64_t)(y0 - M) * W + (x0 - M));
          acc[b] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < MAXS; ++k) {
          if (kWave * k >= n) break;
#pragma unroll
          for (int b = 0; b < kBatch; ++b)
            acc[b] = fma(ev[k], (double)base[b][off[k]], acc[b]);
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
          const double num = wave_sum_dpp(acc[b]) - sg[b] * rnd * es;
          z[b] = adm[b] ? num / (df * sqrt(var[b])) : -INFINITY;
        }
      };

      double qx = 0.0, qy = 0.0, vx = 0.0, vy = 0.0;
      if (part) {
        qx = pso_init(ur[0].x, Sd);
        qy = pso_init(ur[0].y, Sd);
        vx = pso_init(ur[0].z, Sd);
        vy = pso_init(ur[0].w, Sd);
      }
      double pbc = -INFINITY;
      int pbi = side * side, pbx = 0, pby = 0;
#pragma unroll 1
      for (int t = 0; t < kPsoGenerations; ++t) {
        // positions this particle needs: rint(q) clipped, and with the star
        // step its four neighbours inside the window
        const int kx = (int)fmin(fmax(rint(qx), -Sd), Sd);
        const int ky = (int)fmin(fmax(rint(qy), -Sd), Sd);
        int want[kPsoStar];
#pragma unroll
        for (int j = 0; j < kPsoStar; ++j) {
          const int sx = j == 1 ? 1 : j == 2 ? -1 : 0, sy = j == 3 ? 1 : j == 4 ? -1 : 0;
          const int nx = kx + sx, ny = ky + sy;
          const bool ok = part && (MOD || j == 0) && nx >= -S && nx <= S && ny >= -S && ny <= S;
          want[j] = ok ? (ny + S) * side + (nx + S) : -1;
        }
        // claim the positions not computed yet (one lane per position), list them
        int total = 0;
#pragma unroll
        for (int j = 0; j < kPsoStar; ++j) {
          const uint32_t bit = 1u << (want[j] & 31);
          const bool mine = want[j] >= 0 && !(atomicOr(&L.claim[want[j] >> 5], bit) & bit);
          const uint64_t b = __ballot(mine);
          if (mine) L.list[total + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                         __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u))] = want[j];
          total += __popcll(b);
        }
        evals += total;
        wave_lds_sync();
        for (int k0 = 0; k0 < total; k0 += kBatch) {
          int idx[kBatch];
#pragma unroll
          for (int b = 0; b < kBatch; ++b) idx[b] = uniform(L.list[k0 + (k0 + b < total ? b : 0)]);
          double z[kBatch];
          coeff_batch(idx, min(kBatch, total - k0), z);
          // every lane writes the same values
#pragma unroll
          for (int b = 0; b < kBatch; ++b)
            if (k0 + b < total) L.lut[idx[b]] = z[b];
        }
        wave_lds_sync();
        // the particle's coefficient(s), star step, personal best
        if (part) {
          double bc = L.lut[want[0]];
          int bi = want[0], bx = kx, by = ky;
          if (MOD) {
#pragma unroll
            for (int j = 1; j < kPsoStar; ++j) {
              if (want[j] < 0) continue;
              const double c = L.lut[want[j]];
              if (pso_better(c, want[j], bc, bi)) {
                bc = c;
                bi = want[j];
                bx = kx + (j == 1 ? 1 : j == 2 ? -1 : 0);
                by = ky + (j == 3 ? 1 : j == 4 ? -1 : 0);
              }
            }
            qx = (double)bx;
            qy = (double)by;
          }
          if (pso_better(bc, bi, pbc, pbi)) {
            pbc = bc;
            pbi = bi;
            pbx = bx;
            pby = by;
          }
        }
        // swarm best: the fold over the particles in index order.  When every
        // particle within the tie window of the maximum holds the same
        // position the fold ends there; otherwise it runs particle by particle.
        const double cmax = wave_max_f64(pbc);
        double gc = -INFINITY;
        int gi = side * side, gx = 0, gy = 0;
        if (cmax > -INFINITY) {
          const bool near = pbc >= cmax - 2.0 * kTieEps;
          const int lo = wave_min_int(near ? pbi : INT_MAX);
          const int hi = -wave_min_int(near ? -pbi : INT_MAX);
          if (lo == hi) {
            const uint64_t b = __ballot(near);
            const int first = (int)__builtin_ctzll(b);
            gc = readlane_f64(pbc, first);
            gi = lo;
            gx = __builtin_amdgcn_readlane(pbx, first);
            gy = __builtin_amdgcn_readlane(pby, first);
          } else {
            for (int i = 0; i < kPsoParticles; ++i) {
              const double c = readlane_f64(pbc, i);
              const int ii = __builtin_amdgcn_readlane(pbi, i);
              if (pso_better(c, ii, gc, gi)) {
                gc = c;
                gi = ii;
                gx = __builtin_amdgcn_readlane(pbx, i);
                gy = __builtin_amdgcn_readlane(pby, i);
              }
            }
          }
        }
        gbc = gc;
        gbx = gx;
        gby = gy;
        gens = t + 1;
        if ((gc > -INFINITY && gc >= kPsoStopCC) || t == kPsoGenerations - 1) break;
        // Eqs. (2)-(4)
        if (part) {
          const double w = 0.9 - (double)t / (2.0 * kPsoGenerations);
          float4 r = ur[1];
#pragma unroll
          for (int u = 2; u < kPsoGenerations; ++u)
            if (t + 1 == u) r = ur[u];
          const bool hp = pbc > -INFINITY, hg = gc > -INFINITY;
          pso_update(qx, vx, w, (double)r.x, (double)r.z, (double)pbx, hp, (double)gx, hg, Sd);
          pso_update(qy, vy, w, (double)r.y, (double)r.w, (double)pby, hp, (double)gy, hg, Sd);
        }
      }
      status = gbc > -INFINITY ? DIC_POI_OK : DIC_POI_NO_VALID_CANDIDATE;
      // the table of the next POI starts empty
      wave_lds_sync();
    }
    // every lane stores the same (wave-uniform) results
    const bool ok = status == DIC_POI_OK;
    uv_out[2 * g] = ok ? cu + gbx : 0;
    uv_out[2 * g + 1] = ok ? cv + gby : 0;
    zncc_out[g] = ok ? (float)gbc : nanf("");
    status_out[g] = status;
    if (gens_out) gens_out[g] = gens;
    if (evals_out) evals_out[g] = evals;
  }
}

template <bool MOD, int MAXS>
static hipError_t launch_pso_t(const DevState& st, const float* ref, const float* def,
                               const int32_t* poi, const int32_t* seed, const float* rand,
                               int32_t* uv, float* zn, int32_t* status, int32_t* gens,
                               int32_t* evals, int num_cu, hipStream_t s) {
  const size_t wl = pso_wave_lds(st.maxS, st.maxM);
  int waves = 4;
  while (waves > 1 && wl * waves > 64 * 1024) --waves;
  const size_t lds = wl * waves;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&pso_kernel<MOD, MAXS>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  int occ = 0;
  hipError_t e =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, pso_kernel<MOD, MAXS>, waves * kWave, lds);
  if (e != hipSuccess) return e;
  if (occ < 1) return hipErrorInvalidConfiguration;
  int64_t blocks = (int64_t)occ * num_cu;
  const int64_t need = (st.N + waves - 1) / waves;
  if (blocks > need) blocks = need;
  hipLaunchKernelGGL((pso_kernel<MOD, MAXS>), dim3((unsigned)blocks), dim3(waves * kWave), lds, s,
                     st, wl, ref, def, poi, seed, rand, uv, zn, status, gens, evals);
  return hipGetLastError();
}

hipError_t launch_pso(const DevState& st, bool modified, const float* ref, const float* def,
                      const int32_t* poi, const int32_t* seed, const float* rand, int32_t* uv,
                      float* zn, int32_t* status, int32_t* gens, int32_t* evals, int num_cu,
                      hipStream_t s) {
  if (st.N == 0) return hipSuccess;
  const int n = (2 * st.maxM + 1) * (2 * st.maxM + 1);
  const int need = (n + kWave - 1) / kWave;
#define DIC_PSO_CASE(S_)                                                                         \
  if (need <= S_)                                                                                \
    return modified ? launch_pso_t<true, S_>(st, ref, def, poi, seed, rand, uv, zn, status, gens, \
                                             evals, num_cu, s)                                    \
                    : launch_pso_t<false, S_>(st, ref, def, poi, seed, rand, uv, zn, status,      \
                                              gens, evals, num_cu, s);
  DIC_PSO_CASE(4)
  DIC_PSO_CASE(8)
  DIC_PSO_CASE(12)
  DIC_PSO_CASE(16)
  DIC_PSO_CASE(20)
  DIC_PSO_CASE(28)
#undef DIC_PSO_CASE
  return hipErrorInvalidValue;
}

}  // namespace dic
