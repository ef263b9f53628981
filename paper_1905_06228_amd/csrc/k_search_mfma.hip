// Brute-force integer search (Sec. 2.1, Eq. (1)) on the matrix cores:
// bf16 filter, FP64 decision.
//
// The cross terms C(dv, du) = sum_{r,c} t(r, c) g'(r + dv, c + du) of all
// candidates form a correlation, which per template row r is a product of
// two matrices: the window rows r..r+31 (32 x K, K running over window
// columns c') and a Toeplitz matrix B_r(c', du) = t(r, c' - du).  One wave
// per POI accumulates sum_r A_r B_r with v_mfma_f32_32x32x16_bf16 for the
// 32 x 32 candidates dv, du in [0, 32); a window of 33 x 33 candidates adds a
// second tile for dv, du in [1, 33) (its A operand is the next row's, loaded
// once for both tiles) and two corner candidates on the vector ALUs.
//
// Operands are rounded to bf16 (t and g' = g - c0 each to 8 significant
// bits, c0 the mean of the window's centre subset), so each product carries
// a relative error below 2^-7 + 3 * 2^-16 and the FP32 accumulation adds at
// most (terms) * 2^-24.  With Cauchy-Schwarz,
// sum |t| |g'| <= df * sqrt(sum g'^2), the approximate coefficient of every
// candidate is within
//   E = kappa * sqrt(sum g'^2 / sum (g - gbar)^2)
// of Eq. (1), kappa = 8.5e-3 covering all of the above with margin.  The
// exact maximum therefore lies in { c : s_c + E_c >= max_k (s_k - E_k) };
// those few candidates (about two per POI on speckle) are re-scored in FP64
// in index order and the tie rule picks the smallest row-major index within
// 1e-12 of the FP64 maximum: the same decision, and the same coefficient, as
// the FP64 definition.  Window sums come from the FP64 box-sum images.
//
// LDS per wave: the window in bf16 (rows padded to 16 KB + 8 elements so the
// 16-byte reads of 8 consecutive rows hit distinct banks) and the template in
// bf16 as two copies of dword pairs, even and odd phase, so that the 8
// consecutive elements a lane needs for its Toeplitz column start at a dword
// boundary in one of them (the odd copy sits 16 banks away from the even one).
#include "search_common.h"

namespace dic {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
// four floats at any 4-byte aligned global address (one dwordx4 load)
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));

constexpr float kBoundRel = 8.5e-3f;
constexpr int kXcds = 8;   // accelerator complex dies of the MI355X
constexpr int kMaskWords = 36;        // >= ceil(33 * 33 / 32)
constexpr int kMaskWordsWide = 128;   // >= ceil(64 * 64 / 32)

// Per-wave LDS layout for K-block count KB and subsets up to nmax wide; TT
// tiles of 32 candidates per direction (TT = 2: the window is 32 rows and
// columns wider).
struct MfmaLayout {
  int wpb;     // window row pitch (bf16 elements)
  int tpd;     // template row pitch (dwords)
  int win, te, to, mask, edge, total;   // byte offsets / size
};

__host__ __device__ __forceinline__ MfmaLayout mfma_layout(int KB, int nmax, int TT = 1) {
  MfmaLayout L;
  L.wpb = 16 * KB + 32 * (TT - 1) + 8;
  L.tpd = 8 * KB + 16;
  L.win = 0;
  const int wrows = nmax + 32 * TT;
  L.te = (wrows * L.wpb * 2 + 127) / 128 * 128;
  const int tbytes = nmax * L.tpd * 4;
  // odd copy 16 banks (64 bytes) past a 128-byte boundary after the even one
  L.to = (L.te + tbytes + 127) / 128 * 128 + 64;
  L.mask = L.to + tbytes;
  L.edge = L.mask + (TT == 2 ? kMaskWordsWide : kMaskWords) * 4;
  L.total = (L.edge + 64 * 4 + 15) / 16 * 16;
  return L;
}

__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  const __bf16 a = (__bf16)lo, b = (__bf16)hi;
  return (uint32_t)__builtin_bit_cast(uint16_t, a) |
         ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
}

__device__ __forceinline__ bf16x8 load_frag_aligned(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(p));
}

__device__ __forceinline__ bf16x8 load_frag_dwords(const uint32_t* p) {
  const u32x4 v = {p[0], p[1], p[2], p[3]};
  return __builtin_bit_cast(bf16x8, v);
}

// bf16 element x of a template row stored as even-phase dword pairs.
__device__ __forceinline__ float tmpl_elem(const uint32_t* row, int x) {
  const uint32_t d = row[x >> 1];
  return __builtin_bit_cast(float, (x & 1) ? (d & 0xffff0000u) : (d << 16));
}

// sum_r A_r B_r for tile A (dv, du in [0, 32)) and, with TWO, tile B
// (dv, du in [1, 33)).  Lane (n, kg) = (lane % 32, lane / 32).  Tile B's
// term for template row r - 1 pairs window rows r.. (tile B's dv is one
// larger) with the Toeplitz fragment of row r - 1 shifted by one column, so
// both tiles read the same window fragment A(r) at step r:
//   step r:  acc_a += A(r) B(r)      (r < n1)
//            acc_b += A(r) B'(r - 1) (r >= 1)
// The fragments of step r + 1 are requested before the products of step r,
// in two alternating register sets (no copies between steps).
template <int KB>
struct Frags {
  bf16x8 a[KB], b[KB], bp[KB];
};

template <int KB, bool TWO>
__device__ __forceinline__ void mfma_step(const bf16x8* a, const bf16x8* b, const bf16x8* bp,
                                          bool do_a, bool do_b, f32x16& acc_a, f32x16& acc_b) {
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    if (do_a) acc_a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[kb], b[kb], acc_a, 0, 0, 0);
    if (TWO && do_b)
      acc_b = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[kb], bp[kb], acc_b, 0, 0, 0);
  }
}

template <int KB, bool TWO>
__device__ __forceinline__ void correlate_tiles(const uint16_t* win, const uint32_t* te,
                                                const uint32_t* to, int n1, int wpb, int tpd,
                                                f32x16& acc_a, f32x16& acc_b) {
  const int lane = lane_id(), n = lane & 31, kg = lane >> 5;
  const uint16_t* arow = win + n * wpb + 8 * kg;
  const int o0 = 8 * kg - n + 32;   // Toeplitz phase of tile A's column du = n
  const int o1 = o0 - 1;            // tile B: du = n + 1
  const uint32_t* ba = ((o0 & 1) ? to : te) + (o0 >> 1);
  const uint32_t* bb = ((o1 & 1) ? to : te) + (o1 >> 1);
  // window rows r.. (r <= n1), template row rb for tile A and rp for tile B
  auto load = [&](Frags<KB>& f, int r, int rb, int rp) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      f.a[kb] = load_frag_aligned(arow + r * wpb + 16 * kb);
      f.b[kb] = load_frag_dwords(ba + rb * tpd + 8 * kb);
      if (TWO) f.bp[kb] = load_frag_dwords(bb + rp * tpd + 8 * kb);
    }
  };
  Frags<KB> x, y;
  load(x, 0, 0, 0);
  load(y, 1, min(1, n1 - 1), 0);
  mfma_step<KB, TWO>(x.a, x.b, x.bp, true, false, acc_a, acc_b);   // step 0
  // entering step r: y = (A(r), B(r), B'(r - 1))
  int r = 1;
  for (; r + 1 < n1; r += 2) {
    load(x, r + 1, r + 1, r);
    mfma_step<KB, TWO>(y.a, y.b, y.bp, true, true, acc_a, acc_b);
    load(y, r + 2, min(r + 2, n1 - 1), r + 1);
    mfma_step<KB, TWO>(x.a, x.b, x.bp, true, true, acc_a, acc_b);
  }
  if (r < n1) {   // r == n1 - 1: one full step, then the last tile-B step
    load(x, n1, n1 - 1, n1 - 1);
    mfma_step<KB, TWO>(y.a, y.b, y.bp, true, true, acc_a, acc_b);
    mfma_step<KB, TWO>(x.a, x.b, x.bp, false, true, acc_a, acc_b);
  } else {        // r == n1: y = (A(n1), -, B'(n1 - 1))
    mfma_step<KB, TWO>(y.a, y.b, y.bp, false, true, acc_a, acc_b);
  }
}

// Approximate coefficient of candidate (dv, du) of the window (row-major in
// [0, side)^2) from its cross term C and the window statistics st = (mean,
// 1/sqrt(sum (g - mean)^2)) of the box-sum pass, and its error bound E (the
// ratio sum g'^2 / sum (g - mean)^2 is 1 + n ((mean - c0) / sd)^2); -inf for
// an inadmissible or flat candidate.
struct ScoreCtx {
  int x0, y0, cu, cv, S, M, W, H, side;
  float c0, tsum, rdf, nn;
};

__device__ __forceinline__ float score_of(const ScoreCtx& q, float C, int dv, int du, float2 st,
                                          float& E) {
  const int dua = q.cu - q.S + du, dva = q.cv - q.S + dv;
  bool ok = dv < q.side && du < q.side && q.x0 + dua - q.M >= 0 && q.x0 + dua + q.M <= q.W - 1 &&
            q.y0 + dva - q.M >= 0 && q.y0 + dva + q.M <= q.H - 1 && st.y > 0.f;
  // sum t (g - mean) = sum t (g - c0) - (mean - c0) sum t
  const float dm = st.x - q.c0;
  const float sc = fmaf(-dm, q.tsum, C) * st.y * q.rdf;
  const float z = dm * st.y;
  ok = ok && isfinite(sc);
  E = ok ? kBoundRel * sqrtf(fmaf(q.nn * z, z, 1.f)) : 0.f;
  return ok ? sc : -INFINITY;
}

// Index of the box-sum pixel of candidate (dv, du), clamped into the image
// (a clamped candidate is inadmissible and its sums are not used).
__device__ __forceinline__ int64_t box_index(const ScoreCtx& q, int dv, int du) {
  const int x = min(max(q.x0 + q.cu - q.S + du, 0), q.W - 1);
  const int y = min(max(q.y0 + q.cv - q.S + dv, 0), q.H - 1);
  return (int64_t)y * q.W + x;
}

}  // namespace

size_t search_mfma_wave_lds(int kb, int maxM, bool wide) {
  const int nmax = min(16 * kb - 32, 2 * maxM + 1);
  return (size_t)mfma_layout(kb, nmax, wide ? 2 : 1).total;
}

// TT = 1: windows up to 33 x 33 candidates (one tile, or two sharing their
// window fragments for 33 x 33).  TT = 2: windows of 34..64 per side, covered
// by 2 x 2 tiles of 32 x 32 candidates at (dv, du) offsets (32a, 32b), each
// the TT = 1 product on the window shifted by 32a rows and 32b columns.
template <int KB, int TT>
__global__ void __launch_bounds__(64, 2) search_mfma_kernel(
    DevState st, const int32_t* __restrict__ work, int64_t count, int nmax,
    const float* __restrict__ tmpl_arena, const double* __restrict__ box,
    const float* __restrict__ ref, const float* __restrict__ def, const int32_t* __restrict__ poi,
    const int32_t* __restrict__ seed, int32_t* __restrict__ uv_out, float* __restrict__ zncc_out,
    int32_t* __restrict__ status_out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  const MfmaLayout Ly = mfma_layout(KB, nmax, TT);
  uint16_t* win = reinterpret_cast<uint16_t*>(lds_raw + Ly.win);
  uint32_t* te = reinterpret_cast<uint32_t*>(lds_raw + Ly.te);
  uint32_t* to = reinterpret_cast<uint32_t*>(lds_raw + Ly.to);
  uint32_t* mask = reinterpret_cast<uint32_t*>(lds_raw + Ly.mask);
  float* edge = reinterpret_cast<float*>(lds_raw + Ly.edge);
  const int lane = lane_id(), n = lane & 31, kg = lane >> 5;
  constexpr int WC = 16 * KB + 32 * (TT - 1);   // staged window columns
  constexpr int CPR = WC / 8;                   // 8-element chunks per window row
  constexpr int NMAX = 16 * KB - 32;            // widest subset of this K-block count
  constexpr int CH = ((NMAX + 32 * TT) * CPR + kWave - 1) / kWave;   // window chunks per lane
  constexpr int TPD = 8 * KB + 16;
  constexpr int TG = (TPD - 16) / 2;   // 4-column groups of a template row past the left pad
  constexpr int TQ = NMAX / 4;         // the groups a template of this K-block count can fill
  constexpr int TQL = (NMAX * TQ + kWave - 1) / kWave;   // such groups per lane
  static_assert(TQ <= TG, "template groups exceed the row");
  const int wpb = Ly.wpb;
  // both template copies zero, once: the 32 elements left of every row and
  // the groups past TQ stay zero; a POI rewrites groups 0..TQ-1 of its rows
  for (int idx = lane; idx < nmax * TPD; idx += kWave) {
    te[idx] = 0u;
    to[idx] = 0u;
  }

  // Static assignment: every POI costs about the same, and a device-wide
  // counter would serialise an atomic per POI across the XCDs.  Workgroups
  // are dispatched round-robin over the XCDs, so with a grid that is a
  // multiple of kXcds, XCD x takes the x-th contiguous part of the work list
  // (neighbouring POIs, whose windows and box sums then share its L2).
  int64_t item, end, step;
  if (gridDim.x % kXcds == 0) {
    const int x = blockIdx.x % kXcds, per = gridDim.x / kXcds;
    item = count * x / kXcds + blockIdx.x / kXcds;
    end = count * (x + 1) / kXcds;
    step = per;
  } else {
    item = blockIdx.x;
    end = count;
    step = gridDim.x;
  }
  for (; item < end; item += step) {
    const int g = uniform(work[item]);
    const DevPair P = st.pairs[uniform(st.poi_pair[g])];
    const RefRec* R = st.recs + g;
    const int x0 = uniform(poi[2 * g]), y0 = uniform(poi[2 * g + 1]);
    const int cu = seed ? uniform(seed[2 * g]) : 0;
    const int cv = seed ? uniform(seed[2 * g + 1]) : 0;
    const int rstat = uniform(R->status);
    if (rstat != DIC_POI_OK && rstat != DIC_POI_SINGULAR_HESSIAN) {
      if (lane == 0) {
        uv_out[2 * g] = 0;
        uv_out[2 * g + 1] = 0;
        zncc_out[g] = nanf("");
        status_out[g] = rstat;
      }
      continue;
    }
    const int M = P.M, S = P.S, n1 = 2 * M + 1, nn = n1 * n1, side = 2 * S + 1;
    const int W = P.width, H = P.height, K = side * side;
    const float* gimg = def + P.def_off;
    const float* fimg = ref + P.ref_off;
    const int64_t plane = (int64_t)W * H;
    const double* s1img = box + P.box_off + 2 * plane;
    const float2* stimg = reinterpret_cast<const float2*>(box + P.box_off + 4 * plane);
    // The window is staged as g - c0 in bf16: c0 is the mean of the subset at
    // the window centre (clamped into the image) when that subset is
    // admissible and not flat, so the staged values, and the bound E, stay
    // small whatever the window's offset against the reference; else the
    // reference mean.
    float c0 = (float)R->fbar;
    {
      const float2 sc = stimg[(int64_t)min(max(y0 + cv, 0), H - 1) * W +
                              min(max(x0 + cu, 0), W - 1)];
      if (sc.y > 0.f && isfinite(sc.x)) c0 = sc.x;
    }
    const int wx0 = x0 + cu - S - M, wy0 = y0 + cv - S - M;
    const int wn = n1 + side - 1;   // real window side
    const int wrows = n1 + 32 * TT;   // staged rows (a tile reads up to 32 (TT - 1) + n1 + 31)
    const bool two = side == 33;
    ScoreCtx q;
    q.x0 = x0; q.y0 = y0; q.cu = cu; q.cv = cv; q.S = S; q.M = M; q.W = W; q.H = H;
    q.side = side;
    q.c0 = c0;
    q.tsum = R->tsum;
    q.rdf = (float)(1.0 / R->df);
    q.nn = (float)nn;

    // 0. the template t = f - fbar of the reference subset (rounded as
    //    f - (float)fbar, the values whose sum is the record's tsum), as
    //    4-column groups of its rows, requested at once; columns past the
    //    subset are zero.  A group whose four pixels lie in the image row is
    //    one 16-byte load; one reaching past the image's last column (only
    //    past the subset's) loads its subset columns alone.
    const float fb = (float)R->fbar;
    const float* fsub = fimg + (int64_t)(y0 - M) * W + (x0 - M);
    float4 tv[TQL];
#pragma unroll
    for (int k = 0; k < TQL; ++k) {
      const int idx = lane + k * kWave, r = idx / TQ, qq = idx - r * TQ, c = 4 * qq;
      const bool in = idx < n1 * TQ && c < n1;
      const float* src = fsub + (int64_t)(in ? r : 0) * W + (in ? c : 0);
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (in) {
        if (x0 - M + c + 3 <= W - 1) {
          const f32x4u a = *reinterpret_cast<const f32x4u*>(src);
          v = make_float4(a.x, a.y, a.z, a.w);
        } else {
          v.x = src[0];
          if (c + 1 < n1) v.y = src[1];
          if (c + 2 < n1) v.z = src[2];
          if (c + 3 < n1) v.w = src[3];
        }
      }
      tv[k] = make_float4(c < n1 ? v.x - fb : 0.f, c + 1 < n1 ? v.y - fb : 0.f,
                          c + 2 < n1 ? v.z - fb : 0.f, c + 3 < n1 ? v.w - fb : 0.f);
      if (!in) tv[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    }

    wave_lds_sync();   // the previous POI's LDS reads are complete
    // 1. template rows in bf16 after 32 zeros: element x of row r is
    //    t(r, x - 32); the even copy holds pairs (2i, 2i+1), the odd copy
    //    (2i+1, 2i+2).  A group's odd pair (3, 4) takes element 4 from the
    //    next group, which the next lane holds.
#pragma unroll
    for (int k = 0; k < TQL; ++k) {
      const int idx = lane + k * kWave, r = idx / TQ, qq = idx - r * TQ;
      const float4 v = tv[k];
      float nxt = __builtin_bit_cast(
          float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v.x), 0x130, 0xF, 0xF, true));
      if (k + 1 < TQL) {
        const float x1 = tv[k + 1 < TQL ? k + 1 : k].x;
        const float lane0 = __builtin_bit_cast(
            float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x1), 0));
        if (lane == kWave - 1) nxt = lane0;
      }
      if (qq == TQ - 1) nxt = 0.f;
      if (idx < n1 * TQ) {
        const int base = r * TPD + 16 + 2 * qq;
        *reinterpret_cast<uint2*>(te + base) = make_uint2(pack_bf16(v.x, v.y), pack_bf16(v.z, v.w));
        *reinterpret_cast<uint2*>(to + base) = make_uint2(pack_bf16(v.y, v.z), pack_bf16(v.w, nxt));
        if (qq == 0) to[base - 1] = pack_bf16(0.f, v.x);
      }
    }
    if constexpr (TT == 2) {
      mask[lane] = 0u;
      mask[lane + kWave] = 0u;
    } else {
      if (lane < kMaskWords) mask[lane] = 0u;
    }
    // 2. window g - c0 in bf16, CB chunks of 8 columns per lane at a time;
    //    outside the window or the image, and non-finite pixels, are 0 (their
    //    candidates are invalid by the box sums).  A window whose staged
    //    rows and columns all lie in the image (the usual case) is read as
    //    two 16-byte loads per chunk; otherwise every element's address is
    //    clamped into the image.
    const bool interior = wx0 >= 0 && wx0 + WC <= W && wy0 >= 0 && wy0 + wrows <= H;
    auto store_chunk = [&](int k, const float* v) {
      const int idx = lane + k * kWave;
      const int rr = idx / CPR, ch = idx - rr * CPR;
      if (k < CH && rr < wrows) {
        const int Y = wy0 + rr;
        const bool rowok = rr < wn && (interior || (Y >= 0 && Y < H));
        float w[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int col = ch * 8 + e, X = wx0 + col;
          const float x = v[e];
          w[e] = (rowok && col < wn && (interior || (X >= 0 && X < W)) && isfinite(x)) ? x - c0
                                                                                     : 0.f;
        }
        const u32x4 pk = {pack_bf16(w[0], w[1]), pack_bf16(w[2], w[3]), pack_bf16(w[4], w[5]),
                          pack_bf16(w[6], w[7])};
        *reinterpret_cast<u32x4*>(win + rr * wpb + ch * 8) = pk;
      }
    };
    // an interior window's chunks are all requested at once when they fit in
    // registers (one memory round trip)
    constexpr int CBI = CH <= 8 ? CH : 4;
    if (interior) {
#pragma unroll
      for (int k0 = 0; k0 < CH; k0 += CBI) {
        float v[CBI][8];
#pragma unroll
        for (int kk = 0; kk < CBI; ++kk) {
          const int idx = lane + (k0 + kk) * kWave;
          const int rr = idx / CPR, ch = idx - rr * CPR;
          // rows past the staged ones (not stored) read the last staged row
          const f32x4u* src = reinterpret_cast<const f32x4u*>(
              gimg + (int64_t)(wy0 + min(rr, wrows - 1)) * W + wx0 + ch * 8);
          const f32x4u a = src[0], b = src[1];
          v[kk][0] = a.x; v[kk][1] = a.y; v[kk][2] = a.z; v[kk][3] = a.w;
          v[kk][4] = b.x; v[kk][5] = b.y; v[kk][6] = b.z; v[kk][7] = b.w;
        }
#pragma unroll
        for (int kk = 0; kk < CBI; ++kk) store_chunk(k0 + kk, v[kk]);
      }
    } else {
      constexpr int CB = 4;
#pragma unroll
      for (int k0 = 0; k0 < CH; k0 += CB) {
        float v[CB][8];
#pragma unroll
        for (int kk = 0; kk < CB; ++kk) {
          const int idx = lane + (k0 + kk) * kWave;
          const int rr = idx / CPR, ch = idx - rr * CPR;
          const int Yc = min(max(wy0 + rr, 0), H - 1);
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int Xc = min(max(wx0 + ch * 8 + e, 0), W - 1);
            v[kk][e] = gimg[(int64_t)Yc * W + Xc];
          }
        }
#pragma unroll
        for (int kk = 0; kk < CB; ++kk) store_chunk(k0 + kk, v[kk]);
      }
    }
    wave_lds_sync();

    // 3.-5. cross terms on the matrix cores, approximate coefficients and
    //    their bounds, and the bit set of the candidates that may hold the
    //    FP64 maximum
    float tau = -INFINITY;
    if constexpr (TT == 1) {
      // 3. cross terms on the matrix cores
      f32x16 acc_a = {}, acc_b = {};
      if (two)
        correlate_tiles<KB, true>(win, te, to, n1, wpb, TPD, acc_a, acc_b);
      else
        correlate_tiles<KB, false>(win, te, to, n1, wpb, TPD, acc_a, acc_b);
      // box sums of every candidate this lane scores, requested at once: 16 of
      // tile A, then one edge candidate of tile B (lanes 0..62) or the two
      // corners (lane 63); their latency overlaps the corner sums below
      float2 sta[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) sta[j] = stimg[box_index(q, (j & 3) + 8 * (j >> 2) + 4 * kg, n)];
      // edge candidates: lane b < 32 -> (32, b + 1); 32 <= b < 63 -> (b - 31, 32);
      // lane 63 -> corners (32, 0) and (0, 32)
      const int e0v = lane < 32 ? 32 : lane < 63 ? lane - 31 : 32;
      const int e0u = lane < 32 ? lane + 1 : lane < 63 ? 32 : 0;
      const int e1v = 0, e1u = 32;
      const float2 ste0 = stimg[box_index(q, e0v, e0u)];
      const float2 ste1 = stimg[box_index(q, e1v, e1u)];

      // the two corners on the vector ALUs
      float cr1 = 0.f, cr2 = 0.f;   // corners (dv, du) = (32, 0) and (0, 32)
      if (two) {
        double s_a = 0.0, s_b = 0.0;
        const int dr = kWave / n1, dc = kWave - dr * n1;
        int r = lane / n1, c = lane - r * n1;
#pragma unroll 4
        for (int k = lane; k < nn; k += kWave) {
          const double t = (double)tmpl_elem(te + r * TPD, c + 32);
          s_a += t * (double)__builtin_bit_cast(float, (uint32_t)win[(r + 32) * wpb + c] << 16);
          s_b += t * (double)__builtin_bit_cast(float, (uint32_t)win[r * wpb + c + 32] << 16);
          c += dc;
          r += dr;
          if (c >= n1) {
            c -= n1;
            ++r;
          }
        }
        cr1 = (float)wave_sum_dpp(s_a);
        cr2 = (float)wave_sum_dpp(s_b);
        // tile B's edge row dv = 32 and column du = 32, one value per lane
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int i = (j & 3) + 8 * (j >> 2) + 4 * kg;
          if (i == 31) edge[n] = acc_b[j];               // (32, n + 1)
          else if (n == 31) edge[32 + i] = acc_b[j];     // (i + 1, 32), i < 31
        }
        wave_lds_sync();
      }

      // 4. approximate coefficients, their bounds, and the threshold
      float sa[16], ea[16];
      float lo = -INFINITY;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int i = (j & 3) + 8 * (j >> 2) + 4 * kg;
        sa[j] = score_of(q, acc_a[j], i, n, sta[j], ea[j]);
        lo = fmaxf(lo, sa[j] - ea[j]);
      }
      float s0 = -INFINITY, e0 = 0.f, s1 = -INFINITY, e1 = 0.f;
      if (two) {
        const float c_e0 = lane < 63 ? edge[lane] : cr1;
        s0 = score_of(q, c_e0, e0v, e0u, ste0, e0);
        if (lane == 63) s1 = score_of(q, cr2, e1v, e1u, ste1, e1);
        lo = fmaxf(lo, fmaxf(s0 - e0, s1 - e1));
      }
      tau = wave_max_dpp(lo);
      if (tau > -INFINITY) {
#pragma unroll
        for (int j = 0; j < 16; ++j)
          if (sa[j] + ea[j] >= tau) {
            const int cand = ((j & 3) + 8 * (j >> 2) + 4 * kg) * side + n;
            atomicOr(&mask[cand >> 5], 1u << (cand & 31));
          }
        if (s0 + e0 >= tau) {
          const int cand = e0v * side + e0u;
          atomicOr(&mask[cand >> 5], 1u << (cand & 31));
        }
        if (s1 + e1 >= tau) {
          const int cand = e1v * side + e1u;
          atomicOr(&mask[cand >> 5], 1u << (cand & 31));
        }
      }
    } else {
      // 2 x 2 tiles, the one holding the window centre first.  The running
      // threshold only grows, so a tile's bits (set against the threshold
      // after it) are a superset of those the final threshold selects; the
      // FP64 re-score decides among them.
      float lo = -INFINITY;
#pragma unroll 1
      for (int t = 0; t < 4; ++t) {
        const int a = t >> 1, b = t & 1;
        if (32 * a >= side || 32 * b >= side) continue;
        f32x16 acc = {}, acc_unused = {};
        correlate_tiles<KB, false>(win + 32 * a * wpb + 32 * b, te, to, n1, wpb, TPD, acc,
                                   acc_unused);
        float2 stt[16];
#pragma unroll
        for (int j = 0; j < 16; ++j)
          stt[j] = stimg[box_index(q, 32 * a + (j & 3) + 8 * (j >> 2) + 4 * kg, 32 * b + n)];
        float st_s[16], st_e[16];
        float l = lo;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int i = 32 * a + (j & 3) + 8 * (j >> 2) + 4 * kg;
          st_s[j] = score_of(q, acc[j], i, 32 * b + n, stt[j], st_e[j]);
          l = fmaxf(l, st_s[j] - st_e[j]);
        }
        lo = wave_max_dpp(l);
        if (lo > -INFINITY) {
#pragma unroll
          for (int j = 0; j < 16; ++j)
            if (st_s[j] + st_e[j] >= lo) {
              const int cand = (32 * a + (j & 3) + 8 * (j >> 2) + 4 * kg) * side + 32 * b + n;
              atomicOr(&mask[cand >> 5], 1u << (cand & 31));
            }
        }
      }
      tau = lo;
    }

    // the list of the bit set's members in index order (lane e holds the e-th)
    int pick = -1;
    double best = -INFINITY;
    if (tau > -INFINITY) {
      wave_lds_sync();
      constexpr int kHalves = TT == 2 ? 2 : 1;   // mask words per lane
      const int words = (K + 31) / 32;
      uint32_t myword[kHalves];
      uint64_t nonempty[kHalves];
#pragma unroll
      for (int h = 0; h < kHalves; ++h) {
        const int wi = kWave * h + lane;
        myword[h] = wi < words ? mask[wi] : 0u;
        nonempty[h] = __ballot(myword[h] != 0u);
      }
      int count = 0, mycand = 0;
#pragma unroll
      for (int h = 0; h < kHalves; ++h)
        for (uint64_t ws = nonempty[h]; ws; ws &= ws - 1) {
          const int w = __builtin_ctzll(ws);
          for (uint32_t bits = (uint32_t)__builtin_amdgcn_readlane((int)myword[h], w); bits;
               bits &= bits - 1) {
            if (lane == count) mycand = 32 * (kWave * h + w) + __builtin_ctz(bits);
            ++count;
          }
        }

      // 6. FP64 re-score, two candidates per pass over the subset; the
      //    first candidate in index order within 1e-12 of the maximum wins.
      //    Members past the 64th (many exact ties) are walked in the bit set.
      const double fbar = R->fbar, dfd = R->df;
      auto centre = [&](int cand, int& xg, int& yg) {
        const int rr = cand / side, cc = cand - rr * side;
        xg = x0 + cu - S + cc;
        yg = y0 + cv - S + rr;
      };
      auto rescore1 = [&](int cand) -> double {
        int xg, yg;
        centre(cand, xg, yg);
        double z;
        rescore_wave<1>(fimg, gimg, W, x0, y0, &xg, &yg, 1, M, fbar, dfd, s1img, &z);
        return z;
      };
      // calls fn(cand) for the members past the 64th, in index order, while it returns true
      auto walk_rest = [&](auto&& fn) {
        int e = 0;
#pragma unroll
        for (int h = 0; h < kHalves; ++h)
          for (uint64_t ws = nonempty[h]; ws; ws &= ws - 1) {
            const int w = __builtin_ctzll(ws);
            for (uint32_t bits = (uint32_t)__builtin_amdgcn_readlane((int)myword[h], w); bits;
                 bits &= bits - 1, ++e)
              if (e >= kWave && !fn(32 * (kWave * h + w) + __builtin_ctz(bits))) return;
          }
      };
      const int listed = min(count, kWave);
      double keep = -INFINITY, cmax = -INFINITY;
      constexpr int kB = 2;
      for (int e0 = 0; e0 < listed; e0 += kB) {
        const int nb = min(kB, listed - e0);
        int xs[kB], ys[kB];
#pragma unroll
        for (int b = 0; b < kB; ++b)
          centre(__builtin_amdgcn_readlane(mycand, e0 + min(b, nb - 1)), xs[b], ys[b]);
        double z[kB];
        rescore_wave<kB>(fimg, gimg, W, x0, y0, xs, ys, nb, M, fbar, dfd, s1img, z);
#pragma unroll
        for (int b = 0; b < kB; ++b)
          if (b < nb) {
            if (lane == e0 + b) keep = z[b];
            cmax = fmax(cmax, z[b]);
          }
      }
      if (count > listed)
        walk_rest([&](int cand) {
          cmax = fmax(cmax, rescore1(cand));
          return true;
        });
      if (cmax > -INFINITY) {
        const uint64_t hit = __ballot(lane < listed && keep >= cmax - 1e-12);
        if (hit) {
          const int e = __builtin_ctzll(hit);
          pick = __builtin_amdgcn_readlane(mycand, e);
          best = readlane_f64(keep, e);
        } else {
          walk_rest([&](int cand) {
            const double z = rescore1(cand);
            if (z >= cmax - 1e-12) {
              pick = cand;
              best = z;
              return false;
            }
            return true;
          });
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
        const int rr = pick / side, cc = pick - rr * side;
        uv_out[2 * g] = cu - S + cc;
        uv_out[2 * g + 1] = cv - S + rr;
        zncc_out[g] = (float)best;
        status_out[g] = DIC_POI_OK;
      }
    }
  }
}

template <int KB, int TT>
static hipError_t launch_search_mfma_kb(const DevState& st, const SearchGroup& gr, int occ_cap,
                                        const float* ref, const float* def, const int32_t* poi,
                                        const int32_t* seed, int32_t* uv, float* zncc,
                                        int32_t* status, int num_cu, hipStream_t s) {
  const int nmax = min(16 * KB - 32, 2 * st.maxM + 1);
  const size_t lds = search_mfma_wave_lds(KB, st.maxM, TT == 2);
  const void* fn = reinterpret_cast<const void*>(&search_mfma_kernel<KB, TT>);
  if (lds > 65536) {
    hipError_t ea = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (ea != hipSuccess) return ea;
  }
  int occ = 0;
  hipError_t e =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, search_mfma_kernel<KB, TT>, kWave, lds);
  if (e != hipSuccess) return e;
  if (occ < 1) return hipErrorInvalidConfiguration;
  if (occ_cap > 0 && occ > occ_cap) occ = occ_cap;
  int64_t blocks = (int64_t)occ * num_cu;
  if (blocks > gr.count) blocks = gr.count;
  if (blocks >= kXcds) blocks -= blocks % kXcds;
  hipLaunchKernelGGL((search_mfma_kernel<KB, TT>), dim3((unsigned)blocks), dim3(kWave), lds, s,
                     st, st.work + gr.begin, gr.count, nmax, st.tmpl, st.box, ref, def, poi, seed,
                     uv, zncc, status);
  return hipGetLastError();
}

template <int TT>
static hipError_t launch_search_mfma_tt(const DevState& st, const dic_tuning_t& tu,
                                        const SearchGroup* groups, int ngroups, const float* ref,
                                        const float* def, const int32_t* poi,
                                        const int32_t* seed, int32_t* uv, float* zncc,
                                        int32_t* status, int num_cu, hipStream_t s) {
  for (int k = 0; k < ngroups; ++k) {
    const SearchGroup& gr = groups[k];
    if (gr.count == 0) continue;
    hipError_t e = hipErrorInvalidValue;
    if (gr.np == 3)
      e = launch_search_mfma_kb<3, TT>(st, gr, tu.search_occupancy, ref, def, poi, seed, uv,
                                       zncc, status, num_cu, s);
    else if (gr.np == 4)
      e = launch_search_mfma_kb<4, TT>(st, gr, tu.search_occupancy, ref, def, poi, seed, uv,
                                       zncc, status, num_cu, s);
    else if (gr.np == 5)
      e = launch_search_mfma_kb<5, TT>(st, gr, tu.search_occupancy, ref, def, poi, seed, uv,
                                       zncc, status, num_cu, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_search_mfma(const DevState& st, const dic_tuning_t& tu,
                              const SearchGroup* groups, int ngroups, const float* ref,
                              const float* def, const int32_t* poi, const int32_t* seed,
                              int32_t* uv, float* zncc, int32_t* status, int num_cu,
                              hipStream_t s) {
  if (ngroups > kMaxSearchGroups || st.maxS > kMfmaWideMaxS) return hipErrorInvalidValue;
  // windows beyond +-kMfmaMaxS in the plan: every POI takes the 2 x 2 tile form
  if (st.maxS > kMfmaMaxS)
    return launch_search_mfma_tt<2>(st, tu, groups, ngroups, ref, def, poi, seed, uv, zncc,
                                    status, num_cu, s);
  return launch_search_mfma_tt<1>(st, tu, groups, ngroups, ref, def, poi, seed, uv, zncc, status,
                                  num_cu, s);
}

}  // namespace dic
