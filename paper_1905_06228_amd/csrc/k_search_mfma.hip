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
//   kappa * sqrt(sum g'^2 / sum (g - gbar)^2) <= E
// of Eq. (1), kappa = 8.5e-3 covering all of the above with margin and E its
// square-root-free upper bound (Scorer below).  The exact maximum therefore
// lies in { c : s_c + E_c >= max_k (s_k - E_k) }; those few candidates (about
// two per POI on speckle) are re-scored in FP64 in index order and the tie
// rule picks the smallest row-major index within 1e-12 of the FP64 maximum:
// the same decision, and the same coefficient, as the FP64 definition.
// Window sums come from the FP64 box-sum images.
//
// LDS per wave: the window in bf16 (rows padded to 16 KB + 8 elements so the
// 16-byte reads of 8 consecutive rows hit distinct banks) and the template in
// bf16 as two copies of dword pairs, even and odd phase, so that the 8
// consecutive elements a lane needs for its Toeplitz column start at a dword
// boundary in one of them (the odd copy sits 16 banks away from the even one).
// A template row is 32 zeros, then the subset row, then zeros, 16 KB elements
// in all; a Toeplitz read reaches up to 31 elements past its row, into the
// next row's leading zeros (a zero tail follows the last row).
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

// Per-wave LDS layout for K-block count KB and subsets up to nmax wide; TT
// tiles of 32 candidates per direction (TT = 2: the window is 32 columns
// wider; the rows of one tile row of candidates are staged at a time).
struct MfmaLayout {
  int wpb;     // window row pitch (bf16 elements)
  int tpd;     // template row pitch (dwords; rows overlap, see above)
  int win, te, to, edge, total;   // byte offsets / size
};

__host__ __device__ __forceinline__ MfmaLayout mfma_layout(int KB, int nmax, int TT = 1) {
  MfmaLayout L;
  L.wpb = 16 * KB + 32 * (TT - 1) + 8;
  L.tpd = 8 * KB;
  L.win = 0;
  const int wrows = nmax + 32;   // one tile row of candidates (see the kernel)
  L.te = (wrows * L.wpb * 2 + 127) / 128 * 128;
  const int tbytes = (nmax * L.tpd + 16) * 4;   // rows, then the zero tail
  // odd copy 16 banks (64 bytes) past a 128-byte boundary after the even one
  L.to = (L.te + tbytes + 127) / 128 * 128 + 64;
  L.edge = L.to + tbytes;
  L.total = (L.edge + 64 * 4 + 15) / 16 * 16;
  return L;
}

__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  const __bf16 a = (__bf16)lo, b = (__bf16)hi;
  return (uint32_t)__builtin_bit_cast(uint16_t, a) |
         ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
}

// w with lane L (wave-uniform) replaced by the wave-uniform value val
__device__ __forceinline__ uint32_t put_lane(uint32_t w, uint32_t val, int L) {
  return __builtin_amdgcn_inverse_ballot_w64(1ull << L) ? val : w;
}

__device__ __forceinline__ float bf16_bits(uint16_t v) {
  return __builtin_bit_cast(float, (uint32_t)v << 16);
}

__device__ __forceinline__ bf16x8 load_frag_aligned(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(p));
}

__device__ __forceinline__ bf16x8 load_frag_dwords(const uint32_t* p) {
  const u32x4 v = {p[0], p[1], p[2], p[3]};
  return __builtin_bit_cast(bf16x8, v);
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

// `last`: the last K block takes part (see correlate_tiles).
template <int KB, bool TWO>
__device__ __forceinline__ void mfma_step(const bf16x8* a, const bf16x8* b, const bf16x8* bp,
                                          bool do_a, bool do_b, bool last, f32x16& acc_a,
                                          f32x16& acc_b) {
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    if (kb == KB - 1 && !last) break;
    if (do_a) acc_a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[kb], b[kb], acc_a, 0, 0, 0);
    if (TWO && do_b)
      acc_b = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[kb], bp[kb], acc_b, 0, 0, 0);
  }
}

// ncols (TRIM): the tile's candidate columns that are used (du < ncols; the
// others are outside the window).  Column du meets template entries only at
// window columns du .. du + n1 - 1, so when ncols - 1 + n1 <= 16 (KB - 1)
// the last K block adds exact zeros to every used column (the staged window
// is finite) and is skipped, with its fragment reads.  Used for a single
// tile (windows up to 32 candidates a side) and the 2 x 2 tile form's second
// tile column; the two-tile 33 x 33 form needs every block.
template <int KB, bool TWO, bool TRIM>
__device__ __forceinline__ void correlate_tiles(const uint16_t* win, const uint32_t* te,
                                                const uint32_t* to, int n1, int wpb, int tpd,
                                                int lane, int ncols, f32x16& acc_a,
                                                f32x16& acc_b) {
  const bool last = !TRIM || ncols - 1 + n1 > 16 * (KB - 1);
  const int n = lane & 31, kg = lane >> 5;
  const uint16_t* arow = win + n * wpb + 8 * kg;
  const int o0 = 8 * kg - n + 32;   // Toeplitz phase of tile A's column du = n
  const int o1 = o0 - 1;            // tile B: du = n + 1
  const uint32_t* ba = ((o0 & 1) ? to : te) + (o0 >> 1);
  const uint32_t* bb = ((o1 & 1) ? to : te) + (o1 >> 1);
  // window rows r.. (r <= n1), template row rb for tile A and rp for tile B
  auto load = [&](Frags<KB>& f, int r, int rb, int rp) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      if (kb == KB - 1 && !last) break;
      f.a[kb] = load_frag_aligned(arow + r * wpb + 16 * kb);
      f.b[kb] = load_frag_dwords(ba + rb * tpd + 8 * kb);
      if (TWO) f.bp[kb] = load_frag_dwords(bb + rp * tpd + 8 * kb);
    }
  };
  Frags<KB> x, y;
  load(x, 0, 0, 0);
  load(y, 1, min(1, n1 - 1), 0);
  mfma_step<KB, TWO>(x.a, x.b, x.bp, true, false, last, acc_a, acc_b);   // step 0
  // entering step r: y = (A(r), B(r), B'(r - 1))
  int r = 1;
  for (; r + 1 < n1; r += 2) {
    load(x, r + 1, r + 1, r);
    mfma_step<KB, TWO>(y.a, y.b, y.bp, true, true, last, acc_a, acc_b);
    load(y, r + 2, min(r + 2, n1 - 1), r + 1);
    mfma_step<KB, TWO>(x.a, x.b, x.bp, true, true, last, acc_a, acc_b);
  }
  if (r < n1) {   // r == n1 - 1: one full step, then the last tile-B step
    load(x, n1, n1 - 1, n1 - 1);
    mfma_step<KB, TWO>(y.a, y.b, y.bp, true, true, last, acc_a, acc_b);
    mfma_step<KB, TWO>(x.a, x.b, x.bp, false, true, last, acc_a, acc_b);
  } else {        // r == n1: y = (A(n1), -, B'(n1 - 1))
    mfma_step<KB, TWO>(y.a, y.b, y.bp, false, true, last, acc_a, acc_b);
  }
}

// Candidates of the window, (dv, du) row-major in [0, side)^2, centred at
// (bx + du, by + dv); those in [dv_lo, dv_hi] x [du_lo, du_hi] have their
// subset inside the image; `inside` when that is the whole window.
struct CandBox {
  int bx, by, side;
  int du_lo, du_hi, dv_lo, dv_hi;
  bool inside;
};

__device__ __forceinline__ CandBox cand_box(int bx, int by, int side, int M, int W, int H) {
  CandBox c;
  c.bx = bx;
  c.by = by;
  c.side = side;
  c.du_lo = max(0, M - bx);
  c.du_hi = min(side - 1, W - 1 - M - bx);
  c.dv_lo = max(0, M - by);
  c.dv_hi = min(side - 1, H - 1 - M - by);
  c.inside = c.du_lo == 0 && c.dv_lo == 0 && c.du_hi == side - 1 && c.dv_hi == side - 1;
  return c;
}

__device__ __forceinline__ bool admissible(const CandBox& c, int dv, int du) {
  return dv >= c.dv_lo && dv <= c.dv_hi && du >= c.du_lo && du <= c.du_hi;
}

// Box-sum pixel of candidate (dv, du) of the window, clamped into the image
// (a clamped candidate is inadmissible and its sums are not used).
__device__ __forceinline__ int64_t box_index(const CandBox& c, int dv, int du, int W, int H) {
  const int x = min(max(c.bx + du, 0), W - 1);
  const int y = min(max(c.by + dv, 0), H - 1);
  return (int64_t)y * W + x;
}

// Box-sum statistics of the 16 candidates (a0 + i, b0 + n) a lane holds in a
// 32 x 32 tile, i = (j & 3) + 8 (j >> 2) + 4 kg; positions past the window
// read its last row or column.
__device__ __forceinline__ void tile_stats(const CandBox& c, const float2* __restrict__ stimg,
                                           int W, int H, int a0, int b0, int lane, float2* out) {
  const int n = lane & 31, kg = lane >> 5;
  if (c.inside) {
    const int du = min(b0 + n, c.side - 1);
    if (a0 + 32 <= c.side) {
      // row offsets j -> ((j & 3) + 8 (j >> 2)) W are wave-uniform
      const float2* sb = stimg + (int64_t)(c.by + a0) * W + (c.bx + du) + 4 * kg * W;
#pragma unroll
      for (int j = 0; j < 16; ++j) out[j] = sb[(int64_t)((j & 3) + 8 * (j >> 2)) * W];
    } else {
      const float2* sb = stimg + (int64_t)c.by * W + (c.bx + du);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int dv = min(a0 + (j & 3) + 8 * (j >> 2) + 4 * kg, c.side - 1);
        out[j] = sb[__umul24((uint32_t)dv, (uint32_t)W)];
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < 16; ++j)
      out[j] = stimg[box_index(c, a0 + (j & 3) + 8 * (j >> 2) + 4 * kg, b0 + n, W, H)];
  }
}

// Approximate coefficient of a candidate from its cross term C and the
// window statistics st = (mean, 1/sqrt(sum (g - mean)^2)) of the box-sum
// pass, returned as the interval [lo, hi] = coefficient -+ E that holds the
// coefficient of Eq. (1).  E = kappa (1 + n1 |mean - c0| st.y) bounds
// kappa sqrt(sum g'^2 / sum (g - mean)^2) = kappa sqrt(1 + n ((mean - c0) st.y)^2)
// from above (sqrt(1 + a^2) <= 1 + |a|).  An inadmissible or flat candidate
// gets lo = hi = -inf.
struct Scorer {
  float c0, tsum, rdf, kn1;   // kn1 = kappa n1
  __device__ __forceinline__ float operator()(float C, float2 st, bool adm, float& hi) const {
    const float dm = st.x - c0;
    // sum t (g - mean) = sum t (g - c0) - (mean - c0) sum t
    const float sc = fmaf(-dm, tsum, C) * st.y * rdf;
    const float e = fmaf(kn1, fabsf(dm * st.y), kBoundRel);
    const bool ok = adm && st.y > 0.f && isfinite(sc);
    hi = ok ? sc + e : -INFINITY;
    return ok ? sc - e : -INFINITY;
  }
};

}  // namespace

size_t search_mfma_wave_lds(int kb, int maxM, bool wide) {
  const int nmax = min(16 * kb - 32, 2 * maxM + 1);
  return (size_t)mfma_layout(kb, nmax, wide ? 2 : 1).total;
}

// TT = 1: windows up to 33 x 33 candidates (one tile, or two sharing their
// window fragments for 33 x 33).  TT = 2: windows of 34..64 per side, covered
// by 2 x 2 tiles of 32 x 32 candidates at (dv, du) offsets (32a, 32b), each
// the TT = 1 product on the window shifted by 32a rows and 32b columns; the
// window rows of tile row a = 1 replace those of a = 0 in LDS when its
// first tile starts, so a wave holds n1 + 32 rows, not n1 + 64.
//
// The candidates that may hold the maximum form a bit set in registers: word
// 2 dv + du / 32 (bit du % 32) sits in lane (2 dv + du / 32) % 64 of word
// register (2 dv + du / 32) / 64, so the words in register-then-lane order
// list the candidates in index order.  A tile's ballot of its 16 candidate
// rows gives whole words.
template <int KB, int TT>
__global__ void __launch_bounds__(64, KB == 3 ? 3 : 2) search_mfma_kernel(
    DevState st, const int32_t* __restrict__ work, int64_t count, int nmax,
    const double* __restrict__ box, const float* __restrict__ ref, const float* __restrict__ def,
    const int32_t* __restrict__ poi, const int32_t* __restrict__ seed,
    int32_t* __restrict__ uv_out, float* __restrict__ zncc_out, int32_t* __restrict__ status_out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  const MfmaLayout Ly = mfma_layout(KB, nmax, TT);
  uint16_t* win = reinterpret_cast<uint16_t*>(lds_raw + Ly.win);
  uint32_t* te = reinterpret_cast<uint32_t*>(lds_raw + Ly.te);
  uint32_t* to = reinterpret_cast<uint32_t*>(lds_raw + Ly.to);
  float* edge = reinterpret_cast<float*>(lds_raw + Ly.edge);
  const int lane0 = lane_id();
  // the refinement's work counters, zeroed here for the refinement that
  // follows in a correlate, which then needs no reset launch of its own
  // (every lane stores; lanes past the counters repeat the first ones)
  if (blockIdx.x == 0) st.counters[kCtrIcgn + (lane0 & (kMaxRefineGroups - 1))] = 0;
  constexpr int WC = 16 * KB + 32 * (TT - 1);   // staged window columns
  constexpr int CPR = WC / 8;                   // 8-element chunks per window row
  constexpr int NMAX = 16 * KB - 32;            // widest subset of this K-block count
  constexpr int CH = ((NMAX + 32) * CPR + kWave - 1) / kWave;   // window chunks per lane
  constexpr int TPD = 8 * KB;
  constexpr int TG = (TPD - 16) / 2;   // 4-column groups of a template row past the left pad
  constexpr int TQ = NMAX / 4;         // the groups a template of this K-block count can fill
  constexpr int TQL = (NMAX * TQ + kWave - 1) / kWave;   // such groups per lane
  static_assert(TQ <= TG, "template groups exceed the row");
  const int wpb = Ly.wpb;
  // both template copies zero, once: the 32 elements left of every row (the
  // previous row's zeros past its end) and the tail stay zero; a POI rewrites
  // groups 0..TQ-1 of its rows
  for (int idx = lane0; idx < nmax * TPD + 16; idx += kWave) {
    te[idx] = 0u;
    to[idx] = 0u;
  }

  // Static assignment: every POI costs about the same, and a work counter
  // (even one per XCD) costs an atomic per POI (0.51 against 0.43 ms
  // measured).  Workgroups are dispatched round-robin over the XCDs, so with
  // a grid that is a multiple of kXcds, XCD x takes the x-th contiguous part
  // of the work list (neighbouring POIs, whose windows and box sums then
  // share its L2).
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
    const int lane = opaque_lane(), n = lane & 31, kg = lane >> 5;
    const int g = uniform(work[item]);
    const DevPair P = st.pairs[uniform(st.poi_pair[g])];
    const RefRec* R = st.recs + g;
    const int x0 = uniform(poi[2 * g]), y0 = uniform(poi[2 * g + 1]);
    const int cu = seed ? uniform(seed[2 * g]) : 0;
    const int cv = seed ? uniform(seed[2 * g + 1]) : 0;
    const int rstat = uniform(load_status(R));
    if (rstat != DIC_POI_OK && rstat != DIC_POI_SINGULAR_HESSIAN) {
      if (lane == 0) {
        uv_out[2 * g] = 0;
        uv_out[2 * g + 1] = 0;
        zncc_out[g] = nanf("");
        status_out[g] = rstat;
      }
      continue;
    }
    const int M = P.M, S = P.S, n1 = 2 * M + 1, side = 2 * S + 1;
    const int W = P.width, H = P.height;
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
    // staged rows: those of one tile row of candidates (a tile reads n1 + 31);
    // the 2 x 2 form stages the second tile row's rows when it gets there
    const int wrows = n1 + 32;
    const bool two = side == 33;
    const CandBox cb = cand_box(x0 + cu - S, y0 + cv - S, side, M, W, H);
    Scorer sco;
    sco.c0 = c0;
    sco.tsum = R->tsum;
    sco.rdf = (float)(1.0 / R->df);
    sco.kn1 = kBoundRel * (float)n1;

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
    // 2. window g - c0 in bf16, chunks of 8 columns.  When the staged rows
    //    and columns all lie in the image (the usual case) every chunk is two
    //    16-byte loads and its values are stored as they are: rows and
    //    columns past the real window only meet zero template entries or
    //    candidates outside the window.  A non-finite pixel anywhere sends
    //    the window to the checked form, which stores 0 outside the window or
    //    the image and for non-finite pixels (their candidates are invalid by
    //    the box sums) and clamps every element's address into the image.
    //    The window rows r0 .. r0 + rows - 1 go to LDS rows 0 ..
    auto stage_window = [&](int r0, int rows) {
      const int wy = wy0 + r0;
      auto store_checked = [&](int k, const float* v) {
        const int idx = lane + k * kWave;
        const int rr = idx / CPR, ch = idx - rr * CPR;
        if (k < CH && rr < rows) {
          const int Y = wy + rr;
          const bool rowok = r0 + rr < wn && Y >= 0 && Y < H;
          float w[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int col = ch * 8 + e, X = wx0 + col;
            const float x = v[e];
            w[e] = (rowok && col < wn && X >= 0 && X < W && isfinite(x)) ? x - c0 : 0.f;
          }
          const u32x4 pk = {pack_bf16(w[0], w[1]), pack_bf16(w[2], w[3]),
                            pack_bf16(w[4], w[5]), pack_bf16(w[6], w[7])};
          *reinterpret_cast<u32x4*>(win + rr * wpb + ch * 8) = pk;
        }
      };
      const bool interior = wx0 >= 0 && wx0 + WC <= W && wy >= 0 && wy + rows <= H;
      bool staged = false;
      if (interior) {
        // all chunks requested at once when they fit in registers (one memory
        // round trip)
        constexpr int CBI = CH <= 8 ? CH : 4;
        bool bad = false;
#pragma unroll
        for (int k0 = 0; k0 < CH; k0 += CBI) {
          float vw[CBI][8];
#pragma unroll
          for (int kk = 0; kk < CBI; ++kk) {
            const int idx = lane + (k0 + kk) * kWave;
            const int rr = idx / CPR, ch = idx - rr * CPR;
            // rows past the staged ones (not stored) read the last staged row
            const f32x4u* src = reinterpret_cast<const f32x4u*>(
                gimg + (int64_t)(wy + min(rr, rows - 1)) * W + wx0 + ch * 8);
            const f32x4u a = src[0], b = src[1];
            vw[kk][0] = a.x; vw[kk][1] = a.y; vw[kk][2] = a.z; vw[kk][3] = a.w;
            vw[kk][4] = b.x; vw[kk][5] = b.y; vw[kk][6] = b.z; vw[kk][7] = b.w;
          }
#pragma unroll
          for (int kk = 0; kk < CBI; ++kk) {
            const int idx = lane + (k0 + kk) * kWave;
            const int rr = idx / CPR, ch = idx - rr * CPR;
            if (k0 + kk < CH && rr < rows) {
              float w[8];
#pragma unroll
              for (int e = 0; e < 8; ++e) {
                bad |= !isfinite(vw[kk][e]);
                w[e] = vw[kk][e] - c0;
              }
              const u32x4 pk = {pack_bf16(w[0], w[1]), pack_bf16(w[2], w[3]),
                                pack_bf16(w[4], w[5]), pack_bf16(w[6], w[7])};
              *reinterpret_cast<u32x4*>(win + rr * wpb + ch * 8) = pk;
            }
          }
        }
        staged = __ballot(bad) == 0;
      }
      if (!staged) {
        constexpr int CB = 4;
#pragma unroll 1
        for (int k0 = 0; k0 < CH; k0 += CB) {
          float v[CB][8];
#pragma unroll
          for (int kk = 0; kk < CB; ++kk) {
            const int idx = lane + (k0 + kk) * kWave;
            const int rr = idx / CPR, ch = idx - rr * CPR;
            const int Yc = min(max(wy + rr, 0), H - 1);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int Xc = min(max(wx0 + ch * 8 + e, 0), W - 1);
              v[kk][e] = gimg[(int64_t)Yc * W + Xc];
            }
          }
#pragma unroll
          for (int kk = 0; kk < CB; ++kk) store_checked(k0 + kk, v[kk]);
        }
      }
    };
    // one tile of up to 32 candidates a side meets window rows below
    // n1 + side - 1 only in its used rows dv < side: the rows past them are
    // not staged (whatever they hold, an earlier POI's values or nothing
    // yet, reaches only the accumulators of unused dv, which the scores
    // drop by a select)
    stage_window(0, (TT == 1 && !two) ? n1 + side - 1 : wrows);
    // 1. (after the window, so the template's loads, issued first, have
    //    arrived) template rows in bf16 after 32 zeros: element x of row r is
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
        const float first0 = __builtin_bit_cast(
            float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x1), 0));
        if (lane == kWave - 1) nxt = first0;
      }
      if (qq == TQ - 1) nxt = 0.f;
      if (idx < n1 * TQ) {
        const int base = r * TPD + 16 + 2 * qq;
        *reinterpret_cast<uint2*>(te + base) = make_uint2(pack_bf16(v.x, v.y), pack_bf16(v.z, v.w));
        *reinterpret_cast<uint2*>(to + base) = make_uint2(pack_bf16(v.y, v.z), pack_bf16(v.w, nxt));
        if (qq == 0) to[base - 1] = pack_bf16(0.f, v.x);
      }
    }
    wave_lds_sync();

    // 3.-5. cross terms on the matrix cores, the candidates' intervals, and
    //    the bit set of those whose interval reaches the largest lower end
    //    (the FP64 maximum is among them)
    float tau = -INFINITY;
    uint32_t word0 = 0u, word1 = 0u;
    if constexpr (TT == 1) {
      f32x16 acc_a = {}, acc_b = {};
      if (two)
        correlate_tiles<KB, true, false>(win, te, to, n1, wpb, TPD, lane, 33, acc_a, acc_b);
      else
        correlate_tiles<KB, false, true>(win, te, to, n1, wpb, TPD, lane, side, acc_a, acc_b);
      // box sums of every candidate this lane scores, requested at once: 16 of
      // tile A, then one edge candidate of tile B (lanes 0..62) or the two
      // corners (lane 63); their latency overlaps the corner sums below
      float2 sta[16];
      tile_stats(cb, stimg, W, H, 0, 0, lane, sta);
      // edge candidates: lane b < 32 -> (32, b + 1); 32 <= b < 63 -> (b - 31, 32);
      // lane 63 -> corners (32, 0) and (0, 32)
      const int e0v = lane < 32 ? 32 : lane < 63 ? lane - 31 : 32;
      const int e0u = lane < 32 ? lane + 1 : lane < 63 ? 32 : 0;
      const int e1v = 0, e1u = 32;
      float2 ste0 = make_float2(0.f, 0.f), ste1 = make_float2(0.f, 0.f);
      if (two) {
        ste0 = stimg[box_index(cb, e0v, e0u, W, H)];
        ste1 = stimg[box_index(cb, e1v, e1u, W, H)];
      }

      // the two corners on the vector ALUs, (32, 0) in lanes 0..31 and
      // (0, 32) in lanes 32..63, one template column per lane: products of
      // bf16 values are exact in FP32, and the FP32 sums stay inside the
      // accumulation term of the bound
      float cr1 = 0.f, cr2 = 0.f;
      if (two) {
        const uint16_t* tl = reinterpret_cast<const uint16_t*>(te) + 32 + n;
        const uint16_t* wl = kg ? win + n + 32 : win + 32 * wpb + n;
        float s = 0.f;
        for (int c = n; c < n1; c += 32) {
#pragma unroll 4
          for (int r = 0; r < n1; ++r)
            s = fmaf(bf16_bits(tl[r * 2 * TPD]), bf16_bits(wl[r * wpb]), s);
          tl += 32;
          wl += 32;
        }
        s += dpp_f32<0xB1>(s);   // quad_perm [1,0,3,2]
        s += dpp_f32<0x4E>(s);   // quad_perm [2,3,0,1]
        s += dpp_f32<0x141>(s);  // row_half_mirror
        s += dpp_f32<0x140>(s);  // row_mirror
        cr1 = readlane_f32(s, 0) + readlane_f32(s, 16);
        cr2 = readlane_f32(s, 32) + readlane_f32(s, 48);
        // tile B's edge row dv = 32 and column du = 32, one value per lane
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int i = (j & 3) + 8 * (j >> 2) + 4 * kg;
          if (i == 31) edge[n] = acc_b[j];               // (32, n + 1)
          else if (n == 31) edge[32 + i] = acc_b[j];     // (i + 1, 32), i < 31
        }
        wave_lds_sync();
      }

      // 4. the intervals and the threshold
      float hia[16];
      float lo = -INFINITY;
      const bool du_ok = n >= cb.du_lo && n <= cb.du_hi;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int i = (j & 3) + 8 * (j >> 2) + 4 * kg;
        const bool adm = du_ok && i >= cb.dv_lo && i <= cb.dv_hi;
        lo = fmaxf(lo, sco(acc_a[j], sta[j], adm, hia[j]));
      }
      float hi0 = -INFINITY, hi1 = -INFINITY;
      if (two) {
        const float c_e0 = lane < 63 ? edge[lane] : cr1;
        lo = fmaxf(lo, sco(c_e0, ste0, admissible(cb, e0v, e0u), hi0));
        const float l1 = sco(cr2, ste1, lane == 63 && admissible(cb, e1v, e1u), hi1);
        lo = fmaxf(lo, l1);
      }
      tau = wave_max_dpp(lo);
      // 5. the bit set: rows i of tile A give words 2 i (columns 0..31);
      //    column 32 (words 2 i + 1, bit 0) and row 32 (words 64, 65) come
      //    from the edge candidates
      if (tau > -INFINITY) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const uint64_t bl = __ballot(hia[j] >= tau);
          const int i0 = (j & 3) + 8 * (j >> 2);
          word0 = put_lane(word0, (uint32_t)bl, 2 * i0);
          word0 = put_lane(word0, (uint32_t)(bl >> 32), 2 * i0 + 8);
        }
        if (two) {
          const uint64_t b0 = __ballot(hi0 >= tau), b1 = __ballot(hi1 >= tau);
          // bit 31 + i: candidate (i, 32), from lane i + 31 of b0 (i >= 1)
          // and lane 63 of b1 (i = 0)
          const uint64_t c32 = (b0 & 0x7FFFFFFF00000000ull) | ((b1 >> 32) & 0x80000000ull);
          if (lane & 1) word0 = (uint32_t)(c32 >> (31 + (lane >> 1))) & 1u;
          // row 32: (32, 0) from lane 63, (32, 1..31) from lanes 0..30, (32, 32) from lane 31
          const uint32_t r32 = ((uint32_t)b0 << 1) | (uint32_t)(b0 >> 63);
          word1 = put_lane(word1, r32, 0);
          word1 = put_lane(word1, ((uint32_t)b0 >> 31) & 1u, 1);
        }
      }
    } else {
      // 2 x 2 tiles in order.  The running threshold only grows, so a tile's
      // bits (set against the threshold after it) are a superset of those the
      // final threshold selects; the FP64 re-score decides among them.
      float lo = -INFINITY;
#pragma unroll 1
      for (int t = 0; t < 4; ++t) {
        const int a = t >> 1, b = t & 1;
        if (32 * a >= side || 32 * b >= side) continue;
        if (a == 1 && b == 0) {
          // the second tile row's window rows, over the first's
          wave_lds_sync();
          // (only the rows the used candidates dv < side reach: the others
          // keep the first tile row's finite values, met by unused dv only)
          stage_window(32, min(wrows, n1 + side - 32));
          wave_lds_sync();
        }
        f32x16 acc = {}, acc_unused = {};
        correlate_tiles<KB, false, true>(win + 32 * b, te, to, n1, wpb, TPD, lane,
                                         min(32, side - 32 * b), acc, acc_unused);
        float2 stt[16];
        tile_stats(cb, stimg, W, H, 32 * a, 32 * b, lane, stt);
        float hit[16];
        float l = lo;
        const int du = 32 * b + n;
        const bool du_ok = du >= cb.du_lo && du <= cb.du_hi;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int i = 32 * a + (j & 3) + 8 * (j >> 2) + 4 * kg;
          const bool adm = du_ok && i >= cb.dv_lo && i <= cb.dv_hi;
          l = fmaxf(l, sco(acc[j], stt[j], adm, hit[j]));
        }
        lo = wave_max_dpp(l);
        if (lo > -INFINITY) {
          // rows 32 a + i give words 64 a + 2 i + b
          uint32_t wt = 0u;
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            const uint64_t bl = __ballot(hit[j] >= lo);
            const int i0 = (j & 3) + 8 * (j >> 2);
            wt = put_lane(wt, (uint32_t)bl, 2 * i0 + b);
            wt = put_lane(wt, (uint32_t)(bl >> 32), 2 * i0 + 8 + b);
          }
          if (a == 0) word0 |= wt;
          else word1 |= wt;
        }
      }
      tau = lo;
    }

    // the list of the bit set's members in index order (lane e holds the e-th)
    int pick = -1;
    double best = -INFINITY;
    if (tau > -INFINITY) {
      const uint32_t myword[2] = {word0, word1};
      uint64_t nonempty[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) nonempty[h] = __ballot(myword[h] != 0u);
      // candidate of bit `bits`'s lowest set bit in word 64 h + w
      auto cand_of = [&](int h, int w, uint32_t bits) {
        const int wi = 64 * h + w;
        return (wi >> 1) * side + 32 * (wi & 1) + __builtin_ctz(bits);
      };
      int count = 0, mycand = 0;
#pragma unroll
      for (int h = 0; h < 2; ++h)
        for (uint64_t ws = nonempty[h]; ws; ws &= ws - 1) {
          const int w = __builtin_ctzll(ws);
          for (uint32_t bits = (uint32_t)__builtin_amdgcn_readlane((int)myword[h], w); bits;
               bits &= bits - 1) {
            if (lane == count) mycand = cand_of(h, w, bits);
            ++count;
          }
        }

      // 6. FP64 re-score of the members in index order, two per pass over the
      //    subset (one call site, so the pass is inlined once): first all of
      //    them, for the maximum, keeping the first 64 coefficients one per
      //    lane; the first member within 1e-12 of the maximum wins, looked for
      //    among those 64 and, only when none of them is, in a second sweep
      //    over the rest (many exact ties).
      const double fbar = R->fbar, dfd = R->df;
      auto centre = [&](int cand, int& xg, int& yg) {
        const int rr = cand / side, cc = cand - rr * side;
        xg = x0 + cu - S + cc;
        yg = y0 + cv - S + rr;
      };
      // the e-th member (e uniform): a lane of the list, or past the 64th a
      // walk over the bit set
      auto nth = [&](int e) -> int {
        if (e < kWave) return __builtin_amdgcn_readlane(mycand, e);
        int k = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h)
          for (uint64_t ws = nonempty[h]; ws; ws &= ws - 1) {
            const int w = __builtin_ctzll(ws);
            for (uint32_t bits = (uint32_t)__builtin_amdgcn_readlane((int)myword[h], w); bits;
                 bits &= bits - 1, ++k)
              if (k == e) return cand_of(h, w, bits);
          }
        return 0;
      };
      const int listed = min(count, kWave);
      double keep = -INFINITY, cmax = -INFINITY;
      bool sweep = false;   // second sweep: members past the 64th, for the first near-maximum
      for (int e = 0;;) {
        if (!sweep && e >= count) {
          if (cmax == -INFINITY) break;
          const uint64_t hit = __ballot(lane < listed && keep >= cmax - 1e-12);
          if (hit) {
            const int h = __builtin_ctzll(hit);
            pick = __builtin_amdgcn_readlane(mycand, h);
            best = readlane_f64(keep, h);
            break;
          }
          sweep = true;
          e = kWave;
        }
        if (e >= count) break;
        const int nb = min(2, count - e);
        int xs[2], ys[2];
        centre(nth(e), xs[0], ys[0]);
        centre(nth(e + nb - 1), xs[1], ys[1]);
        double z[2];
        rescore_wave<2>(fimg, gimg, W, x0, y0, xs, ys, nb, M, fbar, dfd, s1img, z, lane);
        if (!sweep) {
          if (lane == e) keep = z[0];
          cmax = fmax(cmax, z[0]);
          if (nb == 2) {
            if (lane == e + 1) keep = z[1];
            cmax = fmax(cmax, z[1]);
          }
        } else if (z[0] >= cmax - 1e-12) {
          pick = nth(e);
          best = z[0];
          break;
        } else if (nb == 2 && z[1] >= cmax - 1e-12) {
          pick = nth(e + 1);
          best = z[1];
          break;
        }
        e += nb;
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
                     st, st.work + gr.begin, gr.count, nmax, st.box, ref, def, poi, seed, uv,
                     zncc, status);
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
