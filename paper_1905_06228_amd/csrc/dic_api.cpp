// Host implementation of the C ABI declared in include/dic.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "dic.h"
#include "dic_internal.h"

using namespace dic;

// Device scratch of dic_correlate_noalloc: the plan's workspace for callers
// that cannot allocate device memory.  Each device the library runs on holds
// its own copy for the life of the process.  Host code never passes the
// array's name to a kernel or a copy (on the host it is a stand-in symbol, not
// a device address): it uses the per-device address that hipGetSymbolAddress
// returns (noalloc_scratch below).
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

thread_local std::string g_last_error;

// A named range around one stage for rocprofv3's marker trace: it spans the
// host-side enqueue (or its capture into a graph), not the kernels' run on
// the device, which the kernel trace times.
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

dic_status_t fail(dic_status_t code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define DIC_HIP(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(DIC_ERR_HIP, std::string(#expr) + " failed: " + hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t pairs = 0, poi_pair = 0, work = 0, counters = 0, grads = 0, recs = 0, tmpl = 0,
         box = 0, lut = 0, bsp_flags = 0, fix_off = 0, fix_owner = 0, fix = 0, s_status = 0,
         s_zncc = 0, total = 0;
  int64_t fix_count = 0;
};

const dic_tuning_t kDefaultTuning = {8, 0, 4, 4};  // block, occupancy, waves, slack

// Whether search form `block` can run windows up to +-maxS with subsets up
// to radius maxM.
bool search_fits(int maxM, int maxS, int block) {
  if (block == kMfmaBlock)
    return maxS <= kMfmaWideMaxS &&
           search_mfma_wave_lds(mfma_kb(maxM), maxM, maxS > kMfmaMaxS) <= 160 * 1024;
  return search_lds_bytes(maxM, maxS, block) <= 160 * 1024 &&
         search_threads(maxS, block) <= search_max_threads();
}

bool tuning_valid(const dic_tuning_t& t) {
  const bool blk = t.search_block == 4 || t.search_block == 8 || t.search_block == kMfmaBlock;
  const bool thr = t.search_occupancy >= 0 && t.search_occupancy <= 16;
  return blk && thr && t.icgn_waves >= 1 && t.icgn_waves <= 8 && t.icgn_slack >= 0 &&
         t.icgn_slack <= kMaxRefineSlack;
}

}  // namespace

struct dic_plan_s {
  dic_plan_desc_t desc{};
  std::vector<dic_pair_desc_t> pairs;
  std::vector<DevPair> dpairs;
  std::vector<int32_t> poi_pair, work;
  std::vector<std::pair<int, int64_t>> m_runs;  // (M, length) runs of the work list
  std::vector<RefineGroup> rgroups;  // runs of the work list that share a refinement kernel
  std::vector<int64_t> fix_off;
  // deterministic adjoint: the pair that owns each distinct deformed image
  // (pairs on the same image share its fixed-point accumulator, flushed once)
  std::vector<int32_t> fix_owner;
  int64_t N = 0;
  int maxM = 0, maxS = 0, maxW = 0, maxH = 0;
  Layout lay;
  dic_tuning_t tuning = kDefaultTuning;
  void* ws = nullptr;
  bool bound = false;
  int num_cu = 0;
  DevState st{};
  bool ref_valid = false;
  bool ref_tmpl = false;   // the cached reference preparation wrote the FP32 template
  const void* ref_img = nullptr;
  const void* ref_poi = nullptr;
  bool def_valid = false;
  const void* def_img = nullptr;
  bool lut_valid = false;
  const void* lut_img = nullptr;
  std::map<std::vector<uintptr_t>, hipGraphExec_t> graphs;
  std::vector<hipGraph_t> graph_objs;
  hipStream_t cap_stream = nullptr;
  // second stream for the deformed-side preparation, which runs beside the
  // reference-side one (forked from and joined back to the caller's stream)
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // the reference side's statistics done (main stream), and its Hessian part
  // done (side stream, beside the search)
  hipEvent_t ev_stats = nullptr, ev_ref = nullptr;

  bool fp32() const { return desc.precision == DIC_FP32_BATCHED; }
  bool det() const { return (desc.flags & DIC_FLAG_DETERMINISTIC_BWD) != 0; }
  bool nr() const { return (desc.flags & DIC_FLAG_REFINE_NR) != 0; }
  bool bilinear() const { return (desc.flags & DIC_FLAG_INTERP_BILINEAR) != 0; }
  bool lut() const { return (desc.flags & DIC_FLAG_BICUBIC_LUT) != 0; }
  bool bspline() const { return (desc.flags & DIC_FLAG_INTERP_BSPLINE) != 0; }
  // a per-image table the refinements read: bicubic coefficients or the
  // B-spline coefficient image
  bool table() const { return lut() || bspline(); }
  int interp() const {
    return bilinear()  ? kInterpBilinear
           : lut()     ? kInterpBicubicLut
           : bspline() ? kInterpBSpline
                       : kInterpBicubic;
  }
};

namespace {

void drop_graphs(dic_plan_s* p) {
  for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto g : p->graph_objs) (void)hipGraphDestroy(g);
  p->graphs.clear();
  p->graph_objs.clear();
}

std::string tune_key(const dic_plan_s* p) {
  std::ostringstream k;
  k << "gfx950|" << (p->fp32() ? "f32" : "f64") << "|N" << p->N;
  std::vector<std::pair<int, int>> ms;
  for (auto& d : p->pairs) ms.emplace_back(d.subset_radius, d.search_radius);
  std::sort(ms.begin(), ms.end());
  ms.erase(std::unique(ms.begin(), ms.end()), ms.end());
  for (auto& m : ms) k << "|M" << m.first << "S" << m.second;
  return k.str();
}

// Minimal JSON object of arrays: {"key": [a, b, c, d], ...}.
std::map<std::string, std::vector<int>> read_tune_cache(const char* path) {
  std::map<std::string, std::vector<int>> out;
  std::ifstream in(path);
  if (!in) return out;
  std::stringstream ss;
  ss << in.rdbuf();
  const std::string s = ss.str();
  size_t i = 0;
  while (true) {
    const size_t q0 = s.find('"', i);
    if (q0 == std::string::npos) break;
    const size_t q1 = s.find('"', q0 + 1);
    if (q1 == std::string::npos) break;
    const std::string key = s.substr(q0 + 1, q1 - q0 - 1);
    const size_t b0 = s.find('[', q1), b1 = s.find(']', q1);
    if (b0 == std::string::npos || b1 == std::string::npos || b1 < b0) break;
    std::vector<int> vals;
    std::stringstream vs(s.substr(b0 + 1, b1 - b0 - 1));
    std::string tok;
    while (std::getline(vs, tok, ',')) vals.push_back(std::atoi(tok.c_str()));
    out[key] = vals;
    i = b1 + 1;
  }
  return out;
}

void write_tune_cache(const char* path, const std::map<std::string, std::vector<int>>& m) {
  std::ofstream o(path, std::ios::trunc);
  if (!o) return;
  o << "{\n";
  size_t k = 0;
  for (auto& kv : m) {
    o << "  \"" << kv.first << "\": [";
    for (size_t j = 0; j < kv.second.size(); ++j) o << (j ? ", " : "") << kv.second[j];
    o << "]" << (++k < m.size() ? "," : "") << "\n";
  }
  o << "}\n";
}

dic_status_t check_plan(dic_plan_t p, bool need_bound) {
  if (!p) return fail(DIC_ERR_INVALID_ARGUMENT, "null plan");
  if (need_bound && !p->bound) return fail(DIC_ERR_NOT_BOUND, "plan has no workspace bound");
  return DIC_SUCCESS;
}

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device: the address of `scratch`, null until looked up

// Device address of the current device's copy of `scratch`, looked up once per
// device with that device current.
dic_status_t noalloc_scratch(void** out) {
  int dev = 0, ndev = 0;
  DIC_HIP(hipGetDevice(&dev));
  DIC_HIP(hipGetDeviceCount(&ndev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() < ndev) g_scratch_ptr.resize(ndev, nullptr);
  if (dev < 0 || dev >= ndev) return fail(DIC_ERR_HIP, "current device outside the device count");
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    DIC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr || reinterpret_cast<uintptr_t>(ptr) % kAlign)
      return fail(DIC_ERR_INTERNAL, "static scratch address missing or misaligned");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return DIC_SUCCESS;
}

// Points the plan's device state at the workspace `base` and uploads the pair
// table, the POI -> pair map, the work list and the adjoint's accumulator
// table there (asynchronous on `s`); every cached preparation is marked
// stale.  Copies only: no allocation.
dic_status_t attach_workspace(dic_plan_t p, void* ws, hipStream_t s) {
  int dev = 0;
  DIC_HIP(hipGetDevice(&dev));
  DIC_HIP(hipDeviceGetAttribute(&p->num_cu, hipDeviceAttributeMultiprocessorCount, dev));
  char* base = static_cast<char*>(ws);
  DIC_HIP(hipMemcpyAsync(base + p->lay.pairs, p->dpairs.data(), sizeof(DevPair) * p->dpairs.size(),
                         hipMemcpyHostToDevice, s));
  if (p->N) {
    DIC_HIP(hipMemcpyAsync(base + p->lay.poi_pair, p->poi_pair.data(), sizeof(int32_t) * p->N,
                           hipMemcpyHostToDevice, s));
    DIC_HIP(hipMemcpyAsync(base + p->lay.work, p->work.data(), sizeof(int32_t) * p->N,
                           hipMemcpyHostToDevice, s));
  }
  DIC_HIP(hipMemcpyAsync(base + p->lay.fix_off, p->fix_off.data(), sizeof(int64_t) * p->fix_off.size(),
                         hipMemcpyHostToDevice, s));
  if (!p->fix_owner.empty())
    DIC_HIP(hipMemcpyAsync(base + p->lay.fix_owner, p->fix_owner.data(),
                           sizeof(int32_t) * p->fix_owner.size(), hipMemcpyHostToDevice, s));
  DevState& st = p->st;
  st.pairs = reinterpret_cast<const DevPair*>(base + p->lay.pairs);
  st.poi_pair = reinterpret_cast<const int32_t*>(base + p->lay.poi_pair);
  st.work = reinterpret_cast<const int32_t*>(base + p->lay.work);
  st.counters = reinterpret_cast<int32_t*>(base + p->lay.counters);
  st.grads = reinterpret_cast<float*>(base + p->lay.grads);
  st.recs = reinterpret_cast<RefRec*>(base + p->lay.recs);
  st.tmpl = reinterpret_cast<float*>(base + p->lay.tmpl);
  st.box = reinterpret_cast<double*>(base + p->lay.box);
  st.lut = reinterpret_cast<float*>(base + p->lay.lut);
  st.bsp_flags = reinterpret_cast<int32_t*>(base + p->lay.bsp_flags);
  st.N = p->N;
  st.num_pairs = p->desc.num_pairs;
  st.maxM = p->maxM;
  st.maxS = p->maxS;
  st.max_width = p->maxW;
  st.max_height = p->maxH;
  st.max_iters = p->desc.max_iters;
  st.conv_tol = p->desc.conv_tol;
  p->ws = ws;
  p->bound = true;
  p->ref_valid = false;
  p->def_valid = false;
  p->lut_valid = false;
  return DIC_SUCCESS;
}

// The reference side.  The FP32 search template is written only when the
// vector-ALU search form (which reads it) may run: its tuning, or `tmpl`
// (the autotuner, which tries every form); a cached preparation without it
// is redone when a form that needs it comes.
bool ref_cached(const dic_plan_s* p, const float* ref, const int32_t* poi, bool need_tmpl) {
  return (p->desc.flags & DIC_FLAG_CACHE_REF_PREP) && p->ref_valid && p->ref_img == ref &&
         p->ref_poi == poi && (p->ref_tmpl || !need_tmpl || !p->fp32());
}

void mark_ref(dic_plan_t p, const float* ref, const int32_t* poi, bool need_tmpl) {
  p->ref_valid = true;
  p->ref_tmpl = need_tmpl;
  p->ref_img = ref;
  p->ref_poi = poi;
}

dic_status_t prepare(dic_plan_t p, const float* ref, const int32_t* poi, hipStream_t s,
                     bool force, bool tmpl = false) {
  const Range range("dic: reference preparation");
  const bool need_tmpl = tmpl || p->tuning.search_block != kMfmaBlock;
  if (!force && ref_cached(p, ref, poi, need_tmpl)) return DIC_SUCCESS;
  if (p->fp32()) {
    DIC_HIP(launch_gradients(p->st, ref, s));
    DIC_HIP(launch_ref_prep_f32(p->st, p->rgroups.data(), (int)p->rgroups.size(), ref, poi,
                                need_tmpl, s));
  } else {
    DIC_HIP(launch_ref_prep_f64(p->st, p->dpairs.data(), ref, poi, s));
  }
  mark_ref(p, ref, poi, need_tmpl);
  return DIC_SUCCESS;
}

// Runs of the work list that share the search kernel's template row length
// (vector-ALU form) or K-block count (matrix-core form).
std::vector<SearchGroup> search_groups(const dic_plan_s* p, int block) {
  std::vector<SearchGroup> g;
  int64_t at = 0;
  for (auto& run : p->m_runs) {
    const int np = block == kMfmaBlock ? mfma_kb(run.first) : search_np(run.first, block);
    if (g.empty() || g.back().np != np) g.push_back({np, at, 0});
    g.back().count += run.second;
    at += run.second;
  }
  return g;
}

dic_status_t prepare_deformed(dic_plan_t p, const float* def, hipStream_t s, bool force) {
  const Range range("dic: deformed preparation");
  if (!p->fp32()) return DIC_SUCCESS;
  if (!force && (p->desc.flags & DIC_FLAG_CACHE_REF_PREP) && p->def_valid && p->def_img == def)
    return DIC_SUCCESS;
  DIC_HIP(launch_box_sums(p->st, def, s));
  p->def_valid = true;
  p->def_img = def;
  return DIC_SUCCESS;
}

// The bicubic coefficient table (DIC_FLAG_BICUBIC_LUT) or the B-spline
// coefficient image (DIC_FLAG_INTERP_BSPLINE) of the deformed images,
// cached like the box sums.
dic_status_t prepare_lut(dic_plan_t p, const float* def, hipStream_t s, bool force) {
  if (!p->table()) return DIC_SUCCESS;
  if (!force && (p->desc.flags & DIC_FLAG_CACHE_REF_PREP) && p->lut_valid && p->lut_img == def)
    return DIC_SUCCESS;
  if (p->lut())
    DIC_HIP(launch_bicubic_lut(p->st, def, s));
  else
    DIC_HIP(launch_bspline_coeffs(p->st, def, s));
  p->lut_valid = true;
  p->lut_img = def;
  return DIC_SUCCESS;
}

dic_status_t enqueue_search(dic_plan_t p, const float* ref, const float* def, const int32_t* poi,
                            const int32_t* seed, int32_t* uv, float* zn, int32_t* status,
                            hipStream_t s, bool def_ready = false) {
  const Range range("dic: integer search");
  if (p->fp32()) {
    const std::vector<SearchGroup> groups = search_groups(p, p->tuning.search_block);
    if (!def_ready) {
      dic_status_t r = prepare_deformed(p, def, s, false);
      if (r) return r;
    }
    // the matrix-core form assigns POIs statically and uses no work counter
    if (p->tuning.search_block == kMfmaBlock) {
      DIC_HIP(launch_search_mfma(p->st, p->tuning, groups.data(), (int)groups.size(), ref, def,
                                 poi, seed, uv, zn, status, p->num_cu, s));
    } else {
      DIC_HIP(launch_reset_counters(p->st, s));
      DIC_HIP(launch_search_f32(p->st, p->tuning, groups.data(), (int)groups.size(), ref, def,
                                poi, seed, uv, zn, status, p->num_cu, s));
    }
  } else {
    DIC_HIP(launch_search_f64(p->st, p->dpairs.data(), ref, def, poi, seed, uv, zn, status, s));
  }
  return DIC_SUCCESS;
}

// Sub-pixel refinement: IC-GN, or Newton-Raphson when `nr`.
dic_status_t enqueue_refine(dic_plan_t p, const float* ref, const float* def, const int32_t* poi,
                            const int32_t* uv, const int32_t* status_in, const double* p_init,
                            double* p_out, float* zn, int32_t* iters, int32_t* status,
                            hipStream_t s, bool nr, bool table_ready = false,
                            bool counters_ready = false) {
  const Range range(nr ? "dic: Newton-Raphson refinement" : "dic: IC-GN refinement");
  if (p->fp32()) {
    if (!table_ready) {
      dic_status_t r = prepare_lut(p, def, s, false);
      if (r) return r;
    }
    if (!counters_ready) DIC_HIP(launch_reset_counters(p->st, s));
    const int ng = (int)p->rgroups.size();
    if (nr)
      DIC_HIP(launch_nr_f32(p->st, p->tuning, p->rgroups.data(), ng, ref, def, poi, uv,
                            status_in, p_init, p_out, zn, iters, status, p->num_cu, s,
                            p->interp()));
    else
      DIC_HIP(launch_icgn_f32(p->st, p->tuning, p->rgroups.data(), ng, ref, def, poi, uv,
                              status_in, p_init, p_out, zn, iters, status, p->num_cu, s,
                              p->interp()));
  } else if (nr) {
    DIC_HIP(launch_nr_f64(p->st, p->dpairs.data(), ref, def, poi, uv, status_in, p_init, p_out,
                          zn, iters, status, s));
  } else {
    DIC_HIP(launch_icgn_f64(p->st, p->dpairs.data(), ref, def, poi, uv, status_in, p_init, p_out,
                            zn, iters, status, s));
  }
  return DIC_SUCCESS;
}

struct CorrArgs {
  const float *ref, *def;
  const int32_t* poi;
  const int32_t* seed;
  const double* p_init;
  int32_t* uv;
  float* zn_int;
  int32_t* st_int;
  double* p_out;
  float* zn;
  int32_t* iters;
  int32_t* status;
};

// Search then refine.  In the FP32 form the deformed-side box sums and the
// interpolation table or B-spline coefficients (when not cached) run on the
// plan's side stream beside the reference side's statistics: the two read
// different images and write different sections.  The reference side's
// gradients, Hessian and factor, which only the refinement reads, then run
// on the side stream beside the search (enqueued after it, so the search's
// waves take the device first and the preparation fills what they leave);
// the refinement waits for them.
// With `allow_fork` false everything runs in order on `s` (no side stream is
// created or used).
dic_status_t enqueue_correlate(dic_plan_t p, const CorrArgs& a, hipStream_t s,
                               bool allow_fork = true) {
  const Range range("dic: correlate");
  const bool fork = allow_fork && p->fp32() &&
                    !((p->desc.flags & DIC_FLAG_CACHE_REF_PREP) && p->def_valid &&
                      p->def_img == a.def);
  const bool need_tmpl = p->tuning.search_block != kMfmaBlock;
  const bool split = fork && !ref_cached(p, a.ref, a.poi, need_tmpl);
  if (fork) {
    if (!p->side_stream) DIC_HIP(hipStreamCreateWithFlags(&p->side_stream, hipStreamNonBlocking));
    if (!p->ev_fork) DIC_HIP(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
    if (!p->ev_join) DIC_HIP(hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming));
    if (!p->ev_stats) DIC_HIP(hipEventCreateWithFlags(&p->ev_stats, hipEventDisableTiming));
    if (!p->ev_ref) DIC_HIP(hipEventCreateWithFlags(&p->ev_ref, hipEventDisableTiming));
    DIC_HIP(hipEventRecord(p->ev_fork, s));
    DIC_HIP(hipStreamWaitEvent(p->side_stream, p->ev_fork, 0));
    // the deformed side: box sums, then the refinement's coefficient table
    // or B-spline coefficients (if the plan has one), beside the reference side
    dic_status_t r = prepare_deformed(p, a.def, p->side_stream, false);
    if (r == DIC_SUCCESS) r = prepare_lut(p, a.def, p->side_stream, false);
    if (r != DIC_SUCCESS) return r;
    DIC_HIP(hipEventRecord(p->ev_join, p->side_stream));
  }
  dic_status_t r = DIC_SUCCESS;
  if (split) {
    const Range range("dic: reference statistics");
    DIC_HIP(launch_ref_prep_stats(p->st, p->rgroups.data(), (int)p->rgroups.size(), a.ref,
                                  a.poi, need_tmpl, s));
    DIC_HIP(hipEventRecord(p->ev_stats, s));
  } else {
    r = prepare(p, a.ref, a.poi, s, false);
  }
  if (fork) DIC_HIP(hipStreamWaitEvent(s, p->ev_join, 0));
  if (r != DIC_SUCCESS) return r;
  r = enqueue_search(p, a.ref, a.def, a.poi, a.seed, a.uv, a.zn_int, a.st_int, s, fork);
  if (r != DIC_SUCCESS) return r;
  if (split) {
    const Range range("dic: reference gradients and Hessian (side stream)");
    DIC_HIP(hipStreamWaitEvent(p->side_stream, p->ev_stats, 0));
    DIC_HIP(launch_gradients(p->st, a.ref, p->side_stream));
    DIC_HIP(launch_ref_prep_hessian(p->st, a.ref, a.poi, p->side_stream));
    DIC_HIP(hipEventRecord(p->ev_ref, p->side_stream));
    DIC_HIP(hipStreamWaitEvent(s, p->ev_ref, 0));
    mark_ref(p, a.ref, a.poi, need_tmpl);
  }
  // the FP32 searches leave the refinement's counters at zero (the
  // matrix-core form zeroes them, the vector-ALU form's reset before it
  // covers them and it uses only its own)
  return enqueue_refine(p, a.ref, a.def, a.poi, a.uv, a.st_int, a.p_init, a.p_out, a.zn, a.iters,
                        a.status, s, p->nr(), fork, p->fp32());
}

}  // namespace

extern "C" {

const char* dic_last_error(void) { return g_last_error.c_str(); }

const char* dic_status_string(int32_t status) {
  switch (status) {
    case DIC_SUCCESS: return "success";
    case DIC_ERR_INVALID_ARGUMENT: return "invalid argument";
    case DIC_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case DIC_ERR_HIP: return "HIP runtime error";
    case DIC_ERR_UNSUPPORTED: return "unsupported";
    case DIC_ERR_INTERNAL: return "internal error";
    case DIC_ERR_NOT_BOUND: return "plan not bound to a workspace";
    default: return "unknown status";
  }
}

dic_status_t dic_plan_create(const dic_plan_desc_t* d, dic_plan_t* out) {
  if (!d || !out) return fail(DIC_ERR_INVALID_ARGUMENT, "null desc or out");
  *out = nullptr;
  if (d->num_pairs < 1 || !d->pairs) return fail(DIC_ERR_INVALID_ARGUMENT, "num_pairs < 1 or null pairs");
  if (d->precision != DIC_FP32_BATCHED && d->precision != DIC_FP64_PLAIN)
    return fail(DIC_ERR_INVALID_ARGUMENT, "unknown precision");
  if (d->max_iters < 1 || d->max_iters > 200) return fail(DIC_ERR_INVALID_ARGUMENT, "max_iters outside 1..200");
  if (!(d->conv_tol > 0.0) || !std::isfinite(d->conv_tol))
    return fail(DIC_ERR_INVALID_ARGUMENT, "conv_tol must be positive and finite");
  const uint32_t known = DIC_FLAG_USE_GRAPH | DIC_FLAG_CACHE_REF_PREP |
                         DIC_FLAG_DETERMINISTIC_BWD | DIC_FLAG_REFINE_NR |
                         DIC_FLAG_INTERP_BILINEAR | DIC_FLAG_BICUBIC_LUT |
                         DIC_FLAG_INTERP_BSPLINE;
  if (d->flags & ~known) return fail(DIC_ERR_INVALID_ARGUMENT, "unknown flag bits");
  if ((d->flags & DIC_FLAG_INTERP_BILINEAR) && d->precision != DIC_FP32_BATCHED)
    return fail(DIC_ERR_UNSUPPORTED, "bilinear interpolation needs the FP32 batched form");
  if ((d->flags & DIC_FLAG_BICUBIC_LUT) && d->precision != DIC_FP32_BATCHED)
    return fail(DIC_ERR_UNSUPPORTED, "the bicubic coefficient table needs the FP32 batched form");
  if ((d->flags & DIC_FLAG_INTERP_BSPLINE) && d->precision != DIC_FP32_BATCHED)
    return fail(DIC_ERR_UNSUPPORTED, "B-spline interpolation needs the FP32 batched form");
  {
    const uint32_t im = d->flags & (DIC_FLAG_INTERP_BILINEAR | DIC_FLAG_BICUBIC_LUT |
                                    DIC_FLAG_INTERP_BSPLINE);
    if (im & (im - 1))
      return fail(DIC_ERR_INVALID_ARGUMENT,
                  "DIC_FLAG_INTERP_BILINEAR, DIC_FLAG_BICUBIC_LUT and DIC_FLAG_INTERP_BSPLINE "
                  "are exclusive");
  }
  auto p = new dic_plan_s();
  p->desc = *d;
  p->pairs.assign(d->pairs, d->pairs + d->num_pairs);
  p->desc.pairs = nullptr;
  int64_t next = 0;
  for (int k = 0; k < d->num_pairs; ++k) {
    const dic_pair_desc_t& q = p->pairs[k];
    std::ostringstream why;
    why << "pair " << k << ": ";
    if (q.width < 8 || q.height < 8 || q.width > 65536 || q.height > 65536) why << "width/height outside 8..65536";
    else if (q.subset_radius < 1 || q.subset_radius > kMaxM) why << "subset_radius outside 1..20";
    else if (q.search_radius < 0 || q.search_radius > kMaxS) why << "search_radius outside 0..32";
    else if (2 * q.subset_radius + 3 > std::min(q.width, q.height)) why << "subset does not fit the image";
    else if (q.ref_offset < 0 || q.def_offset < 0) why << "negative image offset";
    else if (q.poi_count < 0) why << "negative poi_count";
    else if (q.poi_offset != next) why << "POI ranges must be contiguous and in pair order";
    else {
      next += q.poi_count;
      continue;
    }
    delete p;
    return fail(DIC_ERR_INVALID_ARGUMENT, why.str());
  }
  if (next > INT32_MAX) {
    delete p;
    return fail(DIC_ERR_INVALID_ARGUMENT, "more than 2^31-1 POIs");
  }
  p->N = next;
  const bool f32 = p->fp32();
  // layout
  Layout& L = p->lay;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  L.pairs = take(sizeof(DevPair) * d->num_pairs);
  L.poi_pair = take(sizeof(int32_t) * p->N);
  L.work = take(sizeof(int32_t) * p->N);
  L.counters = take(sizeof(int32_t) * kNumCounters);
  int64_t gfl = 0, tfl = 0, bxd = 0, lut4 = 0, fix = 0;
  const bool use_lut = (d->flags & DIC_FLAG_BICUBIC_LUT) != 0;
  const bool use_bsp = (d->flags & DIC_FLAG_INTERP_BSPLINE) != 0;
  p->dpairs.resize(d->num_pairs);
  p->fix_off.resize(d->num_pairs);
  for (int k = 0; k < d->num_pairs; ++k) {
    const dic_pair_desc_t& q = p->pairs[k];
    DevPair& P = p->dpairs[k];
    P.width = q.width;
    P.height = q.height;
    P.M = q.subset_radius;
    P.S = q.search_radius;
    P.ref_off = q.ref_offset;
    P.def_off = q.def_offset;
    P.poi_off = q.poi_offset;
    P.poi_count = q.poi_count;
    P.grad_off = gfl;
    P.tmpl_off = tfl;
    P.tmpl_pitch = template_pitch(q.subset_radius);
    P.pad_ = 0;
    P.box_off = bxd;
    P.lut_off = lut4;
    const int64_t tn = (int64_t)(2 * q.subset_radius + 1) * P.tmpl_pitch;
    if (f32) {
      gfl += 2 * (int64_t)q.width * q.height;
      tfl += q.poi_count * tn;
      bxd += 5 * (int64_t)q.width * q.height;
      if (use_lut) lut4 += 4 * (int64_t)q.width * q.height;
      if (use_bsp) lut4 += (2 * (int64_t)q.width * q.height + 3) / 4;
    }
    p->fix_off[k] = fix;
    if (p->det()) {
      // Pairs that name the same deformed image (offset and size) share one
      // accumulator; partly overlapping images would be flushed twice over
      // the same pixels, so they are rejected.
      int shared = -1;
      const int64_t a0 = q.def_offset, a1 = a0 + (int64_t)q.width * q.height;
      for (int j : p->fix_owner) {
        const dic_pair_desc_t& o = p->pairs[j];
        const int64_t b0 = o.def_offset, b1 = b0 + (int64_t)o.width * o.height;
        if (o.def_offset == q.def_offset && o.width == q.width && o.height == q.height) {
          shared = j;
          break;
        }
        if (a0 < b1 && b0 < a1) {
          std::ostringstream why;
          why << "pair " << k << ": with DIC_FLAG_DETERMINISTIC_BWD the deformed image must be "
              << "the same image as, or disjoint from, that of pair " << j;
          delete p;
          return fail(DIC_ERR_INVALID_ARGUMENT, why.str());
        }
      }
      if (shared >= 0) {
        p->fix_off[k] = p->fix_off[shared];
      } else {
        p->fix_owner.push_back(k);
        fix += (int64_t)q.width * q.height;
      }
    }
    p->maxM = std::max(p->maxM, (int)q.subset_radius);
    p->maxS = std::max(p->maxS, (int)q.search_radius);
    p->maxW = std::max(p->maxW, (int)q.width);
    p->maxH = std::max(p->maxH, (int)q.height);
  }
  L.grads = take(sizeof(float) * gfl);
  L.recs = take(sizeof(RefRec) * p->N);
  L.tmpl = take(sizeof(float) * tfl);
  L.box = take(sizeof(double) * bxd);
  L.lut = take(sizeof(float) * 4 * lut4);
  L.bsp_flags = take(use_bsp ? sizeof(int32_t) * d->num_pairs : 0);
  L.fix_off = take(sizeof(int64_t) * d->num_pairs);
  L.fix_owner = take(sizeof(int32_t) * p->fix_owner.size());
  L.fix = take(sizeof(unsigned long long) * fix);
  L.fix_count = fix;
  L.s_status = take(sizeof(int32_t) * p->N);
  L.s_zncc = take(sizeof(float) * p->N);
  L.total = off;
  // POI -> pair and the work list, largest subsets first (stable)
  p->poi_pair.resize(p->N);
  for (int k = 0; k < d->num_pairs; ++k)
    for (int64_t i = 0; i < p->pairs[k].poi_count; ++i)
      p->poi_pair[p->pairs[k].poi_offset + i] = k;
  p->work.resize(p->N);
  for (int64_t i = 0; i < p->N; ++i) p->work[i] = (int32_t)i;
  std::stable_sort(p->work.begin(), p->work.end(), [&](int32_t a, int32_t b) {
    return p->pairs[p->poi_pair[a]].subset_radius > p->pairs[p->poi_pair[b]].subset_radius;
  });
  for (int64_t i = 0; i < p->N; ++i) {
    const int m = p->pairs[p->poi_pair[p->work[i]]].subset_radius;
    if (p->m_runs.empty() || p->m_runs.back().first != m) p->m_runs.emplace_back(m, 0);
    ++p->m_runs.back().second;
  }
  {
    int64_t at = 0;
    for (auto& run : p->m_runs) {
      if (p->rgroups.empty() || refine_class(p->rgroups.back().maxM) != refine_class(run.first))
        p->rgroups.push_back({at, 0, run.first});
      p->rgroups.back().count += run.second;
      at += run.second;
    }
  }
  // the matrix-core search where the window allows it, else the vector-ALU form
  if (f32 && search_fits(p->maxM, p->maxS, kMfmaBlock)) p->tuning.search_block = kMfmaBlock;
  if (f32 && !search_fits(p->maxM, p->maxS, p->tuning.search_block)) {
    delete p;
    return fail(DIC_ERR_UNSUPPORTED, "search window exceeds the 160 KiB LDS of a CU");
  }
  *out = p;
  return DIC_SUCCESS;
}

void dic_plan_destroy(dic_plan_t p) {
  if (!p) return;
  drop_graphs(p);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->side_stream) (void)hipStreamDestroy(p->side_stream);
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  if (p->ev_join) (void)hipEventDestroy(p->ev_join);
  if (p->ev_stats) (void)hipEventDestroy(p->ev_stats);
  if (p->ev_ref) (void)hipEventDestroy(p->ev_ref);
  delete p;
}

dic_status_t dic_plan_workspace_size(dic_plan_t p, size_t* bytes) {
  dic_status_t r = check_plan(p, false);
  if (r) return r;
  if (!bytes) return fail(DIC_ERR_INVALID_ARGUMENT, "null bytes");
  *bytes = p->lay.total;
  return DIC_SUCCESS;
}

dic_status_t dic_plan_get_tuning(dic_plan_t p, dic_tuning_t* out) {
  dic_status_t r = check_plan(p, false);
  if (r) return r;
  if (!out) return fail(DIC_ERR_INVALID_ARGUMENT, "null out");
  *out = p->tuning;
  return DIC_SUCCESS;
}

dic_status_t dic_plan_set_tuning(dic_plan_t p, const dic_tuning_t* in) {
  dic_status_t r = check_plan(p, false);
  if (r) return r;
  if (!in || !tuning_valid(*in)) return fail(DIC_ERR_INVALID_ARGUMENT, "invalid tuning");
  if (p->fp32() && !search_fits(p->maxM, p->maxS, in->search_block))
    return fail(DIC_ERR_UNSUPPORTED,
                "search form does not fit: LDS, workgroup width, or radius above the "
                "matrix-core limit");
  p->tuning = *in;
  drop_graphs(p);
  return DIC_SUCCESS;
}

dic_status_t dic_plan_bind(dic_plan_t p, void* ws, size_t bytes, dic_stream_t stream) {
  dic_status_t r = check_plan(p, false);
  if (r) return r;
  if (!ws) return fail(DIC_ERR_INVALID_ARGUMENT, "null workspace");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(DIC_ERR_INVALID_ARGUMENT, "workspace not 256-byte aligned");
  if (bytes < p->lay.total) return fail(DIC_ERR_WORKSPACE_TOO_SMALL, "workspace smaller than dic_plan_workspace_size");
  r = attach_workspace(p, ws, reinterpret_cast<hipStream_t>(stream));
  if (r) return r;
  drop_graphs(p);
  if (const char* path = std::getenv("DIC_AUTOTUNE_CACHE")) {
    auto m = read_tune_cache(path);
    auto it = m.find(tune_key(p));
    if (it != m.end() && it->second.size() == 4) {
      dic_tuning_t t = {it->second[0], it->second[1], it->second[2], it->second[3]};
      if (tuning_valid(t) && (!p->fp32() || search_fits(p->maxM, p->maxS, t.search_block)))
        p->tuning = t;
    }
  }
  return DIC_SUCCESS;
}

dic_status_t dic_plan_invalidate_reference(dic_plan_t p) {
  dic_status_t r = check_plan(p, false);
  if (r) return r;
  p->ref_valid = false;
  p->def_valid = false;
  p->lut_valid = false;
  drop_graphs(p);
  return DIC_SUCCESS;
}

dic_status_t dic_prepare_reference(dic_plan_t p, const float* ref, const int32_t* poi,
                                   dic_stream_t stream) {
  dic_status_t r = check_plan(p, true);
  if (r) return r;
  if (!ref || (!poi && p->N)) return fail(DIC_ERR_INVALID_ARGUMENT, "null image or POI pointer");
  return prepare(p, ref, poi, reinterpret_cast<hipStream_t>(stream), true);
}

dic_status_t dic_prepare_deformed(dic_plan_t p, const float* def, dic_stream_t stream) {
  dic_status_t r = check_plan(p, true);
  if (r) return r;
  if (!def) return fail(DIC_ERR_INVALID_ARGUMENT, "null image pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  r = prepare_deformed(p, def, s, true);
  if (r) return r;
  return prepare_lut(p, def, s, true);
}

dic_status_t dic_integer_search(dic_plan_t p, const float* ref, const float* def,
                                const int32_t* poi, const int32_t* seed, int32_t* uv, float* zn,
                                int32_t* status, dic_stream_t stream) {
  dic_status_t r = check_plan(p, true);
  if (r) return r;
  if (p->N == 0) return DIC_SUCCESS;
  if (!ref || !def || !poi || !uv || !zn || !status)
    return fail(DIC_ERR_INVALID_ARGUMENT, "null required pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  r = prepare(p, ref, poi, s, false);
  if (r) return r;
  return enqueue_search(p, ref, def, poi, seed, uv, zn, status, s);
}

dic_status_t dic_icgn_refine(dic_plan_t p, const float* ref, const float* def, const int32_t* poi,
                             const int32_t* uv_init, const int32_t* status_in,
                             const double* p_init, double* p_out, float* zn, int32_t* iters,
                             int32_t* status, dic_stream_t stream) {
  dic_status_t r = check_plan(p, true);
  if (r) return r;
  if (p->N == 0) return DIC_SUCCESS;
  if (!ref || !def || !poi || !uv_init || !p_out || !zn || !iters || !status)
    return fail(DIC_ERR_INVALID_ARGUMENT, "null required pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  r = prepare(p, ref, poi, s, false);
  if (r) return r;
  return enqueue_refine(p, ref, def, poi, uv_init, status_in, p_init, p_out, zn, iters, status, s,
                        false);
}

dic_status_t dic_nr_refine(dic_plan_t p, const float* ref, const float* def, const int32_t* poi,
                           const int32_t* uv_init, const int32_t* status_in,
                           const double* p_init, double* p_out, float* zn, int32_t* iters,
                           int32_t* status, dic_stream_t stream) {
  dic_status_t r = check_plan(p, true);
  if (r) return r;
  if (p->N == 0) return DIC_SUCCESS;
  if (!ref || !def || !poi || !uv_init || !p_out || !zn || !iters || !status)
    return fail(DIC_ERR_INVALID_ARGUMENT, "null required pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  r = prepare(p, ref, poi, s, false);
  if (r) return r;
  return enqueue_refine(p, ref, def, poi, uv_init, status_in, p_init, p_out, zn, iters, status, s,
                        true);
}

dic_status_t dic_pso_search(dic_plan_t p, const float* ref, const float* def,
                            const int32_t* poi, const int32_t* seed, const float* swarm_random,
                            int32_t modified, int32_t* uv, float* zn, int32_t* status,
                            int32_t* generations, int32_t* evaluations, dic_stream_t stream) {
  dic_status_t r = check_plan(p, true);
  if (r) return r;
  if (p->N == 0) return DIC_SUCCESS;
  if (!ref || !def || !poi || !swarm_random || !uv || !zn || !status)
    return fail(DIC_ERR_INVALID_ARGUMENT, "null required pointer");
  if (modified != 0 && modified != 1)
    return fail(DIC_ERR_INVALID_ARGUMENT, "modified must be 0 or 1");
  if (!p->fp32())
    return fail(DIC_ERR_UNSUPPORTED, "the swarm search uses the FP32 batched form's box sums");
  const Range range(modified ? "dic: modified swarm search" : "dic: swarm search");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  r = prepare(p, ref, poi, s, false);
  if (r) return r;
  r = prepare_deformed(p, def, s, false);
  if (r) return r;
  DIC_HIP(launch_reset_counters(p->st, s));
  DIC_HIP(launch_pso(p->st, modified != 0, ref, def, poi, seed, swarm_random, uv, zn, status,
                     generations, evaluations, p->num_cu, s));
  return DIC_SUCCESS;
}

dic_status_t dic_correlate(dic_plan_t p, const float* ref, const float* def, const int32_t* poi,
                           const int32_t* seed, const double* p_init, int32_t* uv,
                           float* zn_int, int32_t* st_int, double* p_out, float* zn,
                           int32_t* iters, int32_t* status, dic_stream_t stream) {
  dic_status_t r = check_plan(p, true);
  if (r) return r;
  if (p->N == 0) return DIC_SUCCESS;
  if (!ref || !def || !poi || !uv || !p_out || !zn || !iters || !status)
    return fail(DIC_ERR_INVALID_ARGUMENT, "null required pointer");
  char* base = static_cast<char*>(p->ws);
  CorrArgs a{ref, def, poi, seed, p_init, uv,
             zn_int ? zn_int : reinterpret_cast<float*>(base + p->lay.s_zncc),
             st_int ? st_int : reinterpret_cast<int32_t*>(base + p->lay.s_status),
             p_out, zn, iters, status};
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (!(p->desc.flags & DIC_FLAG_USE_GRAPH)) return enqueue_correlate(p, a, s);
  const bool cached_ref = (p->desc.flags & DIC_FLAG_CACHE_REF_PREP) && p->ref_valid &&
                          (p->ref_tmpl || p->tuning.search_block == kMfmaBlock || !p->fp32()) &&
                          p->ref_img == ref && p->ref_poi == poi && p->def_valid &&
                          p->def_img == def &&
                          (!p->table() || (p->lut_valid && p->lut_img == def));
  std::vector<uintptr_t> key = {
      (uintptr_t)ref, (uintptr_t)def, (uintptr_t)poi, (uintptr_t)seed, (uintptr_t)p_init,
      (uintptr_t)uv, (uintptr_t)a.zn_int, (uintptr_t)a.st_int, (uintptr_t)p_out, (uintptr_t)zn,
      (uintptr_t)iters, (uintptr_t)status, (uintptr_t)cached_ref};
  auto it = p->graphs.find(key);
  if (it == p->graphs.end()) {
    if (!p->cap_stream) DIC_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    DIC_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeRelaxed));
    r = enqueue_correlate(p, a, p->cap_stream);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(p->cap_stream, &graph);
    if (r) {
      if (graph) (void)hipGraphDestroy(graph);
      return r;
    }
    if (e != hipSuccess) return fail(DIC_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return fail(DIC_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    p->graph_objs.push_back(graph);
    it = p->graphs.emplace(key, exec).first;
  }
  DIC_HIP(hipGraphLaunch(it->second, s));
  return DIC_SUCCESS;
}

dic_status_t dic_correlate_noalloc(dic_plan_t p, const float* ref, const float* def,
                                   const int32_t* poi, const int32_t* seed, const double* p_init,
                                   int32_t* uv, float* zn_int, int32_t* st_int, double* p_out,
                                   float* zn, int32_t* iters, int32_t* status,
                                   dic_stream_t stream) {
  dic_status_t r = check_plan(p, false);
  if (r) return r;
  if (p->N == 0) return DIC_SUCCESS;
  if (!ref || !def || !poi || !uv || !p_out || !zn || !iters || !status)
    return fail(DIC_ERR_INVALID_ARGUMENT, "null required pointer");
  if (p->lay.total > kNoallocScratchBytes) {
    std::ostringstream why;
    why << "plan needs " << p->lay.total << " bytes of device workspace; the static scratch of "
        << "dic_correlate_noalloc holds " << kNoallocScratchBytes
        << ": bind a caller workspace (dic_plan_bind) and use dic_correlate";
    return fail(DIC_ERR_WORKSPACE_TOO_SMALL, why.str());
  }
  void* base = nullptr;
  r = noalloc_scratch(&base);
  if (r) return r;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // The plan runs attached to the scratch for this call only: its own binding
  // (workspace, caches, graphs) is put back afterwards, untouched.
  struct Saved {
    void* ws;
    bool bound, ref_valid, ref_tmpl, def_valid, lut_valid;
    const void *ref_img, *ref_poi, *def_img, *lut_img;
    DevState st;
    int num_cu;
  } sv{p->ws,      p->bound,   p->ref_valid, p->ref_tmpl, p->def_valid, p->lut_valid,
       p->ref_img, p->ref_poi, p->def_img,   p->lut_img,  p->st,        p->num_cu};
  r = attach_workspace(p, base, s);
  if (r == DIC_SUCCESS) {
    char* b = static_cast<char*>(base);
    CorrArgs a{ref, def, poi, seed, p_init, uv,
               zn_int ? zn_int : reinterpret_cast<float*>(b + p->lay.s_zncc),
               st_int ? st_int : reinterpret_cast<int32_t*>(b + p->lay.s_status),
               p_out, zn, iters, status};
    r = enqueue_correlate(p, a, s, false);
  }
  p->ws = sv.ws;
  p->bound = sv.bound;
  p->ref_valid = sv.ref_valid;
  p->ref_tmpl = sv.ref_tmpl;
  p->def_valid = sv.def_valid;
  p->lut_valid = sv.lut_valid;
  p->ref_img = sv.ref_img;
  p->ref_poi = sv.ref_poi;
  p->def_img = sv.def_img;
  p->lut_img = sv.lut_img;
  p->st = sv.st;
  p->num_cu = sv.num_cu;
  return r;
}

dic_status_t dic_znssd_backward(dic_plan_t p, const float* ref, const float* def,
                                const int32_t* poi, const double* pw, const float* grad_c,
                                float* c_out, double* grad_p, float* grad_def,
                                dic_stream_t stream) {
  dic_status_t r = check_plan(p, true);
  if (r) return r;
  if (p->N == 0) return DIC_SUCCESS;
  if (!ref || !def || !poi || !pw) return fail(DIC_ERR_INVALID_ARGUMENT, "null required pointer");
  if (p->bilinear() || p->bspline())
    return fail(DIC_ERR_UNSUPPORTED, "the ZNSSD adjoint interpolates bicubically only");
  const Range range("dic: ZNSSD forward and backward");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  r = prepare(p, ref, poi, s, false);
  if (r) return r;
  char* base = static_cast<char*>(p->ws);
  unsigned long long* fix = p->det() ? reinterpret_cast<unsigned long long*>(base + p->lay.fix) : nullptr;
  const int64_t* fix_off = reinterpret_cast<const int64_t*>(base + p->lay.fix_off);
  const int32_t* fix_owner = reinterpret_cast<const int32_t*>(base + p->lay.fix_owner);
  DIC_HIP(launch_znssd(p->st, ref, def, poi, pw, grad_c, c_out, grad_p, grad_def, fix, fix_off,
                       fix_owner, (int)p->fix_owner.size(), p->lay.fix_count, p->num_cu, s));
  return DIC_SUCCESS;
}

dic_status_t dic_seed_update(dic_plan_t p, const double* pw, const int32_t* status,
                             int32_t* seed_uv, double* p_seed, dic_stream_t stream) {
  dic_status_t r = check_plan(p, true);
  if (r) return r;
  if (p->N == 0) return DIC_SUCCESS;
  if (!pw || !status || !seed_uv || !p_seed) return fail(DIC_ERR_INVALID_ARGUMENT, "null pointer");
  DIC_HIP(launch_seed_update(p->N, pw, status, seed_uv, p_seed, reinterpret_cast<hipStream_t>(stream)));
  return DIC_SUCCESS;
}

dic_status_t dic_poi_grid(int32_t width, int32_t height, int32_t M, int32_t S, int32_t step,
                          int32_t* out_xy, int64_t capacity, int64_t* count) {
  if (!count || step < 1 || M < 0 || S < 0 || width < 1 || height < 1 || capacity < 0 ||
      (capacity > 0 && !out_xy))
    return fail(DIC_ERR_INVALID_ARGUMENT, "invalid grid arguments");
  const int64_t m = (int64_t)M + S + 2;
  int64_t nx = 0, ny = 0;
  for (int64_t x = m; x <= width - 1 - m; x += step) ++nx;
  for (int64_t y = m; y <= height - 1 - m; y += step) ++ny;
  *count = nx * ny;
  int64_t k = 0;
  for (int64_t j = 0; j < ny; ++j)
    for (int64_t i = 0; i < nx; ++i, ++k)
      if (k < capacity) {
        out_xy[2 * k] = (int32_t)(m + i * step);
        out_xy[2 * k + 1] = (int32_t)(m + j * step);
      }
  return DIC_SUCCESS;
}

dic_status_t dic_plan_autotune(dic_plan_t p, const float* ref, const float* def,
                               const int32_t* poi, int32_t* uv, float* fs, int32_t* is,
                               double* ps, dic_stream_t stream) {
  dic_status_t r = check_plan(p, true);
  if (r) return r;
  if (!p->fp32() || p->N == 0) return DIC_SUCCESS;
  if (!ref || !def || !poi || !uv || !fs || !is || !ps)
    return fail(DIC_ERR_INVALID_ARGUMENT, "null pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  r = prepare(p, ref, poi, s, true, true);   // every search form may be timed
  if (r) return r;
  r = prepare_deformed(p, def, s, true);
  if (r) return r;
  hipEvent_t e0, e1;
  DIC_HIP(hipEventCreate(&e0));
  DIC_HIP(hipEventCreate(&e1));
  const dic_tuning_t saved = p->tuning;
  dic_tuning_t best = saved;
  auto time_it = [&](auto&& fn, float* ms) -> dic_status_t {
    dic_status_t q = fn();  // warm-up
    if (q) return q;
    DIC_HIP(hipEventRecord(e0, s));
    for (int k = 0; k < 2; ++k) {
      q = fn();
      if (q) return q;
    }
    DIC_HIP(hipEventRecord(e1, s));
    DIC_HIP(hipEventSynchronize(e1));
    DIC_HIP(hipEventElapsedTime(ms, e0, e1));
    return DIC_SUCCESS;
  };
  float best_ms = 1e30f;
  const int blocks[] = {4, 8, kMfmaBlock};
  const int occs[] = {0, 2, 3};
  for (int b : blocks)
    for (int o : occs) {
      dic_tuning_t c = best;
      c.search_block = b;
      c.search_occupancy = o;
      if (!search_fits(p->maxM, p->maxS, b)) continue;
      p->tuning = c;
      float ms = 0.f;
      r = time_it([&] { return enqueue_search(p, ref, def, poi, nullptr, uv, fs, is, s); }, &ms);
      if (r) continue;
      if (ms < best_ms) {
        best_ms = ms;
        best.search_block = c.search_block;
        best.search_occupancy = c.search_occupancy;
      }
    }
  p->tuning = best;
  r = enqueue_search(p, ref, def, poi, nullptr, uv, fs, is, s);
  if (r) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->tuning = saved;
    return r;
  }
  best_ms = 1e30f;
  const int waves[] = {1, 2, 4, 8};
  const int slacks[] = {2, 4, 6};
  for (int w : waves)
    for (int sl : slacks) {
      dic_tuning_t c = best;
      c.icgn_waves = w;
      c.icgn_slack = sl;
      p->tuning = c;
      float ms = 0.f;
      r = time_it([&] {
        return enqueue_refine(p, ref, def, poi, uv, is, nullptr, ps, fs, is + p->N, is + p->N, s,
                              p->nr());
      }, &ms);
      if (r) continue;
      if (ms < best_ms) {
        best_ms = ms;
        best.icgn_waves = w;
        best.icgn_slack = sl;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->tuning = best;
  drop_graphs(p);
  g_last_error.clear();
  if (const char* path = std::getenv("DIC_AUTOTUNE_CACHE")) {
    auto m = read_tune_cache(path);
    m[tune_key(p)] = {best.search_block, best.search_occupancy, best.icgn_waves, best.icgn_slack};
    write_tune_cache(path, m);
  }
  return DIC_SUCCESS;
}

}  // extern "C"
