// knn_api.cpp -- C ABI of the k-NN library: argument checks, launch plans,
// workspaces and reference-set handles.  Every computation runs in the HIP
// kernels of knn_kernels.hip.
#include <cmath>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <tuple>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "knn.h"
#include "knn_host.h"
#include "knn_internal.h"

using namespace knn;
using namespace knn::host;

// ------------------------------------------------------------ error state
namespace knn::host {

thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

int hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return fail(KNN_ERR_OOM, "%s: %s", what, hipGetErrorString(e));
  return fail(KNN_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
int64_t ceil_div(int64_t x, int64_t a) { return (x + a - 1) / a; }

// ------------------------------------------------------ device allocation
// Every device allocation of the library goes through dev_alloc, which also
// carries the allocation-failure test hook: with KNN_FAIL_ALLOC=N in the
// environment, the N-th allocation from then on (1 = the next) fails as if
// the device were out of memory, and the variable is cleared.
int dev_alloc(void** out, size_t bytes, const char* what) {
  *out = nullptr;
  static std::mutex hook_mutex;
  {
    std::lock_guard<std::mutex> lock(hook_mutex);
    const char* v = getenv("KNN_FAIL_ALLOC");
    if (v && *v) {
      const long left = atol(v);
      if (left <= 1) {
        unsetenv("KNN_FAIL_ALLOC");
        return fail(KNN_ERR_OOM, "%s: injected allocation failure (KNN_FAIL_ALLOC)", what);
      }
      char buf[32];
      snprintf(buf, sizeof buf, "%ld", left - 1);
      setenv("KNN_FAIL_ALLOC", buf, 1);
    }
  }
  const hipError_t e = hipMalloc(out, bytes);
  if (e != hipSuccess) {
    *out = nullptr;
    (void)hipGetLastError();
    return hip_fail(e, what);
  }
  return KNN_OK;
}

// --------------------------------------------------- per-stream workspace
// A grow-only device buffer per (device, stream).  A search holds the
// buffer's lock from the moment it takes the buffer until its last launch is
// enqueued, so the launches of two searches on one stream never interleave
// (stream order then keeps one search's kernels from overwriting the
// other's data).  A buffer that grows is released only after the work
// already enqueued on its stream has finished.
int workspace_grow(Workspace& w, hipStream_t stream, size_t bytes) {
  if (w.size >= bytes) return KNN_OK;
  if (w.ptr) {
    hipError_t e = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = hipFree(w.ptr);
    w.ptr = nullptr;
    w.size = 0;
    if (e != hipSuccess) return hip_fail(e, "releasing the workspace");
  }
  const size_t want = std::max(bytes, (size_t)1 << 20);
  int st = dev_alloc(&w.ptr, want, "workspace allocation");
  if (st != KNN_OK) return st;
  w.size = want;
  return KNN_OK;
}

std::mutex g_ws_mutex;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

Workspace* workspace_of(hipStream_t stream) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(g_ws_mutex);
  return &g_ws[{dev, stream}];  // std::map keeps element addresses stable
}

// ---------------------------------------------------------- kernel timing
// Optional start/stop events around every launch, on the launch's stream.
struct TimingRecord {
  std::string name;
  hipEvent_t start;
  hipEvent_t stop;
};

std::mutex g_tm_mutex;
bool g_tm_enabled = false;
thread_local bool g_tm_suppress = false;
std::vector<hipEvent_t> g_tm_pool;
std::vector<TimingRecord> g_tm_pending;
std::map<std::string, std::pair<double, int64_t>> g_tm_totals;

hipEvent_t tm_event() {
  if (!g_tm_pool.empty()) {
    hipEvent_t e = g_tm_pool.back();
    g_tm_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// RAII: records a start event now and a stop event when it goes out of scope.
class TimedLaunch {
 public:
  TimedLaunch(const char* name, hipStream_t s) : stream_(s) {
    if (g_tm_suppress) return;
    std::lock_guard<std::mutex> lock(g_tm_mutex);
    if (!g_tm_enabled) return;
    start_ = tm_event();
    stop_ = tm_event();
    if (start_ && stop_ && hipEventRecord(start_, s) == hipSuccess) {
      name_ = name;
      active_ = true;
    }
  }
  ~TimedLaunch() {
    if (!active_) return;
    std::lock_guard<std::mutex> lock(g_tm_mutex);
    if (hipEventRecord(stop_, stream_) == hipSuccess) g_tm_pending.push_back({name_, start_, stop_});
  }

 private:
  hipStream_t stream_;
  hipEvent_t start_ = nullptr, stop_ = nullptr;
  std::string name_;
  bool active_ = false;
};

int tm_collect() {
  for (auto& r : g_tm_pending) {
    hipError_t e = hipEventSynchronize(r.stop);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.start, r.stop);
    if (e != hipSuccess) return hip_fail(e, "timing events");
    auto& t = g_tm_totals[r.name];
    t.first += ms;
    t.second += 1;
    g_tm_pool.push_back(r.start);
    g_tm_pool.push_back(r.stop);
  }
  g_tm_pending.clear();
  return KNN_OK;
}

const char* fused_name(int kind) {
  switch (kind) {
    case TILE_L2_F32: return "fused_l2_f32";
    case TILE_L2_BF16: return "fused_l2_bf16";
    case TILE_L2_F16: return "fused_l2_f16";
    case TILE_L1_F32: return "fused_l1_f32";
    default: return "fused_linf_f32";
  }
}

// -------------------------------------------------------------- planning
struct Plan {
  int kind = 0;
  int waves = 8;
  int cb = 64;
  int ng = 1;      // k groups per chunk
  int group = 16;  // dims per k group
  int nchunk = 1;
  int P = 1;
  int64_t slice_len = 0;
  int kc = 0;
  int dp = 0;
  int es = 4;
  bool wide = false;  // the 32x32-tile Euclidean kernel with register lists
  bool lane = false;  // the one-query-per-lane Manhattan / infinity-norm kernel
  int nq = 128;       // queries per workgroup
  int G = 1;          // slice lists merged per group before the finalize (1: none)
  int P2 = 1;         // lists per query the finalize merges: ceil(P / G)
};

// Slices of a search: at most kMaxSlices, and at least max(kStepRefs, 4 k')
// references each.  With k' <= 64, more than kFinalMaxKeys / k' lists per
// query are first merged in groups (merge_lists_kernel); larger k' keeps the
// finalize's limit.
int64_t cap_slices(int64_t P, int kc, int64_t m) {
  const int64_t pmax_len = std::max<int64_t>(1, m / std::max<int64_t>(kStepRefs, 4 * (int64_t)kc));
  const int64_t cap = kc <= 64 ? kMaxSlices : std::min<int64_t>(64, kFinalMaxKeys / kc);
  return std::max<int64_t>(1, std::min<int64_t>({P, cap, pmax_len}));
}

// the merge groups of a plan with P slices
void plan_merge(Plan& p) {
  const int64_t p2max = std::min<int64_t>(64, kFinalMaxKeys / p.kc);
  if (p.P <= p2max) {
    p.G = 1;
    p.P2 = p.P;
    return;
  }
  p.G = (int)ceil_div(p.P, p2max);
  p.P2 = (int)ceil_div(p.P, p.G);
}

bool is_half_kind(int kind) { return kind == TILE_L2_BF16 || kind == TILE_L2_F16; }

// dims per k group of a tile kind: four float32 MFMAs (16 dims), one 16-bit
// MFMA (32 dims), or 16 dims of the vector-ALU kinds
int group_dims(int kind) { return is_half_kind(kind) ? 32 : 16; }

// padded dimension of the rows a tile kind reads: a whole number of k groups
int padded_dim(int kind, int d) { return (int)round_up(d, group_dims(kind)); }

int device_cu_count() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      cus = prop.multiProcessorCount;
    if (cus <= 0) cus = 256;
  }
  return cus;
}

// Environment overrides of the launch plan, for tuning sweeps: KNN_FUSED_WAVES,
// KNN_FUSED_CB, KNN_FUSED_NG, KNN_FUSED_P.  A value the plan cannot honour is
// ignored.
int env_int(const char* name) {
  const char* v = getenv(name);
  return v ? atoi(v) : 0;
}

// KNN_SLICE_SHARE=0 turns off the bound a query's slices share (timing comparisons)
bool slice_share_on() {
  const char* v = getenv("KNN_SLICE_SHARE");
  return !(v && atoi(v) == 0);
}

// KNN_RANK_SHARE=0 turns off the rank slots of a query's slices (timing comparisons)
bool rank_share_on() {
  const char* v = getenv("KNN_RANK_SHARE");
  return !(v && atoi(v) == 0);
}

// The rank slots of an instance whose queries are split over P slices (see
// FusedInst::tshare): each slice publishes its r-th best, r = ceil(kc / P)
// (at least ceil(kc / 64), so that a group spans at most 64 slices and the
// r-th key lies in the first 64 of a list); gs = ceil(kc / r) slices make a
// group (gs * r >= kc, gs <= P) and up to 4 groups are read.
void set_rank_plan(FusedInst& fi) {
  fi.rank_r = fi.rank_gs = fi.rank_G = 0;
  if (!fi.tshare || fi.P < kRankMinSlices || !rank_share_on()) return;
  const int r = (int)std::max(ceil_div((int64_t)fi.kc, (int64_t)fi.P), ceil_div((int64_t)fi.kc, (int64_t)64));
  const int gs = (int)ceil_div((int64_t)fi.kc, (int64_t)r);
  fi.rank_r = r;
  fi.rank_gs = gs;
  fi.rank_G = std::max(1, std::min(fi.P / gs, 4));
}

// workspace bytes of the shared bounds and rank slots of n queries over P slices
size_t share_bytes(int64_t n, int P) { return (size_t)n * 4 * (1 + (size_t)P); }

// tiled_refs: the references can be prepared in the 32-row tile layout (one-shot
// searches), which makes the float32 lane kernel the faster one up to far longer slices
int make_plan(int kind, int64_t n, int64_t m, int d, int kc, bool tiled_refs, Plan* out) {
  Plan p;
  p.kind = kind;
  p.kc = kc;
  p.group = group_dims(kind);
  p.dp = padded_dim(kind, d);
  p.es = is_half_kind(kind) ? 2 : 4;
  const int total = p.dp / p.group;
  const int gmax = kind == TILE_L2_F32 ? kMaxGroupsF32 : is_half_kind(kind) ? kMaxGroups16 : kMaxGroupsValu;
  const int ew = env_int("KNN_FUSED_WAVES"), ecb = env_int("KNN_FUSED_CB"), eng = env_int("KNN_FUSED_NG");
  // Euclidean with k' <= 64 and d <= 128: the 32x32-tile kernel with
  // register lists (KNN_FUSED_WIDE=0 selects the general kernel instead)
  const char* ewide = getenv("KNN_FUSED_WIDE");
  const int wide_kc = kind == TILE_L2_F32 ? kWideMaxKc1 : kWideMaxKc;
  if (kind <= TILE_L2_F16 && kc <= wide_kc && p.dp <= kWideMaxDp && !(ewide && atoi(ewide) == 0)) {
    p.wide = true;
    p.waves = 8;
    p.cb = 32;
    p.ng = p.dp / 16;
    p.nchunk = 1;
    p.nq = kWideQueries;
    const int64_t nqb = ceil_div(n, (int64_t)p.nq);
    int64_t P = cap_slices(ceil_div((int64_t)device_cu_count(), nqb), kc, m);
    const int ep = env_int("KNN_FUSED_P");
    if (ep > 0) P = std::min<int64_t>({(int64_t)ep, cap_slices(ep, kc, m), ceil_div(m, kStepRefs)});
    p.slice_len = round_up(ceil_div(m, P), kStepRefs);
    p.P = (int)ceil_div(m, p.slice_len);
    plan_merge(p);
    // Float32 steps are long, so the 32x32 kernel pays off only where its
    // per-query merges are spread over a long scan; shorter slices take the
    // float32 lane kernel (or the general kernel), and one-shot searches,
    // whose references the lane kernel reads in the tile layout, keep the
    // 32x32 kernel only for the longest scans.
    const int64_t min_f32 = tiled_refs && p.dp <= kLaneMaxDp ? kWideMinSliceF32Tiled : kWideMinSliceF32;
    if (!(kind == TILE_L2_F32 && p.slice_len < min_f32)) {
      *out = p;
      return KNN_OK;
    }
    p = Plan{};
    p.kind = kind;
    p.kc = kc;
    p.group = group_dims(kind);
    p.dp = padded_dim(kind, d);
    p.es = 4;
  }
  // Per-lane selection with dp <= 128: Manhattan / infinity norm with one
  // query per lane (64 per wave), float32 Euclidean on 32x32 MFMA tiles with
  // one query per lane pair (32 per wave); up to 4 waves per workgroup as
  // the LDS lists allow (KNN_FUSED_LANE=0 selects the general kernel instead)
  const char* elane = getenv("KNN_FUSED_LANE");
  if ((kind >= TILE_L1_F32 || kind == TILE_L2_F32) && p.dp <= kLaneMaxDp && !(elane && atoi(elane) == 0)) {
    const int qw = kind == TILE_L2_F32 ? 32 : kWaveSize;  // queries per wave
    // the (waves, queue) pair with the most resident waves per CU (two per
    // SIMD at most, for registers), the larger queue where it costs none
    int waves = 0, queue = 0, best = 0;
    const int eq = env_int("KNN_LANE_QUEUE");
    for (int t : {12, 8}) {
      if (eq && t != eq) continue;
      for (int w : {4, 2, 1}) {
        if (ew && w != ew) continue;
        if (w > 1 && (int64_t)(w / 2) * qw >= n) continue;  // no wave without a query
        const size_t lds = lane_lds(w, kc, t);
        if (lds > (size_t)kLdsBytes) continue;
        const int resident = w * std::min<int>(8 / w, (int)(kLdsBytes / lds));
        if (resident > best) {
          best = resident;
          waves = w;
          queue = t;
        }
      }
    }
    if (waves > 0) {
      p.lane = true;
      p.waves = waves;
      p.cb = queue;
      p.ng = p.dp / 16;
      p.nchunk = 1;
      p.nq = waves * qw;
      // two waves per SIMD at most (register budget), fewer where LDS binds
      const int wg_per_cu = best / waves;
      const int64_t nqb = ceil_div(n, (int64_t)p.nq);
      int64_t P = cap_slices(ceil_div((int64_t)device_cu_count() * wg_per_cu, nqb), kc, m);
      const int ep = env_int("KNN_FUSED_P");
      if (ep > 0) P = std::min<int64_t>({(int64_t)ep, cap_slices(ep, kc, m), m});
      p.slice_len = round_up(ceil_div(m, P), 32);
      p.P = (int)ceil_div(m, p.slice_len);
      plan_merge(p);
      *out = p;
      return KNN_OK;
    }
  }
  bool found = false;
  // prefer 8 waves (two per SIMD), then the widest chunk, then the largest
  // candidate buffer (the buffer must hold one step: cb >= 64)
  for (int waves : {8, 4, 2, 1}) {
    if (ew && waves != ew) continue;
    for (int ng = std::min(total, gmax); ng >= 1 && !found; --ng) {
      if (eng && ng != eng) continue;
      // with k' <= 64 a 64-key buffer takes the register merge
      for (int cb : {128, 96, 64}) {
        if (kc <= 64 && cb > 64 && !ecb) continue;
        if (ecb && cb != ecb) continue;
        if (kc + cb > 64 * kMaxMergePerLane) continue;
        if (fused_lds_bytes(kind, waves, kc, cb, ng * p.group) > (size_t)kLdsBytes) continue;
        p.waves = waves;
        p.cb = cb;
        p.ng = ng;
        found = true;
        break;
      }
    }
    if (found) break;
  }
  if (!found)
    return fail(KNN_ERR_UNSUPPORTED, "k' = %d candidates per query do not fit the fused kernel's LDS budget", kc);
  p.nchunk = (int)ceil_div(total, p.ng);
  p.nq = p.waves * kQueriesPerWave;
  const size_t lds = fused_lds_bytes(kind, p.waves, kc, p.cb, p.ng * p.group);
  const int wg_per_cu = std::max<int>(1, (int)(kLdsBytes / lds));
  const int64_t nqb = ceil_div(n, (int64_t)p.nq);
  const int64_t target = (int64_t)device_cu_count() * wg_per_cu;
  int64_t P = cap_slices(ceil_div(target, nqb), kc, m);
  const int ep = env_int("KNN_FUSED_P");
  if (ep > 0) P = std::min<int64_t>({(int64_t)ep, cap_slices(ep, kc, m), ceil_div(m, kStepRefs)});
  p.slice_len = round_up(ceil_div(m, P), kStepRefs);
  p.P = (int)ceil_div(m, p.slice_len);
  plan_merge(p);
  *out = p;
  return KNN_OK;
}

int check_ptr(const void* ptr, const char* name) {
  if (!ptr) return fail(KNN_ERR_INVALID, "%s is NULL", name);
  return KNN_OK;
}

}  // namespace knn::host

namespace knn::host {


int elem_of_kind(int kind) {
  return kind == TILE_L2_BF16 ? ELEM_BF16 : kind == TILE_L2_F16 ? ELEM_F16 : ELEM_F32;
}

// Run one search in the caller's workspace `ws` of `ws_size` bytes.  With
// ws == nullptr only the needed size is stored in *need.
int run_search_ws(const SearchArgs& a, void* ws_in, size_t ws_size, size_t* need) {
  Plan plan;
  int st = make_plan(a.kind, a.n, a.m, a.d, a.kprime, a.R32 != nullptr, &plan);
  if (st != KNN_OK) return st;
  const bool l2 = a.kind <= TILE_L2_F16;
  const bool one_shot = a.R32 != nullptr;
  const bool d_pad_free = plan.dp == a.d;
  // one-shot Euclidean: centre + translated rows; one-shot L1/Linf: the
  // caller's rows serve directly when no padding is needed and they are aligned
  const bool prep_refs = one_shot && (l2 || !d_pad_free || ((uintptr_t)a.R32 % 16) != 0);
  const bool centre_refs = one_shot && l2;
  const float* centre = one_shot ? nullptr : a.centre;
  const bool prep_q = l2 || !d_pad_free || ((uintptr_t)a.Q % 16) != 0;

  const size_t cbytes = centre_refs ? (size_t)round_up((int64_t)a.d * 4, 256) : 0;
  const size_t pbytes0 = 0;
  // the float32 Euclidean lane kernel reads one-shot references in the
  // 32-row tile layout (whole tiles allocated)
  const bool tiled = one_shot && plan.lane && a.kind == TILE_L2_F32;
  const int64_t mrows = tiled ? round_up(a.m, (int64_t)32) : a.m;
  const size_t rbytes = prep_refs ? (size_t)round_up(mrows * plan.dp * plan.es, 256) : 0;
  const size_t hbytes = prep_refs && l2 ? (size_t)round_up(a.m * 4, 256) : 0;
  const size_t qbytes = prep_q ? (size_t)round_up(a.n * plan.dp * plan.es, 256) : 0;
  const size_t kbytes = (size_t)round_up(a.n * plan.P * (int64_t)plan.kc * 8, 256);
  const size_t k2bytes = plan.G > 1 ? (size_t)round_up(a.n * plan.P2 * (int64_t)plan.kc * 8, 256) : 0;
  const size_t tbytes = a.nsubs > 0 ? sub_tables_bytes(a.nsubs, a.n) : 0;
  // the 32x32-tile kernel's slices of one query share their bound
  const bool share = plan.wide && plan.P > 1 && prep_q && slice_share_on();
  const size_t sbytes = share ? (size_t)round_up((int64_t)share_bytes(a.n, plan.P), 256) : 0;
  const size_t total = cbytes + pbytes0 + rbytes + hbytes + qbytes + kbytes + k2bytes + tbytes + sbytes;
  if (need) *need = total;
  if (!ws_in) return KNN_OK;
  if (ws_size < total) return fail(KNN_ERR_INVALID, "workspace of %zu bytes is smaller than the %zu needed", ws_size, total);
  unsigned char* w = (unsigned char*)ws_in;
  float* wcentre = (float*)w;
  unsigned char* wrows = w + cbytes + pbytes0;
  float* wrhalf = (float*)(wrows + rbytes);
  unsigned char* wq = wrows + rbytes + hbytes;
  uint64_t* part = (uint64_t*)(wq + qbytes);
  uint64_t* part2 = (uint64_t*)((unsigned char*)part + kbytes);
  unsigned char* tables = (unsigned char*)part2 + k2bytes;
  uint32_t* tshare = share ? (uint32_t*)(tables + tbytes) : nullptr;
  const int nslots = share && rank_share_on() ? plan.P : 0;

  const void* rows = a.rows;
  int ldr = a.ldr;
  const float* rhalf = a.rhalf;
  if (centre_refs) {
    TimedLaunch tl("centre", a.stream);
    HIP_TRY(launch_centre(a.R32, a.m, a.d, a.d, wcentre, a.stream), "centre launch");
    centre = wcentre;
  }
  if (one_shot) {
    if (prep_refs) {
      TimedLaunch tl("prep_refs", a.stream);
      if (tiled)
        HIP_TRY(launch_prep_rows_tiled(a.R32, a.m, a.d, a.d, centre, (float*)wrows, plan.dp, wrhalf, a.stream),
                "reference preparation launch");
      else
        HIP_TRY(launch_prep_rows(a.R32, a.m, a.d, a.d, centre, wrows, plan.dp, elem_of_kind(a.kind),
                                 l2 ? wrhalf : nullptr, a.stream),
                "reference preparation launch");
      rows = wrows;
      rhalf = l2 ? wrhalf : nullptr;
    } else {
      rows = a.R32;
    }
    ldr = plan.dp;
  }
  const void* qp = a.Q;
  int ldq = a.d;
  if (prep_q) {
    TimedLaunch tl("prep_queries", a.stream);
    HIP_TRY(launch_prep_rows(a.Q, a.n, a.d, a.d, l2 ? centre : nullptr, wq, plan.dp, elem_of_kind(a.kind), nullptr,
                             a.stream, nullptr, tshare, nslots),
            "query preparation launch");
    qp = wq;
    ldq = plan.dp;
  }

  FusedParams fp{};
  FusedInst& fi = fp.one;
  fi.Q = qp;
  fi.R = rows;
  fi.rhalf = rhalf;
  fi.part = part;
  fi.n = a.n;
  fi.m = a.m;
  fi.slice_len = plan.slice_len;
  fi.ldq = ldq;
  fi.ldr = ldr;
  fi.dp = plan.dp;
  fi.nchunk = plan.nchunk;
  fi.P = plan.P;
  fi.kc = plan.kc;
  fi.tshare = tshare;
  set_rank_plan(fi);
  fp.insts = nullptr;
  fp.items = nullptr;
  fp.nitems = 0;
  fp.ng = plan.ng;
  fp.cb = plan.cb;
  fp.waves = plan.waves;
  fp.kc_max = plan.kc;
  fp.wide = plan.wide ? 1 : 0;
  fp.lane = plan.lane ? 1 : 0;
  fp.tiled = tiled ? 1 : 0;
  {
    TimedLaunch tl(fused_name(a.kind), a.stream);
    HIP_TRY(launch_fused(a.kind, fp, a.stream), "fused distance/selection launch");
  }

  if (plan.G > 1) {
    TimedLaunch tl("merge", a.stream);
    HIP_TRY(launch_merge_lists(part, part2, a.n, plan.P, plan.kc, plan.G, plan.P2, a.stream), "slice-list merge launch");
  }

  FinalParams fin{};
  FinalInst& f1 = fin.one;
  f1.part = plan.G > 1 ? part2 : part;
  f1.Q = a.Q;
  f1.ldq = a.d;
  if (one_shot) {
    f1.Rm = a.R32;
    f1.rm_type = ELEM_F32;
    f1.ldr = a.d;
  } else {
    f1.Rm = a.canon;
    f1.rm_type = a.canon_type;
    f1.ldr = a.ld_canon;
  }
  f1.dist = a.dist;
  f1.idx = a.idx;
  f1.n = a.n;
  f1.m = a.m;
  f1.d = a.d;
  f1.P = plan.P2;
  f1.kc = plan.kc;
  f1.kprime = a.kprime;
  f1.k = a.k;
  f1.metric = a.metric;
  fin.insts = nullptr;
  fin.items = nullptr;
  fin.nitems = 0;
  fin.keys_max = plan.P2 * plan.kc;
  fin.p_max = plan.P2;
  fin.kprime_max = a.kprime;
  if (a.nsubs > 0) {
    // one finalize instance per request, each with its own k and k': the
    // first k'_i keys of a row's merged top-k' list are that row's top k'_i
    FinalInst* ti = (FinalInst*)a.tables_host;
    FinalItem* tt = (FinalItem*)((unsigned char*)a.tables_host + round_up(a.nsubs * (int64_t)sizeof(FinalInst), 16));
    int nitems = 0;
    for (int i = 0; i < a.nsubs; ++i) {
      const SubSearch& sb = a.subs[i];
      if (sb.row0 < 0 || sb.n < 1 || sb.row0 + sb.n > a.n || sb.kprime > a.kprime || sb.k > sb.kprime || sb.k < 1)
        return fail(KNN_ERR_INVALID, "request %d of the search does not fit it", i);
      FinalInst fi = f1;
      fi.part = f1.part + sb.row0 * (int64_t)plan.P2 * plan.kc;
      fi.Q = a.Q + sb.row0 * (int64_t)a.d;
      fi.dist = sb.dist;
      fi.idx = sb.idx;
      fi.n = sb.n;
      fi.kprime = sb.kprime;
      fi.k = sb.k;
      ti[i] = fi;
      for (int64_t q = 0; q < sb.n; q += kFinalWaves) tt[nitems++] = FinalItem{i, (int)q};
    }
    HIP_TRY(hipMemcpyAsync(tables, a.tables_host, tbytes, hipMemcpyHostToDevice, a.stream), "finalize tables copy");
    fin.insts = (const FinalInst*)tables;
    fin.items = (const FinalItem*)(tables + ((unsigned char*)tt - (unsigned char*)ti));
    fin.nitems = nitems;
  }
  {
    TimedLaunch tl("finalize", a.stream);
    HIP_TRY(launch_finalize(fin, a.stream), "finalize launch");
  }
  return KNN_OK;
}

size_t sub_tables_bytes(int nsubs, int64_t n) {
  const int64_t items = n / kFinalWaves + nsubs;  // >= sum over requests of ceil(n_i / kFinalWaves)
  return (size_t)round_up(round_up(nsubs * (int64_t)sizeof(FinalInst), 16) + items * (int64_t)sizeof(FinalItem), 256);
}

// ------------------------------------------------- multi-set search
// Several requests (each: some query rows against one resident 16-bit set,
// with its own k) in one launch of the 32x32 register-list kernel.  Layout
// of the workspace: per request its prepared queries and slice lists (and
// merged lists when it has more slices than the finalize takes), then the
// tables -- query preparation jobs, fused instances, fused items, finalize
// instances, finalize items, the item counter -- which the host writes to
// `tables_host` and one copy moves to the device.

int tile_kind(int metric, int precision);

bool multi_supported(const knn_refs_s* r, int precision, int kprime) {
  if (!(precision == KNN_BF16 || precision == KNN_FP16) || r->storage != precision) return false;
  const int kind = tile_kind(KNN_L2, precision);
  return kprime <= kWideMaxKc && padded_dim(kind, r->d) <= kWideMaxDp;
}

namespace {

struct MultiPlan {
  struct Req {
    int P = 1, G = 1, P2 = 1;
    int64_t slice_len = 0;
    size_t q_off = 0, part_off = 0, part2_off = 0, share_off = 0;
  };
  std::vector<Req> req;
  int dp = 0, kind = 0;
  int64_t nitems = 0, nfitems = 0;
  size_t tables_off = 0, jobs_off = 0, insts_off = 0, items_off = 0, finsts_off = 0, fitems_off = 0, counter_off = 0;
  size_t total = 0, tables_bytes = 0;
};

int multi_plan(const MultiReq* reqs, int nreq, int precision, MultiPlan* out) {
  MultiPlan& mp = *out;
  mp = MultiPlan{};
  mp.kind = tile_kind(KNN_L2, precision);
  mp.req.resize(nreq);
  // one slice length for the launch: about two items per CU over all the
  // requests' query blocks, at least 16 steps
  int64_t work = 0;
  for (int i = 0; i < nreq; ++i) {
    const MultiReq& r = reqs[i];
    if (!valid_refs(r.refs) || !multi_supported(r.refs, precision, r.kprime) || r.n < 1 || r.k < 1 ||
        r.k > r.kprime || r.kprime > r.refs->m)
      return fail(KNN_ERR_INVALID, "request %d of the multi-set search is not supported", i);
    if (i > 0 && r.refs->d != reqs[0].refs->d) return fail(KNN_ERR_INVALID, "requests differ in dimension");
    work += ceil_div(r.n, (int64_t)kWideQueries) * r.refs->m;
  }
  mp.dp = padded_dim(mp.kind, reqs[0].refs->d);
  const int64_t target = std::max<int64_t>(16 * kStepRefs, round_up(ceil_div(work, 2 * (int64_t)device_cu_count()),
                                                                     kStepRefs));
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (size_t)round_up((int64_t)std::max<size_t>(bytes, 1), 256);
    return at;
  };
  for (int i = 0; i < nreq; ++i) {
    const MultiReq& r = reqs[i];
    MultiPlan::Req& q = mp.req[i];
    const int64_t m = r.refs->m;
    // slices: up to kMaxSlices, merged in groups first when more than the
    // finalize takes (k' <= 64 only)
    const int64_t p2max = std::min<int64_t>(64, kFinalMaxKeys / r.kprime);
    const int64_t pcap = r.kprime <= 64 ? kMaxSlices : p2max;
    const int64_t P = std::max<int64_t>(1, std::min<int64_t>({pcap, ceil_div(m, target), m / (4 * (int64_t)r.kprime) + 1}));
    q.slice_len = round_up(ceil_div(m, P), kStepRefs);
    q.P = (int)ceil_div(m, q.slice_len);
    q.G = q.P <= p2max ? 1 : (int)ceil_div(q.P, p2max);
    q.P2 = (int)ceil_div(q.P, q.G);
    q.q_off = take((size_t)r.n * mp.dp * 2);
    q.part_off = take((size_t)r.n * q.P * r.kprime * 8);
    if (q.G > 1) q.part2_off = take((size_t)r.n * q.P2 * r.kprime * 8);
    q.share_off = take(share_bytes(r.n, q.P));
    mp.nitems += ceil_div(r.n, (int64_t)kWideQueries) * q.P;
    mp.nfitems += ceil_div(r.n, (int64_t)kFinalWaves);
  }
  mp.tables_off = off;
  size_t toff = 0;
  auto ttake = [&](size_t bytes) {
    const size_t at = toff;
    toff += (size_t)round_up((int64_t)std::max<size_t>(bytes, 1), 16);
    return at;
  };
  mp.jobs_off = ttake(nreq * sizeof(PrepJob));
  mp.insts_off = ttake(nreq * sizeof(FusedInst));
  mp.items_off = ttake((size_t)mp.nitems * sizeof(FusedItem));
  mp.finsts_off = ttake(nreq * sizeof(FinalInst));
  mp.fitems_off = ttake((size_t)mp.nfitems * sizeof(FinalItem));
  mp.counter_off = ttake(sizeof(int));
  mp.tables_bytes = (size_t)round_up((int64_t)toff, 256);
  mp.total = mp.tables_off + mp.tables_bytes;
  return KNN_OK;
}

}  // namespace

int run_multi_ws(const MultiReq* reqs, int nreq, const float* Q, int precision, void* ws_in, size_t ws_size,
                 size_t* need, void* tables_host, size_t* tables_need, hipStream_t stream) {
  if (nreq < 1) return fail(KNN_ERR_INVALID, "no request");
  MultiPlan mp;
  int st = multi_plan(reqs, nreq, precision, &mp);
  if (st != KNN_OK) return st;
  if (need) *need = mp.total;
  if (tables_need) *tables_need = mp.tables_bytes;
  if (!ws_in) return KNN_OK;
  if (ws_size < mp.total) return fail(KNN_ERR_INVALID, "workspace of %zu bytes is smaller than the %zu needed",
                                      ws_size, mp.total);
  if (!tables_host) return fail(KNN_ERR_INVALID, "no host staging for the tables");
  unsigned char* w = (unsigned char*)ws_in;
  unsigned char* tdev = w + mp.tables_off;
  unsigned char* th = (unsigned char*)tables_host;
  PrepJob* jobs = (PrepJob*)(th + mp.jobs_off);
  FusedInst* insts = (FusedInst*)(th + mp.insts_off);
  FusedItem* items = (FusedItem*)(th + mp.items_off);
  FinalInst* finsts = (FinalInst*)(th + mp.finsts_off);
  FinalItem* fitems = (FinalItem*)(th + mp.fitems_off);
  const int elem = elem_of_kind(mp.kind);
  int64_t prep_rows = 0;
  int kc_max = 0, keys_max = 0, p_max = 1, kprime_max = 0;
  // items, longest first: full query blocks of long slices before the rest
  struct Cost {
    int64_t cost;
    FusedItem it;
  };
  std::vector<Cost> all;
  all.reserve((size_t)mp.nitems);
  int64_t nf = 0;
  for (int i = 0; i < nreq; ++i) {
    const MultiReq& r = reqs[i];
    const knn_refs_s* R = r.refs;
    const MultiPlan::Req& q = mp.req[i];
    PrepJob& jb = jobs[i];
    jb = PrepJob{};
    jb.src = Q + r.row0 * (int64_t)R->d;
    jb.dst = w + q.q_off;
    jb.centre = R->centre;
    jb.rhalf = nullptr;
    jb.rows = r.n;
    jb.row0 = prep_rows;
    jb.d = R->d;
    jb.lds = R->d;
    jb.ldd = mp.dp;
    jb.elem = elem;
    jb.tshare = (uint32_t*)(w + q.share_off);
    jb.nslots = rank_share_on() ? q.P : 0;
    prep_rows += r.n;
    FusedInst& fi = insts[i];
    fi = FusedInst{};
    fi.Q = w + q.q_off;
    fi.R = R->rows;
    fi.rhalf = R->rhalf;
    fi.part = (uint64_t*)(w + q.part_off);
    fi.n = r.n;
    fi.m = R->m;
    fi.slice_len = q.slice_len;
    fi.ldq = mp.dp;
    fi.ldr = R->dp;
    fi.dp = mp.dp;
    fi.nchunk = 1;
    fi.P = q.P;
    fi.kc = r.kprime;
    fi.tshare = q.P > 1 && slice_share_on() ? (uint32_t*)(w + q.share_off) : nullptr;
    set_rank_plan(fi);
    const int64_t qb = ceil_div(r.n, (int64_t)kWideQueries);
    for (int64_t b = 0; b < qb; ++b)
      for (int sl = 0; sl < q.P; ++sl) {
        const int64_t refs = std::min<int64_t>(q.slice_len, R->m - sl * q.slice_len);
        all.push_back({refs * (mp.dp + 64), FusedItem{i, (int)b, sl, 0}});
      }
    FinalInst& f = finsts[i];
    f = FinalInst{};
    f.part = (const uint64_t*)(w + (q.G > 1 ? q.part2_off : q.part_off));
    f.Q = Q + r.row0 * (int64_t)R->d;
    f.ldq = R->d;
    if (R->master) {
      f.Rm = R->master;
      f.rm_type = ELEM_F32;
      f.ldr = R->dp32;
    } else {
      f.Rm = R->rows;
      f.rm_type = elem;
      f.ldr = R->dp;
    }
    f.dist = r.dist;
    f.idx = r.idx;
    f.n = r.n;
    f.m = R->m;
    f.d = R->d;
    f.P = q.P2;
    f.kc = r.kprime;
    f.kprime = r.kprime;
    f.k = r.k;
    f.metric = KNN_L2;
    for (int64_t q0 = 0; q0 < r.n; q0 += kFinalWaves) fitems[nf++] = FinalItem{i, (int)q0};
    kc_max = std::max(kc_max, r.kprime);
    keys_max = std::max(keys_max, q.P2 * r.kprime);
    p_max = std::max(p_max, q.P2);
    kprime_max = std::max(kprime_max, r.kprime);
  }
  std::stable_sort(all.begin(), all.end(), [](const Cost& x, const Cost& y) { return x.cost > y.cost; });
  for (size_t j = 0; j < all.size(); ++j) items[j] = all[j].it;
  *(int*)(th + mp.counter_off) = 0;
  HIP_TRY(hipMemcpyAsync(tdev, th, mp.tables_bytes, hipMemcpyHostToDevice, stream), "multi-set tables copy");
  int* counter = (int*)(tdev + mp.counter_off);
  {
    TimedLaunch tl("prep_queries", stream);
    HIP_TRY(launch_prep_batched((const PrepJob*)(tdev + mp.jobs_off), nreq, prep_rows, stream, counter),
            "multi-set query preparation launch");
  }
  FusedParams fp{};
  fp.insts = (const FusedInst*)(tdev + mp.insts_off);
  fp.items = (const FusedItem*)(tdev + mp.items_off);
  fp.nitems = (int)mp.nitems;
  fp.wide = 1;
  fp.ng = mp.dp / 16;
  fp.cb = 32;
  fp.waves = 8;
  fp.kc_max = kc_max;
  // Every request has the same padded dimension; with one key per lane for
  // all of them (k' <= 64) the kernel built for that dimension alone takes
  // the items, in table order, one per workgroup (fewer registers than the
  // kernel that serves every dimension and both list sizes); otherwise that
  // kernel takes them through the counter.
  fp.counter = kc_max <= kWideMaxKc1 ? nullptr : counter;
  {
    TimedLaunch tl(fused_name(mp.kind), stream);
    HIP_TRY(launch_fused(mp.kind, fp, stream), "multi-set fused launch");
  }
  for (int i = 0; i < nreq; ++i) {
    const MultiPlan::Req& q = mp.req[i];
    if (q.G <= 1) continue;
    TimedLaunch tl("merge", stream);
    HIP_TRY(launch_merge_lists((const uint64_t*)(w + q.part_off), (uint64_t*)(w + q.part2_off), reqs[i].n, q.P,
                               reqs[i].kprime, q.G, q.P2, stream),
            "slice-list merge launch");
  }
  FinalParams fin{};
  fin.insts = (const FinalInst*)(tdev + mp.finsts_off);
  fin.items = (const FinalItem*)(tdev + mp.fitems_off);
  fin.nitems = (int)mp.nfitems;
  fin.keys_max = keys_max;
  fin.p_max = p_max;
  fin.kprime_max = kprime_max;
  {
    TimedLaunch tl("finalize", stream);
    HIP_TRY(launch_finalize(fin, stream), "multi-set finalize launch");
  }
  return KNN_OK;
}

// Run one search in the library's per-stream workspace.
int run_search(const SearchArgs& a) {
  size_t need = 0;
  int st = run_search_ws(a, nullptr, 0, &need);
  if (st != KNN_OK) return st;
  Workspace* w = workspace_of(a.stream);
  if (!w) return fail(KNN_ERR_DEVICE, "hipGetDevice failed");
  std::lock_guard<std::mutex> lock(w->mu);
  st = workspace_grow(*w, a.stream, need);
  if (st != KNN_OK) return st;
  return run_search_ws(a, w->ptr, need, nullptr);
}

int check_common(int64_t n, int64_t m, int32_t d, int32_t k, int32_t metric) {
  if (n < 0) return fail(KNN_ERR_INVALID, "n = %lld is negative", (long long)n);
  if (m < 1) return fail(KNN_ERR_INVALID, "m = %lld: at least one reference is required", (long long)m);
  if (m > 0x7fffffffLL) return fail(KNN_ERR_UNSUPPORTED, "m = %lld exceeds 2^31 - 1", (long long)m);
  if (d < 1) return fail(KNN_ERR_INVALID, "d = %d: dimension must be >= 1", d);
  if (k < 1 || k > m) return fail(KNN_ERR_INVALID, "k = %d outside [1, m = %lld]", k, (long long)m);
  if (metric < KNN_L2 || metric > KNN_LINF) return fail(KNN_ERR_INVALID, "unknown metric %d", metric);
  return KNN_OK;
}

int tile_kind(int metric, int precision) {
  if (metric == KNN_L1) return TILE_L1_F32;
  if (metric == KNN_LINF) return TILE_LINF_F32;
  if (precision == KNN_BF16) return TILE_L2_BF16;
  if (precision == KNN_FP16) return TILE_L2_F16;
  return TILE_L2_F32;
}

int default_extra(int precision) { return precision == KNN_FP32 ? 8 : 32; }

int one_shot_args(const float* Q, int64_t n, const float* R, int64_t m, int32_t d, int32_t k, int32_t metric,
                  float* dist, int32_t* idx, hipStream_t stream, SearchArgs* out) {
  int st = check_common(n, m, d, k, metric);
  if (st != KNN_OK || n == 0) return st;
  if ((st = check_ptr(Q, "Q")) || (st = check_ptr(R, "R")) || (st = check_ptr(dist, "dist")) ||
      (st = check_ptr(idx, "idx")))
    return st;
  SearchArgs& a = *out;
  a = SearchArgs{};
  a.Q = Q;
  a.n = n;
  a.d = d;
  a.m = m;
  a.R32 = R;
  a.k = k;
  a.kprime = (int)std::min<int64_t>(m, (int64_t)k + default_extra(KNN_FP32));
  a.metric = metric;
  a.kind = tile_kind(metric, KNN_FP32);
  a.dist = dist;
  a.idx = idx;
  a.stream = stream;
  return KNN_OK;
}


bool valid_refs(knn_refs_t r) { return r && r->magic == 0x6b6e6e52u; }

int refs_search_args(knn_refs_t refs, const float* Q, int64_t n, int32_t k, int32_t metric, int32_t precision,
                     int32_t s_extra, float* dist, int32_t* idx, hipStream_t stream, SearchArgs* out) {
  if (!valid_refs(refs)) return fail(KNN_ERR_INVALID, "not a live reference-set handle");
  int st = check_common(n, refs->m, refs->d, k, metric);
  if (st != KNN_OK) return st;
  if (precision < KNN_FP32 || precision > KNN_FP16) return fail(KNN_ERR_INVALID, "unknown precision %d", precision);
  if (metric == KNN_L2 && precision != refs->storage)
    return fail(KNN_ERR_UNSUPPORTED, "precision %d needs rows stored in that precision (stored: %d)", precision,
                refs->storage);
  if (metric != KNN_L2 && precision != KNN_FP32)
    return fail(KNN_ERR_UNSUPPORTED, "low-precision tiles support the Euclidean distance only");
  if (metric != KNN_L2 && !refs->master)
    return fail(KNN_ERR_UNSUPPORTED, "Manhattan / infinity-norm search needs float32 rows (create with a master)");
  if ((st = check_ptr(Q, "Q")) || (st = check_ptr(dist, "dist")) || (st = check_ptr(idx, "idx"))) return st;
  const int extra = s_extra < 0 ? default_extra(precision) : s_extra;
  SearchArgs& a = *out;
  a = SearchArgs{};
  a.Q = Q;
  a.n = n;
  a.d = refs->d;
  a.m = refs->m;
  a.kind = tile_kind(metric, precision);
  if (metric == KNN_L2) {
    a.rows = refs->rows;
    a.ldr = refs->dp;
    a.rhalf = refs->rhalf;
    a.centre = refs->centre;
  } else {
    a.rows = refs->master;
    a.ldr = refs->dp32;
  }
  if (refs->master) {
    a.canon = refs->master;
    a.canon_type = ELEM_F32;
    a.ld_canon = refs->dp32;
  } else {
    a.canon = refs->rows;
    a.canon_type = elem_of_kind(a.kind);
    a.ld_canon = refs->dp;
  }
  a.k = k;
  a.kprime = (int)std::min<int64_t>(refs->m, (int64_t)k + extra);
  a.metric = metric;
  a.dist = dist;
  a.idx = idx;
  a.stream = stream;
  return KNN_OK;
}

void free_refs(knn_refs_s* h) {
  (void)hipFree(h->rows);
  (void)hipFree(h->rhalf);
  (void)hipFree(h->centre);
  (void)hipFree(h->master);
  (void)hipFree(h->flag);
  h->rows = nullptr;
  h->rhalf = h->centre = h->master = nullptr;
  h->flag = nullptr;
  for (auto& u : h->uses) (void)hipEventDestroy(u.second);
  h->uses.clear();
}

int record_use(std::mutex& mu, std::vector<std::pair<hipStream_t, hipEvent_t>>& uses, hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return KNN_OK;
  std::lock_guard<std::mutex> lock(mu);
  for (auto& u : uses)
    if (u.first == s) {
      HIP_TRY(hipEventRecord(u.second, s), "hipEventRecord(use)");
      return KNN_OK;
    }
  hipEvent_t e = nullptr;
  HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate(use)");
  uses.push_back({s, e});
  HIP_TRY(hipEventRecord(e, s), "hipEventRecord(use)");
  return KNN_OK;
}

// wait for and release every recorded use; returns the first error
hipError_t wait_uses(std::mutex& mu, std::vector<std::pair<hipStream_t, hipEvent_t>>& uses) {
  std::lock_guard<std::mutex> lock(mu);
  hipError_t e = hipSuccess;
  for (auto& u : uses) {
    const hipError_t e2 = hipEventSynchronize(u.second);
    if (e == hipSuccess) e = e2;
    (void)hipEventDestroy(u.second);
  }
  uses.clear();
  return e;
}

int note_use(knn_refs_s* h, hipStream_t s) { return record_use(h->use_mu, h->uses, s); }

}  // namespace knn::host

extern "C" {

int knn_version(void) { return 100; }

const char* knn_last_error(void) { return g_last_error.c_str(); }

int knn_search(const float* Q, int64_t n, const float* R, int64_t m, int32_t d, int32_t k, int32_t metric,
               float* dist, int32_t* idx, void* stream) {
  SearchArgs a{};
  const int st = one_shot_args(Q, n, R, m, d, k, metric, dist, idx, (hipStream_t)stream, &a);
  if (st != KNN_OK || n == 0) return st;
  return run_search(a);
}

int knn_search_mahalanobis(const float* Q, int64_t n, const float* R, int64_t m, int32_t d, const float* L, int32_t k,
                           float* dist, int32_t* idx, void* stream) {
  int st = check_common(n, m, d, k, KNN_L2);
  if (st != KNN_OK) return st;
  if (n == 0) return KNN_OK;
  if ((st = check_ptr(Q, "Q")) || (st = check_ptr(R, "R")) || (st = check_ptr(L, "L")) ||
      (st = check_ptr(dist, "dist")) || (st = check_ptr(idx, "idx")))
    return st;
  // candidates: the k' = k + 8 nearest of the mapped points (Euclidean
  // search); then their exact distances from the caller's rows
  const int kc = (int)std::min<int64_t>(m, (int64_t)k + default_extra(KNN_FP32));
  if ((size_t)4 * (d + 2 * kc) * 4 > (size_t)kLdsBytes)
    return fail(KNN_ERR_UNSUPPORTED, "d = %d is too large for the Mahalanobis re-rank", d);
  {
    SearchArgs probe{};
    if ((st = one_shot_args(Q, n, R, m, d, kc, KNN_L2, dist, idx, (hipStream_t)stream, &probe)) != KNN_OK) return st;
    size_t need = 0;
    if ((st = run_search_ws(probe, nullptr, 0, &need)) != KNN_OK) return st;  // k' beyond the kernels' limit
  }
  hipStream_t s = (hipStream_t)stream;
  const size_t cbytes = round_up((int64_t)d * 4, 256), qbytes = round_up(n * d * 4, 256),
               rbytes = round_up(m * d * 4, 256), kbytes = round_up(n * (int64_t)kc * 4, 256);
  void* scratch = nullptr;
  if (hipMallocAsync(&scratch, cbytes + qbytes + rbytes + 2 * kbytes, s) != hipSuccess) {
    (void)hipGetLastError();
    return fail(KNN_ERR_OOM, "cannot allocate %zu bytes of Mahalanobis scratch", cbytes + qbytes + rbytes + 2 * kbytes);
  }
  float* c = (float*)scratch;
  float* Qt = (float*)((unsigned char*)scratch + cbytes);
  float* Rt = (float*)((unsigned char*)scratch + cbytes + qbytes);
  float* cdist = (float*)((unsigned char*)scratch + cbytes + qbytes + rbytes);
  int32_t* cidx = (int32_t*)((unsigned char*)cdist + kbytes);
  hipError_t e = launch_centre(R, m, d, d, c, s);
  if (e == hipSuccess) e = launch_transform_rows(Q, n, d, c, L, Qt, s);
  if (e == hipSuccess) e = launch_transform_rows(R, m, d, c, L, Rt, s);
  st = e == hipSuccess ? knn_search(Qt, n, Rt, m, d, kc, KNN_L2, cdist, cidx, stream) : hip_fail(e, "Mahalanobis transform");
  if (st == KNN_OK) {
    e = launch_mahalanobis_rerank(Q, R, L, n, d, m, cidx, kc, dist, idx, k, s);
    if (e != hipSuccess) st = hip_fail(e, "Mahalanobis re-rank");
  }
  const hipError_t ef = hipFreeAsync(scratch, s);
  if (st == KNN_OK && ef != hipSuccess) st = hip_fail(ef, "Mahalanobis scratch release");
  return st;
}

int knn_classify(const float* Q, int64_t n, const float* R, int64_t m, int32_t d, const int32_t* labels, int32_t k,
                 int32_t* out, void* stream) {
  int st = check_common(n, m, d, k, KNN_L2);
  if (st != KNN_OK) return st;
  if (n == 0) return KNN_OK;
  if ((st = check_ptr(Q, "Q")) || (st = check_ptr(R, "R")) || (st = check_ptr(labels, "labels")) ||
      (st = check_ptr(out, "out")))
    return st;
  hipStream_t s = (hipStream_t)stream;
  const size_t dbytes = round_up(n * (int64_t)k * 4, 256);
  void* scratch = nullptr;
  if (hipMallocAsync(&scratch, 2 * dbytes, s) != hipSuccess) {
    (void)hipGetLastError();
    return fail(KNN_ERR_OOM, "cannot allocate %zu bytes of classification scratch", 2 * dbytes);
  }
  float* dist = (float*)scratch;
  int32_t* idx = (int32_t*)((unsigned char*)scratch + dbytes);
  st = knn_search(Q, n, R, m, d, k, KNN_L2, dist, idx, stream);
  if (st == KNN_OK) {
    const hipError_t e = launch_vote(idx, n, k, labels, out, s);
    if (e != hipSuccess) st = hip_fail(e, "vote launch");
  }
  const hipError_t ef = hipFreeAsync(scratch, s);
  if (st == KNN_OK && ef != hipSuccess) st = hip_fail(ef, "classification scratch release");
  return st;
}

int knn_entropy(const float* Y, int64_t n, int32_t d, int32_t k, double* out, void* stream) {
  if (n < 2) return fail(KNN_ERR_INVALID, "n = %lld: the estimate needs at least two points", (long long)n);
  if (k < 1 || (int64_t)k > n - 1) return fail(KNN_ERR_INVALID, "k = %d outside [1, n - 1 = %lld]", k, (long long)(n - 1));
  if (d < 1) return fail(KNN_ERR_INVALID, "d = %d: dimension must be >= 1", d);
  int st;
  if ((st = check_ptr(Y, "Y")) || (st = check_ptr(out, "out"))) return st;
  hipStream_t s = (hipStream_t)stream;
  const int64_t kk = (int64_t)k + 1;
  const size_t dbytes = round_up(n * kk * 4, 256), ibytes = round_up(n * kk * 4, 256), tbytes = n * 8;
  void* scratch = nullptr;
  if (hipMallocAsync(&scratch, dbytes + ibytes + tbytes, s) != hipSuccess) {
    (void)hipGetLastError();
    return fail(KNN_ERR_OOM, "cannot allocate %zu bytes of entropy scratch", dbytes + ibytes + tbytes);
  }
  float* dist = (float*)scratch;
  int32_t* idx = (int32_t*)((unsigned char*)scratch + dbytes);
  double* terms = (double*)((unsigned char*)scratch + dbytes + ibytes);
  st = knn_search(Y, n, Y, n, d, k + 1, KNN_L2, dist, idx, stream);
  if (st == KNN_OK) {
    // log c_1(d) = log 2 + (d/2) log pi - log d - log Gamma(d/2); Psi(k) = -gamma + sum_{j<k} 1/j
    double psi = -0.57721566490153286060651209008240243;
    for (int j = 1; j < k; ++j) psi += 1.0 / j;
    const double logc1 = std::log(2.0) + 0.5 * d * std::log(M_PI) - std::log((double)d) - std::lgamma(0.5 * d);
    const double offset = std::log((double)(n - 1)) + logc1 - psi;
    const hipError_t e = launch_entropy(dist, idx, n, k, terms, (double)d / (double)n, offset, out, s);
    if (e != hipSuccess) st = hip_fail(e, "entropy launch");
  }
  const hipError_t ef = hipFreeAsync(scratch, s);
  if (st == KNN_OK && ef != hipSuccess) st = hip_fail(ef, "entropy scratch release");
  return st;
}

int knn_create_refs(const float* R, int64_t m, int32_t d, int32_t storage, int32_t keep_fp32_master, void* stream,
                    knn_refs_t* out) {
  if (!out) return fail(KNN_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (m < 1) return fail(KNN_ERR_INVALID, "m = %lld: at least one reference is required", (long long)m);
  if (m > 0x7fffffffLL) return fail(KNN_ERR_UNSUPPORTED, "m = %lld exceeds 2^31 - 1", (long long)m);
  if (d < 1) return fail(KNN_ERR_INVALID, "d = %d: dimension must be >= 1", d);
  if (storage < KNN_FP32 || storage > KNN_FP16) return fail(KNN_ERR_INVALID, "unknown storage precision %d", storage);
  int st = check_ptr(R, "R");
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  std::unique_ptr<knn_refs_s> h(new (std::nothrow) knn_refs_s);
  if (!h) return fail(KNN_ERR_OOM, "host allocation of the handle failed");
  h->m = m;
  h->d = d;
  h->storage = storage;
  const int kind = storage == KNN_BF16 ? TILE_L2_BF16 : storage == KNN_FP16 ? TILE_L2_F16 : TILE_L2_F32;
  h->dp = padded_dim(kind, d);
  h->dp32 = padded_dim(TILE_L1_F32, d);
  const int es = storage == KNN_FP32 ? 4 : 2;
  const bool master = storage == KNN_FP32 || keep_fp32_master;
  const bool narrow = storage != KNN_FP32;
  auto cleanup = [&](int rc) {
    free_refs(h.get());
    return rc;
  };
  HIP_TRY(hipGetDevice(&h->device), "hipGetDevice");
  if ((st = dev_alloc(&h->rows, (size_t)m * h->dp * es, "reference rows")) ||
      (st = dev_alloc((void**)&h->rhalf, (size_t)m * 4, "reference norms")) ||
      (master && (st = dev_alloc((void**)&h->master, (size_t)m * h->dp32 * 4, "float32 master rows"))) ||
      (master && (st = dev_alloc((void**)&h->centre, (size_t)d * 4, "centre"))) ||
      (narrow && (st = dev_alloc((void**)&h->flag, 256, "range flag"))))
    return cleanup(st);
  // 16-bit storage: the flag is set when a row value rounds to infinity
  unsigned* overflow = h->flag;
  float* centre = h->centre;
  hipError_t e = hipSuccess;
  if (overflow) e = hipMemsetAsync(overflow, 0, 4, s);
  // rows are translated by the centre only when a float32 master keeps the
  // untranslated values for the re-rank
  if (e == hipSuccess && master) e = launch_centre(R, m, d, d, centre, s);
  if (e == hipSuccess)
    e = launch_prep_rows(R, m, d, d, centre, h->rows, h->dp, elem_of_kind(kind), h->rhalf, s, overflow);
  if (e == hipSuccess && master) e = launch_prep_rows(R, m, d, d, nullptr, h->master, h->dp32, ELEM_F32, nullptr, s);
  if (e != hipSuccess) return cleanup(hip_fail(e, "knn_create_refs"));
  if (overflow) {
    // the range check needs the preparation's result: wait for this stream
    unsigned flag = 0;
    e = hipMemcpyAsync(&flag, overflow, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return cleanup(hip_fail(e, "knn_create_refs range check"));
    if (flag)
      return cleanup(fail(KNN_ERR_UNSUPPORTED, "a reference value%s exceeds the %s range",
                          master ? " minus the set's centre" : "", storage == KNN_FP16 ? "float16 (65504)" : "bfloat16"));
  }
  if ((st = note_use(h.get(), s)) != KNN_OK) return cleanup(st);
  *out = h.release();
  return KNN_OK;
}

int knn_destroy_refs(knn_refs_t refs) {
  if (!valid_refs(refs)) return fail(KNN_ERR_INVALID, "not a live reference-set handle");
  refs->magic = 0;
  const hipError_t e = wait_uses(refs->use_mu, refs->uses);
  free_refs(refs);
  delete refs;
  if (e != hipSuccess) return hip_fail(e, "knn_destroy_refs");
  return KNN_OK;
}

int knn_refs_info(knn_refs_t refs, int64_t* m, int32_t* d, int32_t* storage, int32_t* has_fp32_master) {
  if (!valid_refs(refs)) return fail(KNN_ERR_INVALID, "not a live reference-set handle");
  if (m) *m = refs->m;
  if (d) *d = refs->d;
  if (storage) *storage = refs->storage;
  if (has_fp32_master) *has_fp32_master = refs->master != nullptr;
  return KNN_OK;
}

int knn_search_refs(knn_refs_t refs, const float* Q, int64_t n, int32_t k, int32_t metric, int32_t precision,
                    int32_t s_extra, float* dist, int32_t* idx, void* stream) {
  if (n == 0) {
    if (!valid_refs(refs)) return fail(KNN_ERR_INVALID, "not a live reference-set handle");
    return check_common(n, refs->m, refs->d, k, metric);
  }
  SearchArgs a;
  int st = refs_search_args(refs, Q, n, k, metric, precision, s_extra, dist, idx, (hipStream_t)stream, &a);
  if (st != KNN_OK) return st;
  st = run_search(a);
  if (st != KNN_OK) return st;
  return note_use(refs, (hipStream_t)stream);
}

int knn_timing_enable(int32_t enable) {
  std::lock_guard<std::mutex> lock(g_tm_mutex);
  g_tm_enabled = enable != 0;
  return KNN_OK;
}

int knn_timing_read(const char* name, double* total_ms, int64_t* launches) {
  if (!name) return fail(KNN_ERR_INVALID, "name is NULL");
  std::lock_guard<std::mutex> lock(g_tm_mutex);
  int st = tm_collect();
  if (st != KNN_OK) return st;
  auto it = g_tm_totals.find(name);
  if (total_ms) *total_ms = it == g_tm_totals.end() ? 0.0 : it->second.first;
  if (launches) *launches = it == g_tm_totals.end() ? 0 : it->second.second;
  return KNN_OK;
}

int knn_timing_reset(void) {
  std::lock_guard<std::mutex> lock(g_tm_mutex);
  int st = tm_collect();
  g_tm_totals.clear();
  return st;
}

}  // extern "C"

// ------------------------------------------------------------ batched form
namespace knn::host {

// One instance of a batch, as planned.
struct BatchInst {
  knn_problem_t prob;
  int kind = 0;
  int dp = 0;
  int es = 4;
  int kc = 0;
  int kprime = 0;
  int P = 1;
  int group = 0;
  int64_t slice_len = 0;
  size_t q_off = 0;     // prepared queries in the workspace
  size_t part_off = 0;  // candidate lists in the workspace (sized for the most slices a configuration gives)
  size_t share_off = 0; // the one-launch group: bounds shared by the query's slices (FusedInst::tshare)
  int pmost = 1;        // most slices of any configuration the tuner tries (rank slots per query)
};

// A launch configuration of a group: (waves, cb) of the general kernel, or
// (8, kWideCb) for the 32x32-tile kernel with register lists; and the
// reference slice length of the group's work items.
constexpr int kWideCb = 0;

struct GroupConfig {
  int waves = 8;
  int cb = kWideCb;
  int64_t slice = 0;
  // one-launch group: 0 = one launch of the kernel that serves every padded
  // dimension and list size; 1 = one launch per (padded dimension, list
  // size) class of the kernel built for that class alone (fewer registers)
  int split = 0;
};

// items of one (padded dimension, keys per lane) class in the item list
struct ItemRange {
  int start = 0;
  int count = 0;
  int dp = 0;
  int kc_max = 0;
};

// Instances sharing one fused launch.  Every 16-bit Euclidean instance with
// k' <= 128 and a padded dimension <= 128 belongs to the one-launch group
// (`one`), which the 32x32-tile kernel serves with one workgroup per item;
// the others are grouped by tile kind, padded dimension and k' class.
struct BatchGroup {
  int kind = 0;
  int dp = 0;
  int kclass = 0;
  bool one = false;
  int ng = 1;
  int nchunk = 1;
  int kc_max = 0;
  GroupConfig cfg;
  int64_t base_slice = 0;  // the default slice length
  std::vector<int> insts;
  size_t insts_off = 0;    // FusedInst table in the workspace
  size_t items_off = 0;    // FusedItem list (sized for the configuration with the most items)
  int nitems = 0;
  std::vector<ItemRange> ranges;  // split configuration: the classes' items
  bool tuned = false;
};

// queries per workgroup of a configuration
int config_nq(const GroupConfig& c) { return c.cb == kWideCb ? kWideQueries : c.waves * kQueriesPerWave; }

bool group_wide_ok(const BatchGroup& g) {
  const int lim = g.kind == TILE_L2_F32 ? kWideMaxKc1 : kWideMaxKc;
  return g.kind <= TILE_L2_F16 && g.kc_max <= lim && g.dp <= kWideMaxDp;
}

int64_t clamp_slice(int64_t s) { return std::max<int64_t>(16 * kStepRefs, round_up(std::max<int64_t>(1, s), kStepRefs)); }

// candidate launch configurations of a group, the default first
std::vector<GroupConfig> group_configs(const BatchGroup& g) {
  std::vector<GroupConfig> out;
  if (g.one) {
    // tile shape fixed (256 queries x 64 references per step); the tuner
    // picks the slice length, which sets the number and size of the items
    // KNN_BATCH_SPLIT=0 / 1 keeps only the one-launch / the per-class form
    const char* es = getenv("KNN_BATCH_SPLIT");
    for (int split : {0, 1}) {
      if (es && atoi(es) != split) continue;
      for (int64_t s : {g.base_slice, g.base_slice / 2, g.base_slice * 2, g.base_slice / 4})
        out.push_back({8, kWideCb, clamp_slice(s), split});
    }
    return out;
  }
  if (group_wide_ok(g)) out.push_back({8, kWideCb, g.base_slice});
  const int group = group_dims(g.kind);
  for (int waves : {8, 4, 2}) {
    for (int cb : {64, 96, 128}) {
      if (g.kc_max <= 64 && cb != 64) continue;
      if (g.kc_max + cb > 64 * kMaxMergePerLane) continue;
      if (fused_lds_bytes(g.kind, waves, g.kc_max, cb, g.ng * group) > (size_t)kLdsBytes) continue;
      out.push_back({waves, cb, g.base_slice});
    }
  }
  return out;
}

// tuned configurations of this process (and of a text cache file when
// KNN_TUNE_CACHE names one), keyed by "kind/dp/kclass/size bucket": waves,
// cb and the slice length as a fraction of the default (index into the
// candidate list for the one-launch group)
std::mutex g_tune_mutex;
std::map<std::string, std::pair<int, int>> g_tune;
bool g_tune_loaded = false;

std::string tune_key(const BatchGroup& g, int64_t pairs) {
  int bucket = 0;
  while (pairs > 1 && bucket < 60) {
    pairs >>= 2;
    ++bucket;
  }
  char buf[96];
  if (g.one)
    snprintf(buf, sizeof buf, "v4/one/k%d/s%d", g.kind, bucket);
  else
    snprintf(buf, sizeof buf, "v3/k%d/d%d/c%d/s%d", g.kind, g.dp, g.kclass, bucket);
  return buf;
}

void tune_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = getenv("KNN_TUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char key[96];
  int w = 0, cb = 0;
  // one entry per line: "key a b" (general: waves cb; one-launch group: candidate index, -1)
  while (fscanf(f, "%95s %d %d", key, &w, &cb) == 3) g_tune[key] = {w, cb};
  fclose(f);
}

void tune_store() {
  const char* path = getenv("KNN_TUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "w");
  if (!f) return;
  for (auto& kv : g_tune) fprintf(f, "%s %d %d\n", kv.first.c_str(), kv.second.first, kv.second.second);
  fclose(f);
}

}  // namespace knn::host

struct knn_batch_s {
  uint32_t magic = 0x6b6e6e42u;
  int precision = KNN_FP32;
  int flags = 0;
  std::vector<BatchInst> inst;
  std::vector<BatchGroup> groups;
  std::vector<FinalInst> finsts;  // host copy of the finalize table
  void* ws = nullptr;
  size_t ws_size = 0;
  size_t jobs_off = 0;
  size_t counter_off = 0;  // item counter of the one-launch group
  bool has_one = false;
  int64_t prep_rows = 0;
  size_t finsts_off = 0, fitems_off = 0;
  int nfitems = 0, keys_max = 0, p_max = 1, kprime_max = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::mutex use_mu;  // completion of every run, one event per stream
  std::vector<std::pair<hipStream_t, hipEvent_t>> uses;
};

namespace knn::host {

bool valid_batch(knn_batch_t b) { return b && b->magic == 0x6b6e6e42u; }

int64_t pmax_of(const BatchInst& in) { return std::max<int64_t>(1, std::min<int64_t>(64, kFinalMaxKeys / in.kc)); }

// slices of an instance at slice length `slice`: (P, slice_len)
std::pair<int, int64_t> slicing(const BatchInst& in, int64_t slice) {
  const int64_t m = in.prob.refs->m;
  const int64_t P = std::min<int64_t>(pmax_of(in), ceil_div(m, slice));
  const int64_t len = round_up(ceil_div(m, P), kStepRefs);
  return {(int)ceil_div(m, len), len};
}

// items of group g, longest first: cost = query columns of the block x
// references of the slice x (padded dimension + a fixed selection share)
std::vector<FusedItem> group_items(const knn_batch_s& b, const BatchGroup& g, const GroupConfig& c,
                                   std::vector<ItemRange>* ranges = nullptr) {
  struct Cost {
    int64_t cls;   // split configuration: (padded dimension, keys per lane) class
    int64_t cost;
    FusedItem it;
  };
  std::vector<Cost> all;
  const int nq = config_nq(c);
  for (size_t j = 0; j < g.insts.size(); ++j) {
    const BatchInst& in = b.inst[g.insts[j]];
    const auto sl = slicing(in, c.slice);
    const int64_t qb = ceil_div(in.prob.n, nq);
    const int64_t cls = c.split ? in.dp * 2 + (in.kc > kWideMaxKc1 ? 1 : 0) : 0;
    for (int64_t q = 0; q < qb; ++q) {
      const int64_t rows = std::min<int64_t>(nq, in.prob.n - q * nq);
      for (int s = 0; s < sl.first; ++s) {
        const int64_t refs = std::min<int64_t>(sl.second, in.prob.refs->m - s * sl.second);
        // a block costs its full width of queries whatever its fill
        Cost e;
        e.cls = cls;
        e.cost = (int64_t)nq * refs * (in.dp + 64) + rows;
        e.it.inst = (int)j;
        e.it.qblock = (int)q;
        e.it.slice = s;
        e.it.pad = 0;
        all.push_back(e);
      }
    }
  }
  // longest first (within each class when split)
  std::stable_sort(all.begin(), all.end(), [](const Cost& x, const Cost& y) {
    return x.cls != y.cls ? x.cls > y.cls : x.cost > y.cost;
  });
  std::vector<FusedItem> items;
  items.reserve(all.size());
  if (ranges) ranges->clear();
  for (size_t i = 0; i < all.size(); ++i) {
    items.push_back(all[i].it);
    if (!ranges || !c.split) continue;
    const BatchInst& in = b.inst[g.insts[all[i].it.inst]];
    if (i == 0 || all[i].cls != all[i - 1].cls) ranges->push_back({(int)i, 0, in.dp, 0});
    ranges->back().count += 1;
    ranges->back().kc_max = std::max(ranges->back().kc_max, in.kc);
  }
  return items;
}

int upload(void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return KNN_OK;
  HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice), "hipMemcpy(batch descriptors)");
  return KNN_OK;
}

// The group's fused-launch parameters for its current configuration.
FusedParams group_params(knn_batch_s& b, const BatchGroup& g) {
  FusedParams fp{};
  unsigned char* w = (unsigned char*)b.ws;
  fp.insts = (const FusedInst*)(w + g.insts_off);
  fp.items = (const FusedItem*)(w + g.items_off);
  fp.nitems = g.nitems;
  fp.wide = g.cfg.cb == kWideCb ? 1 : 0;
  fp.ng = fp.wide ? g.dp / 16 : g.ng;
  fp.cb = fp.wide ? 32 : g.cfg.cb;
  fp.waves = g.cfg.waves;
  fp.kc_max = g.kc_max;
  fp.counter = g.one ? (int*)(w + b.counter_off) : nullptr;
  return fp;
}

// Apply configuration `c` to group g: slicing of its instances, its
// instance table and items, and the finalize table.
int batch_set_group_config(knn_batch_s& b, BatchGroup& g, const GroupConfig& c) {
  unsigned char* w = (unsigned char*)b.ws;
  std::vector<FusedInst> fis;
  for (int j : g.insts) {
    BatchInst& in = b.inst[j];
    const auto sl = slicing(in, c.slice);
    in.P = sl.first;
    in.slice_len = sl.second;
    const knn_refs_s* r = in.prob.refs;
    FusedInst fi{};
    fi.Q = w + in.q_off;
    if (in.kind <= TILE_L2_F16) {
      fi.R = r->rows;
      fi.ldr = r->dp;
      fi.rhalf = r->rhalf;
    } else {
      fi.R = r->master;
      fi.ldr = r->dp32;
      fi.rhalf = nullptr;
    }
    fi.part = (uint64_t*)(w + in.part_off);
    fi.n = in.prob.n;
    fi.m = r->m;
    fi.slice_len = in.slice_len;
    fi.ldq = in.dp;
    fi.dp = in.dp;
    fi.nchunk = g.nchunk;
    fi.P = in.P;
    fi.kc = in.kc;
    fi.tshare = g.one && in.P > 1 && slice_share_on() ? (uint32_t*)(w + in.share_off) : nullptr;
    set_rank_plan(fi);
    fis.push_back(fi);
    b.finsts[j].P = in.P;
  }
  int st = upload(w + g.insts_off, fis.data(), fis.size() * sizeof(FusedInst));
  if (st != KNN_OK) return st;
  std::vector<FusedItem> items = group_items(b, g, c, &g.ranges);
  st = upload(w + g.items_off, items.data(), items.size() * sizeof(FusedItem));
  if (st != KNN_OK) return st;
  st = upload(w + b.finsts_off, b.finsts.data(), b.finsts.size() * sizeof(FinalInst));
  if (st != KNN_OK) return st;
  b.keys_max = 0;
  b.p_max = 1;
  for (const BatchInst& in : b.inst) {
    b.keys_max = std::max(b.keys_max, in.P * in.kc);
    b.p_max = std::max(b.p_max, in.P);
  }
  g.cfg = c;
  g.nitems = (int)items.size();
  return KNN_OK;
}

// Enqueue group g's fused launch(es) on `s`: one launch, or for a split
// one-launch group one launch per class of the kernel built for it, each
// taking its items in table order.
hipError_t group_launch(knn_batch_s& b, BatchGroup& g, hipStream_t s) {
  FusedParams fp = group_params(b, g);
  if (!(g.one && g.cfg.split)) return launch_fused(g.kind, fp, s);
  const FusedItem* base = fp.items;
  for (const ItemRange& r : g.ranges) {
    FusedParams f = fp;
    f.items = base + r.start;
    f.nitems = r.count;
    f.ng = r.dp / 16;
    f.kc_max = r.kc_max;
    f.counter = nullptr;
    const hipError_t e = launch_fused(g.kind, f, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Enqueue the whole batch on `s`.
int batch_enqueue(knn_batch_s& b, hipStream_t s) {
  unsigned char* w = (unsigned char*)b.ws;
  {
    TimedLaunch tl("prep_queries", s);
    HIP_TRY(launch_prep_batched((const PrepJob*)(w + b.jobs_off), (int)b.inst.size(), b.prep_rows, s,
                                b.has_one ? (int*)(w + b.counter_off) : nullptr),
            "batched query preparation launch");
  }
  for (BatchGroup& g : b.groups) {
    if (g.nitems == 0) continue;
    TimedLaunch tl(fused_name(g.kind), s);
    HIP_TRY(group_launch(b, g, s), "batched fused launch");
  }
  FinalParams fin{};
  fin.insts = (const FinalInst*)(w + b.finsts_off);
  fin.items = (const FinalItem*)(w + b.fitems_off);
  fin.nitems = b.nfitems;
  fin.keys_max = b.keys_max;
  fin.p_max = b.p_max;
  fin.kprime_max = b.kprime_max;
  {
    TimedLaunch tl("finalize", s);
    HIP_TRY(launch_finalize(fin, s), "batched finalize launch");
  }
  return KNN_OK;
}

// Time each candidate configuration of every untuned group (the fused
// launch alone, on the batch's own data) and keep the fastest.
int batch_tune(knn_batch_s& b, hipStream_t s) {
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  tune_load();
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
  HIP_TRY(hipEventCreate(&e1), "hipEventCreate");
  int st = KNN_OK;
  unsigned char* w = (unsigned char*)b.ws;
  for (BatchGroup& g : b.groups) {
    if (g.tuned || g.insts.empty()) continue;
    int64_t pairs = 0;
    for (int j : g.insts) pairs += b.inst[j].prob.n * b.inst[j].prob.refs->m;
    const std::string key = tune_key(g, pairs);
    const std::vector<GroupConfig> cands = group_configs(g);
    auto hit = g_tune.find(key);
    if (hit != g_tune.end()) {
      GroupConfig c = cands[0];
      if (g.one) {
        if (hit->second.first >= 0 && hit->second.first < (int)cands.size()) c = cands[hit->second.first];
      } else {
        for (const GroupConfig& x : cands)
          if (x.waves == hit->second.first && x.cb == hit->second.second) c = x;
      }
      st = batch_set_group_config(b, g, c);
      if (st != KNN_OK) break;
      g.tuned = true;
      continue;
    }
    float best = 1e30f;
    int best_i = 0;
    for (size_t ci = 0; ci < cands.size(); ++ci) {
      st = batch_set_group_config(b, g, cands[ci]);
      if (st != KNN_OK) break;
      auto one_launch = [&]() {
        hipError_t e = hipSuccess;
        if (g.one) e = hipMemsetAsync(w + b.counter_off, 0, sizeof(int), s);  // outside any graph
        if (e == hipSuccess) e = group_launch(b, g, s);
        return e;
      };
      hipError_t e = one_launch();  // warm-up
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      for (int r = 0; r < 3 && e == hipSuccess; ++r) e = one_launch();
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        st = hip_fail(e, "batch tuning");
        break;
      }
      if (ms < best) {
        best = ms;
        best_i = (int)ci;
      }
    }
    if (st != KNN_OK) break;
    st = batch_set_group_config(b, g, cands[best_i]);
    if (st != KNN_OK) break;
    g_tune[key] = g.one ? std::make_pair(best_i, -1) : std::make_pair(cands[best_i].waves, cands[best_i].cb);
    g.tuned = true;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == KNN_OK) tune_store();
  return st;
}

void free_batch(knn_batch_s* b) {
  for (auto& u : b->uses) (void)hipEventDestroy(u.second);
  b->uses.clear();
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->ws) (void)hipFree(b->ws);
}

}  // namespace knn::host

extern "C" {

int knn_batch_create(const knn_problem_t* probs, int32_t count, int32_t precision, int32_t s_extra, int32_t flags,
                     knn_batch_t* out) {
  if (!out) return fail(KNN_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (count < 0) return fail(KNN_ERR_INVALID, "count = %d is negative", count);
  if (count > 0 && !probs) return fail(KNN_ERR_INVALID, "probs is NULL");
  if (precision < KNN_FP32 || precision > KNN_FP16) return fail(KNN_ERR_INVALID, "unknown precision %d", precision);
  std::unique_ptr<knn_batch_s> b(new (std::nothrow) knn_batch_s);
  if (!b) return fail(KNN_ERR_OOM, "host allocation of the batch failed");
  b->precision = precision;
  b->flags = flags;
  const int extra = s_extra < 0 ? default_extra(precision) : s_extra;
  const bool one_ok = env_int("KNN_BATCH_ONE") >= 0;  // KNN_BATCH_ONE=-1: per-group launches (tests)
  // ---- check and group every instance
  std::map<std::tuple<int, int, int>, int> group_of;
  int one_group = -1;
  for (int i = 0; i < count; ++i) {
    const knn_problem_t& pr = probs[i];
    if (!valid_refs(pr.refs)) return fail(KNN_ERR_INVALID, "instance %d: not a live reference-set handle", i);
    const knn_refs_s* r = pr.refs;
    int st = check_common(pr.n, r->m, r->d, pr.k, pr.metric);
    if (st != KNN_OK) return fail(st, "instance %d: %s", i, g_last_error.c_str());
    if (pr.metric == KNN_L2 && precision != r->storage)
      return fail(KNN_ERR_UNSUPPORTED, "instance %d: precision %d needs rows stored in that precision", i, precision);
    if (pr.metric != KNN_L2 && (precision != KNN_FP32 || !r->master))
      return fail(KNN_ERR_UNSUPPORTED, "instance %d: Manhattan / infinity norm need float32 tiles and rows", i);
    if (pr.n > 0 && (!pr.Q || !pr.dist || !pr.idx))
      return fail(KNN_ERR_INVALID, "instance %d: NULL query or output pointer", i);
    BatchInst in;
    in.prob = pr;
    in.kind = tile_kind(pr.metric, precision);
    in.dp = padded_dim(in.kind, r->d);
    in.es = is_half_kind(in.kind) ? 2 : 4;
    in.kprime = (int)std::min<int64_t>(r->m, (int64_t)pr.k + extra);
    in.kc = in.kprime;
    const bool one = one_ok && is_half_kind(in.kind) && in.kc <= kWideMaxKc && in.dp <= kWideMaxDp;
    if (one) {
      if (one_group < 0) {
        BatchGroup g;
        g.kind = in.kind;
        g.one = true;
        one_group = (int)b->groups.size();
        b->groups.push_back(g);
      }
      in.group = one_group;
    } else {
      const int kclass = in.kc <= 64 ? 0 : 1;
      auto key = std::make_tuple(in.kind, in.dp, kclass);
      auto it = group_of.find(key);
      if (it == group_of.end()) {
        BatchGroup g;
        g.kind = in.kind;
        g.dp = in.dp;
        g.kclass = kclass;
        it = group_of.emplace(key, (int)b->groups.size()).first;
        b->groups.push_back(g);
      }
      in.group = it->second;
    }
    BatchGroup& g = b->groups[in.group];
    g.kc_max = std::max(g.kc_max, in.kc);
    g.dp = std::max(g.dp, in.dp);
    if (pr.n > 0) g.insts.push_back((int)b->inst.size());
    b->inst.push_back(in);
  }
  b->has_one = one_group >= 0;
  // ---- default configuration and slice length of each group
  const int cus = device_cu_count();
  for (BatchGroup& g : b->groups) {
    const int group = group_dims(g.kind);
    const int total = g.dp / group;
    const int gmax = g.kind == TILE_L2_F32 ? kMaxGroupsF32 : is_half_kind(g.kind) ? kMaxGroups16 : kMaxGroupsValu;
    if (!g.one) {
      // the widest chunk at which the general kernel fits
      bool general = false;
      for (int ng = std::min(total, gmax); ng >= 1 && !general; --ng) {
        g.ng = ng;
        for (const GroupConfig& c : group_configs(g)) general = general || c.cb != kWideCb;
      }
      if (group_configs(g).empty())
        return fail(KNN_ERR_UNSUPPORTED, "k' = %d candidates per query do not fit the fused kernel's LDS budget",
                    g.kc_max);
      g.nchunk = (int)ceil_div(total, g.ng);
    }
    // slice length: about four items per workgroup slot of the whole device
    // for the default configuration
    const GroupConfig c0 = g.one ? GroupConfig{8, kWideCb, 0} : group_configs(g)[0];
    const int nq = config_nq(c0);
    const size_t lds = c0.cb == kWideCb ? kWideLdsBytes
                                         : fused_lds_bytes(g.kind, c0.waves, g.kc_max, c0.cb, g.ng * group);
    const int64_t slots = (int64_t)cus * std::max<int>(1, (int)(kLdsBytes / lds));
    int64_t blockrefs = 0;
    for (int j : g.insts) blockrefs += ceil_div(b->inst[j].prob.n, nq) * b->inst[j].prob.refs->m;
    g.base_slice = clamp_slice(blockrefs / std::max<int64_t>(1, 4 * slots));
    g.cfg = c0;
    g.cfg.slice = g.base_slice;
  }
  // ---- workspace layout (part lists sized for the most slices any candidate gives)
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (size_t)round_up((int64_t)bytes, 256);
    return at;
  };
  for (BatchInst& in : b->inst) {
    int pmost = 1;
    for (const GroupConfig& c : group_configs(b->groups[in.group])) pmost = std::max(pmost, slicing(in, c.slice).first);
    in.q_off = take((size_t)in.prob.n * in.dp * in.es);
    in.part_off = take((size_t)in.prob.n * pmost * in.kc * 8);
    in.pmost = pmost;
    in.share_off = b->groups[in.group].one ? take(share_bytes(in.prob.n, pmost)) : 0;
  }
  for (BatchGroup& g : b->groups) {
    g.insts_off = take(g.insts.size() * sizeof(FusedInst));
    size_t most = 0;
    for (const GroupConfig& c : group_configs(g)) most = std::max(most, group_items(*b, g, c).size());
    g.items_off = take(most * sizeof(FusedItem));
  }
  b->jobs_off = take(b->inst.size() * sizeof(PrepJob));
  b->finsts_off = take(b->inst.size() * sizeof(FinalInst));
  b->counter_off = take(sizeof(int));
  int64_t nf = 0;
  for (BatchInst& in : b->inst) nf += ceil_div(in.prob.n, kFinalWaves);
  b->fitems_off = take((size_t)nf * sizeof(FinalItem));
  b->ws_size = std::max<size_t>(off, 256);
  if (int st0 = dev_alloc(&b->ws, b->ws_size, "batch workspace")) return st0;
  std::unique_ptr<knn_batch_s, void (*)(knn_batch_s*)> guard(b.get(), [](knn_batch_s* p) { free_batch(p); });
  unsigned char* w = (unsigned char*)b->ws;
  // ---- descriptors: query preparation, finalize, then each group's configuration
  std::vector<PrepJob> jobs;
  std::vector<FinalItem> fitems;
  int64_t row0 = 0;
  for (size_t i = 0; i < b->inst.size(); ++i) {
    const BatchInst& in = b->inst[i];
    const knn_refs_s* r = in.prob.refs;
    const bool l2 = in.kind <= TILE_L2_F16;
    PrepJob jb{};
    jb.src = in.prob.Q;
    jb.dst = w + in.q_off;
    jb.centre = l2 ? r->centre : nullptr;
    jb.rhalf = nullptr;
    jb.rows = in.prob.n;
    jb.row0 = row0;
    jb.d = r->d;
    jb.lds = r->d;
    jb.ldd = in.dp;
    jb.elem = elem_of_kind(in.kind);
    jb.tshare = b->groups[in.group].one ? (uint32_t*)(w + in.share_off) : nullptr;
    jb.nslots = jb.tshare && rank_share_on() ? in.pmost : 0;
    jobs.push_back(jb);
    row0 += in.prob.n;
    FinalInst fi{};
    fi.part = (const uint64_t*)(w + in.part_off);
    fi.Q = in.prob.Q;
    fi.ldq = r->d;
    if (r->master) {
      fi.Rm = r->master;
      fi.rm_type = ELEM_F32;
      fi.ldr = r->dp32;
    } else {
      fi.Rm = r->rows;
      fi.rm_type = elem_of_kind(in.kind);
      fi.ldr = r->dp;
    }
    fi.dist = in.prob.dist;
    fi.idx = in.prob.idx;
    fi.n = in.prob.n;
    fi.m = r->m;
    fi.d = r->d;
    fi.P = 1;
    fi.kc = in.kc;
    fi.kprime = in.kprime;
    fi.k = in.prob.k;
    fi.metric = in.prob.metric;
    b->finsts.push_back(fi);
    for (int64_t q = 0; q < in.prob.n; q += kFinalWaves) fitems.push_back({(int)i, (int)q});
    b->kprime_max = std::max(b->kprime_max, in.kprime);
  }
  b->prep_rows = row0;
  b->nfitems = (int)fitems.size();
  int st = upload(w + b->jobs_off, jobs.data(), jobs.size() * sizeof(PrepJob));
  if (st == KNN_OK) st = upload(w + b->fitems_off, fitems.data(), fitems.size() * sizeof(FinalItem));
  for (BatchGroup& g : b->groups) {
    if (st != KNN_OK) break;
    st = batch_set_group_config(*b, g, g.cfg);
  }
  if (st == KNN_OK) st = upload(w + b->finsts_off, b->finsts.data(), b->finsts.size() * sizeof(FinalInst));
  if (st != KNN_OK) return st;
  guard.release();
  *out = b.release();
  return KNN_OK;
}

}  // extern "C"

namespace knn::host {

int batch_run(knn_batch_t batch, int32_t use_graph, hipStream_t s) {
  if ((batch->flags & KNN_BATCH_TUNE)) {
    int st = batch_tune(*batch, s);
    if (st != KNN_OK) return st;
  }
  if (!use_graph) return batch_enqueue(*batch, s);
  if (!batch->exec) {
    // first graph run: run eagerly (this also sets the kernels' launch
    // attributes), then capture the same sequence for later replays
    int st = batch_enqueue(*batch, s);
    if (st != KNN_OK) return st;
    bool timing;
    {
      std::lock_guard<std::mutex> lock(g_tm_mutex);
      timing = g_tm_enabled;
      g_tm_enabled = false;
    }
    // capture on a private stream (the caller's may be the null stream,
    // which cannot be captured); replays go to the caller's stream
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    hipGraph_t graph = nullptr;
    if (e == hipSuccess) {
      st = batch_enqueue(*batch, cs);
      e = hipStreamEndCapture(cs, &graph);
    }
    if (cs) (void)hipStreamDestroy(cs);
    {
      std::lock_guard<std::mutex> lock(g_tm_mutex);
      g_tm_enabled = timing;
    }
    if (st != KNN_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return hip_fail(e, "graph capture");
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_fail(e, "hipGraphInstantiate");
    }
    batch->graph = graph;
    batch->exec = exec;
    return KNN_OK;
  }
  TimedLaunch tl("batch_graph", s);
  HIP_TRY(hipGraphLaunch(batch->exec, s), "hipGraphLaunch");
  return KNN_OK;
}

}  // namespace knn::host

extern "C" {

int knn_batch_run(knn_batch_t batch, int32_t use_graph, void* stream) {
  if (!valid_batch(batch)) return fail(KNN_ERR_INVALID, "not a live batch handle");
  const int st = batch_run(batch, use_graph, (hipStream_t)stream);
  if (st != KNN_OK) return st;
  return record_use(batch->use_mu, batch->uses, (hipStream_t)stream);
}

int knn_batch_destroy(knn_batch_t batch) {
  if (!valid_batch(batch)) return fail(KNN_ERR_INVALID, "not a live batch handle");
  batch->magic = 0;
  const hipError_t e = wait_uses(batch->use_mu, batch->uses);
  free_batch(batch);
  delete batch;
  if (e != hipSuccess) return hip_fail(e, "knn_batch_destroy");
  return KNN_OK;
}

int knn_search_batched(const knn_problem_t* probs, int32_t count, int32_t precision, int32_t s_extra,
                       void* stream) {
  knn_batch_t b = nullptr;
  int st = knn_batch_create(probs, count, precision, s_extra, 0, &b);
  if (st != KNN_OK) return st;
  st = knn_batch_run(b, 0, stream);
  const int st2 = knn_batch_destroy(b);
  return st != KNN_OK ? st : st2;
}

}  // extern "C"
