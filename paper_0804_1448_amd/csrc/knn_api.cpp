// knn_api.cpp -- C ABI of the k-NN library: argument checks, launch plans,
// workspaces and reference-set handles.  Every computation runs in the HIP
// kernels of knn_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "knn.h"
#include "knn_internal.h"

using namespace knn;

// ------------------------------------------------------------ error state
namespace {

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

#define HIP_TRY(expr, what)                 \
  do {                                      \
    hipError_t e_ = (expr);                 \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
int64_t ceil_div(int64_t x, int64_t a) { return (x + a - 1) / a; }

// --------------------------------------------------- per-stream workspace
// A grow-only device buffer per (device, stream).  Growing frees the old
// buffer; hipFree waits for the device, so work still queued on the old
// buffer completes first.
struct Workspace {
  void* ptr = nullptr;
  size_t size = 0;
};

std::mutex g_ws_mutex;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

int workspace(hipStream_t stream, size_t bytes, void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> lock(g_ws_mutex);
  Workspace& w = g_ws[{dev, stream}];
  if (w.size < bytes) {
    if (w.ptr) {
      hipError_t e = hipFree(w.ptr);
      w.ptr = nullptr;
      w.size = 0;
      if (e != hipSuccess) return hip_fail(e, "hipFree(workspace)");
    }
    size_t want = std::max(bytes, (size_t)1 << 20);
    hipError_t e = hipMalloc(&w.ptr, want);
    if (e != hipSuccess) {
      w.ptr = nullptr;
      return hip_fail(e, "hipMalloc(workspace)");
    }
    w.size = want;
  }
  *out = w.ptr;
  return KNN_OK;
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
};

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
// KNN_FUSED_CB, KNN_FUSED_CW, KNN_FUSED_P.  A value the plan cannot honour is
// ignored.
int env_int(const char* name) {
  const char* v = getenv(name);
  return v ? atoi(v) : 0;
}

int make_plan(int kind, int64_t n, int64_t m, int d, int kc, Plan* out) {
  Plan p;
  p.kind = kind;
  p.kc = kc;
  p.group = group_dims(kind);
  p.dp = padded_dim(kind, d);
  p.es = is_half_kind(kind) ? 2 : 4;
  const int total = p.dp / p.group;
  const int gmax = kind == TILE_L2_F32 ? kMaxGroupsF32 : is_half_kind(kind) ? kMaxGroups16 : kMaxGroupsValu;
  const int ew = env_int("KNN_FUSED_WAVES"), ecb = env_int("KNN_FUSED_CB"), eng = env_int("KNN_FUSED_NG");
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
  const size_t lds = fused_lds_bytes(kind, p.waves, kc, p.cb, p.ng * p.group);
  const int wg_per_cu = std::max<int>(1, (int)(kLdsBytes / lds));
  const int64_t nqb = ceil_div(n, (int64_t)p.waves * kQueriesPerWave);
  const int64_t target = (int64_t)device_cu_count() * wg_per_cu;
  int64_t P = ceil_div(target, nqb);
  const int64_t pmax_keys = kFinalMaxKeys / kc;
  const int64_t pmax_len = std::max<int64_t>(1, m / std::max<int64_t>(kStepRefs, 4 * (int64_t)kc));
  P = std::max<int64_t>(1, std::min<int64_t>({P, (int64_t)32, pmax_keys, pmax_len}));
  const int ep = env_int("KNN_FUSED_P");
  if (ep > 0) P = std::min<int64_t>({(int64_t)ep, pmax_keys, ceil_div(m, kStepRefs)});
  p.slice_len = round_up(ceil_div(m, P), kStepRefs);
  p.P = (int)ceil_div(m, p.slice_len);
  *out = p;
  return KNN_OK;
}

int check_ptr(const void* ptr, const char* name) {
  if (!ptr) return fail(KNN_ERR_INVALID, "%s is NULL", name);
  return KNN_OK;
}

}  // namespace

// ----------------------------------------------------------- handle type
// A resident reference set.
//   rows:   the rows the Euclidean tiles read, in the storage precision,
//           translated by `centre` (when set) and zero-padded to dp.
//   rhalf:  half the squared norm of each stored row.
//   master: float32 rows zero-padded to dp32, untranslated: read by the
//           exact re-rank and by the Manhattan / infinity-norm tiles.  Absent
//           only for 16-bit storage without a master, where the stored
//           (untranslated) rows are canonical.
struct knn_refs_s {
  int64_t m = 0;
  int d = 0;
  int storage = KNN_FP32;
  int dp = 0;    // padded dimension of `rows`
  int dp32 = 0;  // padded dimension of `master`
  void* rows = nullptr;
  float* rhalf = nullptr;
  float* centre = nullptr;
  float* master = nullptr;
  int device = 0;
  uint32_t magic = 0x6b6e6e52u;
};

namespace {

// One search, as the pipeline sees it.
struct SearchArgs {
  const float* Q;        // caller's float32 queries [n][d]
  int64_t n;
  int d;
  int64_t m;
  const float* R32;      // one-shot form: caller's float32 references [m][d]; NULL for a handle
  const void* rows;      // handle form: prepared rows for the tile kind
  int ldr;
  const float* rhalf;
  const float* centre;
  const void* canon;     // canonical rows for the exact re-rank
  int canon_type;
  int ld_canon;
  int k;
  int kprime;
  int metric;
  int kind;
  float* dist;
  int32_t* idx;
  hipStream_t stream;
};

int elem_of_kind(int kind) {
  return kind == TILE_L2_BF16 ? ELEM_BF16 : kind == TILE_L2_F16 ? ELEM_F16 : ELEM_F32;
}

int run_search(const SearchArgs& a) {
  Plan plan;
  int st = make_plan(a.kind, a.n, a.m, a.d, a.kprime, &plan);
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
  const size_t rbytes = prep_refs ? (size_t)round_up(a.m * plan.dp * plan.es, 256) : 0;
  const size_t hbytes = prep_refs && l2 ? (size_t)round_up(a.m * 4, 256) : 0;
  const size_t qbytes = prep_q ? (size_t)round_up(a.n * plan.dp * plan.es, 256) : 0;
  const size_t kbytes = (size_t)round_up(a.n * plan.P * (int64_t)plan.kc * 8, 256);
  void* ws = nullptr;
  st = workspace(a.stream, cbytes + pbytes0 + rbytes + hbytes + qbytes + kbytes, &ws);
  if (st != KNN_OK) return st;
  unsigned char* w = (unsigned char*)ws;
  float* wcentre = (float*)w;
  unsigned char* wrows = w + cbytes + pbytes0;
  float* wrhalf = (float*)(wrows + rbytes);
  unsigned char* wq = wrows + rbytes + hbytes;
  uint64_t* part = (uint64_t*)(wq + qbytes);

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
                             a.stream),
            "query preparation launch");
    qp = wq;
    ldq = plan.dp;
  }

  FusedParams fp;
  fp.Q = qp;
  fp.R = rows;
  fp.rhalf = rhalf;
  fp.part = part;
  fp.n = a.n;
  fp.m = a.m;
  fp.slice_len = plan.slice_len;
  fp.ldq = ldq;
  fp.ldr = ldr;
  fp.dp = plan.dp;
  fp.ng = plan.ng;
  fp.nchunk = plan.nchunk;
  fp.P = plan.P;
  fp.kc = plan.kc;
  fp.cb = plan.cb;
  fp.waves = plan.waves;
  {
    TimedLaunch tl(fused_name(a.kind), a.stream);
    HIP_TRY(launch_fused(a.kind, fp, a.stream), "fused distance/selection launch");
  }

  FinalParams fin;
  fin.part = part;
  fin.Q = a.Q;
  fin.ldq = a.d;
  if (one_shot) {
    fin.Rm = a.R32;
    fin.rm_type = ELEM_F32;
    fin.ldr = a.d;
  } else {
    fin.Rm = a.canon;
    fin.rm_type = a.canon_type;
    fin.ldr = a.ld_canon;
  }
  fin.dist = a.dist;
  fin.idx = a.idx;
  fin.n = a.n;
  fin.m = a.m;
  fin.d = a.d;
  fin.P = plan.P;
  fin.kc = plan.kc;
  fin.kprime = a.kprime;
  fin.k = a.k;
  fin.metric = a.metric;
  {
    TimedLaunch tl("finalize", a.stream);
    HIP_TRY(launch_finalize(fin, a.stream), "finalize launch");
  }
  return KNN_OK;
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

bool valid_refs(knn_refs_t r) { return r && r->magic == 0x6b6e6e52u; }

void free_refs(knn_refs_s* h) {
  (void)hipFree(h->rows);
  (void)hipFree(h->rhalf);
  (void)hipFree(h->centre);
  (void)hipFree(h->master);
}

}  // namespace

extern "C" {

int knn_version(void) { return 100; }

const char* knn_last_error(void) { return g_last_error.c_str(); }

int knn_search(const float* Q, int64_t n, const float* R, int64_t m, int32_t d, int32_t k, int32_t metric,
               float* dist, int32_t* idx, void* stream) {
  int st = check_common(n, m, d, k, metric);
  if (st != KNN_OK) return st;
  if (n == 0) return KNN_OK;
  if ((st = check_ptr(Q, "Q")) || (st = check_ptr(R, "R")) || (st = check_ptr(dist, "dist")) ||
      (st = check_ptr(idx, "idx")))
    return st;
  SearchArgs a{};
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
  a.stream = (hipStream_t)stream;
  return run_search(a);
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
  knn_refs_s* h = new (std::nothrow) knn_refs_s;
  if (!h) return fail(KNN_ERR_OOM, "host allocation of the handle failed");
  h->m = m;
  h->d = d;
  h->storage = storage;
  const int kind = storage == KNN_BF16 ? TILE_L2_BF16 : storage == KNN_FP16 ? TILE_L2_F16 : TILE_L2_F32;
  h->dp = padded_dim(kind, d);
  h->dp32 = padded_dim(TILE_L1_F32, d);
  const int es = storage == KNN_FP32 ? 4 : 2;
  const bool master = storage == KNN_FP32 || keep_fp32_master;
  hipError_t e = hipGetDevice(&h->device);
  if (e == hipSuccess) e = hipMalloc(&h->rows, (size_t)m * h->dp * es);
  if (e == hipSuccess) e = hipMalloc((void**)&h->rhalf, (size_t)m * 4);
  if (e == hipSuccess && master) e = hipMalloc((void**)&h->master, (size_t)m * h->dp32 * 4);
  if (e == hipSuccess && master) e = hipMalloc((void**)&h->centre, (size_t)d * 4);
  // rows are translated by the centre only when a float32 master keeps the
  // untranslated values for the re-rank
  if (e == hipSuccess && master) e = launch_centre(R, m, d, d, h->centre, s);
  if (e == hipSuccess) e = launch_prep_rows(R, m, d, d, h->centre, h->rows, h->dp, elem_of_kind(kind), h->rhalf, s);
  if (e == hipSuccess && master) e = launch_prep_rows(R, m, d, d, nullptr, h->master, h->dp32, ELEM_F32, nullptr, s);
  if (e != hipSuccess) {
    int rc = hip_fail(e, "knn_create_refs");
    free_refs(h);
    delete h;
    return rc;
  }
  *out = h;
  return KNN_OK;
}

int knn_destroy_refs(knn_refs_t refs) {
  if (!valid_refs(refs)) return fail(KNN_ERR_INVALID, "not a live reference-set handle");
  refs->magic = 0;
  hipError_t e = hipDeviceSynchronize();
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
  if (n == 0) return KNN_OK;
  if ((st = check_ptr(Q, "Q")) || (st = check_ptr(dist, "dist")) || (st = check_ptr(idx, "idx"))) return st;
  const int extra = s_extra < 0 ? default_extra(precision) : s_extra;
  SearchArgs a{};
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
  a.stream = (hipStream_t)stream;
  return run_search(a);
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
