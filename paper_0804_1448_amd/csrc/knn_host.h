// knn_host.h -- host-side internals shared by the C ABI (knn_api.cpp) and
// the serving engine (knn_server.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <utility>
#include <vector>

#include "knn.h"
#include "knn_internal.h"

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
  unsigned* flag = nullptr;  // 16-bit storage: range check of the rounded rows
  int device = 0;
  uint32_t magic = 0x6b6e6e52u;
  // completion of the handle's creation and of every search of it the
  // library enqueued, one event per stream (knn_destroy_refs waits for them)
  std::mutex use_mu;
  std::vector<std::pair<hipStream_t, hipEvent_t>> uses;
};

namespace knn::host {

// Rows [row0, row0 + n) of a search that form one request with its own k,
// k' (<= the search's k') and outputs dist [n][k], idx [n][k].
struct SubSearch {
  int64_t row0;
  int64_t n;
  int k;
  int kprime;
  float* dist;
  int32_t* idx;
};

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
  // optional: the rows form `nsubs` requests, each finalized with its own k
  // and k' into its own outputs (dist / idx above unused); their finalize
  // tables are written to `tables_host` (pinned host memory of
  // sub_tables_bytes(nsubs, n) bytes, valid until the search has run) and
  // copied to the workspace on the stream
  const SubSearch* subs = nullptr;
  int nsubs = 0;
  void* tables_host = nullptr;
};

// bytes of the finalize tables of a search of n rows split into nsubs requests
size_t sub_tables_bytes(int nsubs, int64_t n);

int fail(int status, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

// Device allocation with the KNN_FAIL_ALLOC test hook (see knn_api.cpp).
int dev_alloc(void** out, size_t bytes, const char* what);

// Record on `stream` that work using `refs` has been enqueued there.
int note_use(knn_refs_s* refs, hipStream_t stream);

// A grow-only per-stream device buffer; `mu` is held by a search from taking
// the buffer to its last launch.
struct Workspace {
  std::mutex mu;
  void* ptr = nullptr;
  size_t size = 0;
};

#define HIP_TRY(expr, what)                            \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return ::knn::host::hip_fail(e_, what); \
  } while (0)
bool valid_refs(knn_refs_t r);
int check_common(int64_t n, int64_t m, int32_t d, int32_t k, int32_t metric);

// Fill `a` for a search of `refs` (argument checks included; returns a status).
int refs_search_args(knn_refs_t refs, const float* Q, int64_t n, int32_t k, int32_t metric, int32_t precision,
                     int32_t s_extra, float* dist, int32_t* idx, hipStream_t stream, SearchArgs* a);

// Check the arguments of a one-shot float32 search (knn_search) and fill `a`;
// n == 0 returns KNN_OK with `a` untouched.
int one_shot_args(const float* Q, int64_t n, const float* R, int64_t m, int32_t d, int32_t k, int32_t metric,
                  float* dist, int32_t* idx, hipStream_t stream, SearchArgs* a);

// Set on a thread to keep kernel timing from recording events (which may
// allocate) for the launches it makes.
extern thread_local bool g_tm_suppress;

// Run one search in the caller's workspace; with ws == nullptr only the
// needed size is stored in *need.
int run_search_ws(const SearchArgs& a, void* ws, size_t ws_size, size_t* need);

// One request of a multi-set search: query rows [row0, row0 + n) of the
// concatenated float32 queries against resident set `refs`, with its own k
// and k' (k <= k' <= m) and device outputs dist / idx [n][k].
struct MultiReq {
  knn_refs_s* refs;
  int64_t row0;
  int64_t n;
  int k;
  int kprime;
  float* dist;
  int32_t* idx;
};

// Whether a request of k' candidates against `refs` can join a multi-set
// search in `precision` (16-bit sets stored in that precision, d <= 128,
// k' <= 128).
bool multi_supported(const knn_refs_s* refs, int precision, int kprime);

// Euclidean searches of several requests against several resident 16-bit
// sets of one dimension in one launch of the 32x32 register-list kernel:
// one query preparation (which also zeroes the item counter), one fused
// launch over (request, query block, slice) items taken longest first, the
// slice-list merges of requests with many slices, one finalize with each
// request's own k.  Q: the requests' float32 queries concatenated [N][d] on
// the device.  The tables are built in `tables_host` (pinned host memory of
// *tables_need bytes, valid until the search has run) and copied to the
// workspace on `stream`.  With ws == nullptr only *need (workspace bytes)
// and *tables_need are stored.  A request's result does not depend on the
// other requests of the launch.
int run_multi_ws(const MultiReq* reqs, int nreq, const float* Q, int precision, void* ws, size_t ws_size,
                 size_t* need, void* tables_host, size_t* tables_need, hipStream_t stream);

}  // namespace knn::host
