// knn_server.cpp -- serving engine: resident reference sets, requests from
// host memory, continuous batching on a pool of streams, memory admission
// through one device arena.
//
// Each request is the k-NN problem of Section 2.1 of the paper for its own
// query set against one resident reference set; the engine only decides
// which requests share a launch and when, and every batch runs the same
// search pipeline as knn_search_refs on the concatenated queries.  A query
// row's result does not depend on the other rows of its launch, so a
// request's answer is the same alone or batched.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "knn.h"
#include "knn_host.h"

using namespace knn;
using namespace knn::host;

namespace {

using Clock = std::chrono::steady_clock;

int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// First-fit allocator over [0, size) with coalescing free blocks.
class Arena {
 public:
  explicit Arena(int64_t size) : size_(size) {
    if (size > 0) free_[0] = size;
  }
  // offset of a block of `bytes` (256-byte aligned), or -1
  int64_t alloc(int64_t bytes) {
    bytes = align_up(std::max<int64_t>(bytes, 1), 256);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const int64_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used_[off] = bytes;
        in_use_ += bytes;
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return;
    int64_t start = off, len = u->second;
    in_use_ -= len;
    used_.erase(u);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {
      len += next->second;
      free_.erase(next);
    }
    auto nit = free_.lower_bound(start);
    if (nit != free_.begin()) {
      auto prev = std::prev(nit);
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
  }
  int64_t in_use() const { return in_use_; }
  int64_t size() const { return size_; }

 private:
  int64_t size_;
  int64_t in_use_ = 0;
  std::map<int64_t, int64_t> free_;
  std::map<int64_t, int64_t> used_;
};

struct Request {
  uint64_t id = 0;
  int set = 0;
  int64_t n = 0;
  int k = 0;
  const float* q = nullptr;
  float* dist = nullptr;
  int32_t* idx = nullptr;
  Clock::time_point t_submit, t_done;
  int state = 0;  // 0 waiting, 1 on the device, 2 done
  int status = KNN_OK;
};

// One launch: requests of one set (any k), queries concatenated.  The
// search keeps k' = max k + s candidates per row; each request's rows are
// finalized with its own k and k' = k + s, so its result is the one it gets
// alone.
struct Batch {
  int set = 0;           // the set of every request (one-set batches) or of the head (multi-set batches)
  bool multi = false;    // requests of any set in one launch of the 32x32-tile kernel
  int k = 0;             // largest k of the batch
  int64_t n = 0;
  int64_t outs = 0;      // sum of n * k over the requests
  std::vector<Request*> reqs;
  int slot = -1;
  int64_t dev_off = -1;  // arena block
  int64_t q_bytes = 0, d_bytes = 0, i_bytes = 0, t_bytes = 0, ws_bytes = 0;
  Clock::time_point t_ready;  // dry run: completion time
  int64_t seq = 0;            // launch sequence number
  bool launched = false;      // false: failed before reaching the device
  int status = KNN_OK;
};

}  // namespace

struct knn_server_s {
  uint32_t magic = 0x6b6e6e53u;
  knn_server_config_t cfg{};
  bool dry = false;
  bool multi = false;  // 16-bit sets: a batch takes waiting requests of every set
  std::vector<knn_refs_t> sets;
  int device = 0;
  int d = 0;  // dimension of the sets
  // device resources
  void* dev_base = nullptr;
  std::unique_ptr<Arena> dev_arena;
  // per slot: a stream, its completion event and a grow-only pinned staging
  // buffer for the batch's queries and results
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  std::vector<void*> pinned;
  std::vector<int64_t> pinned_size;
  std::vector<bool> slot_busy;
  // state
  std::mutex mu;
  std::condition_variable cv_engine, cv_done;
  std::deque<Request*> waiting;
  std::vector<std::unique_ptr<Batch>> running;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> requests;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread engine;
  knn_server_stats_t stats{};
};

namespace {

bool valid_server(knn_server_t s) { return s && s->magic == 0x6b6e6e53u; }

int64_t set_m(const knn_server_s& s, int set) { return s.dry ? s.cfg.dry_m : s.sets[set]->m; }

// extra candidates of the server's searches
int server_extra(const knn_server_s& s) { return s.cfg.s_extra < 0 ? (s.cfg.precision == KNN_FP32 ? 8 : 32) : s.cfg.s_extra; }

// the multi-set search requests of batch b: each request's rows of the
// concatenated queries, its own k and k' = k + s, its slice of the outputs
std::vector<MultiReq> multi_reqs(const knn_server_s& s, const Batch& b, const float* qd, float* dd, int32_t* id) {
  std::vector<MultiReq> mr;
  mr.reserve(b.reqs.size());
  int64_t row0 = 0, out0 = 0;
  for (Request* r : b.reqs) {
    const int64_t m = s.sets[r->set]->m;
    mr.push_back(MultiReq{s.sets[r->set], row0, r->n, r->k, (int)std::min<int64_t>(m, (int64_t)r->k + server_extra(s)),
                          dd ? dd + out0 : (float*)16, id ? id + out0 : (int32_t*)16});
    row0 += r->n;
    out0 += r->n * r->k;
  }
  (void)qd;
  return mr;
}

// device bytes of a batch: queries, outputs and the search workspace
int batch_sizes(knn_server_s& s, Batch& b) {
  b.q_bytes = align_up(b.n * s.d * 4, 256);
  b.d_bytes = align_up(b.outs * 4, 256);
  b.i_bytes = align_up(b.outs * 4, 256);
  const int nsubs = std::max<int>(1, (int)b.reqs.size());
  b.t_bytes = (int64_t)sub_tables_bytes(nsubs, b.n);
  if (s.dry) {
    // the workspace a real search of this shape would take
    const int64_t kp = std::min<int64_t>(set_m(s, b.set), b.k + (s.cfg.s_extra < 0 ? 32 : s.cfg.s_extra));
    b.ws_bytes = align_up(b.n * align_up(s.d, 32) * 2, 256) + align_up(b.n * 2 * kp * 8, 256);
    return KNN_OK;
  }
  if (b.multi) {
    std::vector<MultiReq> mr = multi_reqs(s, b, nullptr, nullptr, nullptr);
    size_t need = 0, tneed = 0;
    int st = run_multi_ws(mr.data(), (int)mr.size(), (const float*)16, s.cfg.precision, nullptr, 0, &need, nullptr,
                          &tneed, nullptr);
    if (st != KNN_OK) return st;
    b.ws_bytes = align_up((int64_t)need, 256);
    b.t_bytes = align_up((int64_t)tneed, 256);
    return KNN_OK;
  }
  SearchArgs a;
  int st = refs_search_args(s.sets[b.set], (const float*)16, b.n, b.k, KNN_L2, s.cfg.precision, s.cfg.s_extra,
                            (float*)16, (int32_t*)16, nullptr, &a);
  if (st != KNN_OK) return st;
  a.nsubs = nsubs;
  size_t need = 0;
  st = run_search_ws(a, nullptr, 0, &need);
  if (st != KNN_OK) return st;
  b.ws_bytes = align_up((int64_t)need, 256);
  return KNN_OK;
}

int64_t batch_dev_bytes(const Batch& b) { return b.q_bytes + b.d_bytes + b.i_bytes + b.ws_bytes; }
int64_t batch_pin_bytes(const Batch& b) { return b.q_bytes + b.d_bytes + b.i_bytes + b.t_bytes; }

// Grow slot's pinned staging to hold `bytes` (the slot is idle).
int ensure_pinned(knn_server_s& s, int slot, int64_t bytes) {
  if (s.pinned_size[slot] >= bytes) return KNN_OK;
  if (s.pinned[slot]) {
    HIP_TRY(hipHostFree(s.pinned[slot]), "hipHostFree(staging)");
    s.pinned[slot] = nullptr;
    s.pinned_size[slot] = 0;
  }
  const int64_t want = std::max<int64_t>(bytes, (int64_t)1 << 20);
  HIP_TRY(hipHostMalloc(&s.pinned[slot], (size_t)want, hipHostMallocDefault), "hipHostMalloc(staging)");
  s.pinned_size[slot] = want;
  return KNN_OK;
}

// Launch batch b on its stream.  Called without the lock: the batch owns its
// slot (stream, staging) and arena block, and reads only the immutable parts
// of its requests.
int launch(knn_server_s& s, Batch& b) {
  if (s.dry) {
    const double us = s.cfg.dry_us_per_query * (double)b.n;
    b.t_ready = Clock::now() + std::chrono::microseconds((int64_t)us);
    return KNN_OK;
  }
  int rc = ensure_pinned(s, b.slot, batch_pin_bytes(b));
  if (rc != KNN_OK) return rc;
  unsigned char* dev = (unsigned char*)s.dev_base + b.dev_off;
  unsigned char* pin = (unsigned char*)s.pinned[b.slot];
  float* qd = (float*)dev;
  float* dd = (float*)(dev + b.q_bytes);
  int32_t* id = (int32_t*)(dev + b.q_bytes + b.d_bytes);
  void* ws = dev + b.q_bytes + b.d_bytes + b.i_bytes;
  float* qp = (float*)pin;
  int64_t row = 0;
  for (Request* r : b.reqs) {
    memcpy(qp + row * s.d, r->q, (size_t)r->n * s.d * 4);
    row += r->n;
  }
  hipStream_t st = s.streams[b.slot];
  HIP_TRY(hipMemcpyAsync(qd, qp, (size_t)b.n * s.d * 4, hipMemcpyHostToDevice, st), "server H2D");
  if (b.multi) {
    std::vector<MultiReq> mr = multi_reqs(s, b, qd, dd, id);
    rc = run_multi_ws(mr.data(), (int)mr.size(), qd, s.cfg.precision, ws, (size_t)b.ws_bytes, nullptr,
                      pin + b.q_bytes + b.d_bytes + b.i_bytes, nullptr, st);
  }
  if (!b.multi) {
    // one finalize instance per request: rows row0.. with the request's own k
    const int64_t m = s.sets[b.set]->m;
    const int extra = server_extra(s);
    std::vector<SubSearch> subs;
    subs.reserve(b.reqs.size());
    int64_t row0 = 0, out0 = 0;
    for (Request* r : b.reqs) {
      subs.push_back(SubSearch{row0, r->n, r->k, (int)std::min<int64_t>(m, (int64_t)r->k + extra), dd + out0, id + out0});
      row0 += r->n;
      out0 += r->n * r->k;
    }
    SearchArgs a;
    rc = refs_search_args(s.sets[b.set], qd, b.n, b.k, KNN_L2, s.cfg.precision, s.cfg.s_extra, dd, id, st, &a);
    if (rc == KNN_OK) {
      a.subs = subs.data();
      a.nsubs = (int)subs.size();
      a.tables_host = pin + b.q_bytes + b.d_bytes + b.i_bytes;
      rc = run_search_ws(a, ws, (size_t)b.ws_bytes, nullptr);
    }
  }
  if (rc != KNN_OK) return rc;
  HIP_TRY(hipMemcpyAsync(pin + b.q_bytes, dd, (size_t)b.outs * 4, hipMemcpyDeviceToHost, st), "server D2H");
  HIP_TRY(hipMemcpyAsync(pin + b.q_bytes + b.d_bytes, id, (size_t)b.outs * 4, hipMemcpyDeviceToHost, st),
          "server D2H");
  HIP_TRY(hipEventRecord(s.events[b.slot], st), "server event");
  return KNN_OK;
}

bool batch_finished(knn_server_s& s, Batch& b) {
  if (!b.launched) return true;
  if (s.dry) return Clock::now() >= b.t_ready;
  const hipError_t e = hipEventQuery(s.events[b.slot]);
  if (e == hipErrorNotReady) return false;
  if (e != hipSuccess) b.status = KNN_ERR_DEVICE;
  return true;
}

// Copy a finished batch's results to its requests' host arrays.  Called
// without the lock: the requests are still on the device as far as every
// other thread can tell, so nothing else touches their arrays.
void copy_results(knn_server_s& s, Batch& b) {
  int64_t out0 = 0;
  const unsigned char* pin = s.dry ? nullptr : (const unsigned char*)s.pinned[b.slot];
  for (Request* r : b.reqs) {
    const int64_t cnt = r->n * (int64_t)r->k;
    if (s.dry) {
      for (int64_t e = 0; e < cnt; ++e) {
        r->dist[e] = (float)r->set;
        r->idx[e] = (int32_t)(b.seq & 0x7fffffff);
      }
    } else if (b.status == KNN_OK) {
      memcpy(r->dist, pin + b.q_bytes + out0 * 4, (size_t)cnt * 4);
      memcpy(r->idx, pin + b.q_bytes + b.d_bytes + out0 * 4, (size_t)cnt * 4);
    }
    out0 += cnt;
  }
}

// Mark a batch's requests done and release its memory and slot (lock held).
void complete(knn_server_s& s, Batch& b) {
  const Clock::time_point now = Clock::now();
  for (Request* r : b.reqs) {
    r->status = b.status;
    r->state = 2;
    r->t_done = now;
  }
  s.stats.completed += (int64_t)b.reqs.size();
  if (b.dev_off >= 0) s.dev_arena->release(b.dev_off);
  s.slot_busy[b.slot] = false;
}

// whether request r can join a multi-set batch (16-bit server, k + s <= 128)
bool req_multi(const knn_server_s& s, const Request& r) {
  if (!s.multi) return false;
  const int64_t kp = std::min<int64_t>(set_m(s, r.set), (int64_t)r.k + server_extra(s));
  return s.dry ? kp <= kWideMaxKc : multi_supported(s.sets[r.set], s.cfg.precision, (int)kp);
}

// A request that heads the queue but waits for arena memory lets later
// requests that fit go ahead of it for at most this long; after that nothing
// passes it until memory frees up.
constexpr auto kHeadBypass = std::chrono::milliseconds(50);

// The batch headed by waiting request `hi`: it and later waiting requests of
// its set, up to max_batch_queries, cut back until the batch's memory fits
// the arena.  nullptr when even the head alone does not fit (lock held).
std::unique_ptr<Batch> try_batch(knn_server_s& s, size_t hi, int slot) {
  Request* head = s.waiting[hi];
  const bool multi = req_multi(s, *head);
  std::vector<Request*> cand{head};
  int64_t n = head->n;
  for (size_t i = hi + 1; i < s.waiting.size(); ++i) {
    Request* r = s.waiting[i];
    if ((multi ? req_multi(s, *r) : r->set == head->set) && n + r->n <= s.cfg.max_batch_queries) {
      cand.push_back(r);
      n += r->n;
    }
  }
  while (!cand.empty()) {
    auto b = std::make_unique<Batch>();
    b->set = head->set;
    b->multi = multi;
    b->reqs = cand;
    for (Request* r : cand) {
      b->n += r->n;
      b->k = std::max(b->k, r->k);
      b->outs += r->n * (int64_t)r->k;
    }
    const int st = batch_sizes(s, *b);
    const int64_t dev_off = st == KNN_OK ? s.dev_arena->alloc(batch_dev_bytes(*b)) : -1;
    if (dev_off < 0 && st == KNN_OK) {
      if (cand.size() == 1) return nullptr;  // the head does not fit yet
      cand.pop_back();
      continue;
    }
    // (a head that cannot be planned fails without a launch: status set)
    b->status = st;
    b->dev_off = dev_off;
    b->slot = slot;
    for (Request* r : cand) {
      r->state = 1;
      s.waiting.erase(std::find(s.waiting.begin(), s.waiting.end(), r));
    }
    s.slot_busy[slot] = true;
    return b;
  }
  return nullptr;
}

// Form the next batch from the waiting queue, or return nullptr (lock held).
// The oldest waiting request heads it; if that one waits for memory, the
// next requests in arrival order may head a batch instead, until the oldest
// has waited kHeadBypass.
std::unique_ptr<Batch> form_batch(knn_server_s& s) {
  if (s.waiting.empty()) return nullptr;
  int slot = -1;
  for (size_t i = 0; i < s.slot_busy.size(); ++i)
    if (!s.slot_busy[i]) {
      slot = (int)i;
      break;
    }
  if (slot < 0) return nullptr;
  const bool may_bypass = Clock::now() - s.waiting.front()->t_submit < kHeadBypass;
  for (size_t hi = 0; hi < s.waiting.size(); ++hi) {
    if (hi > 0 && !may_bypass) break;
    std::unique_ptr<Batch> b = try_batch(s, hi, slot);
    if (b) return b;
  }
  return nullptr;
}

void engine_loop(knn_server_s* s) {
  if (!s->dry) (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lock(s->mu);
  for (;;) {
    bool progressed = false;
    // completions: results are copied to the host arrays outside the lock
    std::vector<std::unique_ptr<Batch>> finished;
    for (size_t i = 0; i < s->running.size();) {
      if (batch_finished(*s, *s->running[i])) {
        finished.push_back(std::move(s->running[i]));
        s->running.erase(s->running.begin() + (long)i);
      } else {
        ++i;
      }
    }
    if (!finished.empty()) {
      lock.unlock();
      for (auto& b : finished) copy_results(*s, *b);
      lock.lock();
      for (auto& b : finished) complete(*s, *b);
      progressed = true;
      s->cv_done.notify_all();
    }
    // admissions: a batch is formed (requests, slot and memory reserved)
    // under the lock and launched outside it
    for (;;) {
      std::unique_ptr<Batch> b = form_batch(*s);
      if (!b) break;
      b->seq = s->stats.batches++;
      s->stats.queries += b->n;
      if (b->status == KNN_OK) {
        lock.unlock();
        b->status = launch(*s, *b);
        // a launch that failed part way may have queued work on the stream
        b->launched = b->status == KNN_OK || (!s->dry && hipEventRecord(s->events[b->slot],
                                                                         s->streams[b->slot]) == hipSuccess);
        lock.lock();
      }
      s->running.push_back(std::move(b));
      s->stats.peak_batches_in_flight = std::max<int32_t>(s->stats.peak_batches_in_flight, (int32_t)s->running.size());
      s->stats.peak_mem_in_flight = std::max<int64_t>(s->stats.peak_mem_in_flight, s->dev_arena->in_use());
      progressed = true;
    }
    if (s->stop && s->waiting.empty() && s->running.empty()) break;
    if (!progressed) {
      if (s->running.empty())
        s->cv_engine.wait(lock, [&] { return s->stop || !s->waiting.empty(); });
      else
        s->cv_engine.wait_for(lock, std::chrono::microseconds(20));
    }
  }
}

void free_server(knn_server_s* s) {
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
  if (s->dev_base) (void)hipFree(s->dev_base);
  for (void* p : s->pinned)
    if (p) (void)hipHostFree(p);
}

}  // namespace

extern "C" {

int knn_server_create(const knn_refs_t* sets, int32_t nsets, const knn_server_config_t* cfg, knn_server_t* out) {
  if (!out) return fail(KNN_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!cfg) return fail(KNN_ERR_INVALID, "cfg is NULL");
  if (nsets < 1) return fail(KNN_ERR_INVALID, "nsets = %d: at least one set is required", nsets);
  if (cfg->mem_budget <= 0 || cfg->max_batches < 1 || cfg->max_queue < 1 || cfg->max_batch_queries < 1)
    return fail(KNN_ERR_INVALID, "mem_budget, max_batches, max_queue and max_batch_queries must be positive");
  if (cfg->precision < KNN_FP32 || cfg->precision > KNN_FP16)
    return fail(KNN_ERR_INVALID, "unknown precision %d", cfg->precision);
  auto s = std::make_unique<knn_server_s>();
  s->cfg = *cfg;
  s->dry = (cfg->flags & KNN_SERVER_DRY_RUN) != 0;
  if (s->dry) {
    if (cfg->dry_m < 1 || cfg->dry_d < 1 || cfg->dry_us_per_query < 0)
      return fail(KNN_ERR_INVALID, "dry run needs dry_m >= 1, dry_d >= 1, dry_us_per_query >= 0");
    s->d = cfg->dry_d;
    s->sets.assign(nsets, nullptr);
  } else {
    if (!sets) return fail(KNN_ERR_INVALID, "sets is NULL");
    for (int i = 0; i < nsets; ++i) {
      if (!valid_refs(sets[i])) return fail(KNN_ERR_INVALID, "set %d: not a live reference-set handle", i);
      if (sets[i]->storage != cfg->precision)
        return fail(KNN_ERR_UNSUPPORTED, "set %d is not stored in precision %d", i, cfg->precision);
      if (i > 0 && sets[i]->d != sets[0]->d) return fail(KNN_ERR_UNSUPPORTED, "sets differ in dimension");
    }
    s->sets.assign(sets, sets + nsets);
    s->d = sets[0]->d;
    HIP_TRY(hipGetDevice(&s->device), "hipGetDevice");
  }
  // 16-bit sets answer batches of every set's requests in one launch when
  // every request fits that kernel (k + s <= 128 candidates, d <= 128)
  s->multi = (cfg->precision == KNN_BF16 || cfg->precision == KNN_FP16) && s->d <= kWideMaxDp &&
             (cfg->flags & KNN_SERVER_ONE_SET) == 0;
  s->dev_arena = std::make_unique<Arena>(cfg->mem_budget);
  s->slot_busy.assign(cfg->max_batches, false);
  s->pinned.assign(cfg->max_batches, nullptr);
  s->pinned_size.assign(cfg->max_batches, 0);
  s->stats.mem_budget = cfg->mem_budget;
  if (!s->dry) {
    // the sets' preparation may still be queued on the caller's streams
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMalloc(&s->dev_base, (size_t)cfg->mem_budget);
    for (int i = 0; i < cfg->max_batches && e == hipSuccess; ++i) {
      hipStream_t st = nullptr;
      hipEvent_t ev = nullptr;
      e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
      if (e == hipSuccess) s->streams.push_back(st);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e == hipSuccess) s->events.push_back(ev);
    }
    if (e != hipSuccess) {
      int rc = hip_fail(e, "knn_server_create");
      free_server(s.get());
      return rc;
    }
  }
  knn_server_s* raw = s.release();
  raw->engine = std::thread(engine_loop, raw);
  *out = raw;
  return KNN_OK;
}

int knn_server_submit(knn_server_t srv, int32_t set, const float* Q_host, int64_t n, int32_t k, float* dist_host,
                      int32_t* idx_host, uint64_t* ticket) {
  if (!valid_server(srv)) return fail(KNN_ERR_INVALID, "not a live server handle");
  if (!ticket) return fail(KNN_ERR_INVALID, "ticket is NULL");
  if (set < 0 || set >= (int)srv->sets.size()) return fail(KNN_ERR_INVALID, "set %d out of range", set);
  int st = check_common(n, set_m(*srv, set), srv->d, k, KNN_L2);
  if (st != KNN_OK) return st;
  if (n < 1) return fail(KNN_ERR_INVALID, "n = %lld: a request needs at least one query", (long long)n);
  if (!Q_host || !dist_host || !idx_host) return fail(KNN_ERR_INVALID, "NULL query or result array");
  if (n > srv->cfg.max_batch_queries)
    return fail(KNN_ERR_UNSUPPORTED, "n = %lld exceeds max_batch_queries", (long long)n);
  auto r = std::make_unique<Request>();
  r->set = set;
  r->n = n;
  r->k = k;
  r->q = Q_host;
  r->dist = dist_host;
  r->idx = idx_host;
  {
    Batch probe;
    probe.set = set;
    probe.k = k;
    probe.n = n;
    probe.outs = n * (int64_t)k;
    probe.reqs = {r.get()};
    probe.multi = req_multi(*srv, *r);
    std::lock_guard<std::mutex> lock(srv->mu);
    st = batch_sizes(*srv, probe);
    if (st != KNN_OK) return st;
    if (batch_dev_bytes(probe) > srv->cfg.mem_budget)
      return fail(KNN_ERR_UNSUPPORTED, "a request of %lld queries needs %lld bytes, above the memory budget",
                  (long long)n, (long long)batch_dev_bytes(probe));
    if ((int64_t)srv->waiting.size() >= srv->cfg.max_queue) {
      ++srv->stats.rejected_busy;
      return fail(KNN_ERR_BUSY, "%d requests already waiting", (int)srv->waiting.size());
    }
    r->id = srv->next_id++;
    r->t_submit = Clock::now();
    *ticket = r->id;
    srv->waiting.push_back(r.get());
    srv->requests.emplace(r->id, std::move(r));
    ++srv->stats.submitted;
  }
  srv->cv_engine.notify_one();
  return KNN_OK;
}

int knn_server_poll(knn_server_t srv, uint64_t ticket, int32_t* done, double* latency_us) {
  if (!valid_server(srv)) return fail(KNN_ERR_INVALID, "not a live server handle");
  std::lock_guard<std::mutex> lock(srv->mu);
  auto it = srv->requests.find(ticket);
  if (it == srv->requests.end()) return fail(KNN_ERR_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  Request& r = *it->second;
  if (done) *done = r.state == 2;
  if (r.state == 2) {
    if (latency_us) *latency_us = std::chrono::duration<double, std::micro>(r.t_done - r.t_submit).count();
    const int status = r.status;
    srv->requests.erase(it);
    if (status == KNN_ERR_CANCELLED) return fail(status, "request %llu was cancelled", (unsigned long long)ticket);
    if (status != KNN_OK) return fail(status, "request %llu failed on the device", (unsigned long long)ticket);
  }
  return KNN_OK;
}

int knn_server_wait(knn_server_t srv, uint64_t ticket, double* latency_us) {
  if (!valid_server(srv)) return fail(KNN_ERR_INVALID, "not a live server handle");
  {
    std::unique_lock<std::mutex> lock(srv->mu);
    auto it = srv->requests.find(ticket);
    if (it == srv->requests.end()) return fail(KNN_ERR_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    Request* r = it->second.get();
    srv->cv_done.wait(lock, [&] { return r->state == 2; });
  }
  int32_t done = 0;
  return knn_server_poll(srv, ticket, &done, latency_us);
}

int knn_server_cancel(knn_server_t srv, uint64_t ticket) {
  if (!valid_server(srv)) return fail(KNN_ERR_INVALID, "not a live server handle");
  {
    std::lock_guard<std::mutex> lock(srv->mu);
    auto it = srv->requests.find(ticket);
    if (it == srv->requests.end()) return fail(KNN_ERR_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    Request& r = *it->second;
    if (r.state != 0)
      return fail(KNN_ERR_BUSY, "request %llu is already %s", (unsigned long long)ticket,
                  r.state == 1 ? "on the device" : "complete");
    srv->waiting.erase(std::find(srv->waiting.begin(), srv->waiting.end(), &r));
    r.state = 2;
    r.status = KNN_ERR_CANCELLED;
    r.t_done = Clock::now();
    ++srv->stats.cancelled;
    ++srv->stats.completed;
  }
  srv->cv_done.notify_all();
  return KNN_OK;
}

int knn_server_stats(knn_server_t srv, knn_server_stats_t* out) {
  if (!valid_server(srv)) return fail(KNN_ERR_INVALID, "not a live server handle");
  if (!out) return fail(KNN_ERR_INVALID, "out is NULL");
  std::lock_guard<std::mutex> lock(srv->mu);
  *out = srv->stats;
  return KNN_OK;
}

int knn_server_destroy(knn_server_t srv) {
  if (!valid_server(srv)) return fail(KNN_ERR_INVALID, "not a live server handle");
  {
    std::lock_guard<std::mutex> lock(srv->mu);
    srv->stop = true;
  }
  srv->cv_engine.notify_all();
  if (srv->engine.joinable()) srv->engine.join();
  srv->magic = 0;
  if (!srv->dry)
    for (hipStream_t st : srv->streams) (void)hipStreamSynchronize(st);
  free_server(srv);
  delete srv;
  return KNN_OK;
}

}  // extern "C"
