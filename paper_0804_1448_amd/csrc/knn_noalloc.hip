// knn_noalloc.hip -- the one-shot float32 search (knn_search) for callers
// that cannot allocate device memory: its workspace is a fixed array in the
// library's own device memory instead of the per-stream buffer the library
// grows on demand.
//
// The array is a file-scope device variable.  Host code never passes its
// name to a kernel or a copy (on the host the name stands for a host-side
// shadow, not a device address): the device address is looked up once per
// device with hipGetSymbolAddress while that device is current, and only
// that address is used afterwards.
#include <hip/hip_runtime.h>

#include <mutex>

#include "knn.h"
#include "knn_host.h"

// one buffer per device, held until the process ends
static __device__ __align__(256) unsigned char scratch[KNN_NOALLOC_MAX_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up on the
// first call on that device.
int scratch_of_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return knn::host::hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return knn::host::fail(KNN_ERR_UNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return knn::host::hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return knn::host::fail(KNN_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned a null address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return KNN_OK;
}

// keeps the kernel-timing hooks (which record events) off for this thread
struct SuppressTiming {
  bool saved;
  SuppressTiming() : saved(knn::host::g_tm_suppress) { knn::host::g_tm_suppress = true; }
  ~SuppressTiming() { knn::host::g_tm_suppress = saved; }
};

}  // namespace

extern "C" {

int knn_search_noalloc(const float* Q, int64_t n, const float* R, int64_t m, int32_t d, int32_t k, int32_t metric,
                       float* dist, int32_t* idx, void* stream) {
  using namespace knn::host;
  SearchArgs a{};
  int st = one_shot_args(Q, n, R, m, d, k, metric, dist, idx, (hipStream_t)stream, &a);
  if (st != KNN_OK || n == 0) return st;
  size_t need = 0;
  st = run_search_ws(a, nullptr, 0, &need);
  if (st != KNN_OK) return st;
  if (need > (size_t)KNN_NOALLOC_MAX_BYTES)
    return fail(KNN_ERR_UNSUPPORTED, "search needs %zu bytes of workspace; the fixed workspace holds %zu", need,
                (size_t)KNN_NOALLOC_MAX_BYTES);
  void* ws = nullptr;
  st = scratch_of_current_device(&ws);
  if (st != KNN_OK) return st;
  SuppressTiming quiet;
  return run_search_ws(a, ws, need, nullptr);
}

}  // extern "C"
