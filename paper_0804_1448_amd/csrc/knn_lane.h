// knn_lane.h -- Manhattan and infinity-norm distances with one query per
// lane, fused with the per-query top-k' selection.
//
// The problem definition of Section 2.1 admits any distance; the Manhattan
// and infinity-norm distances it names are not contractions, so they run on
// the vector ALUs in float32.  A wave owns 64 queries, one per lane, and keeps
// the lane's whole (padded) query row in registers while it walks one slice
// of the references, NR references per batch.  A reference row is loaded so
// that lane j of each 16-lane row holds dims 64h + 4j .. 64h + 4j + 3 of the
// row's 64-dim chunk h (the four rows load the same 256 bytes); the DPP row
// broadcast (row_newbcast:j) then hands dim 64h + 4j + c to every lane as an
// operand of the subtraction.  Each query-reference-dimension triple costs
// one subtraction and one accumulation (|.| is a source modifier), and the
// distance loop touches no LDS.  Reference rows are loaded one batch ahead.
//
// Selection is per lane.  A lane keeps a sorted list of its kc best keys
// (score, reference index) and a queue of up to T = 8 or 12 candidates, both
// in LDS in slot-major order ([slot][lane]: lanes at one slot hit distinct
// banks), with the list length and queue count in registers.  A score joins
// the queue if it is <= the list's kc-th score (+inf until the list is full;
// NaN, used for rows past the end of the slice, never does).  Distances are
// non-negative, so scores compare as their bit patterns and a key's
// monotone code is the pattern with the sign bit set.  When the
// queue of some lane might not take the next batch, the wave merges: each
// lane sorts its queue with a comparator network, finds by binary search
// along the merge path how many queue keys b belong to the kept
// min(kc, len + queued) keys, and merges the two sorted runs in place from
// the back.  The merge also tightens the lane's threshold.
#pragma once

#include <utility>

#include "knn_device.h"

namespace knn {

template <int J>
__device__ __forceinline__ float row_bcast(float v) {  // lane J of this lane's 16-lane row
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x150 + J, 0xF, 0xF, true));
}

__device__ __forceinline__ float comp(const float4& v, int c) {
  return c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w;
}

__device__ __forceinline__ void cas64(uint64_t& a, uint64_t& b) {
  const bool s = a < b;
  const uint64_t lo = s ? a : b, hi = s ? b : a;
  a = lo;
  b = hi;
}

// Ascending sorts of 8 and 12 keys: Batcher's odd-even merge networks for 8
// and 16 keys (for 12, the comparators among the first 12 positions: the
// four missing keys act as +inf, which no comparator moves down).
constexpr unsigned char kNet8[19][2] = {{0, 2}, {1, 3}, {4, 6}, {5, 7}, {0, 4}, {1, 5}, {2, 6}, {3, 7}, {0, 1}, {2, 3},
                                        {4, 5}, {6, 7}, {2, 4}, {3, 5}, {1, 4}, {3, 6}, {1, 2}, {3, 4}, {5, 6}};
constexpr unsigned char kNet12[42][2] = {
    {0, 1}, {2, 3}, {4, 5}, {6, 7}, {8, 9}, {10, 11}, {0, 2}, {1, 3}, {4, 6}, {5, 7}, {8, 10}, {9, 11}, {1, 2}, {5, 6},
    {9, 10}, {0, 4}, {1, 5}, {2, 6}, {3, 7}, {2, 4}, {3, 5}, {1, 2}, {3, 4}, {5, 6}, {9, 10}, {0, 8}, {1, 9}, {2, 10},
    {3, 11}, {4, 8}, {5, 9}, {6, 10}, {7, 11}, {2, 4}, {3, 5}, {6, 8}, {7, 9}, {1, 2}, {3, 4}, {5, 6}, {7, 8}, {9, 10}};

template <int T>
__device__ __forceinline__ void sort_queue(uint64_t (&x)[T]) {
  static_assert(T == 8 || T == 12, "queue sizes with a network");
  if constexpr (T == 8) {
#pragma unroll
    for (int c = 0; c < 19; ++c) cas64(x[kNet8[c][0]], x[kNet8[c][1]]);
  } else {
#pragma unroll
    for (int c = 0; c < 42; ++c) cas64(x[kNet12[c][0]], x[kNet12[c][1]]);
  }
}

// Merge this lane's queue (qn unsorted keys at X[s * 64]) into its sorted
// list (len keys at L[s * 64]), keeping the min(kc, len + qn) smallest; the
// whole wave calls it, each lane on its own list.  The queue is sorted by a
// network; b, the number of queue keys among the kept, is found by binary
// search along the merge path; the two sorted runs are then merged in place
// from the back, which stops once the queue run is used up (the rest of
// the list is already in place).
// RAW_HI: the queue keys hold the float score bits in their high word (the
// float32 Euclidean kernel appends them so); the merge maps them to the
// monotone code first.
template <int T, bool RAW_HI = false>
__device__ __forceinline__ void lane_merge(uint64_t* L, uint64_t* X, int& len, int& qn, int kc) {
  uint64_t x[T];
#pragma unroll
  for (int s = 0; s < T; ++s) {
    uint64_t v = X[s * kWaveSize];  // slots past the count hold stale keys
    if constexpr (RAW_HI) v = ((uint64_t)mono_code(__uint_as_float((uint32_t)(v >> 32))) << 32) | (uint32_t)v;
    x[s] = s < qn ? v : kEmptyKey;
  }
  sort_queue<T>(x);
#pragma unroll
  for (int s = 0; s < T; ++s) X[s * kWaveSize] = x[s];
  const int kp = min(kc, len + qn);
  // the smallest b in [lo, hi] whose next queue key does not precede the
  // list key it would displace
  int lo = max(0, kp - len), hi = min(qn, kp);
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (X[mid * kWaveSize] < L[(kp - mid - 1) * kWaveSize])
      lo = mid + 1;
    else
      hi = mid;
  }
  int b = lo, a = kp - lo, i = kp - 1;
  while (b > 0) {  // position i takes the larger of L[a-1] and X[b-1]
    const uint64_t xq = X[(b - 1) * kWaveSize];
    const uint64_t xl = a > 0 ? L[(a - 1) * kWaveSize] : 0ull;
    const bool take_list = a > 0 && xl > xq;
    L[i * kWaveSize] = take_list ? xl : xq;
    a -= take_list ? 1 : 0;
    b -= take_list ? 0 : 1;
    --i;
  }
  len = kp;
  qn = 0;
}

// Accumulate dims 64H + 4J .. 64H + 4J + 3 of NR references into acc.
template <int KIND, int NR, int NCH, int H, int J>
__device__ __forceinline__ void lane_dims4(float (&acc)[NR], const float4 (&v)[NR][NCH], const float4& q4) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const float qd = comp(q4, c);
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const float t = fabsf(row_bcast<J>(comp(v[i][H], c)) - qd);
      if constexpr (KIND == TILE_L1_F32)
        acc[i] = acc[i] + t;
      else
        acc[i] = fmaxf(acc[i], t);
    }
  }
}

template <int KIND, int NR, int NCH, int H, size_t... J>
__device__ __forceinline__ void lane_chunk(float (&acc)[NR], const float4 (&v)[NR][NCH], const float4* qv,
                                           std::index_sequence<J...>) {
  (lane_dims4<KIND, NR, NCH, H, (int)J>(acc, v, qv[16 * H + J]), ...);
}

template <int KIND, int NR, int NCH, int DP, size_t... H>
__device__ __forceinline__ void lane_score(float (&acc)[NR], const float4 (&v)[NR][NCH], const float4* qv,
                                           std::index_sequence<H...>) {
  (lane_chunk<KIND, NR, NCH, (int)H>(acc, v, qv, std::make_index_sequence<(DP - 64 * (int)H >= 64 ? 16 : (DP - 64 * (int)H) / 4)>{}),
   ...);
}

// NG: 16-dim groups of the padded dimension (dp = 16 NG <= 128); T: queue
// keys per lane (8 or 12).
template <int KIND, int NG, int T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void lane_kernel(FusedParams p) {
  constexpr int DP = 16 * NG;
  constexpr int NCH = (DP + 63) / 64;  // 64-dim chunks per row
  constexpr int NR = 4;                // references per batch
  static_assert(NR <= T, "a batch must fit an empty queue");
  extern __shared__ __align__(16) unsigned char smem[];

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, W = blockDim.x >> 6;
  int qblock = blockIdx.x, slice = blockIdx.y;
  FusedInst in;
  if (p.items) {
    const FusedItem it = p.items[blockIdx.x];
    in = p.insts[it.inst];
    qblock = it.qblock;
    slice = it.slice;
  } else {
    in = p.one;
  }
  const int64_t qrow = ((int64_t)qblock * W + wave) * kWaveSize + lane;
  const int64_t qsafe = qrow < in.n ? qrow : in.n - 1;
  const int64_t s0 = (int64_t)slice * in.slice_len;
  const int64_t s1 = min(in.m, s0 + in.slice_len);
  const int kc = in.kc;
  uint64_t* L = (uint64_t*)smem + (size_t)wave * (p.kc_max + T) * kWaveSize + lane;  // L[s * 64]: list slot s
  uint64_t* X = L + (size_t)p.kc_max * kWaveSize;                                     // X[s * 64]: queue slot s

  // the lane's query row, dims 4g .. 4g + 3 in qv[g]
  float4 qv[4 * NG];
  {
    const float* qp = (const float*)in.Q + qsafe * (int64_t)in.ldq;
#pragma unroll
    for (int g = 0; g < 4 * NG; ++g) qv[g] = gload4(qp + 4 * g);
  }

  // reference rows r0 .. r0 + NR - 1 (clamped to the slice), lane j of a
  // 16-lane row holding dims 64h + 4j .. +3 of chunk h; lanes past a short
  // last chunk repeat its last 16 bytes (never broadcast)
  const float* Rf = (const float*)in.R;
  const int jl = lane & 15;
  auto load = [&](int64_t r0, float4 (&v)[NR][NCH]) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int64_t r = min(r0 + i, s1 - 1);
      const float* row = Rf + r * (int64_t)in.ldr;
#pragma unroll
      for (int h = 0; h < NCH; ++h) {
        constexpr int full = 16;
        const int nv = (DP - 64 * h) >= 64 ? full : (DP - 64 * h) / 4;
        const int j = nv < full ? min(jl, nv - 1) : jl;
        v[i][h] = gload4(row + 64 * h + 4 * j);
      }
    }
  };

  // threshold as a bit pattern: non-negative floats (and NaN above +inf)
  // order as unsigned integers
  uint32_t thr = 0x7f800000u;
  int len = 0, qn = 0;

  auto merge = [&]() __attribute__((always_inline)) {
    lane_merge<T>(L, X, len, qn, kc);
    if (len == kc) thr = (uint32_t)(L[(kc - 1) * kWaveSize] >> 32) & 0x7fffffffu;
  };

  // queue the batch's scores that pass the threshold; merge if the next
  // batch might not fit some lane's queue
  auto select = [&](const float (&acc)[NR], int64_t r0) __attribute__((always_inline)) {
    uint32_t sc[NR];  // score bit patterns; NaN past the end of the slice
    uint32_t mn = 0xffffffffu;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      sc[i] = r0 + i < s1 ? __float_as_uint(acc[i]) : 0x7fc00000u;
      mn = min(mn, sc[i]);
    }
    if (__builtin_amdgcn_ballot_w64(mn <= thr)) {
      // branch-free append: every key is written at the current count,
      // which advances only for a passing score (a failing key is
      // overwritten or lies past the count)
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        X[qn * kWaveSize] = ((uint64_t)(sc[i] | 0x80000000u) << 32) | (uint32_t)(r0 + i);
        qn += sc[i] <= thr ? 1 : 0;
      }
      if (__builtin_amdgcn_ballot_w64(qn > T - NR)) merge();
    }
  };

  float4 va[NR][NCH], vb[NR][NCH];
  if (s0 < s1) load(s0, va);
  for (int64_t r0 = s0; r0 < s1; r0 += 2 * NR) {
    float acc[NR];
    load(r0 + NR, vb);
#pragma unroll
    for (int i = 0; i < NR; ++i) acc[i] = 0.f;
    lane_score<KIND, NR, NCH, DP>(acc, va, qv, std::make_index_sequence<NCH>{});
    select(acc, r0);
    if (r0 + NR >= s1) break;
    load(r0 + 2 * NR, va);
#pragma unroll
    for (int i = 0; i < NR; ++i) acc[i] = 0.f;
    lane_score<KIND, NR, NCH, DP>(acc, vb, qv, std::make_index_sequence<NCH>{});
    select(acc, r0 + NR);
  }
  if (__builtin_amdgcn_ballot_w64(qn > 0)) merge();

  if (qrow < in.n) {
    uint64_t* dst = in.part + ((size_t)qrow * in.P + slice) * kc;
    for (int s = 0; s < kc; ++s) dst[s] = s < len ? L[s * kWaveSize] : kEmptyKey;
  }
}

// dynamic LDS of one workgroup of `waves` waves: list and queue slots per lane
__host__ __device__ constexpr size_t lane_lds_bytes(int waves, int kc_max, int queue) {
  return (size_t)waves * kWaveSize * (size_t)(kc_max + queue) * 8;
}

template <int KIND, int NG, int T>
hipError_t launch_lane_one(const FusedParams& p, hipStream_t stream) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)lane_kernel<KIND, NG, T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       kLdsBytes);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (p.items && p.nitems <= 0) return hipSuccess;
  const int nq = p.waves * kWaveSize;
  dim3 grid = p.items ? dim3((unsigned)p.nitems) : dim3((unsigned)((p.one.n + nq - 1) / nq), (unsigned)p.one.P);
  hipLaunchKernelGGL((lane_kernel<KIND, NG, T>), grid, dim3(p.waves * kWaveSize),
                     lane_lds_bytes(p.waves, p.kc_max, T), stream, p);
  return hipGetLastError();
}

}  // namespace knn
