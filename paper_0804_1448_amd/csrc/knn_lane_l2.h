// knn_lane_l2.h -- float32 Euclidean scores on the matrix cores, fused with
// per-lane top-k' selection.
//
// The score s(q, r) = |r|^2 / 2 - q.r orders references as |q - r|^2 does for
// a fixed query (Section 2.1's brute force, in the form whose cross term is a
// contraction).  A wave scores 32 queries against 32-reference tiles with
// v_mfma_f32_32x32x2f32: references are the rows (A operand), queries the
// columns (B operand, negated), and the rows' half norms are added to the
// products.  The two k slots of the instruction take the two halves of the
// padded dimension: lanes l and l + 32 hold the even and the odd 16-byte
// chunks of query l % 32 in registers for the whole slice and load the same
// chunks of tile row l % 32 straight from global memory, one tile ahead.  In the
// output, lane l holds query l % 32 against the 16 rows 8 (r / 4) + 4 (l / 32)
// + r % 4 of the tile, so every lane sees one query and half of the slice.
//
// Selection is per lane, as in the Manhattan kernel (knn_lane.h): a sorted
// list and a queue per lane in LDS, merged by lane_merge.  A lane filters
// with an upper bound of its query's kc-th best key so far, from its own list
// and its partner lane's (l ^ 32, the same query's other half): either list's
// kc-th key, and, once the lists hold i and kc - i keys, the larger of their
// i-th and (kc - i)-th keys (kc keys lie at or below it), which tracks the
// query's kc-th best over the whole slice rather than over half of it.  At the
// end of the slice lane l < 32 merges the two lists of its query into the
// slice's output list.
#pragma once

#include "knn_lane.h"

namespace knn {

// NG: 16-dim groups of the padded dimension (dp = 16 NG); T: queue keys.
// TILED: R in the 32-row tile layout, where each 16-byte load instruction of
// a wave reads 1 KB of contiguous memory (row-major rows: 32 rows, 32 bytes
// each).
template <int NG, int T, bool TILED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void lane_l2_kernel(FusedParams p) {
  constexpr int HD = 8 * NG;  // dims per lane half
  constexpr int NL = HD / 4;  // 16-byte loads per half row
  constexpr int QW = 32;      // queries per wave
  extern __shared__ __align__(16) unsigned char smem[];

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, W = blockDim.x >> 6;
  const int col = lane & 31, half = lane >> 5;
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
  const int64_t qrow = ((int64_t)qblock * W + wave) * QW + col;
  const int64_t qsafe = qrow < in.n ? qrow : in.n - 1;
  const int64_t s0 = (int64_t)slice * in.slice_len;
  const int64_t s1 = min(in.m, s0 + in.slice_len);
  const int kc = in.kc;
  uint64_t* L = (uint64_t*)smem + (size_t)wave * (p.kc_max + T) * kWaveSize + lane;  // L[s * 64]: list slot s
  uint64_t* X = L + (size_t)p.kc_max * kWaveSize;                                     // X[s * 64]: queue slot s
  const uint64_t* Lp = L - lane + (lane ^ 32);                                        // the partner's list

  // B operand: the negated query dims 8 g + 4 half + c (16-byte chunks
  // alternate between the lane halves, so that the two lanes of a row load
  // adjacent chunks)
  float qv[HD];
  {
    const float* qp = (const float*)in.Q + qsafe * (int64_t)in.ldq + 4 * half;
#pragma unroll
    for (int g = 0; g < NL; ++g) {
      const float4 v = gload4(qp + 8 * g);
      qv[4 * g] = -v.x;
      qv[4 * g + 1] = -v.y;
      qv[4 * g + 2] = -v.z;
      qv[4 * g + 3] = -v.w;
    }
  }

  // A operand of the tile at t0 (row t0 + col, clamped to the slice), 16
  // bytes at a time, and the half norms of this lane's output rows
  // t0 + 8 g + 4 half + i (clamped to the set)
  const float* Rf = (const float*)in.R;
  auto row_part = [&](int64_t t0, int g) __attribute__((always_inline)) {
    if constexpr (TILED) {  // tiles past the slice end read the last tile of the slice
      const int64_t tile = min(t0, s1 - 1) >> 5;
      return gload4(Rf + ((tile * (2 * NL) + 2 * g + half) * 32 + col) * 4);
    } else {
      return gload4(Rf + min(t0 + col, s1 - 1) * (int64_t)in.ldr + 8 * g + 4 * half);
    }
  };
  // Rows past the end of the slice get a NaN norm, which makes their scores
  // NaN: no comparison accepts them.
  auto norms = [&](int64_t t0, float4 (&nh)[4]) __attribute__((always_inline)) {
    if (t0 + QW <= s1) {  // the whole tile lies in the slice (wave-uniform)
#pragma unroll
      for (int g = 0; g < 4; ++g) nh[g] = gload4(in.rhalf + t0 + 8 * g + 4 * half);
      return;
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int64_t r0 = t0 + 8 * g + 4 * half;
      if (r0 + 3 < s1) {
        nh[g] = gload4(in.rhalf + r0);
      } else {
        const int64_t last = in.m - 1;
        const float nan = __builtin_nanf("");
        nh[g] = make_float4(r0 < s1 ? gload1(in.rhalf + min(r0, last)) : nan,
                            r0 + 1 < s1 ? gload1(in.rhalf + min(r0 + 1, last)) : nan,
                            r0 + 2 < s1 ? gload1(in.rhalf + min(r0 + 2, last)) : nan,
                            r0 + 3 < s1 ? gload1(in.rhalf + min(r0 + 3, last)) : nan);
      }
    }
  };

  // threshold as a monotone score code (the high word of a key), +inf until
  // the lists fill, and as the float it codes.  Scores are filtered with
  // float compares, which NaN (the score of rows past the end of the slice)
  // never passes; -0 and +0 compare equal there, so a key coded just above the
  // threshold may enter the queue, and the merge, which keeps the kc smallest
  // keys, drops it.
  uint32_t thr = 0xff800000u;
  float thr_f = __builtin_inff();
  int len = 0, qn = 0;
  const int ki = kc / 2, kj = kc - kc / 2;  // the split of the two-list bound

  auto merge = [&]() __attribute__((always_inline)) {
    lane_merge<T, true>(L, X, len, qn, kc);
    __builtin_amdgcn_wave_barrier();
    const int plen = (int)xor_lane32<32>((uint32_t)len, lane);
    uint32_t t = thr;
    if (len == kc) t = min(t, (uint32_t)(L[(kc - 1) * kWaveSize] >> 32));
    if (plen == kc) t = min(t, (uint32_t)(Lp[(kc - 1) * kWaveSize] >> 32));
    if (ki > 0 && len >= ki && plen >= kj)
      t = min(t, max((uint32_t)(L[(ki - 1) * kWaveSize] >> 32), (uint32_t)(Lp[(kj - 1) * kWaveSize] >> 32)));
    thr = t;
    thr_f = mono_value(t);
  };

  // queue the tile's scores that pass the threshold, four rows at a time;
  // merge when the next four might not fit some lane's queue
  auto select = [&](const f32x16& acc, int64_t t0) __attribute__((always_inline)) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const uint32_t rb = (uint32_t)(t0 + 8 * g + 4 * half);
      bool pass[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) pass[i] = acc[4 * g + i] <= thr_f;
      if (__builtin_amdgcn_ballot_w64(pass[0] || pass[1] || pass[2] || pass[3])) {
        // branch-free append (a failing key is overwritten or lies past the
        // count); the high word holds the score's float bits, mapped to the
        // monotone code by the merge
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          X[qn * kWaveSize] = ((uint64_t)__float_as_uint(acc[4 * g + i]) << 32) | (rb + (uint32_t)i);
          qn += pass[i] ? 1 : 0;
        }
        if (__builtin_amdgcn_ballot_w64(qn > T - 4)) merge();
      }
    }
  };

  // One register set per operand: as the products of 16 bytes of the
  // current tile are issued, the same 16 bytes of the next tile are loaded
  // into them, a whole tile ahead of their use; the norms are added after
  // the products and reloaded likewise.
  float4 v[NL], nh[4];
#pragma unroll
  for (int g = 0; g < NL; ++g) v[g] = row_part(s0, g);
  norms(s0, nh);
  for (int64_t t0 = s0; t0 < s1; t0 += QW) {
    const int64_t tn = t0 + QW;
    f32x16 acc = {};
#pragma unroll
    for (int g = 0; g < NL; ++g) {
#pragma unroll
      for (int c = 0; c < 4; ++c)
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(comp(v[g], c), qv[4 * g + c], acc, 0, 0, 0);
      v[g] = row_part(tn, g);
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      acc[4 * g] += nh[g].x;
      acc[4 * g + 1] += nh[g].y;
      acc[4 * g + 2] += nh[g].z;
      acc[4 * g + 3] += nh[g].w;
    }
    norms(tn, nh);
    select(acc, t0);
  }
  if (__builtin_amdgcn_ballot_w64(qn > 0)) merge();

  // the query's two half-slice lists merged into the slice's list
  __builtin_amdgcn_wave_barrier();
  const int plen = (int)xor_lane32<32>((uint32_t)len, lane);
  if (half == 0 && qrow < in.n) {
    uint64_t* dst = in.part + ((size_t)qrow * in.P + slice) * kc;
    int a = 0, b = 0;
    for (int s = 0; s < kc; ++s) {
      const uint64_t xa = a < len ? L[a * kWaveSize] : kEmptyKey;
      const uint64_t xb = b < plen ? Lp[b * kWaveSize] : kEmptyKey;
      const bool ta = xa < xb;
      dst[s] = ta ? xa : xb;
      a += ta ? 1 : 0;
      b += ta ? 0 : 1;
    }
  }
}

template <int NG, int T, bool TILED>
hipError_t launch_lane_l2_one(const FusedParams& p, hipStream_t stream) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)lane_l2_kernel<NG, T, TILED>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (p.items && p.nitems <= 0) return hipSuccess;
  const int nq = p.waves * 32;
  dim3 grid = p.items ? dim3((unsigned)p.nitems) : dim3((unsigned)((p.one.n + nq - 1) / nq), (unsigned)p.one.P);
  hipLaunchKernelGGL((lane_l2_kernel<NG, T, TILED>), grid, dim3(p.waves * kWaveSize), lane_lds_bytes(p.waves, p.kc_max, T),
                     stream, p);
  return hipGetLastError();
}

}  // namespace knn
