// knn_kernels.hip -- gfx950 kernels of the brute-force k-NN path.
//
// The brute force of Section 2.1 of the paper computes every query-reference
// distance, sorts each query's distances and keeps the k smallest.  Here the
// two steps are fused: a workgroup scores a block of queries against a slice
// of references tile by tile and keeps, per query, the k' = k + s best
// candidates under the total order (score, reference index); the score
// matrix never leaves the compute unit.  A second kernel merges the
// per-slice candidate lists, recomputes the exact float32 distance of each
// kept candidate in the difference form, orders them by (distance, index)
// and writes the first k.
//
// Euclidean scores use s(q, r) = |r|^2 / 2 - q.r, which orders references as
// |q - r|^2 does for a fixed query (the two differ by |q|^2 / 2 and a factor
// 2).  The cross term q.r is a dense contraction and runs on the matrix cores
// (v_mfma_f32_32x32x2_f32, or v_mfma_f32_32x32x16_{bf16,f16} for the
// low-precision forms) with float32 accumulation; the norm term is preloaded
// into the accumulator.  Manhattan and infinity-norm distances are not
// contractions and run on the vector ALUs in float32.

#include "knn_fused.h"

namespace knn {

// ------------------------------------------------------- point preparation
// Centre of a reference set for the Euclidean scores: the mean of its first
// min(m, kCentreRows) rows.  The distance is invariant under a common
// translation of queries and references, and scores of translated points
// lose far less to cancellation in |r|^2 / 2 - q.r when the data sits away
// from the origin.  One block per 64 dimensions sums the rows in a fixed
// order, so the centre is deterministic.
constexpr int kCentreRows = 256;

__global__ __launch_bounds__(256) void centre_kernel(const float* __restrict__ src, int64_t rows, int d, int lds,
                                                     float* __restrict__ centre) {
  __shared__ float red[4][64];
  const int dl = threadIdx.x & 63, ph = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + dl;
  const int used = (int)(rows < kCentreRows ? rows : kCentreRows);
  float acc = 0.f;
  if (j < d) {
#pragma unroll 16
    for (int i = ph; i < used; i += 4) acc += src[(int64_t)i * lds + j];
  }
  red[ph][dl] = acc;
  __syncthreads();
  if (ph == 0 && j < d) centre[j] = (((red[0][dl] + red[1][dl]) + red[2][dl]) + red[3][dl]) / (float)used;
}

hipError_t launch_centre(const float* src, int64_t rows, int d, int lds, float* centre, hipStream_t stream) {
  hipLaunchKernelGGL(centre_kernel, dim3((unsigned)((d + 63) / 64)), dim3(256), 0, stream, src, rows, d, lds, centre);
  return hipGetLastError();
}

// One wave per row: copy (float32) or round (bf16/f16, nearest even) a row,
// minus `centre` if given, into a zero-padded row of `ldd` elements and, if
// `rhalf` is set, store half the squared norm of the stored (rounded) row.
// TILED (float32 only): element t of row i goes to the 32-row tile layout
// [i / 32][t / 4][i % 32][t % 4], in which the same 16 bytes of 32
// consecutive rows are contiguous.
template <int E, bool TILED = false>
__global__ __launch_bounds__(256) void prep_rows_kernel(const float* __restrict__ src, int64_t rows, int d,
                                                        int lds, const float* __restrict__ centre,
                                                        void* __restrict__ dst, int ldd,
                                                        float* __restrict__ rhalf, unsigned* __restrict__ overflow,
                                                        uint32_t* __restrict__ tshare, int nslots) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= rows) return;
  if (tshare) {
    if (lane == 0) tshare[row] = 0xffffffffu;
    for (int s = lane; s < nslots; s += 64) tshare[rows + s * rows + row] = 0xffffffffu;
  }
  const float* s = src + row * (int64_t)lds;
  float acc = 0.f;
  for (int t = lane; t < ldd; t += 64) {
    float v = t < d ? (centre ? s[t] - centre[t] : s[t]) : 0.f;
    float stored;
    if constexpr (E == ELEM_F32) {
      const int64_t at = TILED ? (((row >> 5) * (ldd >> 2) + (t >> 2)) << 7) + ((row & 31) << 2) + (t & 3) : row * ldd + t;
      ((float*)dst)[at] = v;
      stored = v;
    } else if constexpr (E == ELEM_BF16) {
      uint16_t b = f32_to_bf16_rne(v);
      ((uint16_t*)dst)[row * ldd + t] = b;
      stored = bf16_to_f32(b);
      if (overflow && (b & 0x7fffu) == 0x7f80u) *overflow = 1u;  // finite input rounded to infinity
    } else {
      uint16_t b = f32_to_f16_rne(v);
      ((uint16_t*)dst)[row * ldd + t] = b;
      stored = f16_to_f32(b);
      if (overflow && (b & 0x7fffu) == 0x7c00u) *overflow = 1u;  // |v| beyond the float16 range
    }
    acc += stored * stored;
  }
  if (rhalf) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) rhalf[row] = 0.5f * acc;
  }
}

hipError_t launch_prep_rows_tiled(const float* src, int64_t rows, int d, int lds, const float* centre, float* dst,
                                  int ldd, float* rhalf, hipStream_t stream) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL((prep_rows_kernel<ELEM_F32, true>), dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, stream, src,
                     rows, d, lds, centre, (void*)dst, ldd, rhalf, (unsigned*)nullptr, (uint32_t*)nullptr, 0);
  return hipGetLastError();
}

hipError_t launch_prep_rows(const float* src, int64_t rows, int d, int lds, const float* centre, void* dst, int ldd,
                            int elem, float* rhalf, hipStream_t stream, unsigned* overflow, uint32_t* tshare,
                            int nslots) {
  if (rows <= 0) return hipSuccess;
  dim3 grid((unsigned)((rows + 3) / 4)), block(256);
  if (elem == ELEM_F32)
    hipLaunchKernelGGL(prep_rows_kernel<ELEM_F32>, grid, block, 0, stream, src, rows, d, lds, centre, dst, ldd, rhalf,
                       (unsigned*)nullptr, tshare, nslots);
  else if (elem == ELEM_BF16)
    hipLaunchKernelGGL(prep_rows_kernel<ELEM_BF16>, grid, block, 0, stream, src, rows, d, lds, centre, dst, ldd,
                       rhalf, overflow, tshare, nslots);
  else
    hipLaunchKernelGGL(prep_rows_kernel<ELEM_F16>, grid, block, 0, stream, src, rows, d, lds, centre, dst, ldd, rhalf,
                       overflow, tshare, nslots);
  return hipGetLastError();
}

// ------------------------------------------- fused distance + selection
// (kernel template in knn_fused.h; instantiations in knn_fused_*.hip)

size_t fused_lds_bytes(int kind, int waves, int kc, int cb, int cw) {
  const int es = (kind == TILE_L2_BF16 || kind == TILE_L2_F16) ? 2 : 4;
  return fused_lds_size(es, waves, kc, cb, cw);
}

hipError_t launch_fused(int kind, const FusedParams& p, hipStream_t stream) {
  if (p.wide) return launch_wide(kind, p, stream);
  if (p.lane) return kind == TILE_L2_F32 ? launch_lane_l2(p, stream) : launch_lane(kind, p, stream);
  const bool s = p.kc_max <= 64 && p.cb / 4 <= 16;  // register merge only
  switch (kind) {
    case TILE_L2_F32:
      if (p.ng <= 8) return s ? launch_fused_f32lo_s(p, stream) : launch_fused_f32lo_l(p, stream);
      return s ? launch_fused_f32hi_s(p, stream) : launch_fused_f32hi_l(p, stream);
    case TILE_L2_BF16: return s ? launch_fused_bf16_s(p, stream) : launch_fused_bf16_l(p, stream);
    case TILE_L2_F16: return s ? launch_fused_f16_s(p, stream) : launch_fused_f16_l(p, stream);
    case TILE_L1_F32: return s ? launch_fused_l1_s(p, stream) : launch_fused_l1_l(p, stream);
    case TILE_LINF_F32: return s ? launch_fused_linf_s(p, stream) : launch_fused_linf_l(p, stream);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------ merge + exact re-rank + output
//
// One wave per query.  (1) The P sorted per-slice lists are merged: for few
// lists by rank (the key at position i of list p lands at i + sum over the
// other lists of the number of their keys below it), for many by a k-way
// merge over the list heads held one per lane; the first k' are kept.  (2) Each kept
// candidate's distance is recomputed exactly in float32 in the difference
// form (sum of squared differences, sum of absolute differences, or the
// largest absolute difference) from the canonical rows.  (3) Candidates are
// ordered by (distance, index) and the first k are written; Euclidean
// distances are returned as the square root.

__device__ __forceinline__ float load_canon(const void* base, int type, int64_t off) {
  if (type == ELEM_F32) return ((const float*)base)[off];
  if (type == ELEM_F16) return f16_to_f32(((const uint16_t*)base)[off]);
  return bf16_to_f32(((const uint16_t*)base)[off]);
}

__device__ __forceinline__ float exact_distance(const float* q, const void* rm, int type, int64_t roff, int d,
                                                int metric) {
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  int t = 0;
  for (; t + 4 <= d; t += 4) {
    const float d0 = q[t] - load_canon(rm, type, roff + t);
    const float d1 = q[t + 1] - load_canon(rm, type, roff + t + 1);
    const float d2 = q[t + 2] - load_canon(rm, type, roff + t + 2);
    const float d3 = q[t + 3] - load_canon(rm, type, roff + t + 3);
    if (metric == 0) {
      s0 = fmaf(d0, d0, s0); s1 = fmaf(d1, d1, s1); s2 = fmaf(d2, d2, s2); s3 = fmaf(d3, d3, s3);
    } else if (metric == 1) {
      s0 += fabsf(d0); s1 += fabsf(d1); s2 += fabsf(d2); s3 += fabsf(d3);
    } else {
      s0 = fmaxf(s0, fabsf(d0)); s1 = fmaxf(s1, fabsf(d1)); s2 = fmaxf(s2, fabsf(d2)); s3 = fmaxf(s3, fabsf(d3));
    }
  }
  for (; t < d; ++t) {
    const float d0 = q[t] - load_canon(rm, type, roff + t);
    if (metric == 0) s0 = fmaf(d0, d0, s0);
    else if (metric == 1) s0 += fabsf(d0);
    else s0 = fmaxf(s0, fabsf(d0));
  }
  if (metric == 2) return fmaxf(fmaxf(s0, s1), fmaxf(s2, s3));
  return (s0 + s1) + (s2 + s3);
}

// One lane's share of an exact distance: dims first, first + stride, ...
// in runs of `run` (4 float32 or 8 16-bit values per 16-byte load).  The
// row is zero-padded to a whole number of runs; query values past d are
// taken as zero, so padded dims contribute nothing.
__device__ __forceinline__ float exact_distance_run(const float* q, bool qvec, const void* rm, int type, int64_t roff,
                                                    int d, int metric, int first, int stride, int run) {
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  auto acc4 = [&](float a0, float a1, float a2, float a3) __attribute__((always_inline)) {
    if (metric == 0) {
      s0 = fmaf(a0, a0, s0); s1 = fmaf(a1, a1, s1); s2 = fmaf(a2, a2, s2); s3 = fmaf(a3, a3, s3);
    } else if (metric == 1) {
      s0 += fabsf(a0); s1 += fabsf(a1); s2 += fabsf(a2); s3 += fabsf(a3);
    } else {
      s0 = fmaxf(s0, fabsf(a0)); s1 = fmaxf(s1, fabsf(a1)); s2 = fmaxf(s2, fabsf(a2)); s3 = fmaxf(s3, fabsf(a3));
    }
  };
  auto qload4 = [&](int t) __attribute__((always_inline)) {
    if (qvec && t + 4 <= d) return gload4(q + t);
    return make_float4(t < d ? gload1(q + t) : 0.f, t + 1 < d ? gload1(q + t + 1) : 0.f,
                       t + 2 < d ? gload1(q + t + 2) : 0.f, t + 3 < d ? gload1(q + t + 3) : 0.f);
  };
  for (int t = first; t < d; t += stride) {
    if (type == ELEM_F32) {
      const float4 rv = gload4((const float*)rm + roff + t);
      const float4 qv = qload4(t);
      acc4(qv.x - rv.x, qv.y - rv.y, qv.z - rv.z, qv.w - rv.w);
    } else {
      const uint4 rv = gload16((const uint16_t*)rm + roff + t);
      const uint32_t w[4] = {rv.x, rv.y, rv.z, rv.w};
      float r8[8];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint16_t lo = (uint16_t)(w[i] & 0xffffu), hi = (uint16_t)(w[i] >> 16);
        r8[2 * i] = type == ELEM_F16 ? f16_to_f32(lo) : bf16_to_f32(lo);
        r8[2 * i + 1] = type == ELEM_F16 ? f16_to_f32(hi) : bf16_to_f32(hi);
      }
      const float4 qa = qload4(t), qb = qload4(t + 4);
      acc4(qa.x - r8[0], qa.y - r8[1], qa.z - r8[2], qa.w - r8[3]);
      acc4(qb.x - r8[4], qb.y - r8[5], qb.z - r8[6], qb.w - r8[7]);
    }
  }
  if (metric == 2) return fmaxf(fmaxf(s0, s1), fmaxf(s2, s3));
  return (s0 + s1) + (s2 + s3);
}

// combine the partial results of the 16 lanes of a row (fixed order)
__device__ __forceinline__ float reduce16(float s, int metric, int lane) {
#define KNN_STEP(J)                                                        \
  {                                                                         \
    const float o = __uint_as_float(xor_lane32<J>(__float_as_uint(s), lane)); \
    s = metric == 2 ? fmaxf(s, o) : s + o;                                  \
  }
  KNN_STEP(8) KNN_STEP(4) KNN_STEP(2) KNN_STEP(1)
#undef KNN_STEP
  return s;
}

__host__ __device__ inline size_t finalize_wave_bytes(int keys_max, int p_max, int kprime_max) {
  return (((size_t)keys_max * 8 + (size_t)p_max * 4 + (size_t)kprime_max * 8) + 15) & ~(size_t)15;
}

__global__ __launch_bounds__(256) void finalize_kernel(FinalParams p) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  FinalInst in;
  int64_t q;
  if (p.items) {
    const FinalItem it = p.items[blockIdx.x];
    in = p.insts[it.inst];
    q = (int64_t)it.q0 + wave;
  } else {
    in = p.one;
    q = (int64_t)blockIdx.x * kFinalWaves + wave;
  }
  const int T = in.P * in.kc;
  // per-wave region: keys[T] | lens[P] | cand[kprime] | cdist[kprime], sized
  // for the largest instance of the launch
  const size_t wave_bytes = finalize_wave_bytes(p.keys_max, p.p_max, p.kprime_max);
  unsigned char* base = smem + wave * wave_bytes;
  uint64_t* keys = (uint64_t*)base;
  int* lens = (int*)(keys + T);
  uint32_t* cand = (uint32_t*)(lens + in.P);
  float* cdist = (float*)(cand + in.kprime);
  if (q >= in.n) return;

  const uint64_t* src = in.part + q * (int64_t)T;
  for (int e = lane; e < T; e += 64) keys[e] = src[e];
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  for (int pl = lane; pl < in.P; pl += 64) {
    const uint64_t* L = keys + pl * in.kc;
    int lo = 0, hi = in.kc;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (L[mid] != kEmptyKey) lo = mid + 1; else hi = mid;
    }
    lens[pl] = lo;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();

  int nvalid = 0;
  for (int pl = 0; pl < in.P; ++pl) nvalid += lens[pl];
  const int nc = min(in.kprime, nvalid);

  if (in.P <= 8 && in.kc <= 32 && in.kprime <= 32) {
    // up to 8 lists of at most 32 keys: a bitonic merge tree in registers.
    // Register j holds list 2j ascending in lanes 0..31 and list 2j+1
    // descending in lanes 32..63; the lane-wise minimum across the halves is
    // a bitonic sequence holding the 32 smallest keys of the pair, which five
    // exchange stages sort (ascending for even j, descending for odd j, so
    // that the next level pairs an ascending with a descending run).
    const int i = lane & 31, up = lane >> 5;
    uint64_t v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int pl = 2 * j + up, e = up ? 31 - i : i;
      v[j] = pl < in.P && e < lens[pl] ? keys[pl * in.kc + e] : kEmptyKey;
    }
    auto clean32 = [&](uint64_t x, bool asc) __attribute__((always_inline)) {
      x = bitonic_step<16>(x, lane, asc);
      x = bitonic_step<8>(x, lane, asc);
      x = bitonic_step<4>(x, lane, asc);
      x = bitonic_step<2>(x, lane, asc);
      return bitonic_step<1>(x, lane, asc);
    };
    const int nreg = (in.P + 1) / 2;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j < nreg) v[j] = clean32(min(v[j], xor_lane64<32>(v[j], lane)), (j & 1) == 0);
    // level 2: runs 0 (ascending) and 1 (descending), 2 and 3, lane-wise
    if (nreg > 1) v[0] = clean32(min(v[0], v[1]), true);
    if (nreg > 2) v[2] = clean32(min(v[2], nreg > 3 ? v[3] : kEmptyKey), false);
    if (nreg > 2) v[0] = clean32(min(v[0], v[2]), true);
    if (lane < nc) cand[lane] = (uint32_t)v[0];
  } else if (in.P <= 4 || in.P > 64) {
    // few lists: each key's merged position by binary searches in the others
    for (int e = lane; e < T; e += 64) {
      const int pl = e / in.kc, i = e - pl * in.kc;
      if (i >= lens[pl] || i >= in.kprime) continue;
      const uint64_t x = keys[e];
      int rank = i;
      for (int o = 0; o < in.P && rank < in.kprime; ++o) {
        if (o == pl) continue;
        const uint64_t* L = keys + o * in.kc;
        int lo = 0, hi = lens[o];
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (L[mid] < x) lo = mid + 1; else hi = mid;
        }
        rank += lo;
      }
      if (rank < in.kprime) cand[rank] = (uint32_t)x;
    }
  } else {
    // many lists (5..64): a k-way merge.  Lane p holds the head of list
    // p; each round the wave minimum of the heads (keys are distinct) is
    // the next key in merged order, and its list advances.
    int hp = 0;
    uint64_t head = lane < in.P && lens[lane] > 0 ? keys[lane * in.kc] : kEmptyKey;
    for (int r = 0; r < nc; ++r) {
      uint64_t mn = head;
      mn = min(mn, xor_lane64<32>(mn, lane));
      mn = min(mn, xor_lane64<16>(mn, lane));
      mn = min(mn, xor_lane64<8>(mn, lane));
      mn = min(mn, xor_lane64<4>(mn, lane));
      mn = min(mn, xor_lane64<2>(mn, lane));
      mn = min(mn, xor_lane64<1>(mn, lane));
      if (head == mn) {
        cand[r] = (uint32_t)mn;
        ++hp;
        head = hp < lens[lane] ? keys[lane * in.kc + hp] : kEmptyKey;
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();

  const float* qrow = in.Q + q * (int64_t)in.ldq;
  // Rows that allow 16-byte loads are re-ranked by 16 lanes per candidate
  // (four candidates at a time, each lane a run of 4 or 8 consecutive dims,
  // the 16 partial results combined by a fixed tree); others one per lane.
  const bool vec_rows =
      ((uintptr_t)in.Rm % 16) == 0 && (in.rm_type == ELEM_F32 ? in.ldr % 4 == 0 : in.ldr % 8 == 0);
  if (vec_rows) {
    const int sub = lane & 15, grp = lane >> 4;
    const int run = in.rm_type == ELEM_F32 ? 4 : 8;  // dims per lane and pass
    const bool qvec = ((uintptr_t)qrow % 16) == 0;
    for (int j0 = 0; j0 < nc; j0 += 4) {
      const int j = j0 + grp;
      const uint32_t r = j < nc ? cand[j] : 0u;
      const bool live = j < nc && r < (uint64_t)in.m;
      float s = 0.f;
      if (live) s = exact_distance_run(qrow, qvec, in.Rm, in.rm_type, (int64_t)r * in.ldr, in.d, in.metric,
                                       run * sub, run * 16, run);
      s = reduce16(s, in.metric, lane);
      if (sub == 0 && j < nc) cdist[j] = live ? s : __builtin_huge_valf();
    }
  } else {
    for (int j = lane; j < nc; j += 64) {
      const uint32_t r = cand[j];
      cdist[j] = r < (uint64_t)in.m
                     ? exact_distance(qrow, in.Rm, in.rm_type, (int64_t)r * in.ldr, in.d, in.metric)
                     : __builtin_huge_valf();
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();

  for (int j = lane; j < nc; j += 64) {
    const float dj = cdist[j];
    const uint32_t rj = cand[j];
    int rank = 0;
    for (int i = 0; i < nc; ++i) {
      const float di = cdist[i];
      rank += (di < dj) || (di == dj && cand[i] < rj);
    }
    if (rank < in.k) {
      in.dist[q * in.k + rank] = in.metric == 0 ? sqrtf(dj) : dj;
      in.idx[q * in.k + rank] = (int32_t)rj;
    }
  }
}

hipError_t launch_finalize(const FinalParams& p, hipStream_t stream) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)finalize_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       kLdsBytes);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const unsigned blocks = p.items ? (unsigned)p.nitems : (unsigned)((p.one.n + kFinalWaves - 1) / kFinalWaves);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_kernel, dim3(blocks), dim3(kFinalWaves * kWaveSize),
                     finalize_lds_bytes(p.keys_max, p.p_max, p.kprime_max), stream, p);
  return hipGetLastError();
}

size_t finalize_lds_bytes(int keys_max, int p_max, int kprime_max) {
  return finalize_wave_bytes(keys_max, p_max, kprime_max) * kFinalWaves;
}

// ------------------------------------------- merge of slice lists (kc <= 64)
// Groups of G consecutive sorted lists of each query are merged into one:
// part [n][P][kc] -> out [n][P2][kc], P2 = ceil(P / G).  One wave per
// (query, group): the running list sits one key per lane, ascending; the
// next list is loaded in reverse, so that the lane-wise minimum of the two
// is a bitonic sequence holding the 64 smallest keys of both, which six
// exchange stages sort.  Empty slots (all ones) sort last.
__global__ __launch_bounds__(256) void merge_lists_kernel(const uint64_t* __restrict__ part, uint64_t* __restrict__ out,
                                                          int64_t n, int P, int kc, int G, int P2) {
  const int lane = threadIdx.x & 63;
  const int64_t wv = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wv >= n * P2) return;
  const int64_t q = wv / P2;
  const int g = (int)(wv - q * P2);
  const uint64_t* src = part + q * (int64_t)P * kc;
  const int l0 = g * G, l1 = min(P, l0 + G);
  uint64_t acc = lane < kc ? src[(int64_t)l0 * kc + lane] : kEmptyKey;
  for (int l = l0 + 1; l < l1; ++l) {
    const int e = 63 - lane;
    const uint64_t x = e < kc ? src[(int64_t)l * kc + e] : kEmptyKey;
    acc = bitonic_clean64(acc < x ? acc : x, lane);
  }
  if (lane < kc) out[(q * P2 + g) * (int64_t)kc + lane] = acc;
}

hipError_t launch_merge_lists(const uint64_t* part, uint64_t* out, int64_t n, int P, int kc, int G, int P2,
                              hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  if (kc < 1 || kc > 64 || G < 1 || P2 != (P + G - 1) / G) return hipErrorInvalidValue;
  const int64_t waves = n * P2;
  hipLaunchKernelGGL(merge_lists_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, stream, part, out, n, P, kc,
                     G, P2);
  return hipGetLastError();
}

// ------------------------------------------------ Mahalanobis transform
// Y[i][j] = sum_t (X[i][t] - c[t]) L[t][j]: rows mapped by L^T after a common
// translation by c (which cancels in every difference), one thread per output
// element, the sum in ascending t with fused multiply-adds.
__global__ __launch_bounds__(256) void transform_rows_kernel(const float* __restrict__ X, int64_t rows, int d,
                                                             const float* __restrict__ c,
                                                             const float* __restrict__ L, float* __restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * d) return;
  const int64_t i = e / d;
  const int j = (int)(e - i * d);
  const float* x = X + i * d;
  float acc = 0.f;
  for (int t = 0; t < d; ++t) acc = fmaf(x[t] - c[t], L[(int64_t)t * d + j], acc);
  Y[e] = acc;
}

hipError_t launch_transform_rows(const float* X, int64_t rows, int d, const float* c, const float* L, float* Y,
                                 hipStream_t stream) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(transform_rows_kernel, dim3((unsigned)((rows * d + 255) / 256)), dim3(256), 0, stream, X, rows,
                     d, c, L, Y);
  return hipGetLastError();
}

// Exact re-rank of Mahalanobis candidates: for each query's kc candidates
// (found by the Euclidean search of the mapped points), the distance
// ||L^T (q - r)|| from the caller's rows: the difference q - r in float32,
// then y = L^T (q - r) and sum y^2 accumulated in double precision in a
// fixed order, rounded to float32; the k best by (distance, index) are
// written.  One wave per query.
__global__ __launch_bounds__(256) void mahalanobis_rerank_kernel(const float* __restrict__ Q,
                                                                 const float* __restrict__ R,
                                                                 const float* __restrict__ L, int64_t n, int d,
                                                                 int64_t m, const int32_t* __restrict__ cidx, int kc,
                                                                 float* __restrict__ dist, int32_t* __restrict__ idx,
                                                                 int k) {
  extern __shared__ __align__(16) unsigned char smem_mr[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t q = (int64_t)blockIdx.x * 4 + wave;
  float* diff = (float*)smem_mr + (size_t)wave * (d + 2 * kc);
  float* cd = diff + d;
  int32_t* ci = (int32_t*)(cd + kc);
  if (q >= n) return;
  const float* qrow = Q + q * (int64_t)d;
  for (int j = 0; j < kc; ++j) {
    int32_t r = cidx[q * kc + j];
    const bool live = r >= 0 && (int64_t)r < m;
    if (!live) r = 0;
    const float* rrow = R + (int64_t)r * d;
    for (int t = lane; t < d; t += 64) diff[t] = qrow[t] - rrow[t];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    double s = 0.0;
    for (int u = lane; u < d; u += 64) {
      double y = 0.0;
      for (int t = 0; t < d; ++t) y = fma((double)L[(int64_t)t * d + u], (double)diff[t], y);
      s = fma(y, y, s);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) {
      cd[j] = live ? (float)sqrt(s) : __builtin_huge_valf();
      ci[j] = live ? r : 0x7fffffff;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  for (int j = lane; j < kc; j += 64) {
    const float dj = cd[j];
    const int32_t rj = ci[j];
    int rank = 0;
    for (int i = 0; i < kc; ++i) rank += (cd[i] < dj) || (cd[i] == dj && ci[i] < rj);
    if (rank < k) {
      dist[q * k + rank] = dj;
      idx[q * k + rank] = rj;
    }
  }
}

hipError_t launch_mahalanobis_rerank(const float* Q, const float* R, const float* L, int64_t n, int d, int64_t m,
                                     const int32_t* cidx, int kc, float* dist, int32_t* idx, int k,
                                     hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const size_t lds = (size_t)4 * (d + 2 * kc) * 4;
  if (lds > (size_t)kLdsBytes) return hipErrorInvalidValue;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)mahalanobis_rerank_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(mahalanobis_rerank_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), lds, stream, Q, R, L, n, d,
                     m, cidx, kc, dist, idx, k);
  return hipGetLastError();
}

// ------------------------------------------------ k-NN classification
// Majority label of each query's k nearest (idx [n][k], nearest first): the
// count of neighbour j's label among the k, maximised over j; the first j
// (nearest) with the top count wins, so a tie between classes goes to the
// class of the nearest neighbour among the tied classes.  One thread per
// query, k^2 label comparisons.
__global__ __launch_bounds__(256) void vote_kernel(const int32_t* __restrict__ idx, int64_t n, int k,
                                                   const int32_t* __restrict__ labels, int32_t* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= n) return;
  const int32_t* row = idx + q * (int64_t)k;
  int best = -1, best_count = 0;
  for (int j = 0; j < k; ++j) {
    const int32_t lj = labels[row[j]];
    int c = 0;
    for (int t = 0; t < k; ++t) c += labels[row[t]] == lj ? 1 : 0;
    if (c > best_count) {
      best_count = c;
      best = lj;
    }
  }
  out[q] = best;
}

hipError_t launch_vote(const int32_t* idx, int64_t n, int k, const int32_t* labels, int32_t* out,
                       hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(vote_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, idx, n, k, labels, out);
  return hipGetLastError();
}

// ------------------------------------------------ k-NN entropy estimate
// log rho_k(y_i) for every point from its k + 1 nearest in (distance, index)
// order: the point's own entry (distance 0) is dropped, which leaves the k-th
// other neighbour at position k if the point was among the k + 1, else at
// position k - 1 (then k + 1 other points lie at distance 0).
__global__ __launch_bounds__(256) void entropy_terms_kernel(const float* __restrict__ dist,
                                                            const int32_t* __restrict__ idx, int64_t n, int k,
                                                            double* __restrict__ terms) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t row = i * (int64_t)(k + 1);
  bool self = false;
  for (int j = 0; j <= k; ++j) self |= idx[row + j] == (int32_t)i;
  terms[i] = log((double)dist[row + (self ? k : k - 1)]);
}

// out = scale * (sum of terms) + offset: one workgroup, each thread a fixed
// strided subset in order, then a fixed tree over the threads
__global__ __launch_bounds__(1024) void entropy_sum_kernel(const double* __restrict__ terms, int64_t n, double scale,
                                                           double offset, double* __restrict__ out) {
  __shared__ double part[1024];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) s += terms[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = scale * part[0] + offset;
}

hipError_t launch_entropy(const float* dist, const int32_t* idx, int64_t n, int k, double* terms, double scale,
                          double offset, double* out, hipStream_t stream) {
  hipLaunchKernelGGL(entropy_terms_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, dist, idx, n, k,
                     terms);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(entropy_sum_kernel, dim3(1), dim3(1024), 0, stream, terms, n, scale, offset, out);
  return hipGetLastError();
}

// ------------------------------------------------ batched point preparation
// One wave per row over the concatenated rows of several arrays; a row's
// job is found by binary search over the jobs' first rows.
__global__ __launch_bounds__(256) void prep_batched_kernel(const PrepJob* __restrict__ jobs, int njobs,
                                                           int64_t total_rows, int* __restrict__ zero) {
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (zero && g == 0 && lane == 0) *zero = 0;  // item counter of the launch that follows
  if (g >= total_rows) return;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].row0 <= g) lo = mid; else hi = mid - 1;
  }
  const PrepJob jb = jobs[lo];
  const int64_t row = g - jb.row0;
  if (jb.tshare) {
    if (lane == 0) jb.tshare[row] = 0xffffffffu;
    for (int s = lane; s < jb.nslots; s += 64) jb.tshare[jb.rows + s * jb.rows + row] = 0xffffffffu;
  }
  const float* s = jb.src + row * (int64_t)jb.lds;
  float acc = 0.f;
  for (int t = lane; t < jb.ldd; t += 64) {
    const float v = t < jb.d ? (jb.centre ? s[t] - jb.centre[t] : s[t]) : 0.f;
    float stored;
    if (jb.elem == ELEM_F32) {
      ((float*)jb.dst)[row * jb.ldd + t] = v;
      stored = v;
    } else if (jb.elem == ELEM_BF16) {
      const uint16_t b = f32_to_bf16_rne(v);
      ((uint16_t*)jb.dst)[row * jb.ldd + t] = b;
      stored = bf16_to_f32(b);
    } else {
      const uint16_t b = f32_to_f16_rne(v);
      ((uint16_t*)jb.dst)[row * jb.ldd + t] = b;
      stored = f16_to_f32(b);
    }
    acc += stored * stored;
  }
  if (jb.rhalf) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) jb.rhalf[row] = 0.5f * acc;
  }
}

hipError_t launch_prep_batched(const PrepJob* jobs_dev, int njobs, int64_t total_rows, hipStream_t stream,
                               int* zero) {
  if ((total_rows <= 0 || njobs <= 0) && !zero) return hipSuccess;
  const int64_t rows = total_rows > 0 && njobs > 0 ? total_rows : 0;
  hipLaunchKernelGGL(prep_batched_kernel, dim3((unsigned)std::max<int64_t>(1, (rows + 3) / 4)), dim3(256), 0, stream,
                     jobs_dev, njobs, rows, zero);
  return hipGetLastError();
}

}  // namespace knn
