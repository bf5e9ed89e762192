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

#include "knn_internal.h"

namespace knn {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------- helpers

// float -> monotone unsigned code: a < b as floats (non-NaN) iff code(a) < code(b)
__device__ __forceinline__ uint32_t mono_code(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float mono_value(uint32_t c) {
  return __uint_as_float((c & 0x80000000u) ? (c & 0x7fffffffu) : ~c);
}

__device__ __forceinline__ uint64_t make_key(float score, uint32_t ref) {
  return ((uint64_t)mono_code(score) << 32) | ref;
}

// round to nearest even; NaN/Inf are outside the contract
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ uint16_t f32_to_f16_rne(float f) {
  _Float16 h = (_Float16)f;
  return __builtin_bit_cast(uint16_t, h);
}

__device__ __forceinline__ float f16_to_f32(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

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
  if (j < d)
    for (int i = ph; i < used; i += 4) acc += src[(int64_t)i * lds + j];
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
template <int E>
__global__ __launch_bounds__(256) void prep_rows_kernel(const float* __restrict__ src, int64_t rows, int d,
                                                        int lds, const float* __restrict__ centre,
                                                        void* __restrict__ dst, int ldd,
                                                        float* __restrict__ rhalf) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= rows) return;
  const float* s = src + row * (int64_t)lds;
  float acc = 0.f;
  for (int t = lane; t < ldd; t += 64) {
    float v = t < d ? (centre ? s[t] - centre[t] : s[t]) : 0.f;
    float stored;
    if constexpr (E == ELEM_F32) {
      ((float*)dst)[row * ldd + t] = v;
      stored = v;
    } else if constexpr (E == ELEM_BF16) {
      uint16_t b = f32_to_bf16_rne(v);
      ((uint16_t*)dst)[row * ldd + t] = b;
      stored = bf16_to_f32(b);
    } else {
      uint16_t b = f32_to_f16_rne(v);
      ((uint16_t*)dst)[row * ldd + t] = b;
      stored = f16_to_f32(b);
    }
    acc += stored * stored;
  }
  if (rhalf) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) rhalf[row] = 0.5f * acc;
  }
}

hipError_t launch_prep_rows(const float* src, int64_t rows, int d, int lds, const float* centre, void* dst, int ldd,
                            int elem, float* rhalf, hipStream_t stream) {
  if (rows <= 0) return hipSuccess;
  dim3 grid((unsigned)((rows + 3) / 4)), block(256);
  if (elem == ELEM_F32)
    hipLaunchKernelGGL(prep_rows_kernel<ELEM_F32>, grid, block, 0, stream, src, rows, d, lds, centre, dst, ldd, rhalf);
  else if (elem == ELEM_BF16)
    hipLaunchKernelGGL(prep_rows_kernel<ELEM_BF16>, grid, block, 0, stream, src, rows, d, lds, centre, dst, ldd,
                       rhalf);
  else
    hipLaunchKernelGGL(prep_rows_kernel<ELEM_F16>, grid, block, 0, stream, src, rows, d, lds, centre, dst, ldd, rhalf);
  return hipGetLastError();
}

// ------------------------------------------------------ wave-private merge
// One query's sorted list L (len keys) and unsorted candidate buffer B
// (c keys) are replaced by the first kc keys of their union, sorted.  All
// keys are distinct (a reference enters a query's buffer at most once per
// slice).  Each lane places up to NR keys by rank: a list key at position e
// moves to e + #{b in B: b < key}; a buffer key goes to #{x in L: x < key} +
// #{b in B: b < key}.
template <int NR>
__device__ __forceinline__ void merge_ranked(uint64_t* L, const uint64_t* B, int len, int c, int kc, int lane) {
  const int T = len + c;
  uint64_t x[NR];
  int below[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int e = lane + 64 * r;
    x[r] = kEmptyKey;
    below[r] = 0;
    if (e < T) x[r] = e < len ? L[e] : B[e - len];
  }
  int j = 0;
  for (; j + 4 <= c; j += 4) {
    const uint64_t b0 = B[j], b1 = B[j + 1], b2 = B[j + 2], b3 = B[j + 3];
#pragma unroll
    for (int r = 0; r < NR; ++r)
      below[r] += (int)(b0 < x[r]) + (int)(b1 < x[r]) + (int)(b2 < x[r]) + (int)(b3 < x[r]);
  }
  for (; j < c; ++j) {
    const uint64_t b = B[j];
#pragma unroll
    for (int r = 0; r < NR; ++r) below[r] += (int)(b < x[r]);
  }
  int top = 1;
  while (top * 2 <= len) top *= 2;
  int rank[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int e = lane + 64 * r;
    rank[r] = 0x7fffffff;
    if (e < len) {
      rank[r] = e + below[r];
    } else if (e < T) {
      int pos = 0;  // number of list keys below x[r]
      for (int st = top; st > 0; st >>= 1)
        if (pos + st <= len && L[pos + st - 1] < x[r]) pos += st;
      rank[r] = pos + below[r];
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (rank[r] < kc) L[rank[r]] = x[r];
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void wave_merge(uint64_t* L, const uint64_t* B, int* lenp, int* cntp, int kc, int lane) {
  const int len = *lenp, c = *cntp;
  const int nr = (len + c + 63) >> 6;
  switch (nr) {
    case 0: break;
    case 1: merge_ranked<1>(L, B, len, c, kc, lane); break;
    case 2: merge_ranked<2>(L, B, len, c, kc, lane); break;
    case 3: merge_ranked<3>(L, B, len, c, kc, lane); break;
    case 4: merge_ranked<4>(L, B, len, c, kc, lane); break;
    case 5: merge_ranked<5>(L, B, len, c, kc, lane); break;
    case 6: merge_ranked<6>(L, B, len, c, kc, lane); break;
    case 7: merge_ranked<7>(L, B, len, c, kc, lane); break;
    default: merge_ranked<8>(L, B, len, c, kc, lane); break;
  }
  __builtin_amdgcn_wave_barrier();
  if (lane == 0) {
    *lenp = min(kc, len + c);
    *cntp = 0;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------- fused distance + selection
//
// Workgroup = `waves` waves (up to 8, two per SIMD); wave w owns 16 queries
// q0 + 16w .. q0 + 16w + 15 and their selection state; all waves share the
// reference tiles staged in LDS.  A step scores 64 references (four 16x16
// tiles) against the wave's 16 queries.  In the 16x16 MFMA output layout
// lane l holds column l % 16 (its query) and rows 4*(l/16) + i, i = 0..3, of
// each tile; the vector-ALU kernels compute the same lane -> (query,
// reference) layout so that the selection code is shared.
//
// Selection per query: a sorted list of the kc best keys so far and a buffer
// of up to cb unsorted candidates, both in LDS.  A score enters the buffer
// only if it is <= the list's kc-th score (the threshold, +inf until the
// list is full).  After each tile (at most 16 new candidates per query) a
// buffer that could overflow on the next tile is merged into the list by the
// whole wave, which also tightens the threshold.

constexpr int kPrefetchVecs = kPrefetchVecsHost;  // 16-byte global loads per thread per staged chunk

template <int KIND>
struct TileCfg {
  static constexpr bool mfma = KIND <= TILE_L2_F16;
  static constexpr bool half16 = KIND == TILE_L2_BF16 || KIND == TILE_L2_F16;
  static constexpr int es = half16 ? 2 : 4;  // element size in bytes
};

template <int KIND>
__global__ __launch_bounds__(512) void fused_select_kernel(FusedParams p) {
  using Cfg = TileCfg<KIND>;
  constexpr int ES = Cfg::es;
  extern __shared__ __align__(16) unsigned char smem[];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, col = lane & 15, kq = lane >> 4;
  const int nthreads = blockDim.x;
  const int nq = p.waves * kQueriesPerWave;
  const int64_t q0 = (int64_t)blockIdx.x * nq;
  const int ql = wave * kQueriesPerWave + col;
  const int64_t qrow = q0 + ql;
  const int64_t qsafe = qrow < p.n ? qrow : p.n - 1;
  const int64_t s0 = (int64_t)blockIdx.y * p.slice_len;
  const int64_t s1 = min(p.m, s0 + p.slice_len);
  const int ntiles = (int)((s1 - s0 + kStepRefs - 1) / kStepRefs);
  const int kc = p.kc, cb = p.cb;

  uint64_t* lists = (uint64_t*)smem;
  uint64_t* bufs = lists + (size_t)nq * kc;
  int* counts = (int*)(bufs + (size_t)nq * cb);
  int* lens = counts + nq;
  float* nbuf = (float*)(lens + nq);
  unsigned char* rbuf = (unsigned char*)(nbuf + 2 * kStepRefs);
  const int tile_bytes = kStepRefs * p.rstride * ES;

  for (int i = tid; i < nq; i += nthreads) {
    counts[i] = 0;
    lens[i] = 0;
  }

  // ---- query operands in registers (MFMA kinds), one chunk of dims at a
  // time.  Lane group kq = l / 16 supplies the k slots of the MFMA; group g
  // of four float32 MFMAs covers dims 16g .. 16g+15, lane group kq holding
  // 16g+4kq .. 16g+4kq+3; a 16-bit MFMA s covers 32s .. 32s+31, lane group
  // kq holding 32s+8kq .. 32s+8kq+7.  The reference tile is read with the
  // same mapping, so every product pairs the same dimension.  Queries are
  // negated so that the MFMA adds -q.r to the preloaded |r|^2 / 2.
  float4 qf[16];
  uint4 qh[8];
  auto load_q = [&](int c) {
    const int cb0 = c * p.cw;
    const int cwc = min(p.cw, p.dp - cb0);
    if constexpr (Cfg::mfma && !Cfg::half16) {
      const float* qp = (const float*)p.Q + qsafe * (int64_t)p.ldq + cb0;
#pragma unroll
      for (int g = 0; g < 16; ++g) {
        qf[g] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (g * 16 < cwc && qrow < p.n) {
          const float4 v = *(const float4*)(qp + g * 16 + 4 * kq);
          qf[g] = make_float4(-v.x, -v.y, -v.z, -v.w);
        }
      }
    } else if constexpr (Cfg::mfma) {
      const uint16_t* qp = (const uint16_t*)p.Q + qsafe * (int64_t)p.ldq + cb0;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        qh[s] = make_uint4(0u, 0u, 0u, 0u);
        if (s * 32 < cwc && qrow < p.n) {
          const uint4 v = *(const uint4*)(qp + s * 32 + 8 * kq);
          qh[s] = make_uint4(v.x ^ 0x80008000u, v.y ^ 0x80008000u, v.z ^ 0x80008000u, v.w ^ 0x80008000u);
        }
      }
    }
  };
  if (p.nchunk == 1) load_q(0);

  // ---- staging of reference tiles through registers (double-buffered LDS)
  uint4 pf[kPrefetchVecs];
  float pfn = 0.f;
  int pf_vpr = 0;  // 16-byte vectors per staged row of the prefetched chunk
  auto load_stage = [&](int step) {
    const int tile = step / p.nchunk, c = step - tile * p.nchunk;
    const int64_t rb = s0 + (int64_t)tile * kStepRefs;
    const int vpr = min(p.cw, p.dp - c * p.cw) * ES / 16;
    const int nvec = kStepRefs * vpr;
    pf_vpr = vpr;
    const unsigned char* gR = (const unsigned char*)p.R;
#pragma unroll
    for (int r = 0; r < kPrefetchVecs; ++r) {
      const int e = tid + r * nthreads;
      pf[r] = make_uint4(0u, 0u, 0u, 0u);
      if (e < nvec) {
        const int row = e / vpr, cv = e - row * vpr;
        const int64_t g = rb + row;
        if (g < s1) pf[r] = *(const uint4*)(gR + (g * p.ldr + (int64_t)c * p.cw) * ES + cv * 16);
      }
    }
    if constexpr (Cfg::mfma) {
      if (tid < kStepRefs) pfn = (rb + tid < s1) ? p.rhalf[rb + tid] : 0.f;
    }
  };
  auto store_stage = [&](int buf) {
    unsigned char* dst = rbuf + buf * tile_bytes;
    const int vpr = pf_vpr, nvec = kStepRefs * vpr;
#pragma unroll
    for (int r = 0; r < kPrefetchVecs; ++r) {
      const int e = tid + r * nthreads;
      if (e < nvec) {
        const int row = e / vpr, cv = e - row * vpr;
        *(uint4*)(dst + row * p.rstride * ES + cv * 16) = pf[r];
      }
    }
    if constexpr (Cfg::mfma) {
      if (tid < kStepRefs) nbuf[buf * kStepRefs + tid] = pfn;
    }
  };

  const int nsteps = ntiles * p.nchunk;
  float thr = __builtin_huge_valf();
  f32x4 acc[kTilesPerStep];

  if (nsteps > 0) {
    load_stage(0);
    store_stage(0);
  }
  __syncthreads();

  for (int step = 0; step < nsteps; ++step) {
    const int buf = step & 1;
    const int tile = step / p.nchunk, c = step - tile * p.nchunk;
    if (step + 1 < nsteps) load_stage(step + 1);
    const unsigned char* rt = rbuf + buf * tile_bytes;

    if (c == 0) {
#pragma unroll
      for (int t = 0; t < kTilesPerStep; ++t) {
        if constexpr (Cfg::mfma) {
          const float4 v = *(const float4*)(nbuf + buf * kStepRefs + t * 16 + 4 * kq);
          acc[t][0] = v.x;
          acc[t][1] = v.y;
          acc[t][2] = v.z;
          acc[t][3] = v.w;
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[t][i] = 0.f;
        }
      }
    }

    // ---- distance tiles on this chunk
    const int cwc = min(p.cw, p.dp - c * p.cw);
    if (p.nchunk > 1) load_q(c);
    if constexpr (Cfg::mfma && !Cfg::half16) {
#pragma unroll
      for (int g = 0; g < 16; ++g) {
        if (g * 16 < cwc) {
#pragma unroll
          for (int t = 0; t < kTilesPerStep; ++t) {
            const float4 a = *(const float4*)(rt + ((t * 16 + col) * p.rstride + g * 16 + 4 * kq) * ES);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, qf[g].x, acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, qf[g].y, acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, qf[g].z, acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, qf[g].w, acc[t], 0, 0, 0);
          }
        }
      }
    } else if constexpr (Cfg::mfma) {
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        if (s * 32 < cwc) {
#pragma unroll
          for (int t = 0; t < kTilesPerStep; ++t) {
            const uint4 a = *(const uint4*)(rt + ((t * 16 + col) * p.rstride + s * 32 + 8 * kq) * ES);
            if constexpr (KIND == TILE_L2_BF16)
              acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                               __builtin_bit_cast(bf16x8, qh[s]), acc[t], 0, 0, 0);
            else
              acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                              __builtin_bit_cast(f16x8, qh[s]), acc[t], 0, 0, 0);
          }
        }
      }
    } else {
      // vector ALU: lane (query col, group kq) accumulates its 16 rows over
      // the chunk's dims; every lane of a 16-lane group reads the same
      // reference row (an LDS broadcast).
      const float* qp = (const float*)p.Q + qsafe * (int64_t)p.ldq + c * p.cw;
      const unsigned char* rbase = rt + (4 * kq) * p.rstride * ES;
      for (int t4 = 0; t4 < cwc; t4 += 4) {
        const float4 qv = *(const float4*)(qp + t4);
#pragma unroll
        for (int t = 0; t < kTilesPerStep; ++t) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float4 rv = *(const float4*)(rbase + ((t * 16 + i) * p.rstride + t4) * ES);
            const float a0 = fabsf(qv.x - rv.x), a1 = fabsf(qv.y - rv.y);
            const float a2 = fabsf(qv.z - rv.z), a3 = fabsf(qv.w - rv.w);
            if constexpr (KIND == TILE_L1_F32)
              acc[t][i] = (((acc[t][i] + a0) + a1) + a2) + a3;
            else
              acc[t][i] = fmaxf(fmaxf(acc[t][i], fmaxf(a0, a1)), fmaxf(a2, a3));
          }
        }
      }
    }

    // ---- selection once the tiles have seen every chunk
    if (c == p.nchunk - 1) {
      const int64_t tb = s0 + (int64_t)tile * kStepRefs;
      const int rowlim = (int)min((int64_t)kStepRefs, s1 - tb) - 4 * kq;  // row 16t+4kq+i valid iff 16t+i < rowlim
      float mn = __builtin_huge_valf();
#pragma unroll
      for (int t = 0; t < kTilesPerStep; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) mn = fminf(mn, acc[t][i]);
      if (ballot(mn <= thr)) {
#pragma unroll
        for (int t = 0; t < kTilesPerStep; ++t) {
          uint32_t mask = 0;
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (acc[t][i] <= thr && t * 16 + i < rowlim) mask |= 1u << i;
          const int cnt = __popc(mask);
          if (!ballot(cnt != 0)) continue;
          int base = 0;
          if (cnt) base = atomicAdd(&counts[ql], cnt);
          uint64_t* dst = bufs + (size_t)ql * cb + base;
          const uint32_t rref = (uint32_t)(tb + t * 16 + 4 * kq);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (mask & (1u << i)) {
              *dst = make_key(acc[t][i], rref + (uint32_t)i);
              ++dst;
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
          uint64_t needm = ballot(kq == 0 && counts[ql] > cb - kTileRefs);
          if (needm) {
            while (needm) {
              const int j = __builtin_ctzll(needm);
              needm &= needm - 1;
              const int qs = wave * kQueriesPerWave + j;
              wave_merge(lists + (size_t)qs * kc, bufs + (size_t)qs * cb, lens + qs, counts + qs, kc, lane);
            }
            if (lens[ql] == kc) thr = mono_value((uint32_t)(lists[(size_t)ql * kc + kc - 1] >> 32));
          }
        }
      }
    }

    if (step + 1 < nsteps) store_stage(buf ^ 1);
    __syncthreads();
  }

  // ---- flush the buffers and write this slice's sorted lists
  {
    uint64_t needm = ballot(kq == 0 && counts[ql] > 0);
    while (needm) {
      const int j = __builtin_ctzll(needm);
      needm &= needm - 1;
      const int qs = wave * kQueriesPerWave + j;
      wave_merge(lists + (size_t)qs * kc, bufs + (size_t)qs * cb, lens + qs, counts + qs, kc, lane);
    }
  }
  const int tot = kQueriesPerWave * kc;
  for (int e = lane; e < tot; e += 64) {
    const int j = e / kc, pos = e - j * kc;
    const int qs = wave * kQueriesPerWave + j;
    const int64_t qg = q0 + qs;
    if (qg < p.n) {
      const uint64_t key = pos < lens[qs] ? lists[(size_t)qs * kc + pos] : kEmptyKey;
      p.part[(qg * p.P + blockIdx.y) * kc + pos] = key;
    }
  }
}

size_t fused_lds_bytes(int kind, int waves, int kc, int cb, int cw) {
  const int es = (kind == TILE_L2_BF16 || kind == TILE_L2_F16) ? 2 : 4;
  const int pad = 16 / es;
  const size_t nq = (size_t)waves * kQueriesPerWave;
  return nq * (size_t)(kc + cb) * 8 + nq * 8 + 2 * kStepRefs * 4 + 2 * (size_t)kStepRefs * (cw + pad) * es;
}

template <int KIND>
static hipError_t launch_fused_t(const FusedParams& p, hipStream_t stream) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)fused_select_kernel<KIND>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const size_t lds = fused_lds_bytes(KIND, p.waves, p.kc, p.cb, p.cw);
  const int nq = p.waves * kQueriesPerWave;
  dim3 grid((unsigned)((p.n + nq - 1) / nq), (unsigned)p.P);
  dim3 block(p.waves * kWaveSize);
  hipLaunchKernelGGL(fused_select_kernel<KIND>, grid, block, lds, stream, p);
  return hipGetLastError();
}

hipError_t launch_fused(int kind, const FusedParams& p, hipStream_t stream) {
  switch (kind) {
    case TILE_L2_F32: return launch_fused_t<TILE_L2_F32>(p, stream);
    case TILE_L2_BF16: return launch_fused_t<TILE_L2_BF16>(p, stream);
    case TILE_L2_F16: return launch_fused_t<TILE_L2_F16>(p, stream);
    case TILE_L1_F32: return launch_fused_t<TILE_L1_F32>(p, stream);
    case TILE_LINF_F32: return launch_fused_t<TILE_LINF_F32>(p, stream);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------ merge + exact re-rank + output
//
// One wave per query.  (1) The P sorted per-slice lists are merged by rank:
// the key at position i of list p lands at i + sum over the other lists of
// the number of their keys below it; the first k' are kept.  (2) Each kept
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

__global__ __launch_bounds__(256) void finalize_kernel(FinalParams p) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t q = (int64_t)blockIdx.x * kFinalWaves + wave;
  const int T = p.P * p.kc;
  // per-wave region: keys[T] | lens[P] | cand[kprime] | cdist[kprime]
  const size_t wave_bytes = (((size_t)T * 8 + (size_t)p.P * 4 + (size_t)p.kprime * 8) + 15) & ~(size_t)15;
  unsigned char* base = smem + wave * wave_bytes;
  uint64_t* keys = (uint64_t*)base;
  int* lens = (int*)(keys + T);
  uint32_t* cand = (uint32_t*)(lens + p.P);
  float* cdist = (float*)(cand + p.kprime);
  if (q >= p.n) return;

  const uint64_t* src = p.part + q * (int64_t)T;
  for (int e = lane; e < T; e += 64) keys[e] = src[e];
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  for (int pl = lane; pl < p.P; pl += 64) {
    const uint64_t* L = keys + pl * p.kc;
    int lo = 0, hi = p.kc;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (L[mid] != kEmptyKey) lo = mid + 1; else hi = mid;
    }
    lens[pl] = lo;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();

  int nvalid = 0;
  for (int pl = 0; pl < p.P; ++pl) nvalid += lens[pl];
  const int nc = min(p.kprime, nvalid);

  for (int e = lane; e < T; e += 64) {
    const int pl = e / p.kc, i = e - pl * p.kc;
    if (i >= lens[pl] || i >= p.kprime) continue;
    const uint64_t x = keys[e];
    int rank = i;
    for (int o = 0; o < p.P && rank < p.kprime; ++o) {
      if (o == pl) continue;
      const uint64_t* L = keys + o * p.kc;
      int lo = 0, hi = lens[o];
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (L[mid] < x) lo = mid + 1; else hi = mid;
      }
      rank += lo;
    }
    if (rank < p.kprime) cand[rank] = (uint32_t)x;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();

  const float* qrow = p.Q + q * (int64_t)p.ldq;
  for (int j = lane; j < nc; j += 64) {
    const uint32_t r = cand[j];
    cdist[j] = r < (uint64_t)p.m ? exact_distance(qrow, p.Rm, p.rm_type, (int64_t)r * p.ldr, p.d, p.metric)
                                 : __builtin_huge_valf();
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
    if (rank < p.k) {
      p.dist[q * p.k + rank] = p.metric == 0 ? sqrtf(dj) : dj;
      p.idx[q * p.k + rank] = (int32_t)rj;
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
  if (p.n <= 0) return hipSuccess;
  const int T = p.P * p.kc;
  const size_t wave_bytes = (((size_t)T * 8 + (size_t)p.P * 4 + (size_t)p.kprime * 8) + 15) & ~(size_t)15;
  dim3 grid((unsigned)((p.n + kFinalWaves - 1) / kFinalWaves)), block(kFinalWaves * kWaveSize);
  hipLaunchKernelGGL(finalize_kernel, grid, block, wave_bytes * kFinalWaves, stream, p);
  return hipGetLastError();
}

}  // namespace knn
