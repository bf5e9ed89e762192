// knn_fused.h -- the fused distance-tile + per-query top-k' selection kernel.
//
// The brute force of Section 2.1 of the paper computes every query-reference
// distance, sorts each query's distances and keeps the k smallest.  Here the
// two steps are fused: a workgroup scores a block of queries against a slice
// of references and keeps, per query, the k' best candidates under the
// total order (score, reference index).  The score matrix never leaves the
// compute unit; the finalize kernel (knn_kernels.hip) merges the per-slice
// lists and re-ranks the kept candidates exactly.
//
// Euclidean scores use s(q, r) = |r|^2 / 2 - q.r, which orders references as
// |q - r|^2 does for a fixed query (they differ by |q|^2 / 2 and a factor 2).
// The cross term is a dense contraction on the matrix cores
// (v_mfma_f32_16x16x4_f32, or v_mfma_f32_16x16x32_{bf16,f16}) with float32
// accumulation, the norm term preloaded into the accumulator.  Manhattan and
// infinity-norm distances are not contractions and run on the vector ALUs in
// float32, in the same lane layout.
//
// Geometry.  A workgroup has `waves` waves (up to 8: two per SIMD); wave w
// owns 16 queries and their selection state.  A step scores 64 references
// (four 16x16 tiles) against each wave's 16 queries.  In the 16x16 MFMA
// output layout lane l holds column l % 16 (its query) and rows
// 4*(l/16) + i, i = 0..3, of each tile.  Reference tiles are copied from
// global memory straight into LDS (global_load_lds_dwordx4), double
// buffered, one barrier per step; 16-byte slots of a staged row are XOR
// swizzled by the row index so that the operand reads of 8 consecutive rows
// hit distinct banks.
//
// Selection per query: a sorted list of the kc best keys so far and a buffer
// of unsorted candidates, both in LDS.  The buffer is split into four
// segments of `sub` keys, one per lane of the query, so that a lane appends
// to its own segment with a count kept in a register.  A score enters the
// buffer only if it is <= the list's kc-th score (the threshold; +inf until
// the list is full).  A query's buffer is merged into its list (by the whole
// wave) only when one of its lanes' survivors of the current step would
// overflow that lane's segment; the merge also tightens the threshold.
// Scores of rows past the end of the slice are set to NaN, which no
// comparison accepts.
#pragma once

#include "knn_device.h"

namespace knn {

template <int KIND>
struct TileCfg {
  static constexpr bool mfma = KIND <= TILE_L2_F16;
  static constexpr bool half16 = KIND == TILE_L2_BF16 || KIND == TILE_L2_F16;
  static constexpr int es = half16 ? 2 : 4;      // element size in bytes
  static constexpr int group = half16 ? 32 : 16;  // dims per k group
};

// SMALL: every instance of the launch has k' <= 64 and the buffer holds 64
// keys (16 per lane), so every merge is the register bitonic merge and the
// rank-merge code is not compiled in.
template <int KIND, int NG, bool SMALL>
__global__ __launch_bounds__(512) void fused_kernel(FusedParams p) {
  using Cfg = TileCfg<KIND>;
  constexpr int ES = Cfg::es, G = Cfg::group;
  constexpr int CW = NG * G;            // dims per chunk
  constexpr int VPR = CW * ES / 16;     // 16-byte slots per staged row (a multiple of 4)
  constexpr int TILE_BYTES = kStepRefs * VPR * 16;
  // slot swizzle: 3 bits where the row has 8 or more slot groups (MFMA
  // operand reads of 8 consecutive rows), 2 bits otherwise and for the
  // vector-ALU kinds (whose reads are 16-lane broadcasts)
  constexpr int SWZ = (Cfg::mfma && VPR % 8 == 0) ? 7 : 3;
  extern __shared__ __align__(16) unsigned char smem[];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, col = lane & 15, kq = lane >> 4;
  const int W = p.waves;
  const int nq = W * kQueriesPerWave;
  // this workgroup's instance, query block and reference slice
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
  const int64_t q0 = (int64_t)qblock * nq;
  const int ql = wave * kQueriesPerWave + col;
  const int64_t qrow = q0 + ql;
  const int64_t qsafe = qrow < in.n ? qrow : in.n - 1;
  const int64_t s0 = (int64_t)slice * in.slice_len;
  const int64_t s1 = min(in.m, s0 + in.slice_len);
  const int ntiles = (int)((s1 - s0 + kStepRefs - 1) / kStepRefs);
  const int kc = in.kc, cb = p.cb;

  // per-query buffer: 4 segments of `sub` keys, each padded by one key and
  // the query's block by one more, so that lanes appending in parallel
  // spread over the LDS banks
  const int sub = p.cb / 4;
  const int seg_stride = sub + 1;
  const int q_stride = 4 * seg_stride + 1;
  uint64_t* lists = (uint64_t*)smem;
  uint64_t* bufs = lists + (size_t)nq * kc;
  int* lens = (int*)(bufs + (size_t)nq * q_stride);
  // The double-buffered tiles (and norms) are separate static arrays and the
  // step loop below is unrolled by two, so that every read of one buffer is
  // provably disjoint from the asynchronous copy into the other: the copy's
  // completion is then awaited only at the end of the step.
  __shared__ __align__(16) unsigned char tile0[TILE_BYTES], tile1[TILE_BYTES];
  __shared__ __align__(16) float norm0[kStepRefs], norm1[kStepRefs];

  for (int i = tid; i < nq; i += blockDim.x) lens[i] = 0;

  // ---- query operands of the MFMA kinds in registers, one chunk of dims
  // at a time: lane group kq supplies the k slots; float32 group g (four
  // MFMAs) covers dims 16g..16g+15 with kq holding 16g+4kq..+3, a 16-bit
  // MFMA s covers 32s..32s+31 with kq holding 32s+8kq..+7.  The staged
  // reference tile is read with the same mapping, so every product pairs
  // the same dimension.  Queries are negated: the MFMA adds -q.r to the
  // preloaded |r|^2 / 2.  Dims past the chunk's valid groups are zero.  (The
  // vector-ALU kinds read their query values from memory, one group ahead.)
  float4 qf[NG];
  uint4 qh[NG];
  auto load_q = [&](int c) __attribute__((always_inline)) {
    const int ngv = min(NG, (in.dp - c * CW) / G);
    if constexpr (Cfg::mfma && !Cfg::half16) {
      const float* qp = (const float*)in.Q + qsafe * (int64_t)in.ldq + c * CW;
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        qf[g] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (g < ngv) {
          const float4 v = *(const float4*)(qp + g * 16 + 4 * kq);
          qf[g] = make_float4(-v.x, -v.y, -v.z, -v.w);
        }
      }
    } else if constexpr (Cfg::mfma) {
      const uint16_t* qp = (const uint16_t*)in.Q + qsafe * (int64_t)in.ldq + c * CW;
#pragma unroll
      for (int s = 0; s < NG; ++s) {
        qh[s] = make_uint4(0u, 0u, 0u, 0u);
        if (s < ngv) {
          const uint4 v = *(const uint4*)(qp + s * 32 + 8 * kq);
          qh[s] = make_uint4(v.x ^ 0x80008000u, v.y ^ 0x80008000u, v.z ^ 0x80008000u, v.w ^ 0x80008000u);
        }
      }
    }
  };
  if (in.nchunk == 1) load_q(0);

  // ---- staging: slot (row, logical chunk j) of a tile lives at
  // row * VPR + (j ^ (row & SWZ)); a wave instruction fills 64 consecutive
  // slots.  Rows past the slice end and chunks past the row's valid dims
  // load clamped (valid) addresses; their scores are masked, and their
  // products meet zero query operands.
  auto stage = [&](int stile, int sc, unsigned char* dst, float* ndst) __attribute__((always_inline)) {
    const int64_t rb = s0 + (int64_t)stile * kStepRefs;
    const int vvalid = min(VPR, (in.dp - sc * CW) * ES / 16);
    const int rlast = (int)min((int64_t)kStepRefs, s1 - rb) - 1;  // last valid row of the tile
    const unsigned char* gR = (const unsigned char*)in.R + (rb * in.ldr + (int64_t)sc * CW) * ES;
    const int rowbytes = in.ldr * ES;
    for (int i = wave; i < VPR; i += W) {
      const int s = 64 * i + lane;
      const int row = s / VPR, jp = s - row * VPR;
      const int j = min(jp ^ (row & SWZ), vvalid - 1);
      __builtin_amdgcn_global_load_lds(gR + min(row, rlast) * rowbytes + j * 16, (lds_void*)(dst + i * 1024), 16, 0,
                                       0);
    }
    if constexpr (Cfg::mfma) {
      if (wave == W - 1)
        __builtin_amdgcn_global_load_lds(in.rhalf + rb + min(lane, rlast), (lds_void*)ndst, 4, 0, 0);
    }
  };

  const int nsteps = ntiles * in.nchunk;
  float thr = __builtin_huge_valf();
  int lcnt = 0;  // keys in this lane's buffer segment
  uint64_t* myseg = bufs + (size_t)ql * q_stride + kq * seg_stride;
  f32x4 acc[kTilesPerStep];

  // merge the buffers of the wave's queries flagged in `qmask` (bit j =
  // query j of the wave) into their lists, then refresh this lane's count
  // and threshold if its query was merged
  auto merge_queries = [&](uint32_t qmask) __attribute__((always_inline)) {
    wave_sync();
    uint32_t todo = qmask;
    while (todo) {
      const int j = __builtin_ctz(todo);
      todo &= todo - 1;
      const int qs = wave * kQueriesPerWave + j;
      Segs sg;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        sg.seg[k] = bufs + (size_t)qs * q_stride + k * seg_stride;
        sg.cnt[k] = __builtin_amdgcn_readlane(lcnt, j + 16 * k);
      }
      int nl;
      if constexpr (SMALL)
        nl = wave_merge64(lists + (size_t)qs * kc, sg, lens[qs], kc, lane);
      else
        nl = wave_merge(lists + (size_t)qs * kc, sg, lens[qs], kc, sub, lane);
      if (lane == 0) lens[qs] = nl;
      wave_sync();
    }
    if ((qmask >> col) & 1) {
      lcnt = 0;
      if (lens[ql] == kc) thr = mono_value((uint32_t)(lists[(size_t)ql * kc + kc - 1] >> 32));
    }
  };
  auto query_bits = [](uint64_t lanes) __attribute__((always_inline)) {  // lanes col + 16k -> bit col
    return (uint32_t)((lanes | (lanes >> 16) | (lanes >> 32) | (lanes >> 48)) & 0xffffu);
  };

  if (nsteps > 0) stage(0, 0, tile0, norm0);
  wait_vmem();
  __syncthreads();

  // ---- selection over the complete tile `tl` held in acc
  auto select_tile = [&](int tl) __attribute__((always_inline)) {
    const int64_t tb = s0 + (int64_t)tl * kStepRefs;
    if (tb + kStepRefs > s1) {  // last, partial step of the slice
      const int rowlim = (int)(s1 - tb);
#pragma unroll
      for (int t = 0; t < kTilesPerStep; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (t * 16 + 4 * kq + i >= rowlim) acc[t][i] = __builtin_nanf("");
    }
    float mn = fminf(fminf(acc[0][0], acc[0][1]), fminf(acc[0][2], acc[0][3]));
#pragma unroll
    for (int t = 1; t < kTilesPerStep; ++t)
      mn = fminf(mn, fminf(fminf(acc[t][0], acc[t][1]), fminf(acc[t][2], acc[t][3])));
    if (ballot(mn <= thr)) {
      int n = 0;
#pragma unroll
      for (int t = 0; t < kTilesPerStep; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) n += acc[t][i] <= thr ? 1 : 0;
      const uint32_t ovf = query_bits(ballot(lcnt + n > sub));
      if (ovf) merge_queries(ovf);  // segments that cannot take this step's survivors
      const uint32_t rref = (uint32_t)(tb + 4 * kq);
#pragma unroll
      for (int t = 0; t < kTilesPerStep; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (acc[t][i] <= thr) {
            myseg[lcnt] = make_key(acc[t][i], rref + (uint32_t)(t * 16 + i));
            ++lcnt;
          }
    }
  };

  int tile = 0, c = 0;
  // one step: stage the next chunk into (wt, nwr), score the chunk held in
  // (rt, nrd), select if the tile is complete, then wait for the copy and
  // synchronize
  auto run_step = [&](int step, const unsigned char* rt, const float* nrd, unsigned char* wt, float* nwr) __attribute__((always_inline)) {
    if (step + 1 < nsteps) {
      const bool wrap = c + 1 == in.nchunk;
      stage(wrap ? tile + 1 : tile, wrap ? 0 : c + 1, wt, nwr);
    }

    if (c == 0) {
#pragma unroll
      for (int t = 0; t < kTilesPerStep; ++t) {
        if constexpr (Cfg::mfma) {
          const float4 v = *(const float4*)(nrd + t * 16 + 4 * kq);
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
    if (in.nchunk > 1) load_q(c);
    if constexpr (Cfg::mfma) {
      const int sw = col & SWZ;  // swizzle of rows 16t + col
#pragma unroll
      for (int g = 0; g < NG; ++g) {
#pragma unroll
        for (int t = 0; t < kTilesPerStep; ++t) {
          const int slot = (t * 16 + col) * VPR + ((4 * g + kq) ^ sw);
          if constexpr (!Cfg::half16) {
            const float4 a = *(const float4*)(rt + slot * 16);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, qf[g].x, acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, qf[g].y, acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, qf[g].z, acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, qf[g].w, acc[t], 0, 0, 0);
          } else {
            const uint4 a = *(const uint4*)(rt + slot * 16);
            if constexpr (KIND == TILE_L2_BF16)
              acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                               __builtin_bit_cast(bf16x8, qh[g]), acc[t], 0, 0, 0);
            else
              acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                              __builtin_bit_cast(f16x8, qh[g]), acc[t], 0, 0, 0);
          }
        }
      }
    } else {
      // vector ALU: lane (query col, group kq) accumulates rows 16t+4kq+i over
      // the chunk's dims, 16 at a time; the 16 lanes of a group read the same
      // reference row (an LDS broadcast).  Row 16t+4kq+i has swizzle i & 3.
      const int ngv = min(NG, (in.dp - c * CW) / G);
      const float* qp = (const float*)in.Q + qsafe * (int64_t)in.ldq + c * CW;
      const unsigned char* rrow = rt + (4 * kq) * VPR * 16;
      // one group of 16 dims: query values qq[0..3], reference rows from LDS
      // The 64 reads of a group (4 dims of one of 16 rows each) go through
      // a ring of 8 registers, so that 8 are in flight while the vector ALU
      // works on earlier ones.
      auto group = [&](int g, const float4* qq) __attribute__((always_inline)) {
        const unsigned char* rg = rrow + g * 64;
        auto rd = [&](int u) __attribute__((always_inline)) {  // u = 16 jj + 4 t + i
          const int jj = u >> 4, t = (u >> 2) & 3, i = u & 3;
          return *(const float4*)(rg + ((t * 16 + i) * VPR + (jj ^ (i & 3))) * 16);
        };
        constexpr int DEPTH = 8;
        float4 ring[DEPTH];
#pragma unroll
        for (int u = 0; u < DEPTH; ++u) ring[u] = rd(u);
#pragma unroll
        for (int u = 0; u < 64; ++u) {
          const float4 rv = ring[u % DEPTH];
          if (u + DEPTH < 64) ring[u % DEPTH] = rd(u + DEPTH);
          const int jj = u >> 4, t = (u >> 2) & 3, i = u & 3;
          const float4 q4 = qq[jj];
          const float a0 = fabsf(q4.x - rv.x), a1 = fabsf(q4.y - rv.y);
          const float a2 = fabsf(q4.z - rv.z), a3 = fabsf(q4.w - rv.w);
          if constexpr (KIND == TILE_L1_F32)
            acc[t][i] = (((acc[t][i] + a0) + a1) + a2) + a3;
          else
            acc[t][i] = fmaxf(fmaxf(acc[t][i], fmaxf(a0, a1)), fmaxf(a2, a3));
        }
      };
      // groups in pairs, the query values of the next group loaded one group
      // ahead into the other register set (no copies between them)
      float4 qa[4], qb[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) qa[j] = *(const float4*)(qp + 4 * j);
#pragma unroll 1
      for (int g = 0; g < ngv; g += 2) {
        if (g + 1 < ngv) {
#pragma unroll
          for (int j = 0; j < 4; ++j) qb[j] = *(const float4*)(qp + (g + 1) * 16 + 4 * j);
        }
        group(g, qa);
        if (g + 1 < ngv) {
          if (g + 2 < ngv) {
#pragma unroll
            for (int j = 0; j < 4; ++j) qa[j] = *(const float4*)(qp + (g + 2) * 16 + 4 * j);
          }
          group(g + 1, qb);
        }
      }
    }

    // ---- selection once the tiles have seen every chunk
    if (c == in.nchunk - 1) select_tile(tile);

    wait_vmem();
    __syncthreads();
    if (++c == in.nchunk) {
      c = 0;
      ++tile;
    }
  };
  for (int step = 0; step < nsteps; step += 2) {
    run_step(step, tile0, norm0, tile1, norm1);
    if (step + 1 < nsteps) run_step(step + 1, tile1, norm1, tile0, norm0);
  }
  merge_queries(query_bits(ballot(lcnt > 0)));  // end of the slice: flush

  // ---- write this slice's sorted lists
  const int tot = kQueriesPerWave * kc;
  for (int e = lane; e < tot; e += 64) {
    const int j = e / kc, pos = e - j * kc;
    const int qs = wave * kQueriesPerWave + j;
    const int64_t qg = q0 + qs;
    if (qg < in.n) {
      const uint64_t key = pos < lens[qs] ? lists[(size_t)qs * kc + pos] : kEmptyKey;
      in.part[(qg * in.P + slice) * kc + pos] = key;
    }
  }
}

// LDS bytes of one fused workgroup: the dynamic selection state plus the
// static tile and norm buffers.
__host__ __device__ constexpr size_t fused_dyn_lds(int waves, int kc, int cb) {
  return (size_t)waves * kQueriesPerWave * ((size_t)(kc + cb + 5) * 8 + 4);
}
__host__ __device__ constexpr size_t fused_lds_size(int es, int waves, int kc, int cb, int cw) {
  return fused_dyn_lds(waves, kc, cb) + 2 * kStepRefs * 4 + 2 * (size_t)kStepRefs * cw * es;
}

template <int KIND, int NG, bool SMALL>
hipError_t launch_fused_one(const FusedParams& p, hipStream_t stream) {
  static bool attr_set = false;
  if (!attr_set) {
    hipFuncAttributes fa;
    hipError_t e = hipFuncGetAttributes(&fa, (const void*)fused_kernel<KIND, NG, SMALL>);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)fused_kernel<KIND, NG, SMALL>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            kLdsBytes - (int)fa.sharedSizeBytes);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const size_t lds = fused_dyn_lds(p.waves, p.kc_max, p.cb);
  const int nq = p.waves * kQueriesPerWave;
  if (p.items && p.nitems <= 0) return hipSuccess;
  dim3 grid = p.items ? dim3((unsigned)p.nitems) : dim3((unsigned)((p.one.n + nq - 1) / nq), (unsigned)p.one.P);
  dim3 block(p.waves * kWaveSize);
  hipLaunchKernelGGL((fused_kernel<KIND, NG, SMALL>), grid, block, lds, stream, p);
  return hipGetLastError();
}

// launch the instantiation whose chunk width matches p.ng (one of NGS)
template <int KIND, bool SMALL, int... NGS>
hipError_t dispatch_ng(const FusedParams& p, hipStream_t stream) {
  hipError_t r = hipErrorInvalidValue;
  (void)((p.ng == NGS ? (r = launch_fused_one<KIND, NGS, SMALL>(p, stream), true) : false) || ...);
  return r;
}

}  // namespace knn
