// knn_wide.h -- fused distance + per-query top-k' kernel for the
// Euclidean tiles with k' <= 64 and at most 128 dimensions, on 32x32 MFMA
// tiles: float32 operands (v_mfma_f32_32x32x2f32) or 16-bit operands
// (v_mfma_f32_32x32x16_{bf16,f16}), float32 accumulation.  The brute force
// of Section 2.1; the k' candidates are re-ranked exactly in float32 by the
// finalize kernel.
//
// It differs from the general kernel of knn_fused.h in three ways, all for
// matrix-core throughput:
//  * 32x32 MFMA tiles: a wave scores 32 queries (one output column each)
//    against 32 references per instruction, so every reference fragment read
//    from LDS feeds twice as many products as a 16x16 tile;
//  * the sorted k'-lists live in registers, one key per lane and one
//    register pair per query (64 registers for 32 queries); only the
//    candidate buffers stay in LDS, which leaves room for
//  * more reference tiles in flight: with 16-bit tiles (short steps) two
//    steps run between workgroup barriers, and the copies of the next two
//    are issued while they are scored (four tile buffers); float32 steps are
//    long enough for one step per barrier and one step of lookahead;
// and the two waves that share a SIMD run their scoring and selection
// phases in opposite order, so that one wave's selection overlaps the
// other's matrix instructions.
//
// Lane l of a wave owns query 32 * wave + l % 32 and, in each 32x32 output
// tile, the 16 rows 8 * (r / 4) + 4 * (l / 32) + r % 4 (r = 0..15); the two
// lanes of a query each keep a segment of candidate keys (20 with 16-bit
// tiles, 16 with float32 tiles, whose larger staged rows leave less LDS).
// Scores, keys and the (score, index) order are those of knn_fused.h.
#pragma once

#include "knn_device.h"

namespace knn {

typedef uint32_t u32x32 __attribute__((ext_vector_type(32)));

constexpr int kWideWaves = 8;
constexpr int kWideQueriesPerWave = 32;
constexpr int kWideQueriesWG = kWideWaves * kWideQueriesPerWave;  // queries per workgroup
static_assert(kWideQueriesWG == kWideQueries, "host and kernel agree on the query block");

// Minimum of three scores with v_min3_f32 as it stands.  The scores come from
// matrix instructions or are the quiet NaN that marks rows past the end of
// the slice, which the instruction passes over like fminf; fminf itself would
// first canonicalize every operand.
__device__ __forceinline__ float min3_raw(float a, float b, float c) {
  float r;
  asm("v_min3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// Geometry of one instantiation (KIND, NKG).
template <int KIND, int NKG>
struct WideGeom {
  static constexpr bool F32 = KIND == TILE_L2_F32;
  static constexpr int ES = F32 ? 4 : 2;                 // element bytes
  static constexpr int GRP = F32 ? 1 : 2;                // steps between barriers
  static constexpr int STAGES = 2 * GRP;                 // tile buffers: two groups
  static constexpr int SUB = F32 ? 16 : 20;              // keys per lane segment
  static constexpr int SEG = SUB + 1;                    // padded against bank conflicts
  static constexpr int VPR = NKG * 16 * ES / 16;         // 16-byte slots of a row's data
  static constexpr int RS = VPR + 1;                     // slots per staged row: data + one pad slot
  static constexpr int TILE_BYTES = kStepRefs * RS * 16; // 64 references
  static constexpr int TILES_LDS = STAGES * TILE_BYTES;
  static constexpr int NORMS_LDS = STAGES * kStepRefs;   // floats
  static constexpr int BUFS_LDS = kWideWaves * 64 * SEG; // keys
  static_assert(TILES_LDS + NORMS_LDS * 4 + (size_t)BUFS_LDS * 8 <= kWideLdsBytes, "LDS of one workgroup");
};

// One work item of the kernel: the queries of block `qblock` of instance
// `in` against reference slice `slice`, with lists of up to 64 * LK keys
// (LK = 1: k' <= 64; LK = 2: k' <= 128, 16-bit tiles only).  The LDS arrays
// are the caller's (sized by WideGeom); the item leaves no state behind in
// them that a later item reads.
// NKG: 16-dimension k groups of the padded dimension (dp = 16 * NKG; even
// for the 16-bit kinds, whose rows are padded to 32).
template <int KIND, int NKG, int LK, int SHARE>
__device__ __forceinline__ void wide_item(const FusedInst& in, int qblock, int slice, unsigned char* tiles,
                                          float* norms, uint64_t* bufs) {
  static_assert(KIND == TILE_L2_F32 || KIND == TILE_L2_BF16 || KIND == TILE_L2_F16, "Euclidean tiles only");
  using G = WideGeom<KIND, NKG>;
  constexpr bool F32 = G::F32;
  static_assert(NKG >= 1 && NKG <= 8 && (F32 || NKG % 2 == 0), "dp <= 128");
  static_assert(LK == 1 || (LK == 2 && !F32), "two keys per lane for the 16-bit kinds only");
  constexpr int ES = G::ES;
  constexpr int STAGES = G::STAGES;
  constexpr int SUB = G::SUB;
  constexpr int SEG = G::SEG;
  constexpr int VPR = G::VPR;
  constexpr int NU = VPR / 2;                        // slot pairs: a lane half reads one slot of each
  constexpr int RS = G::RS;
  constexpr int TILE_BYTES = G::TILE_BYTES;
  constexpr int NI = RS;                             // wave-wide copy instructions per tile
  constexpr int PER_WAVE = (NI + kWideWaves - 1) / kWideWaves;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, c = lane & 31, h = lane >> 5;
  const int64_t q0 = (int64_t)qblock * kWideQueriesWG + wave * kWideQueriesPerWave;
  const int64_t qrow = q0 + c;
  const int64_t qsafe = qrow < in.n ? qrow : in.n - 1;
  const int64_t s0 = (int64_t)slice * in.slice_len;
  const int64_t s1 = min(in.m, s0 + in.slice_len);
  const int nsteps = (int)((s1 - s0 + kStepRefs - 1) / kStepRefs);
  const int kc = in.kc;

  // ---- query operands, negated so that the MFMA adds -q.r to |r|^2 / 2.
  // Slot pair u of a row holds 16 bytes for each lane half h: 16-bit dims
  // 16u + 8h..+7 (one 32x32x16 instruction), or float32 dims 8u + 4h..+3
  // (four 32x32x2 instructions, one per dim of the lane's run).  The staged
  // reference rows are read with the same mapping.
  uint4 qv[NU];
  {
    const unsigned char* qp = (const unsigned char*)in.Q + (qsafe * (int64_t)in.ldq) * ES + 16 * h;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const uint4 v = *(const uint4*)(qp + 32 * u);
      const uint32_t sgn = F32 ? 0x80000000u : 0x80008000u;
      qv[u] = make_uint4(v.x ^ sgn, v.y ^ sgn, v.z ^ sgn, v.w ^ sgn);
    }
  }

  // ---- asynchronous global-to-LDS copies, written as assembly so that the
  // compiler's wait tracking (which cannot always tell the three tile buffers
  // apart) does not add full waits before reads of the other buffers.  They
  // are ordered by the explicit vmcnt waits and the barrier (whose memory
  // clobber keeps every LDS access on its side).  Each copy takes a
  // wave-uniform 64-bit base in scalar registers and a 32-bit per-lane byte
  // offset; M0 carries the LDS address of the wave's 64 destination slots
  // and is restored afterwards.
  auto copy16 = [](const void* gbase, uint32_t voff, uint32_t lds) __attribute__((always_inline)) {
    uint32_t save;
    asm volatile(
        "s_mov_b32 %0, m0\n\ts_mov_b32 m0, %3\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, %2\n\ts_mov_b32 m0, %0"
        : "=&s"(save)
        : "v"(voff), "s"(gbase), "s"(lds));
  };
  auto copy4 = [](const void* gbase, uint32_t voff, uint32_t lds) __attribute__((always_inline)) {
    uint32_t save;
    asm volatile(
        "s_mov_b32 %0, m0\n\ts_mov_b32 m0, %3\n\ts_nop 0\n\tglobal_load_lds_dword %1, %2\n\ts_mov_b32 m0, %0"
        : "=&s"(save)
        : "v"(voff), "s"(gbase), "s"(lds));
  };
  auto uniform_ptr = [](const void* ptr) __attribute__((always_inline)) {
    const uint64_t v = (uint64_t)(uintptr_t)ptr;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (const unsigned char*)(uintptr_t)(((uint64_t)hi << 32) | lo);
  };

  // ---- staging of a step into tile buffer `b`: copy instruction i fills
  // slots 64i..64i+63; slot j of row r lives at r * RS + j, the pad slot
  // (j = VPR) repeating the row's last data slot.  With a row stride of an
  // odd number of 16-byte slots the operand reads of 8 consecutive rows hit
  // distinct banks, and every (tile, k group) read is a fixed offset from
  // one per-lane address.  Every wave issues the same number of copies
  // (instructions past NI repeat earlier ones, and every wave copies the
  // norms: identical bytes to identical places), so one immediate vmcnt
  // serves all waves.  The per-lane row, byte offset and LDS slot of each
  // copy are the same for every step; only the last, partial step of a
  // slice clamps its rows to the slice.
  const int rowbytes = in.ldr * ES;
  int crow[PER_WAVE];
  uint32_t cjo[PER_WAVE], coff[PER_WAVE], clds[PER_WAVE];
#pragma unroll
  for (int u = 0; u < PER_WAVE; ++u) {
    const int i = (wave + kWideWaves * u) % NI;
    const int sl = 64 * i + lane;
    const int row = sl / RS, jp = sl - row * RS;
    crow[u] = row;
    cjo[u] = (uint32_t)min(jp, VPR - 1) * 16;
    coff[u] = (uint32_t)(row * rowbytes) + cjo[u];
    clds[u] = __builtin_amdgcn_readfirstlane((uint32_t)i * 1024);
  }
  const uint32_t tiles_lds = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_void*)tiles);
  const uint32_t norms_lds = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_void*)norms);
  auto stage = [&](int st, int b) __attribute__((always_inline)) {
    const int64_t rb = s0 + (int64_t)st * kStepRefs;
    const unsigned char* gR = uniform_ptr((const unsigned char*)in.R + rb * (int64_t)rowbytes);
    const unsigned char* gN = uniform_ptr(in.rhalf + rb);
    const uint32_t tl = tiles_lds + (uint32_t)(b * TILE_BYTES), nl = norms_lds + (uint32_t)(b * kStepRefs * 4);
    if (rb + kStepRefs <= s1) {
#pragma unroll
      for (int u = 0; u < PER_WAVE; ++u) copy16(gR, coff[u], tl + clds[u]);
      copy4(gN, (uint32_t)lane * 4, nl);
    } else {  // the last, partial step: rows past the slice repeat its last row
      const int rlast = (int)(s1 - rb) - 1;
#pragma unroll
      for (int u = 0; u < PER_WAVE; ++u) copy16(gR, (uint32_t)(min(crow[u], rlast) * rowbytes) + cjo[u], tl + clds[u]);
      copy4(gN, (uint32_t)min(lane, rlast) * 4, nl);
    }
  };

  // ---- selection state
  u32x32 Llo, Lhi;    // list key e of query j: lane e of register pair j
  u32x32 Llo2, Lhi2;  // LK = 2: list key 64 + e of query j
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    Llo[j] = 0xffffffffu;
    Lhi[j] = 0xffffffffu;
    if constexpr (LK == 2) {
      Llo2[j] = 0xffffffffu;
      Lhi2[j] = 0xffffffffu;
    }
  }
  // A lane whose row lies past n admits nothing (in the kernels with rank
  // slots, which serve the small searches; the others keep the plain start).
  float thr = SHARE == 2 && qrow >= in.n ? -__builtin_huge_valf() : __builtin_huge_valf();
  int lcnt = 0;
  uint64_t* myseg = bufs + (size_t)(wave * 64 + lane) * SEG;
  const uint64_t* wbufs = bufs + (size_t)wave * 64 * SEG;

  // The rank bound of this lane's query: for each of rank_G groups of
  // rank_gs consecutive slices, the largest of their rank slots (the two
  // lane halves read half a group each), and the smallest of those maxima.
  // Loads go out eight at a time (four with two-key lists) before any is
  // waited for.
  auto rank_bound = [&]() __attribute__((always_inline)) -> uint32_t {
    constexpr int RL = LK == 1 ? 8 : 4;
    const int gs = in.rank_gs, half = (gs + 1) >> 1, cnt = h ? gs - half : half;
    const uint32_t* sl = in.tshare + in.n * (int64_t)(1 + h * half) + qsafe;  // slot of slice h * half
    uint32_t best = 0xffffffffu;
    for (int g = 0; g < in.rank_G; ++g) {
      uint32_t mx = 0;
      for (int i0 = 0; i0 < cnt; i0 += RL) {
        uint32_t v[RL];
#pragma unroll
        for (int i = 0; i < RL; ++i) {
          v[i] = 0;
          if (i0 + i < cnt)
            v[i] = __hip_atomic_load(sl + (int64_t)(g * gs + i0 + i) * in.n, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
        }
#pragma unroll
        for (int i = 0; i < RL; ++i) mx = max(mx, v[i]);
      }
      mx = max(mx, xor_lane32<32>(mx, lane));
      best = min(best, mx);
    }
    return qrow < in.n ? best : 0xffffffffu;
  };

  // merge the buffers of the queries in `qm` (bit j = query j of the wave)
  // into their lists; refresh the threshold and count of their two lanes
  auto merge_queries = [&](uint32_t qm) __attribute__((always_inline)) {
    wave_sync();
    while (qm) {
      const int j = __builtin_ctz(qm);
      qm &= qm - 1;
      const int cnt0 = __builtin_amdgcn_readlane(lcnt, j);
      const int cnt1 = __builtin_amdgcn_readlane(lcnt, j + 32);
      // the buffered keys of the query's two lanes (float bits of the score,
      // mapped here), sorted descending over the wave
      const uint64_t* sp0 = wbufs + (size_t)j * SEG;
      const uint64_t* sp1 = wbufs + (size_t)(j + 32) * SEG;
      auto key_at = [](const uint64_t* p, int i) __attribute__((always_inline)) {
        const uint64_t r = p[i];
        return ((uint64_t)mono_code(__uint_as_float((uint32_t)(r >> 32))) << 32) | (uint32_t)r;
      };
      uint64_t x = kEmptyKey;
      const int e = lane & 31;
      if (e < (h ? cnt1 : cnt0)) x = key_at(h ? sp1 : sp0, e);
      x = bitonic_sort64(x, lane, true);
      const uint64_t l = ((uint64_t)Lhi[j] << 32) | Llo[j];
      uint64_t m = l < x ? l : x;
      uint32_t kth;
      if constexpr (LK == 1) {
        m = bitonic_clean64(m, lane);
        kth = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(m >> 32), kc - 1);
      } else {
        // list = A (keys 0..63) then B (64..127), both ascending; x descending.
        // min(A, x) holds the 64 smallest of A and x, max(A, x) the rest,
        // both bitonic.  Every key of min(A, x) is at most max(A) <= min(B),
        // so the new list is sort(min(A, x)) followed by the 64 smallest of
        // max(A, x) and B.
        uint64_t hi = l < x ? x : l;
        m = bitonic_clean64(m, lane);
        hi = bitonic_clean64_desc(hi, lane);
        const uint64_t b = ((uint64_t)Lhi2[j] << 32) | Llo2[j];
        uint64_t m2 = b < hi ? b : hi;
        m2 = bitonic_clean64(m2, lane);
        Llo2[j] = (uint32_t)m2;
        Lhi2[j] = (uint32_t)(m2 >> 32);
        kth = kc > 64 ? (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(m2 >> 32), kc - 65)
                      : (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(m >> 32), kc - 1);
      }
      Llo[j] = (uint32_t)m;
      Lhi[j] = (uint32_t)(m >> 32);
      // publish the slice's kc-th best to the query's other slices (an atomic
      // without return: nothing waits for it), and its rank_r-th best to its
      // rank slot (a store that bypasses the XCD's L2, as the loads that read it)
      if constexpr (SHARE >= 1)
        if (in.tshare && kth != 0xffffffffu && lane == 0 && q0 + j < in.n) atomicMin(in.tshare + q0 + j, kth);
      if constexpr (SHARE == 2) {
        if (in.tshare && in.rank_r > 0) {
          const uint32_t rv = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(m >> 32),
                                                                  __builtin_amdgcn_readfirstlane(in.rank_r - 1));
          if (rv != 0xffffffffu && lane == 0 && q0 + j < in.n)
            __hip_atomic_store(in.tshare + in.n * (1 + (int64_t)slice) + q0 + j, rv, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      if (c == j) {
        lcnt = 0;
        if (kth != 0xffffffffu) thr = fminf(thr, mono_value(kth));
      }
    }
    wave_sync();
  };

  f32x16 acc[2];

  // ---- scoring phase: the 64 references of step `st` against the wave's
  // 32 queries, |r|^2 / 2 preloaded into the accumulators
  auto score = [&](int b) __attribute__((always_inline)) {
    // a wave issuing matrix instructions goes first on its SIMD, so the other
    // wave's selection fills the gaps rather than delaying them
    __builtin_amdgcn_s_setprio(2);
    const unsigned char* rt = tiles + b * TILE_BYTES;
    const float* nrd = norms + b * kStepRefs;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const float4 v = *(const float4*)(nrd + 32 * t + 8 * jj + 4 * h);
        acc[t][4 * jj + 0] = v.x;
        acc[t][4 * jj + 1] = v.y;
        acc[t][4 * jj + 2] = v.z;
        acc[t][4 * jj + 3] = v.w;
      }
    }
    const unsigned char* ra = rt + (c * RS + h) * 16;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const uint4 a = *(const uint4*)(ra + (32 * t * RS + 2 * u) * 16);
        if constexpr (F32) {
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.x), __uint_as_float(qv[u].x), acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.y), __uint_as_float(qv[u].y), acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.z), __uint_as_float(qv[u].z), acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.w), __uint_as_float(qv[u].w), acc[t], 0, 0, 0);
        } else if constexpr (KIND == TILE_L2_BF16) {
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                           __builtin_bit_cast(bf16x8, qv[u]), acc[t], 0, 0, 0);
        } else {
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                          __builtin_bit_cast(f16x8, qv[u]), acc[t], 0, 0, 0);
        }
      }
    }
    // schedule: the eight norm reads and the first PF operand reads, then
    // the matrix instructions of one read per further read, so that PF reads
    // are in flight while the instructions run
    constexpr int NA = 2 * NU, PF = NA < 4 ? NA : 4, MPR = F32 ? 4 : 1;
    __builtin_amdgcn_sched_group_barrier(0x100, 8 + PF, 0);
#pragma unroll
    for (int i = 0; i < NA - PF; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, MPR, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, MPR * PF, 0);
    __builtin_amdgcn_s_setprio(0);
  };

  // ---- selection phase over the scores of step `st` (in acc).  The minima
  // of the tile's groups of 4 scores decide whether the tile, and then each
  // group, has a candidate anywhere in the wave; a group's candidates are
  // appended after the lanes whose segments cannot take them have had their
  // queries merged.
  auto select = [&](int st) __attribute__((always_inline)) {
    const int64_t tb = s0 + (int64_t)st * kStepRefs;
    if (tb + kStepRefs > s1) {  // last, partial step of the slice
      const int lim = (int)(s1 - tb) - 4 * h;  // rows of this lane: 32t + 8(r/4) + 4h + r%4
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          if (32 * t + 8 * (r >> 2) + (r & 3) >= lim) acc[t][r] = __builtin_nanf("");
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        float mq[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        mq[q] = min3_raw(min3_raw(acc[t][4 * q], acc[t][4 * q + 1], acc[t][4 * q + 2]), acc[t][4 * q + 3],
                         acc[t][4 * q + 3]);
      const float mn = min3_raw(min3_raw(mq[0], mq[1], mq[2]), mq[3], mq[3]);
      if (ballot(mn <= thr)) {
        const uint32_t rref = (uint32_t)(tb + 32 * t + 4 * h);
        // Per group of 4 scores with a candidate in the wave: a lane whose
        // buffer cannot take its passing scores has its query merged first
        // (so buffers fill to SUB keys before a merge), then branch-free
        // appends: every score is stored at the lane's count, which advances
        // only for the scores that pass (a failing one is overwritten or lies
        // past the count; the index stays at most SUB < SEG).  The high word
        // holds the score's float bits; the merge maps them to the monotone
        // code.  A merge only lowers the threshold, so the count taken before
        // it bounds the keys appended after it.
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (!ballot(mq[q] <= thr)) continue;  // no candidate in this group anywhere in the wave
          const int np = (acc[t][4 * q] <= thr) + (acc[t][4 * q + 1] <= thr) + (acc[t][4 * q + 2] <= thr) +
                         (acc[t][4 * q + 3] <= thr);
          const uint64_t ov = ballot(lcnt + np > SUB);
          const uint32_t qm = (uint32_t)(ov | (ov >> 32));
          if (qm) merge_queries(qm);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float v = acc[t][4 * q + i];
            myseg[lcnt] = ((uint64_t)__float_as_uint(v) << 32) | (rref + (uint32_t)(8 * q + i));
            lcnt += v <= thr ? 1 : 0;
          }
        }
      }
    }
  };

  // ---- step loop.  Waves 0-3 score step s and then select it; waves 4-7
  // (which share the SIMDs with 0-3) first select step s-1 and then score
  // step s, so on each SIMD one wave's selection runs beside the other's
  // matrix instructions.  One extra pass lets waves 4-7 select the last
  // step.  Steps run in groups of GRP between workgroup barriers: the first
  // step of a group stages the next group into the other half of the tile
  // buffers (which every wave finished reading before the last barrier;
  // near the end of the slice, repeats of the last step into buffers no
  // later step reads, so every group issues the same copies), and the last
  // step of a group waits for those copies before the barrier.  With two
  // steps per barrier a wave whose selection runs long in one step can catch
  // up in the next before the others wait for it.
  const bool lead = wave < kWideWaves / 2;
  constexpr int GRP = G::GRP;
  if (nsteps > 0) {
#pragma unroll
    for (int i = 0; i < GRP; ++i) stage(min(i, nsteps - 1), i);
    wait_vmem();
    barrier_keep_copies();
  }
  int bs = 0;   // tile buffer of `step`
  int gi = 0;   // position of `step` in its group
  // A wave whose 32 query rows all lie past n (the last query block of a
  // small search) skips this loop: see the one after it.  Only the kernels
  // with rank slots (many slices per query, and every item launch) carry that
  // path: the others keep the plain loop, whose schedule it would change.
  const bool live = SHARE < 2 || __builtin_amdgcn_readfirstlane((int)(q0 < in.n));
  const int last = live ? nsteps : -1;
  for (int step = 0; step <= last; ++step) {
    if (gi == 0 && step < nsteps) {
      // group start: stage the next group into the other half of the buffers
#pragma unroll
      for (int i = 0; i < GRP; ++i) stage(min(step + GRP + i, nsteps - 1), (bs ^ GRP) + i);
    }
    if (lead) {
      if (step < nsteps) {
        score(bs);
        select(step);
      }
    } else {
      if (step > 0) select(step - 1);
      if (step < nsteps) score(bs);
    }
    if (step < nsteps && (gi == GRP - 1 || step == nsteps - 1)) {
      wait_vmem();  // the next group's copies have landed
      barrier_keep_copies();
      // the lanes of a query read the bounds its other slices have published
      // (waited for at once: nothing stays live across the steps for them):
      // the smallest kc-th best every 32 steps, and the rank bound after
      // steps 2^i - 1, when a slice's own list is young and the bound of the
      // other slices' keys matters most
      if constexpr (SHARE == 1) {
        if (in.tshare && (step & 31) == 31 && qrow < in.n) {
          const uint32_t sh = __hip_atomic_load(in.tshare + qrow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (sh != 0xffffffffu) thr = fminf(thr, mono_value(sh));
        }
      } else if constexpr (SHARE == 2) {
        if (in.tshare && ((step & 31) == 31 || ((step + 1) & step) == 0)) {
          uint32_t b = 0xffffffffu;
          if (in.rank_r > 0 && ((step + 1) & step) == 0) b = rank_bound();
          if ((step & 31) == 31 && qrow < in.n)
            b = min(b, __hip_atomic_load(in.tshare + qrow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
          if (b != 0xffffffffu) thr = fminf(thr, mono_value(b));
        }
      }
    }
    bs = bs == STAGES - 1 ? 0 : bs + 1;
    gi = gi == GRP - 1 ? 0 : gi + 1;
  }
  if (!live) {
    // Such a wave only issues its share of the copies and takes the same
    // barriers, so the other wave on its SIMD has the matrix cores and vector
    // ALUs to itself.  Its lists stay empty and are not written.
    int db = 0, dg = 0;
    for (int step = 0; step < nsteps; ++step) {
      if (dg == 0) {
#pragma unroll
        for (int i = 0; i < GRP; ++i) stage(min(step + GRP + i, nsteps - 1), (db ^ GRP) + i);
      }
      if (dg == GRP - 1 || step == nsteps - 1) {
        wait_vmem();
        barrier_keep_copies();
      }
      db = db == STAGES - 1 ? 0 : db + 1;
      dg = dg == GRP - 1 ? 0 : dg + 1;
    }
  }
  {  // end of the slice: flush every buffer
    const uint64_t pend = ballot(lcnt > 0);
    merge_queries((uint32_t)(pend | (pend >> 32)));
  }
  wait_vmem();  // no copy may land after the workgroup's LDS is released

  // ---- write this slice's sorted lists: key e of query j from lane e
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    const int64_t qg = q0 + j;
    if (qg < in.n && lane < kc)
      in.part[(qg * in.P + slice) * kc + lane] = ((uint64_t)Lhi[j] << 32) | Llo[j];
    if constexpr (LK == 2)
      if (qg < in.n && lane + 64 < kc)
        in.part[(qg * in.P + slice) * kc + 64 + lane] = ((uint64_t)Lhi2[j] << 32) | Llo2[j];
  }
}

// One instance per launch: grid (query blocks, slices) of p.one, or one item
// of p.items per workgroup.  SHARE: 0 no bound shared between a query's
// slices, 1 the smallest kc-th best, 2 that and the rank slots.
template <int KIND, int NKG, int SHARE>
__global__ __launch_bounds__(512) void wide_kernel(FusedParams p) {
  using G = WideGeom<KIND, NKG>;
  __shared__ __align__(16) unsigned char tiles[G::TILES_LDS];
  __shared__ __align__(16) float norms[G::NORMS_LDS];
  __shared__ __align__(16) uint64_t bufs[G::BUFS_LDS];
  if (p.items) {
    const FusedItem it = p.items[blockIdx.x];
    const FusedInst in = p.insts[it.inst];
    wide_item<KIND, NKG, 1, SHARE>(in, it.qblock, it.slice, tiles, norms, bufs);
  } else {
    wide_item<KIND, NKG, 1, SHARE>(p.one, blockIdx.x, blockIdx.y, tiles, norms, bufs);
  }
}

// The same with two keys per lane (k' <= 128; 16-bit tiles).
template <int KIND, int NKG, int SHARE>
__global__ __launch_bounds__(512) void wide2_kernel(FusedParams p) {
  using G = WideGeom<KIND, NKG>;
  __shared__ __align__(16) unsigned char tiles[G::TILES_LDS];
  __shared__ __align__(16) float norms[G::NORMS_LDS];
  __shared__ __align__(16) uint64_t bufs[G::BUFS_LDS];
  if (p.items) {
    const FusedItem it = p.items[blockIdx.x];
    const FusedInst in = p.insts[it.inst];
    wide_item<KIND, NKG, 2, SHARE>(in, it.qblock, it.slice, tiles, norms, bufs);
  } else {
    wide_item<KIND, NKG, 2, SHARE>(p.one, blockIdx.x, blockIdx.y, tiles, norms, bufs);
  }
}

// Batched form in one launch: 16-bit instances of any padded dimension up
// to 128 and k' up to 128.  The grid has one workgroup per item; each
// workgroup takes the next item (instance, query block, slice) in the order
// of p.items -- longest first -- from the counter p.counter, which the
// launch before this one on the stream zeroes.  The counter, not the block
// index, fixes the order in which items start across the dispatchers of
// the eight XCDs, so the longest items start first device-wide.  Every
// workgroup takes exactly one item; none waits for another.
template <int KIND>
__global__ __launch_bounds__(512) void wide_batch_kernel(FusedParams p) {
  using G = WideGeom<KIND, 8>;
  __shared__ __align__(16) unsigned char tiles[G::TILES_LDS];
  __shared__ __align__(16) float norms[G::NORMS_LDS];
  __shared__ __align__(16) uint64_t bufs[G::BUFS_LDS];
  __shared__ int taken;
  if (threadIdx.x == 0) taken = atomicAdd(p.counter, 1);
  __syncthreads();
  const int i = __builtin_amdgcn_readfirstlane(taken);  // uniform: item and instance fields in scalar registers
  if (i >= p.nitems) return;
  const FusedItem it = p.items[i];
  const FusedInst in = p.insts[it.inst];
  const bool two = in.kc > kWideMaxKc1;
  switch (in.dp) {
    case 32:
      if (two) wide_item<KIND, 2, 2, 2>(in, it.qblock, it.slice, tiles, norms, bufs);
      else wide_item<KIND, 2, 1, 2>(in, it.qblock, it.slice, tiles, norms, bufs);
      break;
    case 64:
      if (two) wide_item<KIND, 4, 2, 2>(in, it.qblock, it.slice, tiles, norms, bufs);
      else wide_item<KIND, 4, 1, 2>(in, it.qblock, it.slice, tiles, norms, bufs);
      break;
    case 96:
      if (two) wide_item<KIND, 6, 2, 2>(in, it.qblock, it.slice, tiles, norms, bufs);
      else wide_item<KIND, 6, 1, 2>(in, it.qblock, it.slice, tiles, norms, bufs);
      break;
    default:
      if (two) wide_item<KIND, 8, 2, 2>(in, it.qblock, it.slice, tiles, norms, bufs);
      else wide_item<KIND, 8, 1, 2>(in, it.qblock, it.slice, tiles, norms, bufs);
      break;
  }
}

// Item launches take the instantiation with both shared bounds; a single
// search takes the one its bounds call for (one slice per query: none, which
// runs fastest; fewer than kRankMinSlices slices: the kc-th best alone, as
// the rank code costs registers there for little gain).
template <int KIND, int NKG>
hipError_t launch_wide_one(const FusedParams& p, hipStream_t stream) {
  if (p.items && p.nitems <= 0) return hipSuccess;
  dim3 grid = p.items ? dim3((unsigned)p.nitems)
                      : dim3((unsigned)((p.one.n + kWideQueriesWG - 1) / kWideQueriesWG), (unsigned)p.one.P);
  const int share = p.items ? 2 : !p.one.tshare ? 0 : p.one.rank_r > 0 ? 2 : 1;
  const dim3 block(kWideWaves * kWaveSize);
  if constexpr (KIND != TILE_L2_F32) {
    if (p.kc_max > kWideMaxKc1) {
      if (share == 2) hipLaunchKernelGGL((wide2_kernel<KIND, NKG, 2>), grid, block, 0, stream, p);
      else if (share == 1) hipLaunchKernelGGL((wide2_kernel<KIND, NKG, 1>), grid, block, 0, stream, p);
      else hipLaunchKernelGGL((wide2_kernel<KIND, NKG, 0>), grid, block, 0, stream, p);
      return hipGetLastError();
    }
  }
  if (share == 2) hipLaunchKernelGGL((wide_kernel<KIND, NKG, 2>), grid, block, 0, stream, p);
  else if (share == 1) hipLaunchKernelGGL((wide_kernel<KIND, NKG, 1>), grid, block, 0, stream, p);
  else hipLaunchKernelGGL((wide_kernel<KIND, NKG, 0>), grid, block, 0, stream, p);
  return hipGetLastError();
}

// launch_wide_one for the padded widths of a 16-bit tile kind (p.ng k groups)
template <int KIND>
hipError_t dispatch_half(const FusedParams& p, hipStream_t stream) {
  switch (p.ng) {
    case 2: return launch_wide_one<KIND, 2>(p, stream);
    case 4: return launch_wide_one<KIND, 4>(p, stream);
    case 6: return launch_wide_one<KIND, 6>(p, stream);
    case 8: return launch_wide_one<KIND, 8>(p, stream);
    default: return hipErrorInvalidValue;
  }
}

template <int KIND>
hipError_t launch_wide_batch_one(const FusedParams& p, hipStream_t stream) {
  if (p.nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL((wide_batch_kernel<KIND>), dim3((unsigned)p.nitems), dim3(kWideWaves * kWaveSize), 0, stream, p);
  return hipGetLastError();
}

}  // namespace knn
