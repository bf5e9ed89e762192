// knn_device.h -- device helpers shared by the k-NN kernels: selection keys,
// 16-bit rounding and the wave-private rank merge.
#pragma once

#include "knn_internal.h"

namespace knn {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void lds_void;

// Loads through the global address space: the compiler counts them on
// vmcnt alone (a flat load also counts on lgkmcnt, which forces a full wait
// before every LDS access and defeats loads issued ahead of their use).
__device__ __forceinline__ float4 gload4(const float* ptr) {
  const f32x4 v = *(const __attribute__((address_space(1))) f32x4*)ptr;
  return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ float gload1(const float* ptr) {
  return *(const __attribute__((address_space(1))) float*)ptr;
}

__device__ __forceinline__ uint4 gload16(const void* ptr) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 v = *(const __attribute__((address_space(1))) u32x4*)ptr;
  return make_uint4(v.x, v.y, v.z, v.w);
}

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

// Wait until at most N vector memory operations of this wave are
// outstanding (the asynchronous global-to-LDS tile copies included).  The
// builtin, unlike inline assembly, is visible to the compiler's own wait
// tracking, which then knows which copies have landed.  gfx9 encoding:
// vmcnt in bits 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 left at their
// maxima.
template <int N>
__device__ __forceinline__ void wait_vmem_n() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt(0x0F70 | (N & 15) | ((N >> 4) << 14));
}
__device__ __forceinline__ void wait_vmem() { wait_vmem_n<0>(); }

// Workgroup barrier without the fence of __syncthreads, which would also
// wait for this wave's outstanding global-to-LDS copies: used where copies
// for later steps are meant to stay in flight across the barrier (each wave
// waits for the copies it needs with an explicit vmcnt first).
__device__ __forceinline__ void barrier_keep_copies() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// compiler and LDS ordering point inside one wave
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------ wave-private merge
// One query's sorted list L (len keys) and its candidate buffer -- four
// segments seg[k] of cnt[k] unsorted keys, one per lane group -- are
// replaced by the first kc keys of their union, sorted.  All keys are
// distinct (a reference enters a query's buffer at most once per slice).
// Each lane places up to NR keys by rank: a list key at position e moves to
// e + #{b in buffer: b < key}; a buffer key goes to #{x in L: x < key} +
// #{b in buffer: b < key}.
struct Segs {
  const uint64_t* seg[4];
  int cnt[4];
};

__device__ __forceinline__ uint64_t seg_at(const Segs& b, int e) {
  if (e < b.cnt[0]) return b.seg[0][e];
  e -= b.cnt[0];
  if (e < b.cnt[1]) return b.seg[1][e];
  e -= b.cnt[1];
  if (e < b.cnt[2]) return b.seg[2][e];
  return b.seg[3][e - b.cnt[2]];
}

template <int NR>
__device__ __forceinline__ void merge_ranked(uint64_t* L, const Segs& b, int len, int c, int kc, int lane) {
  const int T = len + c;
  uint64_t x[NR];
  int below[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int e = lane + 64 * r;
    x[r] = kEmptyKey;
    below[r] = 0;
    if (e < T) x[r] = e < len ? L[e] : seg_at(b, e - len);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint64_t* B = b.seg[k];
    const int ck = b.cnt[k];
    int j = 0;
    for (; j + 4 <= ck; j += 4) {
      const uint64_t b0 = B[j], b1 = B[j + 1], b2 = B[j + 2], b3 = B[j + 3];
#pragma unroll
      for (int r = 0; r < NR; ++r)
        below[r] += (int)(b0 < x[r]) + (int)(b1 < x[r]) + (int)(b2 < x[r]) + (int)(b3 < x[r]);
    }
    for (; j < ck; ++j) {
      const uint64_t bj = B[j];
#pragma unroll
      for (int r = 0; r < NR; ++r) below[r] += (int)(bj < x[r]);
    }
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
  wave_sync();
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (rank[r] < kc) L[rank[r]] = x[r];
  wave_sync();
}

// ------------------------------------------------ register bitonic merge
// Cross-lane exchange with lane ^ J, all on the vector ALU: DPP moves for
// J <= 8 (quad permutes, row shifts, row rotate); for J = 16 and 32 the
// gfx950 lane-swap instructions.  v_permlane16_swap with both operands equal
// to v leaves v's even 16-lane rows in the first result and its odd rows in
// the second, each row duplicated over its pair; v_permlane32_swap does the
// same for 32-lane halves.  A lane then takes the copy of its partner row.
// Every lane reads a lane of its own row (quad permutes, row rotate), or, for
// the row shifts, a lane whose value the caller discards where the shift
// leaves the row; so no "old" value is needed (bound control: such lanes read
// zero), which saves the move that would initialize one.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
}

template <int J>
__device__ __forceinline__ uint32_t xor_lane32(uint32_t v, int lane) {
  if constexpr (J == 1) return dpp_mov<0xB1>(v);       // quad_perm [1,0,3,2]
  else if constexpr (J == 2) return dpp_mov<0x4E>(v);  // quad_perm [2,3,0,1]
  else if constexpr (J == 4) {
    const uint32_t up = dpp_mov<0x104>(v);              // row_shl:4 (from lane + 4)
    const uint32_t dn = dpp_mov<0x114>(v);              // row_shr:4 (from lane - 4)
    return (lane & 4) ? dn : up;
  } else if constexpr (J == 8) return dpp_mov<0x128>(v);  // row_ror:8
  else if constexpr (J == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (lane & 16) ? r[0] : r[1];
  } else {
    static_assert(J == 32, "lane distance");
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (lane & 32) ? r[0] : r[1];
  }
}

template <int J>
__device__ __forceinline__ uint64_t xor_lane64(uint64_t v, int lane) {
  const uint32_t lo = xor_lane32<J>((uint32_t)v, lane);
  const uint32_t hi = xor_lane32<J>((uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

// one compare-exchange stage: the lane whose bit J is clear keeps the
// smaller key when `ascending`, the larger otherwise
template <int J>
__device__ __forceinline__ uint64_t bitonic_step(uint64_t v, int lane, bool ascending) {
  const uint64_t o = xor_lane64<J>(v, lane);
  const bool keep_min = ((lane & J) == 0) == ascending;
  const bool lt = v < o;
  return (lt == keep_min) ? v : o;
}

// sort one key per lane over the 64 lanes, ascending or descending
__device__ __forceinline__ uint64_t bitonic_sort64(uint64_t v, int lane, bool descending) {
  v = bitonic_step<1>(v, lane, (lane & 2) == 0);
  v = bitonic_step<2>(v, lane, (lane & 4) == 0);
  v = bitonic_step<1>(v, lane, (lane & 4) == 0);
  v = bitonic_step<4>(v, lane, (lane & 8) == 0);
  v = bitonic_step<2>(v, lane, (lane & 8) == 0);
  v = bitonic_step<1>(v, lane, (lane & 8) == 0);
  v = bitonic_step<8>(v, lane, (lane & 16) == 0);
  v = bitonic_step<4>(v, lane, (lane & 16) == 0);
  v = bitonic_step<2>(v, lane, (lane & 16) == 0);
  v = bitonic_step<1>(v, lane, (lane & 16) == 0);
  v = bitonic_step<16>(v, lane, (lane & 32) == 0);
  v = bitonic_step<8>(v, lane, (lane & 32) == 0);
  v = bitonic_step<4>(v, lane, (lane & 32) == 0);
  v = bitonic_step<2>(v, lane, (lane & 32) == 0);
  v = bitonic_step<1>(v, lane, (lane & 32) == 0);
  const bool up = !descending;
  v = bitonic_step<32>(v, lane, up);
  v = bitonic_step<16>(v, lane, up);
  v = bitonic_step<8>(v, lane, up);
  v = bitonic_step<4>(v, lane, up);
  v = bitonic_step<2>(v, lane, up);
  v = bitonic_step<1>(v, lane, up);
  return v;
}

// sort a bitonic sequence of one key per lane ascending
__device__ __forceinline__ uint64_t bitonic_clean64(uint64_t v, int lane) {
  v = bitonic_step<32>(v, lane, true);
  v = bitonic_step<16>(v, lane, true);
  v = bitonic_step<8>(v, lane, true);
  v = bitonic_step<4>(v, lane, true);
  v = bitonic_step<2>(v, lane, true);
  v = bitonic_step<1>(v, lane, true);
  return v;
}

// sort a bitonic sequence of one key per lane descending
__device__ __forceinline__ uint64_t bitonic_clean64_desc(uint64_t v, int lane) {
  v = bitonic_step<32>(v, lane, false);
  v = bitonic_step<16>(v, lane, false);
  v = bitonic_step<8>(v, lane, false);
  v = bitonic_step<4>(v, lane, false);
  v = bitonic_step<2>(v, lane, false);
  v = bitonic_step<1>(v, lane, false);
  return v;
}

// Merge of a list of len <= kc <= 64 keys with a buffer of at most 64 keys
// held one per lane: lane j loads buffer key j (segment j / 16, entry
// j % 16).  The buffer is sorted descending across the wave; with the list
// ascending, their lane-wise minimum holds the 64 smallest keys of the
// union as a bitonic sequence, which six exchange stages sort.
__device__ __forceinline__ int wave_merge64(uint64_t* L, const Segs& b, int len, int kc, int lane) {
  const int c = b.cnt[0] + b.cnt[1] + b.cnt[2] + b.cnt[3];
  const int sg = lane >> 4, e = lane & 15;
  const uint64_t* segp = sg == 0 ? b.seg[0] : sg == 1 ? b.seg[1] : sg == 2 ? b.seg[2] : b.seg[3];
  const int segc = sg == 0 ? b.cnt[0] : sg == 1 ? b.cnt[1] : sg == 2 ? b.cnt[2] : b.cnt[3];
  uint64_t x = e < segc ? segp[e] : kEmptyKey;
  const uint64_t l = lane < len ? L[lane] : kEmptyKey;
  x = bitonic_sort64(x, lane, true);
  uint64_t m = l < x ? l : x;
  m = bitonic_clean64(m, lane);
  wave_sync();
  if (lane < kc) L[lane] = m;
  wave_sync();
  return min(kc, len + c);
}

// Merge the buffer segments into list L; returns the new list length.
__device__ __forceinline__ int wave_merge(uint64_t* L, const Segs& b, int len, int kc, int sub, int lane) {
  if (kc <= 64 && sub <= 16) return wave_merge64(L, b, len, kc, lane);
  const int c = b.cnt[0] + b.cnt[1] + b.cnt[2] + b.cnt[3];
  const int nr = (len + c + 63) >> 6;
  switch (nr) {
    case 0: break;
    case 1: merge_ranked<1>(L, b, len, c, kc, lane); break;
    case 2: merge_ranked<2>(L, b, len, c, kc, lane); break;
    case 3: merge_ranked<3>(L, b, len, c, kc, lane); break;
    case 4: merge_ranked<4>(L, b, len, c, kc, lane); break;
    case 5: merge_ranked<5>(L, b, len, c, kc, lane); break;
    case 6: merge_ranked<6>(L, b, len, c, kc, lane); break;
    case 7: merge_ranked<7>(L, b, len, c, kc, lane); break;
    default: merge_ranked<8>(L, b, len, c, kc, lane); break;
  }
  return min(kc, len + c);
}

}  // namespace knn
