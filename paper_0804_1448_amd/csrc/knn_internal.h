// knn_internal.h -- types shared by the host dispatch (knn_api.cpp) and the
// HIP kernels (knn_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace knn {

// Selection keys: a candidate (score, reference index) is packed into one
// 64-bit integer whose unsigned order is the lexicographic (score, index)
// order: the high word is the score's IEEE bits mapped to a monotone
// unsigned code, the low word the index.  An all-ones key marks an empty
// slot and sorts after every real candidate.
constexpr uint64_t kEmptyKey = ~0ull;

// Distance tile kinds.
enum TileKind : int {
  TILE_L2_F32 = 0,   // Euclidean cross term on MFMA, float32 operands
  TILE_L2_BF16 = 1,  // Euclidean cross term on MFMA, bfloat16 operands
  TILE_L2_F16 = 2,   // Euclidean cross term on MFMA, float16 operands
  TILE_L1_F32 = 3,   // Manhattan on the vector ALUs
  TILE_LINF_F32 = 4, // infinity norm on the vector ALUs
};

// Storage element types of a prepared point array.
enum ElemType : int { ELEM_F32 = 0, ELEM_BF16 = 1, ELEM_F16 = 2 };

// Fixed geometry of the fused distance + selection kernel.
constexpr int kWaveSize = 64;
constexpr int kQueriesPerWave = 16;   // one MFMA 16x16 output column per query
constexpr int kTileRefs = 16;         // references per MFMA tile
constexpr int kTilesPerStep = 4;
constexpr int kStepRefs = kTileRefs * kTilesPerStep;  // references scored per step
constexpr int kMaxWaves = 8;          // waves per fused workgroup
constexpr int kMaxMergePerLane = 8;   // (list + buffer) <= 64 * 8 keys
constexpr int kMaxGroupsF32 = 16;     // float32 MFMA k groups (16 dims) per chunk
constexpr int kMaxGroups16 = 8;       // 16-bit MFMA k groups (32 dims) per chunk
constexpr int kMaxGroupsValu = 8;     // vector-ALU groups (16 dims) per chunk
constexpr int kLdsBytes = 160 * 1024; // LDS per compute unit on gfx950

// One search instance of the fused distance + top-k' selection kernel: a
// query set against a reference set.
struct FusedInst {
  const void* Q;        // prepared queries [n][ldq] (element type of the tile kind)
  const void* R;        // prepared references [m][ldr]
  const float* rhalf;   // 0.5 * squared norm of each prepared reference (Euclidean only)
  uint64_t* part;       // out: per-slice sorted candidate lists [n][P][kc]
  int64_t n;
  int64_t m;
  int64_t slice_len;    // references per slice (multiple of kStepRefs)
  int ldq;              // row stride of Q, elements
  int ldr;              // row stride of R, elements
  int dp;               // padded dimension (multiple of the tile kind's k group)
  int nchunk;           // ceil(dp / chunk width); the last chunk may be shorter
  int P;                // number of slices
  int kc;               // list capacity = k'
  // Bounds shared by the slices of a query, or NULL.  tshare[q]: the
  // smallest kc-th best (monotone score code) any slice of query q has
  // published.  With rank_r > 0 the rank slots follow, slice-major:
  // tshare[n + s * n + q] holds slice s's rank_r-th best for query q.  Any
  // rank_gs slices hold between them at least rank_gs * rank_r >= kc keys at
  // or below the largest of their slots, so the smallest such maximum over
  // rank_G groups of consecutive slices bounds the query's kc-th best over
  // the whole set as well.  All ones (no key yet) at the start.
  uint32_t* tshare;
  int rank_r;
  int rank_gs;
  int rank_G;
};

// One workgroup's share of a batched launch.
struct FusedItem {
  int inst;    // index into the instance table
  int qblock;  // query block (waves * 16 queries)
  int slice;   // reference slice
  int pad;
};

// Launch parameters of the fused kernel.  With `items == nullptr` the grid is
// (query blocks, slices) of the single instance `one`; otherwise workgroup b
// processes items[b] of the instance table `insts`.
struct FusedParams {
  FusedInst one;
  const FusedInst* insts;
  const FusedItem* items;
  int nitems;           // workgroups of a batched launch
  int ng;               // k groups per chunk (the kernel's compile-time chunk width)
  int cb;               // candidate buffer capacity per query (4 segments)
  int waves;            // waves per workgroup
  int kc_max;           // largest kc of the launch (sizes the LDS lists)
  int wide;             // 1: the 32x32-tile Euclidean kernel with register lists (ng = dp / 16)
  int lane;             // 1: a per-lane-selection kernel (ng = dp / 16; cb = queue keys per lane)
  int tiled;            // float32 Euclidean lane kernel: R in the 32-row tile layout (launch_prep_rows_tiled)
  int* counter;         // one-launch batched form: next item to take (zeroed before the launch)
};

// One instance of the merge + exact re-rank + finalize kernel.
struct FinalInst {
  const uint64_t* part; // [n][P][kc] sorted candidate lists (empty slots = kEmptyKey)
  const float* Q;       // original float32 queries [n][ldq]
  const void* Rm;       // canonical reference rows [m][ldr]
  float* dist;          // out [n][k]
  int32_t* idx;         // out [n][k]
  int64_t n;
  int64_t m;            // number of references (bounds every candidate index)
  int ldq;
  int ldr;
  int rm_type;          // ElemType of Rm
  int d;
  int P;
  int kc;
  int kprime;           // candidates re-ranked (<= P * kc)
  int k;
  int metric;           // 0 L2, 1 L1, 2 Linf
};

// One finalize workgroup of a batched launch: kFinalWaves consecutive
// queries of one instance.
struct FinalItem {
  int inst;
  int q0;
};

struct FinalParams {
  FinalInst one;
  const FinalInst* insts;
  const FinalItem* items;
  int nitems;
  int keys_max;         // largest P * kc of the launch
  int kprime_max;       // largest k' of the launch
  int p_max;            // largest P of the launch
};

// One array of a batched point preparation.
struct PrepJob {
  const float* src;     // [rows][lds] float32
  void* dst;            // [rows][ldd] in element type `elem`
  const float* centre;  // subtracted from every row, or NULL
  float* rhalf;         // half squared norms of the stored rows, or NULL
  int64_t rows;
  int64_t row0;         // first global row of this job in the launch
  int d;
  int lds;
  int ldd;
  int elem;
  uint32_t* tshare;     // per-row shared bounds of the search to reset (all ones), or NULL
  int nslots;           // rank slots per row after them (FusedInst::tshare), also reset
};

constexpr int kFinalWaves = 4;          // queries per finalize workgroup
constexpr int kFinalMaxKeys = 2048;     // P * kc limit of one finalize wave
constexpr int kMaxSlices = 256;         // slices of one search (above kFinalMaxKeys / kc: merged first, kc <= 64)
constexpr int kFinalMaxCand = 512;      // k' limit of the re-rank

// Launchers (knn_kernels.hip).  All enqueue on `stream` and return the HIP
// status of the launch.
// overflow (16-bit elements only, may be NULL): set to 1 when a finite value
// rounds to infinity in the element type
// tshare (may be NULL): per-row shared bounds of the search that follows and
// `nslots` rank slots per row after them (FusedInst::tshare), set to all ones
hipError_t launch_prep_rows(const float* src, int64_t rows, int d, int lds, const float* centre, void* dst,
                            int ldd, int elem, float* rhalf, hipStream_t stream, unsigned* overflow = nullptr,
                            uint32_t* tshare = nullptr, int nslots = 0);
// float32 rows in the 32-row tile layout [i / 32][t / 4][i % 32][t % 4]
// (ldd a multiple of 4; dst holds round_up(rows, 32) rows)
hipError_t launch_prep_rows_tiled(const float* src, int64_t rows, int d, int lds, const float* centre, float* dst,
                                  int ldd, float* rhalf, hipStream_t stream);
hipError_t launch_centre(const float* src, int64_t rows, int d, int lds, float* centre, hipStream_t stream);
size_t fused_lds_bytes(int kind, int waves, int kc, int cb, int cw);
hipError_t launch_fused(int kind, const FusedParams& p, hipStream_t stream);
// one per instantiation unit knn_fused_<kind>_<s|l>.hip (s: k' <= 64 only)
#define KNN_FUSED_UNIT(name) hipError_t launch_fused_##name(const FusedParams& p, hipStream_t stream);
KNN_FUSED_UNIT(f32lo_s) KNN_FUSED_UNIT(f32lo_l) KNN_FUSED_UNIT(f32hi_s) KNN_FUSED_UNIT(f32hi_l)
KNN_FUSED_UNIT(bf16_s) KNN_FUSED_UNIT(bf16_l) KNN_FUSED_UNIT(f16_s) KNN_FUSED_UNIT(f16_l)
KNN_FUSED_UNIT(l1_s) KNN_FUSED_UNIT(l1_l) KNN_FUSED_UNIT(linf_s) KNN_FUSED_UNIT(linf_l)
#undef KNN_FUSED_UNIT
// Euclidean kernel with 32x32 tiles and register-resident lists (k' <= 64,
// dp <= 128; float32 or 16-bit tiles): 8 waves of 32 queries per workgroup
constexpr int kWideQueries = 256;
constexpr int kWideMaxKc1 = 64;   // one list key per lane
constexpr int kWideMaxKc = 128;   // two keys per lane (16-bit tiles only)
constexpr int kWideMaxDp = 128;
constexpr int64_t kWideMinSliceF32 = 16384;  // float32 tiles: shortest slice worth the 32x32 kernel
// the same when the references can be read in the 32-row tile layout by the
// float32 lane kernel (measured: the lane kernel wins at slices of 16384 and
// 19200, the 32x32 kernel at 2^20)
constexpr int64_t kWideMinSliceF32Tiled = 131072;
constexpr int kRankMinSlices = 8;  // fewest slices per query for the rank slots (FusedInst::tshare)
constexpr size_t kWideLdsBytes = 153 * 1024;  // static LDS of the widest instantiation (16-bit, dp = 128)
hipError_t launch_wide(int kind, const FusedParams& p, hipStream_t stream);
hipError_t launch_wide_f32(const FusedParams& p, hipStream_t stream);   // float32 tiles (knn_wide_f32.hip)
hipError_t launch_wide_bf16(const FusedParams& p, hipStream_t stream);  // BF16 tiles (knn_wide_bf16.hip)
hipError_t launch_wide_f16(const FusedParams& p, hipStream_t stream);   // FP16 tiles (knn_wide_f16.hip)
// Manhattan / infinity-norm kernel with one query per lane (dp <= 128):
// `waves` waves of 64 queries per workgroup, each lane with a sorted list of
// kc keys and a queue of `cb` (8 or 12) keys in LDS
constexpr int kLaneMaxDp = 128;
hipError_t launch_lane(int kind, const FusedParams& p, hipStream_t stream);
// float32 Euclidean with per-lane selection on 32x32 MFMA tiles (dp <= 128):
// `waves` waves of 32 queries, lists as in the Manhattan kernel
hipError_t launch_lane_l2(const FusedParams& p, hipStream_t stream);
size_t lane_lds(int waves, int kc, int queue);
hipError_t launch_finalize(const FinalParams& p, hipStream_t stream);
// merge groups of G consecutive sorted slice lists per query (kc <= 64):
// part [n][P][kc] -> out [n][P2][kc], P2 = ceil(P / G)
hipError_t launch_merge_lists(const uint64_t* part, uint64_t* out, int64_t n, int P, int kc, int G, int P2,
                              hipStream_t stream);
// k-NN classification: out[q] = majority of labels[idx[q][0..k-1]] (ties to
// the nearest of the tied classes)
hipError_t launch_vote(const int32_t* idx, int64_t n, int k, const int32_t* labels, int32_t* out, hipStream_t stream);
// Mahalanobis: Y = (X - c) L for rows of X [rows][d], c [d], L [d][d] (row-major)
hipError_t launch_transform_rows(const float* X, int64_t rows, int d, const float* c, const float* L, float* Y,
                                 hipStream_t stream);
// Mahalanobis: exact distances ||L^T (q - r)|| of kc candidates per query
// (cidx [n][kc]) from the caller's rows, the k best written to dist / idx [n][k]
hipError_t launch_mahalanobis_rerank(const float* Q, const float* R, const float* L, int64_t n, int d, int64_t m,
                                     const int32_t* cidx, int kc, float* dist, int32_t* idx, int k,
                                     hipStream_t stream);
// k-NN entropy: per-point log rho_k from the k + 1 nearest (dist/idx
// [n][k + 1]) into terms[n], then out = scale * sum(terms) + offset
hipError_t launch_entropy(const float* dist, const int32_t* idx, int64_t n, int k, double* terms, double scale,
                          double offset, double* out, hipStream_t stream);

// zero (may be NULL): an int set to 0 by the launch (the item counter of the
// batched launch that follows on the stream)
hipError_t launch_prep_batched(const PrepJob* jobs_dev, int njobs, int64_t total_rows, hipStream_t stream,
                               int* zero = nullptr);
size_t finalize_lds_bytes(int keys_max, int p_max, int kprime_max);

}  // namespace knn
