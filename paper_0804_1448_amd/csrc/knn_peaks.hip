// knn_peaks.hip -- micro-benchmarks that measure the issue rates the
// roofline fractions of the k-NN kernels are taken against: the vector ALU
// rate of the Manhattan kernel's inner operations, the float32 and BF16
// matrix-core rates of the Euclidean kernels, the LDS read rate their
// operand reads draw on, and the shader clock they ran at.  Built as its own library (libknn_peaks.so), used by the benchmark
// only; not part of the k-NN C ABI.
//
// Every kernel runs `iters` iterations of independent instruction chains on
// every lane of every wave and writes one value per lane (so nothing is
// dead code).  Wave 0 of workgroup 0 also records the shader-clock counter
// (s_memtime) and the constant 100 MHz counter (s_memrealtime) around its
// loop, from which the host derives the clock of the run.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void stamp(uint64_t* clk, int which) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    clk[2 * which] = __builtin_amdgcn_s_memtime();
    clk[2 * which + 1] = __builtin_amdgcn_s_memrealtime();
  }
}

template <int I>
__device__ __forceinline__ float sub_abs_add(float acc, float a, float b) {
  const float bb = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(b), 0x150 + I, 0xF, 0xF, false));
  return acc + __builtin_fabsf(a - bb);
}

// The Manhattan kernel's two operations per pair and dimension: a
// subtraction whose second operand is another lane's value broadcast by a
// DPP row_newbcast, then an add of the absolute value.  Eight independent
// accumulators keep the pipeline full.
__global__ __launch_bounds__(256) void valu_kernel(float* out, uint64_t* clk, int iters, float seed) {
  const int lane = threadIdx.x & 63;
  float a[8], acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = seed * (float)(lane + 8 * i + 1);
    acc[i] = 0.f;
  }
  float b = seed * (float)(threadIdx.x + 3);
  stamp(clk, 0);
  for (int it = 0; it < iters; ++it) {
    acc[0] = sub_abs_add<0>(acc[0], a[0], b);
    acc[1] = sub_abs_add<1>(acc[1], a[1], b);
    acc[2] = sub_abs_add<2>(acc[2], a[2], b);
    acc[3] = sub_abs_add<3>(acc[3], a[3], b);
    acc[4] = sub_abs_add<4>(acc[4], a[4], b);
    acc[5] = sub_abs_add<5>(acc[5], a[5], b);
    acc[6] = sub_abs_add<6>(acc[6], a[6], b);
    acc[7] = sub_abs_add<7>(acc[7], a[7], b);
    b = b + 1.0f;
  }
  stamp(clk, 1);
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += acc[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// v_mfma_f32_32x32x16_bf16: eight independent accumulator chains.
__global__ __launch_bounds__(256) void mfma_bf16_kernel(float* out, uint64_t* clk, int iters, float seed) {
  const int lane = threadIdx.x & 63;
  bf16x8 a, b;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = (__bf16)(seed * (float)(lane + i));
    b[i] = (__bf16)(seed * (float)(lane - i));
  }
  f32x16 c0 = {}, c1 = {}, c2 = {}, c3 = {}, c4 = {}, c5 = {}, c6 = {}, c7 = {};
  stamp(clk, 0);
  for (int it = 0; it < iters; ++it) {
    c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c3, 0, 0, 0);
    c4 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c4, 0, 0, 0);
    c5 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c5, 0, 0, 0);
    c6 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c6, 0, 0, 0);
    c7 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c7, 0, 0, 0);
  }
  stamp(clk, 1);
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += c0[i] + c1[i] + c2[i] + c3[i] + c4[i] + c5[i] + c6[i] + c7[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// v_mfma_f32_32x32x2f32: eight independent accumulator chains.
__global__ __launch_bounds__(256) void mfma_f32_kernel(float* out, uint64_t* clk, int iters, float seed) {
  const int lane = threadIdx.x & 63;
  const float a = seed * (float)(lane + 1), b = seed * (float)(lane + 2);
  f32x16 c0 = {}, c1 = {}, c2 = {}, c3 = {}, c4 = {}, c5 = {}, c6 = {}, c7 = {};
  stamp(clk, 0);
  for (int it = 0; it < iters; ++it) {
    c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c3, 0, 0, 0);
    c4 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c4, 0, 0, 0);
    c5 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c5, 0, 0, 0);
    c6 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c6, 0, 0, 0);
    c7 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c7, 0, 0, 0);
  }
  stamp(clk, 1);
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += c0[i] + c1[i] + c2[i] + c3[i] + c4[i] + c5[i] + c6[i] + c7[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// v_mfma_f32_32x32x16_bf16 with CH independent accumulator chains per wave:
// how many chains (and waves per SIMD) keep the matrix core busy.
template <int CH>
__global__ __launch_bounds__(256) void mfma_chains_kernel(float* out, uint64_t* clk, int iters, float seed) {
  const int lane = threadIdx.x & 63;
  bf16x8 a, b;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = (__bf16)(seed * (float)(lane + i));
    b[i] = (__bf16)(seed * (float)(lane - i));
  }
  f32x16 c[CH];
#pragma unroll
  for (int j = 0; j < CH; ++j) c[j] = f32x16{};
  stamp(clk, 0);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < CH; ++j) c[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c[j], 0, 0, 0);
  }
  stamp(clk, 1);
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < CH; ++j)
#pragma unroll
    for (int i = 0; i < 16; ++i) s += c[j][i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// ds_read_b128 rate: per iteration each wave reads eight consecutive 1 KB
// blocks of a 32 KB LDS buffer, lane l the l-th 16-byte chunk of a block
// (the access of the 32x32 kernel's operand reads, without bank conflicts);
// the eight reads share one address register and differ by their immediate
// offsets.  The words read are summed into one value (two v_add3_u32 per
// read) so that every read stays live; the first block steps by 3 (mod 16)
// per iteration, so no unrolled copy of the loop repeats an address, and
// `rot`, taken from a launch argument, keeps the sequence from being known at
// compile time.  32 KB per workgroup: at most four
// workgroups (16 waves) per CU.
__global__ __launch_bounds__(256) void lds_read_kernel(float* out, uint64_t* clk, int iters, float seed) {
  __shared__ __align__(16) uint4 buf[2048];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const uint32_t sb = __float_as_uint(seed);
  for (int i = t; i < 2048; i += 256) buf[i] = make_uint4(i, i * 3u, i * 5u, (i * 7u) ^ sb);
  __syncthreads();
  const int rot = (int)(sb & 15u);
  uint32_t acc = 0;
  stamp(clk, 0);
  for (int it = 0; it < iters; ++it) {
    const uint4* p = buf + ((it * 3 + wave + rot) & 15) * 64 + lane;  // blocks 0..22 of 32
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint4 v = p[u * 64];
      acc = acc + v.x + v.y + v.z + v.w;
    }
  }
  stamp(clk, 1);
  out[blockIdx.x * blockDim.x + threadIdx.x] = __uint_as_float(acc);
}

}  // namespace

extern "C" {

// BF16 32x32x16 loop with `chains` (1, 2, 4 or 8) independent accumulator
// chains per wave; work per wave and iteration: chains * 32768 flops.
int knn_peak_launch_chains(int chains, int blocks, int iters, float* out, uint64_t* clk, void* stream) {
  if (blocks < 1 || iters < 1 || !out || !clk) return (int)hipErrorInvalidValue;
  const hipStream_t s = (hipStream_t)stream;
  const float seed = 1.0f / 1024.0f;
  switch (chains) {
    case 1: hipLaunchKernelGGL(mfma_chains_kernel<1>, dim3(blocks), dim3(256), 0, s, out, clk, iters, seed); break;
    case 2: hipLaunchKernelGGL(mfma_chains_kernel<2>, dim3(blocks), dim3(256), 0, s, out, clk, iters, seed); break;
    case 4: hipLaunchKernelGGL(mfma_chains_kernel<4>, dim3(blocks), dim3(256), 0, s, out, clk, iters, seed); break;
    case 8: hipLaunchKernelGGL(mfma_chains_kernel<8>, dim3(blocks), dim3(256), 0, s, out, clk, iters, seed); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

// Launch micro-benchmark `which` (0 vector ALU, 1 BF16 matrix, 2 float32
// matrix, 3 LDS reads) with `blocks` workgroups of 256 lanes, `iters`
// iterations each, on `stream`.  out: device float [blocks * 256]; clk:
// device uint64 [4] (shader-clock and 100 MHz counters before and after the
// loop of workgroup 0).  Work per launch, per lane and iteration: 16 vector
// operations (8 subtractions + 8 absolute adds); 8 * 32768 BF16 flops per
// wave; 8 * 4096 float32 flops per wave; 8 * 1024 bytes read from LDS per
// wave.  Returns the HIP status of the launch.
int knn_peak_launch(int which, int blocks, int iters, float* out, uint64_t* clk, void* stream) {
  if (blocks < 1 || iters < 1 || !out || !clk) return (int)hipErrorInvalidValue;
  const hipStream_t s = (hipStream_t)stream;
  const float seed = 1.0f / 1024.0f;
  switch (which) {
    case 0: hipLaunchKernelGGL(valu_kernel, dim3(blocks), dim3(256), 0, s, out, clk, iters, seed); break;
    case 1: hipLaunchKernelGGL(mfma_bf16_kernel, dim3(blocks), dim3(256), 0, s, out, clk, iters, seed); break;
    case 2: hipLaunchKernelGGL(mfma_f32_kernel, dim3(blocks), dim3(256), 0, s, out, clk, iters, seed); break;
    case 3: hipLaunchKernelGGL(lds_read_kernel, dim3(blocks), dim3(256), 0, s, out, clk, iters, seed); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

}  // extern "C"
