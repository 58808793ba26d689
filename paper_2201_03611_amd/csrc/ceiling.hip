// Measured ceilings of the machine, for the roofline fractions that sit beside
// the spec-sheet peaks: a streaming device copy (HBM) and back-to-back matrix
// instructions on every SIMD (one per arithmetic the GEMM modes use).  They
// compute nothing of the patterns; they only bound what the pattern kernels
// can reach on the GPU they run on.
#include <stdint.h>

#include <algorithm>

#include "common.h"

namespace rise {
namespace {

constexpr int kThreads = 256;

// One 16-byte chunk per thread, one pass: workgroup b copies the 4 KB block b,
// so the blocks in flight at any moment cover one dense address range in
// dispatch order (the loop only runs when the grid is capped below the block
// count).  Measured on 2 GiB: 6.16 TB/s, against 5.7-5.8 TB/s with 16 KB per
// workgroup and 4.5 TB/s for a grid-stride loop over eight workgroups per CU
// with four loads in flight per thread (the runtime's device copy: 4.5 TB/s).
__global__ __launch_bounds__(kThreads) void copy_stream(i32x4* __restrict__ dst,
                                                        const i32x4* __restrict__ src,
                                                        int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

// Each wave runs `iters` rounds of four independent matrix instructions (four
// accumulators, so consecutive instructions never wait on each other) and
// writes one value per lane so that nothing is removed by the compiler.
constexpr int kChains = 4;

__global__ __launch_bounds__(kThreads) void mfma_f32_loop(float* __restrict__ sink, int64_t iters) {
  const int lane = threadIdx.x & 63;
  float a = 1.0f + lane * 1e-3f, b = 1.0f - lane * 1e-3f;
  f32x16 acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; c++)
#pragma unroll
    for (int r = 0; r < 16; r++) acc[c][r] = 0.f;
  for (int64_t it = 0; it < iters; it++) {
#pragma unroll
    for (int c = 0; c < kChains; c++)
      acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; c++)
#pragma unroll
    for (int r = 0; r < 16; r++) s += acc[c][r];
  sink[(int64_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void mfma_bf16_loop(float* __restrict__ sink, int64_t iters) {
  const int lane = threadIdx.x & 63;
  bf16x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; e++) {
    a[e] = (__bf16)(1.0f + lane * 1e-3f);
    b[e] = (__bf16)(1.0f - e * 1e-3f);
  }
  f32x16 acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; c++)
#pragma unroll
    for (int r = 0; r < 16; r++) acc[c][r] = 0.f;
  for (int64_t it = 0; it < iters; it++) {
#pragma unroll
    for (int c = 0; c < kChains; c++)
      acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; c++)
#pragma unroll
    for (int r = 0; r < 16; r++) s += acc[c][r];
  sink[(int64_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void mfma_fp8_loop(float* __restrict__ sink, int64_t iters) {
  const int lane = threadIdx.x & 63;
  i32x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; e++) {
    a[e] = 0x38383838 + lane;  // E4M3 bytes near 1.0
    b[e] = 0x38383838 - e;
  }
  f32x16 acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; c++)
#pragma unroll
    for (int r = 0; r < 16; r++) acc[c][r] = 0.f;
  for (int64_t it = 0; it < iters; it++) {
#pragma unroll
    for (int c = 0; c < kChains; c++)
      acc[c] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, acc[c], 0, 0, 0, 127, 0, 127);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; c++)
#pragma unroll
    for (int r = 0; r < 16; r++) s += acc[c][r];
  sink[(int64_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

}  // namespace
}  // namespace rise

using namespace rise;

extern "C" {

rise_status rise_ceiling_copy(void* dst, const void* src, size_t bytes, void* stream) {
  clear_error();
  if (bytes == 0) return RISE_OK;
  if (!dst || !src) return fail(RISE_ERR_NULL, "rise_ceiling_copy: NULL pointer");
  if (bytes % 16 || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15))
    return fail(RISE_ERR_SHAPE, "rise_ceiling_copy: 16-byte aligned pointers and size");
  const uintptr_t d = (uintptr_t)dst, s = (uintptr_t)src;
  if (d < s + bytes && s < d + bytes) return fail(RISE_ERR_ALIAS, "rise_ceiling_copy: overlap");
  const int64_t n = (int64_t)(bytes / 16);
  // one pass up to 2^22 blocks (16 GiB); the grid's work-item count stays far
  // below 2^32 and larger copies stride
  const int64_t blocks = std::min<int64_t>((n + kThreads - 1) / kThreads, (int64_t)1 << 22);
  hipLaunchKernelGGL(copy_stream, dim3((unsigned)blocks), dim3(kThreads), 0, (hipStream_t)stream,
                     (i32x4*)dst, (const i32x4*)src, n);
  return check_launch("rise_ceiling_copy");
}

size_t rise_ceiling_mfma_sink_floats(void) { return (size_t)device_cu_count() * 4 * kThreads; }

rise_status rise_ceiling_mfma(rise_mode mode, int64_t iters, float* sink, size_t sink_floats,
                              double* flops, void* stream) {
  clear_error();
  if (!sink || !flops) return fail(RISE_ERR_NULL, "rise_ceiling_mfma: NULL pointer");
  if (iters < 1 || iters > ((int64_t)1 << 32))
    return fail(RISE_ERR_SHAPE, "rise_ceiling_mfma: iters in [1, 2^32]");
  if (sink_floats < rise_ceiling_mfma_sink_floats())
    return fail(RISE_ERR_WORKSPACE, "rise_ceiling_mfma: sink below rise_ceiling_mfma_sink_floats()");
  // four workgroups of four waves per CU: four waves per SIMD
  const int blocks = device_cu_count() * 4;
  const double waves = (double)blocks * (kThreads / 64);
  double per = 0;
  hipStream_t s = (hipStream_t)stream;
  switch (mode) {
    case RISE_MODE_F32:
      per = 2.0 * 32 * 32 * 2;
      hipLaunchKernelGGL(mfma_f32_loop, dim3(blocks), dim3(kThreads), 0, s, sink, iters);
      break;
    case RISE_MODE_BF16:
      per = 2.0 * 32 * 32 * 16;
      hipLaunchKernelGGL(mfma_bf16_loop, dim3(blocks), dim3(kThreads), 0, s, sink, iters);
      break;
    case RISE_MODE_FP8:
      per = 2.0 * 32 * 32 * 64;
      hipLaunchKernelGGL(mfma_fp8_loop, dim3(blocks), dim3(kThreads), 0, s, sink, iters);
      break;
    default:
      return fail(RISE_ERR_UNSUPPORTED, "rise_ceiling_mfma: modes F32, BF16 and FP8");
  }
  *flops = per * kChains * (double)iters * waves;
  return check_launch("rise_ceiling_mfma");
}

}  // extern "C"
