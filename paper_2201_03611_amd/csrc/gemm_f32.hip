// FP32 GEMM on the gfx950 FP32 matrix cores (v_mfma_f32_32x32x2_f32): one
// workgroup per output tile, tiles visited in an XCD-contiguous, grouped order
// so that concurrently running tiles share A and B panels in their XCD's L2.
// Two schedules of the K loop (reduceSeq over split(BK) slabs, each slab staged
// in LDS: toMem(Local), paper Sec. V-B/C):
//   register-staged (tiles::gemm_f32_tile): every shape and alignment, slabs
//     fetched into registers and written to a double-buffered LDS slab;
//   asynchronous ring (gemm_f32_async_kernel, the 256 x 128 x 16 tile when K
//     is a multiple of 16 and rows are 16-byte aligned): slabs copied from
//     global memory straight into a ring of three LDS slabs two slabs ahead,
//     two workgroups per CU.
#include "common.h"
#include "tiles.h"

namespace rise {
namespace {

using tiles::kThreads;

template <int BM, int BN, int BK, bool TA, bool TB, bool VEC>
__global__ __launch_bounds__(kThreads, 2) void gemm_f32_kernel(
    float* __restrict__ C, int64_t ldc, const float* __restrict__ A, int64_t lda,
    const float* __restrict__ B, int64_t ldb, int M, int N, int K, int tiles_m, int tiles_n) {
  __shared__ float lds[tiles::F32Cfg<BM, BN, BK, TA, TB>::LDS_FLOATS];
  int tm, tn;
  grouped_tile(xcd_contiguous(blockIdx.x, gridDim.x), tiles_m, tiles_n, 8, tm, tn);
  tiles::gemm_f32_tile<BM, BN, BK, TA, TB, VEC>(C, ldc, A, lda, B, ldb, M, N, K, tm * BM, tn * BN,
                                                lds);
}

// Asynchronous-ring schedule (tiles::gemm_f32_async_tile): one workgroup per
// 256 x 128 tile, two resident per CU.
template <int BM, int BN, int STAGES, bool TA, bool TB>
__global__ __launch_bounds__(kThreads, 2) void gemm_f32_async_kernel(
    float* __restrict__ C, int64_t ldc, const float* __restrict__ A, int64_t lda,
    const float* __restrict__ B, int64_t ldb, int M, int N, int K, int tiles_m, int tiles_n) {
  __shared__ f32x4 lds[tiles::F32AsyncCfg<BM, BN, STAGES>::LDS_CHUNKS];
  int tm, tn;
  grouped_tile(xcd_contiguous(blockIdx.x, gridDim.x), tiles_m, tiles_n, 8, tm, tn);
  tiles::gemm_f32_async_tile<BM, BN, STAGES, TA, TB>(C, ldc, A, lda, B, ldb, M, N, K, tm * BM,
                                                     tn * BN, lds);
}

template <bool TA, bool TB>
rise_status launch_async(const GemmF32Args& a, hipStream_t s) {
  constexpr int BM = 256, BN = 128;
  const int tiles_m = (a.M + BM - 1) / BM, tiles_n = (a.N + BN - 1) / BN;
  hipLaunchKernelGGL((gemm_f32_async_kernel<BM, BN, 3, TA, TB>), dim3(tiles_m * tiles_n),
                     dim3(kThreads), 0, s, a.C, a.ldc, a.A, a.lda, a.B, a.ldb, a.M, a.N, a.K,
                     tiles_m, tiles_n);
  return check_launch("gemm_f32_async_kernel");
}

bool async_eligible(const GemmF32Args& a) {
  return tiles::f32_async_eligible(a.A, a.lda, a.B, a.ldb, a.M, a.N, a.K, a.ta, a.tb);
}

template <int BM, int BN, int BK, bool TA, bool TB, bool VEC>
rise_status launch_cfg(const GemmF32Args& a, hipStream_t s) {
  int tiles_m = (a.M + BM - 1) / BM, tiles_n = (a.N + BN - 1) / BN;
  dim3 grid(tiles_m * tiles_n), block(kThreads);
  hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, BK, TA, TB, VEC>), grid, block, 0, s, a.C, a.ldc,
                     a.A, a.lda, a.B, a.ldb, a.M, a.N, a.K, tiles_m, tiles_n);
  return check_launch("gemm_f32_kernel");
}

template <int BM, int BN, int BK>
rise_status launch_ops(const GemmF32Args& a, bool vec, hipStream_t s) {
  if (vec) {
    if (!a.ta && !a.tb) return launch_cfg<BM, BN, BK, false, false, true>(a, s);
    if (!a.ta && a.tb) return launch_cfg<BM, BN, BK, false, true, true>(a, s);
    if (a.ta && !a.tb) return launch_cfg<BM, BN, BK, true, false, true>(a, s);
    return launch_cfg<BM, BN, BK, true, true, true>(a, s);
  }
  if (!a.ta && !a.tb) return launch_cfg<BM, BN, BK, false, false, false>(a, s);
  if (!a.ta && a.tb) return launch_cfg<BM, BN, BK, false, true, false>(a, s);
  if (a.ta && !a.tb) return launch_cfg<BM, BN, BK, true, false, false>(a, s);
  return launch_cfg<BM, BN, BK, true, true, false>(a, s);
}

const rise_tile kTiles[] = {{128, 128, 32}, {128, 64, 32}, {64, 128, 32}, {64, 64, 32},
                            {256, 128, 16}};

}  // namespace

bool gemm_f32_tile_supported(const rise_tile& t) {
  for (const auto& k : kTiles)
    if (k.bm == t.bm && k.bn == t.bn && k.bk == t.bk) return true;
  return false;
}

int gemm_f32_tiles(rise_tile* out, int cap) {
  int n = (int)(sizeof(kTiles) / sizeof(kTiles[0]));
  for (int i = 0; out && i < n && i < cap; i++) out[i] = kTiles[i];
  return n;
}

rise_tile gemm_f32_default_tile(int M, int N, int K) {
  // Largest tile that still gives every CU at least one tile: 256 x 128 has the
  // best operand reuse from LDS (measured 123-125 TFLOP/s at 4096^3 and 8192^3).
  long t256 = (long)((M + 255) / 256) * ((N + 127) / 128);
  if (t256 >= 256) return rise_tile{256, 128, 16};
  long t128 = (long)((M + 127) / 128) * ((N + 127) / 128);
  if (t128 >= 256) return rise_tile{128, 128, 32};
  long t64 = (long)((M + 127) / 128) * ((N + 63) / 64);
  if (t64 >= 256) return rise_tile{128, 64, 32};
  return rise_tile{64, 64, 32};
}

rise_status launch_gemm_f32(const GemmF32Args& a, const rise_tile& t, hipStream_t s) {
  auto aligned = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  bool vec = aligned(a.A) && aligned(a.B) && a.lda % 4 == 0 && a.ldb % 4 == 0;
  if (t.bm == 128 && t.bn == 128) return launch_ops<128, 128, 32>(a, vec, s);
  if (t.bm == 128 && t.bn == 64) return launch_ops<128, 64, 32>(a, vec, s);
  if (t.bm == 64 && t.bn == 128) return launch_ops<64, 128, 32>(a, vec, s);
  if (t.bm == 64 && t.bn == 64) return launch_ops<64, 64, 32>(a, vec, s);
  if (t.bm == 256 && t.bn == 128) {
    if (async_eligible(a)) {
      if (!a.ta && !a.tb) return launch_async<false, false>(a, s);
      if (!a.ta && a.tb) return launch_async<false, true>(a, s);
      if (a.ta && !a.tb) return launch_async<true, false>(a, s);
      return launch_async<true, true>(a, s);
    }
    return launch_ops<256, 128, 16>(a, vec, s);
  }
  return fail(RISE_ERR_UNSUPPORTED, "gemm_f32: unsupported tile");
}

}  // namespace rise
