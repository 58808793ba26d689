// FP32 GEMM on the gfx950 FP32 matrix cores (v_mfma_f32_32x32x2_f32).
//
// Pattern -> hardware mapping (paper Sec. IV-B/C: splitJoinMap, the map
// lowerings and fuseReduceMap; Sec. V-C: toMem and reduceSeq):
//   A |> split(BM) |> mapWorkGroup  and  transpose(B) |> split(BN) |> mapWorkGroup
//       -> one workgroup per BM x BN tile of C (XCD-contiguous, grouped order);
//   the tile's 2 x 2 sub-tiles       -> mapLocal over the four waves;
//   split(BK) on the reduction + reduceSeq(Private)
//       -> K loop over BK-wide slabs, accumulators in registers;
//   toMem(Local) of each slab        -> LDS, double buffered: the global fetch of
//       slab i+1 is in flight while the matrix cores consume slab i;
//   zip |> map(*) |> reduce(+)       -> v_mfma_f32_32x32x2_f32 (2 k per issue);
//   join . join                      -> guarded row-major stores of C.
// Operands may be read through transpose (op T) without copies: the loader
// swaps which dimension is contiguous.  Ragged M/N/K use guarded loads that
// supply zeros (exact for the sum) and guarded stores.
#include "common.h"

namespace rise {
namespace {

constexpr int kThreads = 256;

template <int BM, int BN, int BK, bool TA, bool TB, bool VEC>
struct F32Tile {
  // LDS layout: k-major slabs, [BK][BM + pad] and [BK][BN + pad].  Transposing
  // writes (operand stored K-contiguous) use an odd pad so that the scalar
  // writes of a half-wave hit distinct banks; direct float4 writes use pad 4
  // to keep rows 16-byte aligned.
  static constexpr int PA = TA ? 4 : 1;
  static constexpr int PB = TB ? 1 : 4;
  static constexpr int LA = BM + PA;
  static constexpr int LB = BN + PB;
  static constexpr int NA = BM * BK / 4 / kThreads;  // float4 chunks per thread
  static constexpr int NB = BN * BK / 4 / kThreads;
  static_assert(NA >= 1 && NB >= 1, "tile too small for 256 threads");
  static_assert(BM * BK / 4 % kThreads == 0 && BN * BK / 4 % kThreads == 0, "tile split");
};

__device__ __forceinline__ f32x4 load4_guarded(const float* p, int64_t stride_e, int valid) {
  // valid = number of in-bounds elements (0..4) along the contiguous direction
  f32x4 v = {0.f, 0.f, 0.f, 0.f};
  if (valid > 0) v.x = p[0];
  if (valid > 1) v.y = p[stride_e];
  if (valid > 2) v.z = p[2 * stride_e];
  if (valid > 3) v.w = p[3 * stride_e];
  return v;
}

template <bool VEC>
__device__ __forceinline__ f32x4 load_chunk(const float* base, int64_t row_off, int col,
                                            int rows_ok, int cols) {
  // reads 4 consecutive elements starting at base[row_off + col] if the row is
  // in bounds; elements at col + e >= cols read as zero
  if (!rows_ok) return f32x4{0.f, 0.f, 0.f, 0.f};
  const float* p = base + row_off + col;
  int valid = cols - col;
  if (VEC && valid >= 4) return *reinterpret_cast<const f32x4*>(p);
  return load4_guarded(p, 1, valid > 4 ? 4 : valid);
}

template <int BM, int BN, int BK, bool TA, bool TB, bool VEC>
__global__ __launch_bounds__(kThreads, 2) void gemm_f32_kernel(
    float* __restrict__ C, int64_t ldc, const float* __restrict__ A, int64_t lda,
    const float* __restrict__ B, int64_t ldb, int M, int N, int K, int tiles_m, int tiles_n) {
  using T = F32Tile<BM, BN, BK, TA, TB, VEC>;
  constexpr int WM = BM / 2, WN = BN / 2;  // wave tile (2 x 2 waves)
  constexpr int TM = WM / 32, TN = WN / 32;
  static_assert(TM >= 1 && TN >= 1, "wave tile below one 32x32 block");

  __shared__ float As[2][BK][T::LA];
  __shared__ float Bs[2][BK][T::LB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave >> 1) * WM;
  const int wn0 = (wave & 1) * WN;

  int tm, tn;
  grouped_tile(xcd_contiguous(blockIdx.x, gridDim.x), tiles_m, tiles_n, 8, tm, tn);
  const int m0 = tm * BM;
  const int n0 = tn * BN;

  f32x4 ra[T::NA], rb[T::NB];

  // ---- global -> registers for slab k0 ------------------------------------
  auto fetch = [&](int k0) {
#pragma unroll
    for (int p = 0; p < T::NA; p++) {
      int c = tid + kThreads * p;
      if (!TA) {  // stored M x K, K contiguous
        int row = c / (BK / 4), kc = (c % (BK / 4)) * 4;
        ra[p] = load_chunk<VEC>(A, (int64_t)(m0 + row) * lda, k0 + kc, m0 + row < M, K);
      } else {  // stored K x M, M contiguous
        int k = c / (BM / 4), mc = (c % (BM / 4)) * 4;
        ra[p] = load_chunk<VEC>(A, (int64_t)(k0 + k) * lda, m0 + mc, k0 + k < K, M);
      }
    }
#pragma unroll
    for (int p = 0; p < T::NB; p++) {
      int c = tid + kThreads * p;
      if (!TB) {  // stored K x N, N contiguous
        int k = c / (BN / 4), nc = (c % (BN / 4)) * 4;
        rb[p] = load_chunk<VEC>(B, (int64_t)(k0 + k) * ldb, n0 + nc, k0 + k < K, N);
      } else {  // stored N x K, K contiguous
        int n = c / (BK / 4), kc = (c % (BK / 4)) * 4;
        rb[p] = load_chunk<VEC>(B, (int64_t)(n0 + n) * ldb, k0 + kc, n0 + n < N, K);
      }
    }
  };

  // ---- registers -> LDS slab buffer ----------------------------------------
  auto stash = [&](int buf) {
#pragma unroll
    for (int p = 0; p < T::NA; p++) {
      int c = tid + kThreads * p;
      if (!TA) {
        int row = c / (BK / 4), kc = (c % (BK / 4)) * 4;
        As[buf][kc + 0][row] = ra[p].x;
        As[buf][kc + 1][row] = ra[p].y;
        As[buf][kc + 2][row] = ra[p].z;
        As[buf][kc + 3][row] = ra[p].w;
      } else {
        int k = c / (BM / 4), mc = (c % (BM / 4)) * 4;
        *reinterpret_cast<f32x4*>(&As[buf][k][mc]) = ra[p];
      }
    }
#pragma unroll
    for (int p = 0; p < T::NB; p++) {
      int c = tid + kThreads * p;
      if (!TB) {
        int k = c / (BN / 4), nc = (c % (BN / 4)) * 4;
        *reinterpret_cast<f32x4*>(&Bs[buf][k][nc]) = rb[p];
      } else {
        int n = c / (BK / 4), kc = (c % (BK / 4)) * 4;
        Bs[buf][kc + 0][n] = rb[p].x;
        Bs[buf][kc + 1][n] = rb[p].y;
        Bs[buf][kc + 2][n] = rb[p].z;
        Bs[buf][kc + 3][n] = rb[p].w;
      }
    }
  };

  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; i++)
#pragma unroll
    for (int j = 0; j < TN; j++)
#pragma unroll
      for (int r = 0; r < 16; r++) acc[i][j][r] = 0.f;

  const int nk = (K + BK - 1) / BK;
  if (nk > 0) {
    fetch(0);
    stash(0);
    __syncthreads();
  }
  const int kl = lane >> 5;   // which k of the pair this lane supplies
  const int il = lane & 31;   // row of A / column of B this lane supplies
  for (int kt = 0; kt < nk; kt++) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) fetch((kt + 1) * BK);  // in flight while the slab below is consumed
#pragma unroll
    for (int s = 0; s < BK / 2; s++) {
      float a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; i++) a[i] = As[cur][2 * s + kl][wm0 + i * 32 + il];
#pragma unroll
      for (int j = 0; j < TN; j++) b[j] = Bs[cur][2 * s + kl][wn0 + j * 32 + il];
#pragma unroll
      for (int i = 0; i < TM; i++)
#pragma unroll
        for (int j = 0; j < TN; j++)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) stash(cur ^ 1);
    __syncthreads();
  }

  // ---- epilogue: D layout of a 32x32 block: lane l holds column l % 32 and
  // rows 8*(r/4) + 4*(l/32) + r%4 for r = 0..15 ------------------------------
#pragma unroll
  for (int i = 0; i < TM; i++)
#pragma unroll
    for (int j = 0; j < TN; j++) {
      const int col = n0 + wn0 + j * 32 + il;
      if (col >= N) continue;
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int row = m0 + wm0 + i * 32 + 8 * (r >> 2) + 4 * kl + (r & 3);
        if (row < M) C[(int64_t)row * ldc + col] = acc[i][j][r];
      }
    }
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
  if (t.bm == 256 && t.bn == 128) return launch_ops<256, 128, 16>(a, vec, s);
  return fail(RISE_ERR_UNSUPPORTED, "gemm_f32: unsupported tile");
}

}  // namespace rise
