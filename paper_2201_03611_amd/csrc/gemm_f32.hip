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
#include "async_copy.h"
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

// ---------------------------------------------------------------------------
// Asynchronous-ring schedule.
// Each operand's slab (16 values of k by BM or BN values of m or n) is staged
// in the orientation it is stored in, so every 16-byte chunk goes from global
// memory to LDS unchanged (global_load_lds: lane i's 16 bytes land at the
// wave-uniform base + 16 i; the swizzle below is applied on the global side by
// choosing which chunk each lane fetches):
//   rows along k (A as stored, B read through transpose): MN rows of 4 chunks;
//     chunk p of row r holds logical chunk p ^ ((r >> 2) & 3), so the 16 rows
//     one 16-lane group reads at one logical chunk fall in 16 distinct 16-byte
//     slots of a 256-byte (64-bank) LDS line;
//   rows along m or n (A read through transpose, B as stored): 16 rows of MN/4
//     chunks; chunk p of row k holds logical chunk p ^ (8 ((k >> 3) & 1)), so
//     rows k and k + 8, which the two halves of a wave read together, use
//     different banks.
// The 32x32x2 MFMA's k pair is (k, k + 8) at step t = 0..7 of a slab (lane
// half kl supplies k = 8 kl + t): the sum over a slab is the same, and a lane
// of a rows-along-k operand then reads its values of four steps with one
// 16-byte LDS read.
// Ragged M and N: rows (chunks) past the edge are fetched from the last valid
// row (chunk) and only feed outputs that are not stored.  K is a whole number
// of slabs (checked by the launcher), so no k beyond K is ever added.
template <int MN, bool ALONG_K>
struct AsyncSlab {
  static constexpr int CHUNKS = MN * 4;  // 16-byte chunks of a 16 x MN slab
  // source of slab chunk `idx` for slab 0, and the advance per slab
  __device__ static const float* src(const float* X, int64_t ld, int mn0, int mn_total, int idx,
                                     int64_t& step) {
    if (ALONG_K) {
      const int r = idx >> 2, c = (idx & 3) ^ ((r >> 2) & 3);
      const int row = min(mn0 + r, mn_total - 1);
      step = 16;
      return X + (int64_t)row * ld + 4 * c;
    }
    const int k = idx / (MN / 4), c = (idx % (MN / 4)) ^ (8 * ((k >> 3) & 1));
    const int col = min(mn0 + 4 * c, mn_total - 4);
    step = 16 * ld;
    return X + (int64_t)k * ld + col;
  }
  // values at k = 8 kl + 4 h + s (s = 0..3) of row/column r of the slab
  __device__ static f32x4 frag(const f32x4* slab, int r, int kl, int h) {
    if (ALONG_K) return slab[r * 4 + ((2 * kl + h) ^ ((r >> 2) & 3))];
    const float* f = reinterpret_cast<const float*>(slab);
    f32x4 v;
#pragma unroll
    for (int s = 0; s < 4; s++) {
      const int k = 8 * kl + 4 * h + s;
      v[s] = f[k * MN + 4 * ((r >> 2) ^ (8 * ((k >> 3) & 1))) + (r & 3)];
    }
    return v;
  }
};

template <int BM, int BN, int STAGES, bool TA, bool TB>
__global__ __launch_bounds__(kThreads, 2) void gemm_f32_async_kernel(
    float* __restrict__ C, int64_t ldc, const float* __restrict__ A, int64_t lda,
    const float* __restrict__ B, int64_t ldb, int M, int N, int K, int tiles_m, int tiles_n) {
  using SA = AsyncSlab<BM, !TA>;
  using SB = AsyncSlab<BN, TB>;
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 32, TN = WN / 32;
  constexpr int SL = SA::CHUNKS + SB::CHUNKS;  // chunks per ring stage: A slab, then B slab
  constexpr int NCP = SL / kThreads;           // copies per thread per slab
  static_assert(SL % kThreads == 0 && SA::CHUNKS % 64 == 0, "a copy is all A or all B");
  static_assert(STAGES >= 3, "ring of at least three slabs");
  __shared__ f32x4 lds[STAGES][SL];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * WM, wn0 = (wave & 1) * WN;
  int tm, tn;
  grouped_tile(xcd_contiguous(blockIdx.x, gridDim.x), tiles_m, tiles_n, 8, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;

  const float* src[NCP];
  int64_t step[NCP];
#pragma unroll
  for (int j = 0; j < NCP; j++) {
    const int slot = (wave * NCP + j) * 64 + lane;
    src[j] = slot < SA::CHUNKS ? SA::src(A, lda, m0, M, slot, step[j])
                               : SB::src(B, ldb, n0, N, slot - SA::CHUNKS, step[j]);
  }
  const int nk = K / 16;
  auto issue = [&](int kt) {  // slab min(kt, nk - 1) -> ring stage kt % STAGES
    const int64_t kk = kt < nk ? kt : nk - 1;
    const int buf = kt % STAGES;
#pragma unroll
    for (int j = 0; j < NCP; j++) async::copy16(src[j] + kk * step[j], &lds[buf][(wave * NCP + j) * 64]);
  };

  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; i++)
#pragma unroll
    for (int j = 0; j < TN; j++)
#pragma unroll
      for (int r = 0; r < 16; r++) acc[i][j][r] = 0.f;

  const int kl = lane >> 5, il = lane & 31;
#pragma unroll
  for (int st = 0; st < STAGES - 1; st++) issue(st);
  for (int kt = 0; kt < nk; kt++) {
    const int buf = kt % STAGES;
    async::wait_vmcnt<(STAGES - 2) * NCP>();  // this wave's copies of slab kt have landed
    async::wait_lgkmcnt0();                   // and its reads of slab kt - 1 are done
    async::barrier();                         // so every copy of slab kt is visible and
    issue(kt + STAGES - 1);                   // the stage of slab kt - 1 can be refilled
    const f32x4* As = &lds[buf][0];
    const f32x4* Bs = &lds[buf][SA::CHUNKS];
#pragma unroll
    for (int h = 0; h < 2; h++) {
      f32x4 a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; i++) a[i] = SA::frag(As, wm0 + 32 * i + il, kl, h);
#pragma unroll
      for (int j = 0; j < TN; j++) b[j] = SB::frag(Bs, wn0 + 32 * j + il, kl, h);
#pragma unroll
      for (int s = 0; s < 4; s++)
#pragma unroll
        for (int i = 0; i < TM; i++)
#pragma unroll
          for (int j = 0; j < TN; j++)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][s], b[j][s], acc[i][j], 0, 0, 0);
    }
  }
  async::wait_vmcnt<0>();  // the clamped copies past the last slab land before the exit

  // join . join: D layout of a 32x32 block, lane l holds column l % 32 and rows
  // 8 (r / 4) + 4 (l / 32) + r % 4; stores guarded on edge tiles only
  const bool full = m0 + BM <= M && n0 + BN <= N;
#pragma unroll
  for (int i = 0; i < TM; i++)
#pragma unroll
    for (int j = 0; j < TN; j++) {
      const int col = n0 + wn0 + j * 32 + il;
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int row = m0 + wm0 + i * 32 + 8 * (r >> 2) + 4 * kl + (r & 3);
        if (full || (row < M && col < N)) C[(int64_t)row * ldc + col] = acc[i][j][r];
      }
    }
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

// the asynchronous ring copies whole 16-byte chunks and whole slabs of 16 k
bool async_eligible(const GemmF32Args& a) {
  auto aligned = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  return a.K > 0 && a.K % 16 == 0 && a.M > 0 && a.N > 0 && aligned(a.A) && aligned(a.B) &&
         a.lda % 4 == 0 && a.ldb % 4 == 0 && (!a.ta || a.M % 4 == 0) && (a.tb || a.N % 4 == 0);
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
