// Tile-level device functions shared by the one-problem kernels and the
// persistent batched kernel.  Each function computes one output tile with the
// whole 256-thread workgroup and takes its LDS through a pointer, so a kernel
// that runs several kinds of tiles can overlay them in one buffer.
#pragma once

#include "async_copy.h"
#include "common.h"

namespace rise {
namespace tiles {

constexpr int kThreads = 256;

__device__ __forceinline__ int clampi(int v, int lo, int hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// ===========================================================================
// FP32 GEMM tile (v_mfma_f32_32x32x2_f32): C[m0:m0+BM, n0:n0+BN] = A B
// ===========================================================================
template <int BM, int BN, int BK, bool TA, bool TB>
struct F32Cfg {
  // LDS layout: k-major slabs, [BK][BM + pad] and [BK][BN + pad], double buffered.
  // Transposing writes (operand stored K-contiguous) use an odd pad so that the
  // scalar writes of a half-wave hit distinct banks; direct float4 writes use
  // pad 4 to keep rows 16-byte aligned.
  static constexpr int PA = TA ? 4 : 1;
  static constexpr int PB = TB ? 1 : 4;
  static constexpr int LA = BM + PA;
  static constexpr int LB = BN + PB;
  static constexpr int NA = BM * BK / 4 / kThreads;  // float4 chunks per thread
  static constexpr int NB = BN * BK / 4 / kThreads;
  static constexpr int LDS_FLOATS = 2 * BK * (LA + LB);
  static_assert(NA >= 1 && NB >= 1, "tile too small for 256 threads");
  static_assert(BM * BK / 4 % kThreads == 0 && BN * BK / 4 % kThreads == 0, "tile split");
};

__device__ __forceinline__ f32x4 load4_guarded(const float* p, int valid) {
  // valid = number of in-bounds elements (<= 4) along the contiguous direction
  f32x4 v = {0.f, 0.f, 0.f, 0.f};
  if (valid > 0) v.x = p[0];
  if (valid > 1) v.y = p[1];
  if (valid > 2) v.z = p[2];
  if (valid > 3) v.w = p[3];
  return v;
}

template <bool VEC>
__device__ __forceinline__ f32x4 load_chunk(const float* base, int64_t row_off, int col,
                                            bool row_ok, int cols) {
  // 4 consecutive elements from base[row_off + col]; out-of-range elements read 0
  if (!row_ok) return f32x4{0.f, 0.f, 0.f, 0.f};
  const float* p = base + row_off + col;
  const int valid = cols - col;
  if (VEC && valid >= 4) return *reinterpret_cast<const f32x4*>(p);
  return load4_guarded(p, valid > 4 ? 4 : valid);
}

// Pattern -> hardware mapping (paper Sec. IV-B/C: splitJoinMap, the map lowerings
// and fuseReduceMap; Sec. V-C: toMem and reduceSeq): the workgroup owns one
// split(BM) x split(BN) tile (mapWorkGroup); its 2 x 2 sub-tiles go to the four
// waves (mapLocal); split(BK) + reduceSeq(Private) is the K loop with register
// accumulators; each slab is staged in LDS (toMem(Local)), double buffered so the
// global fetch of slab i+1 is in flight while the matrix cores consume slab i;
// zip |> map(*) |> reduce(+) is v_mfma_f32_32x32x2_f32; join . join is the
// guarded row-major store.  Operands may be read through transpose (TA, TB)
// without copies.  Ragged M/N/K: guarded loads supply zeros (exact for the
// sum), stores are guarded.
template <int BM, int BN, int BK, bool TA, bool TB, bool VEC>
__device__ __forceinline__ void gemm_f32_tile(float* __restrict__ C, int64_t ldc,
                                              const float* __restrict__ A, int64_t lda,
                                              const float* __restrict__ B, int64_t ldb, int M,
                                              int N, int K, int m0, int n0, float* lds) {
  using T = F32Cfg<BM, BN, BK, TA, TB>;
  constexpr int WM = BM / 2, WN = BN / 2;  // wave tile (2 x 2 waves)
  constexpr int TM = WM / 32, TN = WN / 32;
  static_assert(TM >= 1 && TN >= 1, "wave tile below one 32x32 block");
  auto As = reinterpret_cast<float(*)[BK][T::LA]>(lds);
  auto Bs = reinterpret_cast<float(*)[BK][T::LB]>(lds + 2 * BK * T::LA);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave >> 1) * WM;
  const int wn0 = (wave & 1) * WN;

  f32x4 ra[T::NA], rb[T::NB];
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
  const int kl = lane >> 5;  // which k of the pair this lane supplies
  const int il = lane & 31;  // row of A / column of B this lane supplies
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

  // D layout of a 32x32 block: lane l holds column l % 32 and rows
  // 8*(r/4) + 4*(l/32) + r%4 for r = 0..15
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

// ===========================================================================
// FP32 GEMM tile, asynchronous-ring schedule.
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

template <int BM, int BN, int STAGES>
struct F32AsyncCfg {
  static constexpr int SL = BM * 4 + BN * 4;   // chunks per ring stage: A slab, then B slab
  static constexpr int LDS_CHUNKS = STAGES * SL;
};

// The operands' storage allows the asynchronous ring: 16-byte chunks and
// whole slabs of 16 k (K > 0, K % 16 == 0, 16-byte aligned rows, and the rows
// along m or n whole chunks).
__host__ __device__ inline bool f32_async_eligible(const float* A, int64_t lda, const float* B,
                                                   int64_t ldb, int M, int N, int K, bool ta,
                                                   bool tb) {
  return K > 0 && K % 16 == 0 && M > 0 && N > 0 && ((uintptr_t)A & 15) == 0 &&
         ((uintptr_t)B & 15) == 0 && lda % 4 == 0 && ldb % 4 == 0 && (!ta || M % 4 == 0) &&
         (tb || N % 4 == 0);
}

// C[m0:m0+BM, n0:n0+BN] = A B with the whole 256-thread workgroup (2 x 2
// waves); lds holds F32AsyncCfg::LDS_CHUNKS 16-byte chunks.  No copy is in
// flight into lds when it returns.
template <int BM, int BN, int STAGES, bool TA, bool TB>
__device__ __forceinline__ void gemm_f32_async_tile(float* __restrict__ C, int64_t ldc,
                                                    const float* __restrict__ A, int64_t lda,
                                                    const float* __restrict__ B, int64_t ldb,
                                                    int M, int N, int K, int m0, int n0,
                                                    f32x4* lds_base) {
  using SA = AsyncSlab<BM, !TA>;
  using SB = AsyncSlab<BN, TB>;
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 32, TN = WN / 32;
  constexpr int SL = F32AsyncCfg<BM, BN, STAGES>::SL;
  constexpr int NCP = SL / kThreads;           // copies per thread per slab
  static_assert(SL % kThreads == 0 && SA::CHUNKS % 64 == 0, "a copy is all A or all B");
  static_assert(STAGES >= 3, "ring of at least three slabs");
  static_assert(TM >= 1 && TN >= 1 && BM >= 64 && BN >= 64, "tile of at least 64 x 64");
  auto lds = reinterpret_cast<f32x4(*)[SL]>(lds_base);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * WM, wn0 = (wave & 1) * WN;

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

// ===========================================================================
// BF16 GEMM tile for bf16-stored operands (v_mfma_f32_32x32x16_bf16, FP32
// accumulation): A is M x K row-major; B is either N x K (TB, K contiguous, read
// directly) or K x N (read through transpose: each 8-element chunk along N is
// scattered into the K-contiguous LDS layout).  Requires lda, ldb multiples of 8
// and 16-byte aligned bases; K ragged in units of 8 (zero-filled chunks).
// ===========================================================================
template <int BM, int BN, int BK>
struct Bf16Cfg {
  static constexpr int CH = BK / 8;  // 16-byte chunks per slab row
  // B stored K x N sits in LDS as stored: BK rows of BN values, the row pitch
  // padded by 64 bytes so the four rows one transposed read touches fall in
  // four different quarters of a 256-byte bank line
  static constexpr int BPITCH = BN * 2 + 64;  // bytes
  static constexpr int B_KN_CHUNKS = 2 * BK * BPITCH / 16;
  static constexpr int LDS_CHUNKS =
      2 * BM * CH + (2 * BN * CH > B_KN_CHUNKS ? 2 * BN * CH : B_KN_CHUNKS);
};

// Four bf16 values of one column from four consecutive LDS rows (gfx950
// ds_read_b64_tr_b16).  Within each group of 16 lanes, lane s supplies the
// address of 4 consecutive 16-bit values M[s][0..3] and lane i receives
// M[4 j + i / 4][i % 4] as element j: with lane s = 4 j + q pointing at
// columns c0 + 4 q .. c0 + 4 q + 3 of row r0 + j, lane i receives column
// c0 + i of rows r0 .. r0 + 3.
typedef short s16x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ s16x4_t lds_read_tr16(const void* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  typedef __attribute__((address_space(3))) s16x4_t lds_s16x4_t;
  return __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4_t*)p);
#else
  (void)p;
  return s16x4_t{0, 0, 0, 0};
#endif
}

// row r, 16-byte chunk c -> LDS chunk index; the XOR key changes every 16/CH rows
// so 16 consecutive rows at one logical chunk hit distinct slots of a 256-byte
// (64-bank) line
template <int CH>
__device__ __forceinline__ int swz16(int r, int c) {
  constexpr int per = 16 / CH;  // rows sharing one 256-byte bank line
  return r * CH + (c ^ ((r / per) % CH));
}

template <int BM, int BN, int BK, bool TB>
__device__ __forceinline__ void gemm_bf16_tile(float* __restrict__ C, int64_t ldc,
                                               const uint16_t* __restrict__ A, int64_t lda,
                                               const uint16_t* __restrict__ B, int64_t ldb, int M,
                                               int N, int K, int m0, int n0, i32x4* lds) {
  using T = Bf16Cfg<BM, BN, BK>;
  constexpr int CH = T::CH;
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 32, TN = WN / 32;
  constexpr int LA = BM * CH / kThreads;                // A chunks per thread
  constexpr int LB = BN * CH / kThreads;                // B chunks per thread (both layouts)
  static_assert(LA >= 1 && LB >= 1 && TM >= 1 && TN >= 1, "tile");
  i32x4* As = lds;
  i32x4* Bs = lds + 2 * BM * CH;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * WM, wn0 = (wave & 1) * WN;
  const int il = lane & 31, kh = lane >> 5;

  i32x4 ra[LA], rb[LB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < LA; q++) {
      const int c = tid + kThreads * q, r = c / CH, ch = c % CH;
      const int k = k0 + ch * 8;
      ra[q] = (m0 + r < M && k < K)
                  ? *reinterpret_cast<const i32x4*>(A + (int64_t)(m0 + r) * lda + k)
                  : i32x4{0, 0, 0, 0};
    }
#pragma unroll
    for (int q = 0; q < LB; q++) {
      const int c = tid + kThreads * q;
      if (TB) {  // B stored N x K
        const int r = c / CH, ch = c % CH, k = k0 + ch * 8;
        rb[q] = (n0 + r < N && k < K)
                    ? *reinterpret_cast<const i32x4*>(B + (int64_t)(n0 + r) * ldb + k)
                    : i32x4{0, 0, 0, 0};
      } else {  // B stored K x N: chunk = 8 consecutive n at one k
        const int k = c / (BN / 8), nc = (c % (BN / 8)) * 8;
        rb[q] = (k0 + k < K && n0 + nc < N)
                    ? *reinterpret_cast<const i32x4*>(B + (int64_t)(k0 + k) * ldb + n0 + nc)
                    : i32x4{0, 0, 0, 0};
      }
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int q = 0; q < LA; q++) {
      const int c = tid + kThreads * q;
      As[buf * BM * CH + swz16<CH>(c / CH, c % CH)] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < LB; q++) {
      const int c = tid + kThreads * q;
      if (TB) {
        Bs[buf * BN * CH + swz16<CH>(c / CH, c % CH)] = rb[q];
      } else {  // 8 consecutive n of row k, stored as they are
        const int k = c / (BN / 8), nc = (c % (BN / 8)) * 8;
        Bs[(buf * BK * T::BPITCH + k * T::BPITCH + nc * 2) / 16] = rb[q];
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
  for (int kt = 0; kt < nk; kt++) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) fetch((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK / 16; ks++) {
      const int c = 2 * ks + kh;
      bf16x8 a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; i++)
        a[i] = __builtin_bit_cast(bf16x8, As[cur * BM * CH + swz16<CH>(wm0 + 32 * i + il, c)]);
      if (TB) {
#pragma unroll
        for (int j = 0; j < TN; j++)
          b[j] = __builtin_bit_cast(bf16x8, Bs[cur * BN * CH + swz16<CH>(wn0 + 32 * j + il, c)]);
      } else {
        // lane (il, kh) needs column wn0 + 32 j + il at k = 16 ks + 8 kh .. + 7:
        // two transposed reads of four rows each (see lds_read_tr16)
        const int i16 = lane & 15, g16 = (lane >> 4) & 1;
        const char* bsb = reinterpret_cast<const char*>(Bs) + cur * BK * T::BPITCH;
        const int row = 16 * ks + 8 * kh + i16 / 4;
#pragma unroll
        for (int j = 0; j < TN; j++) {
          const int col = wn0 + 32 * j + 16 * g16 + 4 * (i16 % 4);
          const s16x4_t lo = lds_read_tr16(bsb + row * T::BPITCH + col * 2);
          const s16x4_t hi = lds_read_tr16(bsb + (row + 4) * T::BPITCH + col * 2);
          b[j] = __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
        }
      }
#pragma unroll
      for (int i = 0; i < TM; i++)
#pragma unroll
        for (int j = 0; j < TN; j++)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) stash(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < TM; i++)
#pragma unroll
    for (int j = 0; j < TN; j++) {
      const int col = n0 + wn0 + j * 32 + il;
      if (col >= N) continue;
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int row = m0 + wm0 + i * 32 + 8 * (r >> 2) + 4 * kh + (r & 3);
        if (row < M) C[(int64_t)row * ldc + col] = acc[i][j][r];
      }
    }
}

// ===========================================================================
// Stencil tile, LDS halo schedule: out rows [y0, y0+TY) x columns [x0, x0+256)
//   pad2D (clamp/zero)     -> index remapping while the halo tile is fetched;
//   slide2D                -> one (TY + 2R) x (256 + 8) halo tile staged in LDS
//                             (toMem(Local), paper Sec. V-B/C) with coalesced
//                             16-byte loads;
//   map(map(...))          -> each lane owns 4 adjacent outputs of a row and walks
//                             down TY / 4 rows, keeping the k rows of its window
//                             in registers;
//   zip |> map(*) |> reduce -> k*k FMAs per output (fuseReduceMap, Sec. IV-B),
//                             weights in scalar registers;
//   join                   -> 16-byte coalesced stores.
// ===========================================================================
constexpr int kStencilTX = 256;   // columns per tile (64 lanes x 4)
constexpr int kHalo = 4;          // LDS columns left and right of the tile
constexpr int kLChunks = (kStencilTX + 2 * kHalo) / 4;  // 16-byte chunks per LDS row

template <int K, int TY>
struct StencilCfg {
  static constexpr int R = (K - 1) / 2;
  static constexpr int ROWS = TY + 2 * R;
  static constexpr int LDS_CHUNKS = ROWS * kLChunks;
  static constexpr int PER = (LDS_CHUNKS + kThreads - 1) / kThreads;  // chunks per thread
};
template <int K, int TY>
using StencilRegs = f32x4[StencilCfg<K, TY>::PER];  // one thread's share of a halo tile

// a 16-byte vector of floats that may sit at any 4-byte boundary (gfx950 runs
// global memory in unaligned-access mode: one dwordx4 access either way)
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));

// Global -> registers: the (TY + 2R) x (256 + 8) halo tile of output rows
// [y0, y0 + TY), columns [x0, x0 + 256), with pad2D applied as index remapping.
// Chunks wholly inside the image row are one 16-byte load (aligned when VEC,
// otherwise at the row's own 4-byte alignment); edge chunks go element-wise.
template <int K, bool VEC, int TY>
__device__ __forceinline__ void stencil_fetch(StencilRegs<K, TY>& st,
                                              const float* __restrict__ in, int64_t ld_in,
                                              int H, int W, int zero_pad, int y0, int x0) {
  using Cfg = StencilCfg<K, TY>;
  const int tid = threadIdx.x;
#pragma unroll
  for (int p = 0; p < Cfg::PER; p++) {
    const int c = tid + p * kThreads;
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (c < Cfg::LDS_CHUNKS) {
      const int lr = c / kLChunks, cc = c - lr * kLChunks;
      int gy = y0 - Cfg::R + lr;
      const int gx = x0 - kHalo + cc * 4;
      bool row_ok = true;
      if (gy < 0 || gy >= H) {
        if (zero_pad) row_ok = false;
        gy = clampi(gy, 0, H - 1);
      }
      if (row_ok) {
        const float* rp = in + (int64_t)gy * ld_in;
        if (gx >= 0 && gx + 3 < W) {
          if (VEC)
            v = *reinterpret_cast<const f32x4*>(rp + gx);
          else
            v = *reinterpret_cast<const f32x4u*>(rp + gx);
        } else {
          float e[4];
#pragma unroll
          for (int q = 0; q < 4; q++) {
            const int xx = gx + q;
            if (xx < 0 || xx >= W)
              e[q] = zero_pad ? 0.f : rp[clampi(xx, 0, W - 1)];
            else
              e[q] = rp[xx];
          }
          v = f32x4{e[0], e[1], e[2], e[3]};
        }
      }
    }
    st[p] = v;
  }
}

// Registers -> LDS (row-major (TY + 2R) x 66 chunks of 16 bytes).
template <int K, int TY>
__device__ __forceinline__ void stencil_stash(const StencilRegs<K, TY>& st,
                                              f32x4* lds) {
  using Cfg = StencilCfg<K, TY>;
#pragma unroll
  for (int p = 0; p < Cfg::PER; p++) {
    const int c = threadIdx.x + p * kThreads;
    if (c < Cfg::LDS_CHUNKS) lds[c] = st[p];
  }
}

// Aligned rows (VEC and W % 4 == 0, which the callers check): every 16-byte
// chunk of the halo tile is either wholly inside or wholly outside the image
// (its columns start at a multiple of 4), so the fetch can be branch-free: each chunk is loaded from a clamped,
// always valid address, and a 2-bit mode per chunk says what pad2D makes of
// it (0 as loaded, 1 zero, 2 the first element repeated, 3 the last element
// repeated); the mode is applied when the chunk is written to LDS, so the
// loads stay in flight until then.
template <int K, int TY>
__device__ __forceinline__ void stencil_fetch_aligned(StencilRegs<K, TY>& st, uint32_t& mode,
                                                      const float* __restrict__ in, int64_t ld_in,
                                                      int H, int W, int zero_pad, int y0, int x0) {
  using Cfg = StencilCfg<K, TY>;
  static_assert(2 * Cfg::PER <= 32, "mode bits");
  uint32_t m_all = 0;
#pragma unroll
  for (int p = 0; p < Cfg::PER; p++) {
    const int c = min((int)threadIdx.x + p * kThreads, Cfg::LDS_CHUNKS - 1);
    const int lr = c / kLChunks, cc = c - lr * kLChunks;
    const int gy = y0 - Cfg::R + lr, gx = x0 - kHalo + cc * 4;
    uint32_t m = 0;
    if (gx < 0) m = 2;
    if (gx >= W) m = 3;
    if (zero_pad && (m != 0 || gy < 0 || gy >= H)) m = 1;
    const int gyc = clampi(gy, 0, H - 1), gxc = clampi(gx, 0, W - 4);
    st[p] = *reinterpret_cast<const f32x4*>(in + (int64_t)gyc * ld_in + gxc);
    m_all |= m << (2 * p);
  }
  mode = m_all;
}

template <int K, int TY>
__device__ __forceinline__ void stencil_stash_aligned(const StencilRegs<K, TY>& st, uint32_t mode,
                                                      f32x4* lds) {
  using Cfg = StencilCfg<K, TY>;
#pragma unroll
  for (int p = 0; p < Cfg::PER; p++) {
    const int c = threadIdx.x + p * kThreads;
    if (c < Cfg::LDS_CHUNKS) {
      const uint32_t m = (mode >> (2 * p)) & 3u;
      f32x4 v = st[p];
      if (m == 1) v = f32x4{0.f, 0.f, 0.f, 0.f};
      if (m == 2) v = f32x4{v.x, v.x, v.x, v.x};
      if (m == 3) v = f32x4{v.w, v.w, v.w, v.w};
      lds[c] = v;
    }
  }
}

// LDS -> k*k weighted sums.  Wave v computes output rows [y0 + v*TY/4,
// y0 + (v+1)*TY/4); lane l owns columns x0 + 4l .. x0 + 4l + 3.
// The window rows stream through registers: row j feeds every output row o
// with 0 <= j - o < k, so each output takes its k*k products in the order dy
// outer, dx inner.  ROWWISE (the default for k >= 7; the batched kernels take
// it from k = 5, to fit eight workgroups per CU) keeps that streaming in
// the schedule: the next row's LDS reads are issued before this row's FMAs,
// and empty asm statements after the FMAs take the accumulators and the LDS
// row index as operands they may change, so the FMAs must be done before them
// and the reads two rows on cannot be hoisted above them; two window rows and
// the accumulators are live instead of the whole window (k = 7 on 16-row
// tiles: 43 VGPRs instead of 124).
// EDGES (clamp padding with whole 16-byte chunks): the chunk left of column 0
// (lane 0 when `left`) and every chunk right of column lim - 1 (lim is the
// image width on the right-edge tile) read as the edge element, whatever the
// LDS tile holds there.
template <int K, int TY, bool EDGES = false, bool ROWWISE = (K >= 7)>
__device__ __forceinline__ void stencil_compute(float (&res)[TY / 4][4], const float (&wt)[K][K],
                                                const f32x4* lds, bool left = false,
                                                int lim = 0, int x = 0) {
  constexpr int R = (K - 1) / 2;
  constexpr int RW = TY / 4;      // output rows per wave
  constexpr int NR = RW + 2 * R;  // window rows
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // this lane's chunk of window row 0 (an index, so the pin below leaves the
  // pointer's LDS address space known); row j is kLChunks * j chunks further
  int base = wave * RW * kLChunks + lane;
  // LDS chunk `lane` = columns x-4..x-1, lane+1 = x..x+3, lane+2 = x+4..x+7
  auto load_row = [&](int j, f32x4 (&c)[3]) {
    const f32x4* row = lds + base + j * kLChunks;
    c[1] = row[1];
    if (R > 0) {
      c[0] = row[0];
      c[2] = row[2];
      if (EDGES) {
        if (left && lane == 0) c[0] = f32x4{c[1].x, c[1].x, c[1].x, c[1].x};
        if (x + 4 >= lim) c[2] = f32x4{c[1].w, c[1].w, c[1].w, c[1].w};
      }
    } else {
      c[0] = c[2] = c[1];
    }
  };
#pragma unroll
  for (int o = 0; o < RW; o++)
#pragma unroll
    for (int q = 0; q < 4; q++) res[o][q] = 0.f;
  f32x4 cur[3], nxt[3];
  load_row(0, cur);
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if (j + 1 < NR) load_row(j + 1, nxt);
    float win[12];
#pragma unroll
    for (int c = 0; c < 3; c++) {
      win[4 * c] = cur[c].x; win[4 * c + 1] = cur[c].y;
      win[4 * c + 2] = cur[c].z; win[4 * c + 3] = cur[c].w;
    }
#pragma unroll
    for (int o = 0; o < RW; o++) {
      const int dy = j - o;
      if (dy < 0 || dy >= K) continue;
#pragma unroll
      for (int q = 0; q < 4; q++)
#pragma unroll
        for (int dx = 0; dx < K; dx++)
          res[o][q] = fmaf(win[4 + q + dx - R], wt[dy][dx], res[o][q]);
    }
    if (ROWWISE) {  // volatile asm statements keep their order: accumulators, then the index
#pragma unroll
      for (int o = 0; o < RW; o++)
        asm volatile("" : "+v"(res[o][0]), "+v"(res[o][1]), "+v"(res[o][2]), "+v"(res[o][3]));
      asm volatile("" : "+v"(base));
    }
#pragma unroll
    for (int c = 0; c < 3; c++) cur[c] = nxt[c];
  }
}

// join: 16-byte row stores of the wave's outputs (guarded at the image edge;
// rows that are not 16-byte aligned use unaligned 16-byte stores).
// NT selects non-temporal stores (the output is not read again by this pass).
template <bool VEC, int TY, bool NT>
__device__ __forceinline__ void stencil_store(float* __restrict__ out, int64_t ld_out, int H,
                                              int W, const float (&res)[TY / 4][4], int y0,
                                              int x0) {
  constexpr int RW = TY / 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x = x0 + lane * 4;
#pragma unroll
  for (int o = 0; o < RW; o++) {
    const int y = y0 + wave * RW + o;
    if (y < H) {
      float* op = out + (int64_t)y * ld_out;
      if (x + 3 < W) {
        if (VEC) {
          const f32x4 v = f32x4{res[o][0], res[o][1], res[o][2], res[o][3]};
          if (NT)
            __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(op + x));
          else
            *reinterpret_cast<f32x4*>(op + x) = v;
        } else {
          const f32x4u v = f32x4u{res[o][0], res[o][1], res[o][2], res[o][3]};
          if (NT)
            __builtin_nontemporal_store(v, reinterpret_cast<f32x4u*>(op + x));
          else
            *reinterpret_cast<f32x4u*>(op + x) = v;
        }
      } else {
#pragma unroll
        for (int q = 0; q < 4; q++)
          if (x + q < W) op[x + q] = res[o][q];
      }
    }
  }
}

template <int K, bool VEC, int TY, bool NT, bool ROWWISE = (K >= 7)>
__device__ __forceinline__ void stencil_compute_store(float* __restrict__ out, int64_t ld_out,
                                                      int H, int W, const float (&wt)[K][K],
                                                      int y0, int x0, const f32x4* lds) {
  float res[TY / 4][4];
  stencil_compute<K, TY, false, ROWWISE>(res, wt, lds);
  stencil_store<VEC, TY, NT>(out, ld_out, H, W, res, y0, x0);
}

// SCALAR: the weight pointer is read from memory (not a kernel argument), so
// the compiler cannot tell that the loads are uniform and not overwritten while
// the kernel runs; it would read them with vector loads.  They are read through
// the constant address space instead: scalar loads straight into scalar
// registers (the weights are the same for every lane and only read).
template <int K, bool SCALAR = false>
__device__ __forceinline__ void stencil_weights(float (&wt)[K][K], const float* __restrict__ w) {
  typedef const __attribute__((address_space(4))) float cfloat;
  cfloat* cw = (cfloat*)(uintptr_t)w;
#pragma unroll
  for (int dy = 0; dy < K; dy++)
#pragma unroll
    for (int dx = 0; dx < K; dx++) wt[dy][dx] = SCALAR ? cw[dy * K + dx] : w[dy * K + dx];
}

// One tile, start to finish (fetch, stage, barrier, compute, store).
// NT: non-temporal output stores (the output is not read again soon); without
// it the output stays in the caches for a consumer that reads it next.
template <int K, bool VEC, int TY, bool NT = true, bool SCALAR_W = false,
          bool ROWWISE = (K >= 7)>
__device__ __forceinline__ void stencil_lds_tile(float* __restrict__ out, int64_t ld_out,
                                                 const float* __restrict__ in, int64_t ld_in,
                                                 int H, int W, const float* __restrict__ w,
                                                 int zero_pad, int y0, int x0, f32x4* lds) {
  StencilRegs<K, TY> st;
  using Cfg = StencilCfg<K, TY>;
  float wt[K][K];
  if (SCALAR_W) stencil_weights<K, true>(wt, w);  // scalar loads, in flight during the fetch
  if (y0 >= Cfg::R && y0 + TY + Cfg::R <= H && x0 >= kHalo && x0 + kStencilTX + kHalo <= W) {
    // interior tile: no padding, every chunk at a fixed offset from the corner
    // (16-byte aligned when VEC, otherwise at the rows' own 4-byte alignment)
    const float* corner = in + (int64_t)(y0 - Cfg::R) * ld_in + (x0 - kHalo);
#pragma unroll
    for (int p = 0; p < Cfg::PER; p++) {
      const int c = min((int)threadIdx.x + p * kThreads, Cfg::LDS_CHUNKS - 1);
      const int lr = c / kLChunks, cc = c - lr * kLChunks;
      const float* q = corner + (int64_t)lr * ld_in + 4 * cc;
      st[p] = VEC ? *reinterpret_cast<const f32x4*>(q) : f32x4(*reinterpret_cast<const f32x4u*>(q));
    }
    stencil_stash<K, TY>(st, lds);
  } else if (VEC && (W & 3) == 0) {
    uint32_t mode;
    stencil_fetch_aligned<K, TY>(st, mode, in, ld_in, H, W, zero_pad, y0, x0);
    stencil_stash_aligned<K, TY>(st, mode, lds);
  } else {
    stencil_fetch<K, VEC, TY>(st, in, ld_in, H, W, zero_pad, y0, x0);
    stencil_stash<K, TY>(st, lds);
  }
  __syncthreads();
  if (!SCALAR_W) stencil_weights<K, false>(wt, w);
  stencil_compute_store<K, VEC, TY, NT, ROWWISE>(out, ld_out, H, W, wt, y0, x0, lds);
}

}  // namespace tiles
}  // namespace rise
