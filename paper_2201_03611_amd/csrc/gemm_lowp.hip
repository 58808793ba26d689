// Reduced-precision GEMM on the gfx950 matrix cores, FP32 accumulation.
//
// The operands arrive prepared (prep.hip): A as Mp x Kp rows and B as Np x Kp
// rows of transpose(B), K contiguous and zero padded to whole tiles, so the K
// loop needs no bounds checks (zero padding adds exact zeros to the sum).
//
// Pattern -> hardware mapping (paper Sec. IV-B/C, V-C):
//   split(BM) / split(BN) + mapWorkGroup -> one workgroup per BM x BN tile of C
//   mapLocal                             -> 2 x 2 waves, each (BM/2) x (BN/2)
//   split(BK) + reduceSeq(Private)       -> K loop, accumulators in registers
//   toMem(Local)                         -> double-buffered LDS slabs; 16-byte
//                                           chunks XOR-swizzled by row so the
//                                           fragment reads are conflict free
//   zip |> map(*) |> reduce(+)           -> v_mfma_f32_32x32x16_bf16, or
//                                           v_mfma_scale_f32_32x32x64_f8f6f4
//                                           with the E8M0 block scales applied
//                                           inside the instruction
//   split compensation                   -> the extra products (hi.lo, lo.hi,
//                                           ...) accumulate into the same
//                                           registers: no extra pass over C.
#include "async_copy.h"
#include "gemm_lowp.h"

#include <type_traits>

namespace rise {
namespace {

constexpr int kThreads = 256;

// row r, 16-byte chunk c of a slab with CH chunks per row -> chunk index in LDS.
// gfx950's LDS serves a 16-lane group of ds_read_b128 from one 256-byte line of
// 64 banks; the XOR key changes every 16/CH rows so that 16 consecutive rows
// read at the same logical chunk land in 16 distinct 16-byte slots.
template <int CH>
__device__ __forceinline__ int swz(int r, int c) {
  constexpr int per = 16 / CH;  // rows sharing one 256-byte bank line
  return r * CH + (c ^ ((r / per) % CH));
}

// join . join: the wave's TM x TN blocks of 32 x 32 (D layout: lane l holds
// column l % 32, rows 8*(r/4) + 4*(l/32) + r%4), guarded only on edge tiles.
template <int TM, int TN>
__device__ __forceinline__ void store_tile(float* __restrict__ C, int64_t ldc, int M, int N,
                                           int r0, int c0, int lane, const f32x16 (&acc)[TM][TN]) {
  const int il = lane & 31, kh = lane >> 5;
  if (r0 + 32 * TM <= M && c0 + 32 * TN <= N) {
    float* base = C + (int64_t)(r0 + 4 * kh) * ldc + c0 + il;
#pragma unroll
    for (int i = 0; i < TM; i++)
#pragma unroll
      for (int j = 0; j < TN; j++)
#pragma unroll
        for (int r = 0; r < 16; r++)
          base[(int64_t)(i * 32 + 8 * (r >> 2) + (r & 3)) * ldc + j * 32] = acc[i][j][r];
    return;
  }
#pragma unroll
  for (int i = 0; i < TM; i++)
#pragma unroll
    for (int j = 0; j < TN; j++) {
      const int col = c0 + j * 32 + il;
      if (col >= N) continue;
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int row = r0 + i * 32 + 8 * (r >> 2) + 4 * kh + (r & 3);
        if (row < M) C[(int64_t)row * ldc + col] = acc[i][j][r];
      }
    }
}

template <int MODE>
struct Parts {
  static constexpr int n = MODE == RISE_MODE_BF16 ? 1 : MODE == RISE_MODE_BF16X3 ? 2 : 3;
  // kept products (part of A, part of B): parts i, j with i + j <= n - 1
  static constexpr int nprod = n == 1 ? 1 : n == 2 ? 3 : 6;
  __device__ static constexpr int pa(int q) {
    constexpr int a[6] = {0, 0, 1, 0, 1, 2};
    return a[q];
  }
  __device__ static constexpr int pb(int q) {
    constexpr int b[6] = {0, 1, 0, 2, 1, 0};
    return b[q];
  }
};

// NW waves per workgroup in an (NW/2) x 2 grid: with 8 waves two waves share
// each SIMD, so one wave's barrier and LDS waits are covered by the other's
// MFMAs (at 0.75 fragment reads per MFMA instead of 0.5, which the LDS
// bandwidth available to 8 waves sustains).
template <int BM, int BN, int BK, int MODE, int NW>
__global__ __launch_bounds__(64 * NW, 1) void packed_bf16_kernel(
    float* __restrict__ C, int64_t ldc, const uint16_t* __restrict__ Ap,
    const uint16_t* __restrict__ Bp, int M, int N, int Kp, int Mp, int Np, int tiles_m,
    int tiles_n) {
  using P = Parts<MODE>;
  constexpr int NP = P::n;
  constexpr int CH = BK / 8;                 // 16-byte chunks per slab row
  constexpr int T = 64 * NW;                 // threads
  constexpr int WM = BM / (NW / 2), WN = BN / 2;
  constexpr int TM = WM / 32, TN = WN / 32;
  constexpr int LA = BM * BK / 8 / T;        // chunks per thread per part
  constexpr int LB = BN * BK / 8 / T;
  static_assert(LA >= 1 && LB >= 1, "tile too small");

  __shared__ i32x4 As[2][NP][BM * CH];
  __shared__ i32x4 Bs[2][NP][BN * CH];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * WM, wn0 = (wave & 1) * WN;
  int tm, tn;
  grouped_tile(xcd_contiguous(blockIdx.x, gridDim.x), tiles_m, tiles_n, 4, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int64_t planeA = (int64_t)Mp * Kp, planeB = (int64_t)Np * Kp;

  // NSET register sets of the global prefetch.  With two (the 128 x 128 tiles,
  // which have the registers for it) slab kt+2 is requested while slab kt+1,
  // requested one slab earlier, is written to LDS, so every global load has
  // about two slabs of MFMA time to arrive; the 256 x 256 tiles keep one set.
  constexpr int NSET = BM >= 256 ? 1 : 2;
  static_assert(NW == 4 || NW == 8, "wave grid");
  i32x4 ra[NSET][NP][LA], rb[NSET][NP][LB];
  auto fetch = [&](int set, int k0) {
#pragma unroll
    for (int p = 0; p < NP; p++) {
#pragma unroll
      for (int q = 0; q < LA; q++) {
        int c = tid + T * q, r = c / CH, ch = c % CH;
        ra[set][p][q] = *reinterpret_cast<const i32x4*>(Ap + p * planeA + (int64_t)(m0 + r) * Kp + k0 + ch * 8);
      }
#pragma unroll
      for (int q = 0; q < LB; q++) {
        int c = tid + T * q, r = c / CH, ch = c % CH;
        rb[set][p][q] = *reinterpret_cast<const i32x4*>(Bp + p * planeB + (int64_t)(n0 + r) * Kp + k0 + ch * 8);
      }
    }
  };
  auto stash = [&](int set, int buf) {
#pragma unroll
    for (int p = 0; p < NP; p++) {
#pragma unroll
      for (int q = 0; q < LA; q++) {
        int c = tid + T * q;
        As[buf][p][swz<CH>(c / CH, c % CH)] = ra[set][p][q];
      }
#pragma unroll
      for (int q = 0; q < LB; q++) {
        int c = tid + T * q;
        Bs[buf][p][swz<CH>(c / CH, c % CH)] = rb[set][p][q];
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

  // Software pipeline of one wave: the fragments of k-step ks+1 are read from
  // LDS while the matrix cores work on step ks, and on the last step of a slab
  // the prefetched next slab is written to the other LDS buffer instead.  The
  // sched_group_barrier hints interleave one LDS instruction after each MFMA so
  // the LDS traffic hides under the 32-cycle MFMAs.
  constexpr int KS = BK / 16;                     // k-steps per slab
  constexpr int NMF = P::nprod * TM * TN;         // MFMAs per k-step
  constexpr int NRD = NP * (TM + TN);             // fragment reads per k-step
  constexpr int NWR = NP * (LA + LB);             // LDS writes of one slab
  const int il = lane & 31, kh = lane >> 5;
  bf16x8 fa[2][NP][TM], fb[2][NP][TN];
  auto read_frags = [&](int buf, int ks, int slot) {
    const int c = 2 * ks + kh;  // this lane's 8 consecutive k within the slab
#pragma unroll
    for (int p = 0; p < NP; p++) {
#pragma unroll
      for (int i = 0; i < TM; i++)
        fa[slot][p][i] = __builtin_bit_cast(bf16x8, As[buf][p][swz<CH>(wm0 + 32 * i + il, c)]);
#pragma unroll
      for (int j = 0; j < TN; j++)
        fb[slot][p][j] = __builtin_bit_cast(bf16x8, Bs[buf][p][swz<CH>(wn0 + 32 * j + il, c)]);
    }
  };
  auto mfmas = [&](int slot) {
#pragma unroll
    for (int q = P::nprod - 1; q >= 0; q--)  // small products first
#pragma unroll
      for (int i = 0; i < TM; i++)
#pragma unroll
        for (int j = 0; j < TN; j++)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[slot][P::pa(q)][i],
                                                              fb[slot][P::pb(q)][j], acc[i][j], 0,
                                                              0, 0);
  };

  const int nk = Kp / BK;
  auto last = [&](int k) { return k < nk ? k : nk - 1; };  // clamp prefetches in bounds
  // one slab: prefetch slab kt+2 into register set `set`, consume LDS buffer kt & 1,
  // and on the last k-step write slab kt+1 (register set set ^ 1) to the other buffer
  auto slab = [&](int kt, int set) {
    const int cur = kt & 1;
    fetch(set, last(kt + NSET) * BK);
    __builtin_amdgcn_sched_group_barrier(0x020, NP * (LA + LB), 0);  // global loads first
#pragma unroll
    for (int ks = 0; ks < KS; ks++) {
      const int slot = ks & 1;
      if (ks + 1 < KS) {
        read_frags(cur, ks + 1, slot ^ 1);
        mfmas(slot);
#pragma unroll
        for (int t = 0; t < (NRD < NMF ? NRD : NMF); t++) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
        }
      } else {
        stash(NSET == 2 ? set ^ 1 : 0, cur ^ 1);
        mfmas(slot);
#pragma unroll
        for (int t = 0; t < (NWR < NMF ? NWR : NMF); t++) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
          __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // one LDS write
        }
      }
    }
    __syncthreads();
    if (kt + 1 < nk) read_frags(cur ^ 1, 0, 0);
  };
  if (nk > 0) {
    fetch(0, 0);
    if (NSET == 2) fetch(NSET - 1, last(1) * BK);
    stash(0, 0);
    __syncthreads();
    read_frags(0, 0, 0);
  }
  // slab kt uses register set kt % NSET for its prefetch: unrolled by two so the
  // register sets are indexed statically
  int kt = 0;
  for (; kt + 1 < nk; kt += 2) {
    slab(kt, 0);
    slab(kt + 1, NSET - 1);
  }
  if (kt < nk) slab(kt, 0);

  store_tile<TM, TN>(C, ldc, M, N, m0 + wm0, n0 + wn0, lane, acc);
}

// FP8 E4M3 with E8M0 block scales (32 elements along K per scale).
template <int BM, int BN>
__global__ __launch_bounds__(kThreads, 1) void packed_fp8_kernel(
    float* __restrict__ C, int64_t ldc, const uint8_t* __restrict__ Ap,
    const uint8_t* __restrict__ Bp, int M, int N, int Kp, int Mp, int Np, int tiles_m,
    int tiles_n) {
  constexpr int BK = 128;                      // bytes = elements per slab row
  constexpr int CH = BK / 16;                  // 8 chunks
  constexpr int SB = BK / 32;                  // scale bytes per slab row
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 32, TN = WN / 32;
  constexpr int LA = BM * CH / kThreads, LB = BN * CH / kThreads;
  static_assert(BM <= kThreads && BN <= kThreads, "one scale word per thread");

  __shared__ i32x4 As[2][BM * CH];
  __shared__ i32x4 Bs[2][BN * CH];
  __shared__ uint32_t Asc[2][BM];  // SB = 4 scale bytes of a row packed in one word
  __shared__ uint32_t Bsc[2][BN];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * WM, wn0 = (wave & 1) * WN;
  int tm, tn;
  grouped_tile(xcd_contiguous(blockIdx.x, gridDim.x), tiles_m, tiles_n, 4, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const uint8_t* As_g = Ap + (int64_t)Mp * Kp;  // scale planes follow the code planes
  const uint8_t* Bs_g = Bp + (int64_t)Np * Kp;
  const int sstride = Kp / 32;

  i32x4 ra[LA], rb[LB];
  uint32_t sa = 0, sb = 0;
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < LA; q++) {
      int c = tid + kThreads * q, r = c / CH, ch = c % CH;
      ra[q] = *reinterpret_cast<const i32x4*>(Ap + (int64_t)(m0 + r) * Kp + k0 + ch * 16);
    }
#pragma unroll
    for (int q = 0; q < LB; q++) {
      int c = tid + kThreads * q, r = c / CH, ch = c % CH;
      rb[q] = *reinterpret_cast<const i32x4*>(Bp + (int64_t)(n0 + r) * Kp + k0 + ch * 16);
    }
    if (tid < BM) sa = *reinterpret_cast<const uint32_t*>(As_g + (int64_t)(m0 + tid) * sstride + k0 / 32);
    if (tid < BN) sb = *reinterpret_cast<const uint32_t*>(Bs_g + (int64_t)(n0 + tid) * sstride + k0 / 32);
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int q = 0; q < LA; q++) {
      int c = tid + kThreads * q;
      As[buf][swz<CH>(c / CH, c % CH)] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < LB; q++) {
      int c = tid + kThreads * q;
      Bs[buf][swz<CH>(c / CH, c % CH)] = rb[q];
    }
    if (tid < BM) Asc[buf][tid] = sa;
    if (tid < BN) Bsc[buf][tid] = sb;
  };

  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; i++)
#pragma unroll
    for (int j = 0; j < TN; j++)
#pragma unroll
      for (int r = 0; r < 16; r++) acc[i][j][r] = 0.f;

  const int nk = Kp / BK;
  if (nk > 0) {
    fetch(0);
    stash(0);
    __syncthreads();
  }
  const int il = lane & 31, kh = lane >> 5;
  for (int kt = 0; kt < nk; kt++) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) fetch((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK / 64; ks++) {
      // Operand registers 0-3 of both lane halves form scale block 2*ks (the
      // scale comes from the lane in half 0), registers 4-7 form block 2*ks+1
      // (scale from half 1).  So half kh takes 16-byte chunk kh of each of the
      // two 32-byte blocks, and supplies the scale of block 2*ks + kh.
      const int c0 = 4 * ks + kh, c1 = 4 * ks + 2 + kh;
      const int sh = 8 * (2 * ks + kh);
      i32x8 a[TM], b[TN];
      int xa[TM], xb[TN];
#pragma unroll
      for (int i = 0; i < TM; i++) {
        const int r = wm0 + 32 * i + il;
        i32x4 lo = As[cur][swz<CH>(r, c0)], hi = As[cur][swz<CH>(r, c1)];
        a[i] = i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
        xa[i] = (int)((Asc[cur][r] >> sh) & 0xffu);
      }
#pragma unroll
      for (int j = 0; j < TN; j++) {
        const int r = wn0 + 32 * j + il;
        i32x4 lo = Bs[cur][swz<CH>(r, c0)], hi = Bs[cur][swz<CH>(r, c1)];
        b[j] = i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
        xb[j] = (int)((Bsc[cur][r] >> sh) & 0xffu);
      }
#pragma unroll
      for (int i = 0; i < TM; i++)
#pragma unroll
        for (int j = 0; j < TN; j++)
          acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[i], b[j], acc[i][j], 0, 0,
                                                                     0, xa[i], 0, xb[j]);
    }
    if (more) stash(cur ^ 1);
    __syncthreads();
  }

  store_tile<TM, TN>(C, ldc, M, N, m0 + wm0, n0 + wn0, lane, acc);
}

// ---------------------------------------------------------------------------
// Asynchronous slab copies (gfx950 global_load_lds: lane i's bytes land at the
// wave-uniform LDS base + size * i, no registers hold data in transit).  Copy
// completion is tracked only by vmcnt, so waits are explicit, and barriers are
// bare s_barrier (a workgroup fence would wait for every copy in flight).
// (the instruction text exists only in the device pass)
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt field is 6 bits");
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
#endif
}
__device__ __forceinline__ void wait_lgkmcnt0() {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#endif
}
__device__ __forceinline__ void raw_barrier() {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("s_barrier" ::: "memory");
#endif
}
// 16 (4) bytes per lane, global -> LDS at lds_base + 16 (4) * lane
// (lds_base wave-uniform), through the inline-asm copies of async_copy.h
__device__ __forceinline__ void copy16_to_lds(const void* src, void* lds_base) {
  async::copy16(src, lds_base);
}
__device__ __forceinline__ void copy4_to_lds(const void* src, void* lds_base) {
  async::copy4(src, lds_base);
}

// ---------------------------------------------------------------------------
// 256 x 256 tiles over K-blocked operands, every format.  A K-blocked part
// holds the K block b of row r (KBB bytes: 64 FP8 codes, 32 bf16 values, or 16
// for the split formats) at (b * rows + r) * KBB, so the blocks of consecutive
// rows are contiguous (an FP8 row's two scale bytes of a block sit together in
// the scale plane).  The register staging of the row-major kernels does not
// fit beside the 256 accumulator registers of a 256 x 256 tile, so each slab
// (one K block of the tile's 512 rows in every part, 32 KB, or 48 KB for
// bf16x6, plus 1 KB of FP8 scales) goes from global memory straight into LDS
// with global_load_lds: a copy instruction moves 1 KB of consecutive rows,
// i.e. whole 128-byte lines, which a row-major slab this thin would fetch in
// pieces.  Slabs flow through a ring of STAGES LDS buffers:
//   wait for this wave's copies of slab kt+1 and its fragment reads of slab kt;
//   barrier (slab kt+1 visible; every wave holds slab kt in registers);
//   copy slab kt+STAGES into the buffer of slab kt, read slab kt+1's
//   fragments and run slab kt's MFMAs, the copies and reads interleaved
//   between MFMAs,
// so a copy has STAGES - 1 slabs of MFMA time to land and fragment reads never
// stall the matrix core.  The copies are the inline-asm ones of async_copy.h,
// so the compiler adds no wait for them in front of the fragment reads (issued
// through the builtin into two LDS arrays, codes and scales, they drew a
// vmcnt(0) before every slab's first read).
// Per accumulator the products run in the same order as in the row-major
// kernels (k-steps in order; split products small first), so results match
// them bit for bit.
__device__ __forceinline__ void wait_lgkmcnt0_visible() {
  // s_waitcnt lgkmcnt(0) (vmcnt and expcnt fields at their maxima) as an
  // instruction the compiler's own wait insertion accounts for
  __builtin_amdgcn_s_waitcnt(0xC07F);
}

template <int MODE>
struct KBlock {
  static constexpr bool fp8 = MODE == RISE_MODE_FP8;
  static constexpr int parts = fp8 ? 1 : Parts<MODE>::n;
  static constexpr int nprod = fp8 ? 1 : Parts<MODE>::nprod;
  static constexpr int bytes = parts == 1 ? 64 : 32;  // KBB: bytes of a K block per part
  static constexpr int elems = bytes / (fp8 ? 1 : 2);  // K per slab
  static constexpr int ksteps = fp8 ? 1 : elems / 16;  // MFMA k-steps per slab
  static constexpr int stages = parts == 3 ? 3 : 4;
};

template <int MODE>
__global__ __launch_bounds__(kThreads, 1) void packed_kblock_kernel(
    float* __restrict__ C, int64_t ldc, const void* __restrict__ Apv,
    const void* __restrict__ Bpv, int M, int N, int Kp, int Mp, int Np, int tiles_m,
    int tiles_n) {
  using KC = KBlock<MODE>;
  constexpr bool FP8 = KC::fp8;
  constexpr int NP = KC::parts, KBB = KC::bytes, KS = KC::ksteps, STAGES = KC::stages;
  constexpr int ES = FP8 ? 1 : 2;             // bytes per element
  constexpr int BM = 256, BN = 256, CH = KBB / 16;
  constexpr int ROWS = BM + BN;
  constexpr int CODE_SLOTS = ROWS * CH;       // 16-byte chunks of one part of a buffer
  constexpr int NCP = CODE_SLOTS / kThreads;  // copies per thread per part per slab
  constexpr int NPS = NP * NCP + (FP8 ? 1 : 0);  // copies per wave per slab
  constexpr int SCW = FP8 ? ROWS * 2 / 4 : 0; // scale words of one slab
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 32, TN = WN / 32;
  static_assert(!FP8 || SCW == kThreads, "one scale word per thread");
  static_assert((STAGES - 1) * NPS < 64, "vmcnt field");
  static_assert(NCP % 2 == 0, "a wave's copies stay within A or within B rows");

  __shared__ i32x4 lds[STAGES * NP * CODE_SLOTS + STAGES * SCW / 4];
  i32x4* const codes = lds;
  uint32_t* const scale_words = reinterpret_cast<uint32_t*>(lds + STAGES * NP * CODE_SLOTS);
  const uint8_t* const scale_bytes = reinterpret_cast<const uint8_t*>(scale_words);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * WM, wn0 = (wave & 1) * WN;
  int tm, tn;
  grouped_tile(xcd_contiguous(blockIdx.x, gridDim.x), tiles_m, tiles_n, 4, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;

  // waves 0, 1 copy the A rows of a slab, waves 2, 3 the B rows; slot
  // (wave * NCP + q) * 64 + lane of a part's buffer holds row slot / CH,
  // physical chunk slot % CH, i.e. the logical chunk given by the swizzle's
  // inverse
  const bool isB = wave >= 2;
  const int64_t prows = isB ? Np : Mp;
  const uint8_t* const plane = reinterpret_cast<const uint8_t*>(isB ? Bpv : Apv);
  const int64_t part_bytes = prows * Kp * ES;
  const uint8_t* const splane = plane + part_bytes;  // FP8 scales follow the codes
  const int64_t row0 = isB ? n0 : m0;
  int coff[NCP];  // bytes
#pragma unroll
  for (int q = 0; q < NCP; q++) {
    const int slot = (wave * NCP + q) * 64 + lane;
    const int r = slot / CH, pc = slot % CH;
    const int c = pc ^ ((r / (16 / CH)) % CH);
    coff[q] = (isB ? r - BM : r) * KBB + c * 16;
  }
  // FP8 scale word tid of a slab: bytes 4 tid .. 4 tid + 3 of the A rows'
  // pairs (words 0-127) then the B rows' pairs (words 128-255)
  const int soff = (isB ? tid - kThreads / 2 : tid) * 4;

  const int nk = Kp / KC::elems;
  auto issue = [&](int kt) {  // slab min(kt, nk - 1) -> buffer kt % STAGES
    const int64_t k = kt < nk ? kt : nk - 1;
    const int buf = kt % STAGES;
    const uint8_t* cb = plane + (k * prows + row0) * KBB;
#pragma unroll
    for (int p = 0; p < NP; p++)
#pragma unroll
      for (int q = 0; q < NCP; q++)
        copy16_to_lds(cb + p * part_bytes + coff[q],
                      codes + (buf * NP + p) * CODE_SLOTS + (wave * NCP + q) * 64);
    if constexpr (FP8)
      copy4_to_lds(splane + (k * prows + row0) * 2 + soff, scale_words + buf * SCW + wave * 64);
  };

  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; i++)
#pragma unroll
    for (int j = 0; j < TN; j++)
#pragma unroll
      for (int r = 0; r < 16; r++) acc[i][j][r] = 0.f;

  // fragments of one slab, two register sets alternating by slab.  FP8: the
  // operand and scale layout of packed_fp8_kernel's k-step 0; bf16: k-step s
  // of the slab takes chunk 2 s + kh (lanes 0-31 k 0-7, lanes 32-63 k 8-15)
  const int il = lane & 31, kh = lane >> 5;
  i32x8 fa8[2][TM], fb8[2][TN];
  int xa[2][TM], xb[2][TN];
  bf16x8 fa16[2][NP][KS][TM], fb16[2][NP][KS][TN];
  auto reads = [&](int buf, int set) {
#pragma unroll
    for (int p = 0; p < NP; p++) {
      const i32x4* cb = codes + (buf * NP + p) * CODE_SLOTS;
#pragma unroll
      for (int i = 0; i < TM; i++) {
        const int r = wm0 + 32 * i + il;
        if constexpr (FP8) {
          const i32x4 lo = cb[swz<CH>(r, kh)], hi = cb[swz<CH>(r, 2 + kh)];
          fa8[set][i] = i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
          xa[set][i] = scale_bytes[buf * SCW * 4 + r * 2 + kh];
        } else {
#pragma unroll
          for (int ks = 0; ks < KS; ks++)
            fa16[set][p][ks][i] = __builtin_bit_cast(bf16x8, cb[swz<CH>(r, 2 * ks + kh)]);
        }
      }
#pragma unroll
      for (int j = 0; j < TN; j++) {
        const int r = BM + wn0 + 32 * j + il;
        if constexpr (FP8) {
          const i32x4 lo = cb[swz<CH>(r, kh)], hi = cb[swz<CH>(r, 2 + kh)];
          fb8[set][j] = i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
          xb[set][j] = scale_bytes[buf * SCW * 4 + r * 2 + kh];
        } else {
#pragma unroll
          for (int ks = 0; ks < KS; ks++)
            fb16[set][p][ks][j] = __builtin_bit_cast(bf16x8, cb[swz<CH>(r, 2 * ks + kh)]);
        }
      }
    }
  };
  auto step = [&](int kt, auto set_tag) {
    constexpr int set = decltype(set_tag)::value;
    wait_vmcnt<(STAGES - 2) * NPS>();  // this wave's copies of slab kt+1 have landed
    wait_lgkmcnt0_visible();           // and its fragments of slab kt are in registers
    __builtin_amdgcn_sched_barrier(0);
    raw_barrier();
    __builtin_amdgcn_sched_barrier(0);
    issue(kt + STAGES);                // refills the buffer of slab kt
    reads((kt + 1) % STAGES, set ^ 1);  // slab kt+1 (past the end: a clamped copy, unused)
    if constexpr (FP8) {
#pragma unroll
      for (int i = 0; i < TM; i++)
#pragma unroll
        for (int j = 0; j < TN; j++)
          acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
              fa8[set][i], fb8[set][j], acc[i][j], 0, 0, 0, xa[set][i], 0, xb[set][j]);
    } else {
      using P = Parts<MODE>;
#pragma unroll
      for (int ks = 0; ks < KS; ks++)
#pragma unroll
        for (int q = P::nprod - 1; q >= 0; q--)  // small products first
#pragma unroll
          for (int i = 0; i < TM; i++)
#pragma unroll
            for (int j = 0; j < TN; j++)
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                  fa16[set][P::pa(q)][ks][i], fb16[set][P::pb(q)][ks][j], acc[i][j], 0, 0, 0);
    }
    // one MFMA, then a copy while copies remain, then the fragment reads
    constexpr int NMF = KS * KC::nprod * TM * TN;
    constexpr int NRD = FP8 ? 3 * (TM + TN) : NP * KS * (TM + TN);
    constexpr int RPM = (NRD + NMF - 1) / NMF;
#pragma unroll
    for (int t = 0; t < NMF; t++) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      if (t < NPS) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
      if (t * RPM < NRD) __builtin_amdgcn_sched_group_barrier(0x100, RPM, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
  };

  if (nk > 0) {
#pragma unroll
    for (int st = 0; st < STAGES; st++) issue(st);
    wait_vmcnt<(STAGES - 1) * NPS>();  // slab 0 has landed
    __builtin_amdgcn_sched_barrier(0);
    raw_barrier();
    __builtin_amdgcn_sched_barrier(0);
    reads(0, 0);
  }
  int kt = 0;
  for (; kt + 1 < nk; kt += 2) {
    step(kt, std::integral_constant<int, 0>{});
    step(kt + 1, std::integral_constant<int, 1>{});
  }
  if (kt < nk) step(kt, std::integral_constant<int, 0>{});
  wait_vmcnt<0>();  // the clamped tail copies land before the workgroup ends
  wait_lgkmcnt0_visible();

  store_tile<TM, TN>(C, ldc, M, N, m0 + wm0, n0 + wn0, lane, acc);
}

struct TileRow {
  rise_mode mode;
  rise_tile t;
};
const TileRow kTiles[] = {
    {RISE_MODE_BF16, {256, 256, 64}},   {RISE_MODE_BF16, {128, 128, 64}},
    {RISE_MODE_BF16, {256, 256, 32}},   {RISE_MODE_BF16X3, {256, 256, 16}},
    {RISE_MODE_BF16X3, {256, 256, 32}}, {RISE_MODE_BF16X3, {128, 128, 32}},
    {RISE_MODE_BF16X6, {256, 256, 16}}, {RISE_MODE_BF16X6, {128, 128, 16}},
    {RISE_MODE_FP8, {256, 256, 128}},   {RISE_MODE_FP8, {128, 128, 128}},
};

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

constexpr int kBf16Waves256 = 4;  // waves per workgroup of the 256 x 256 tiles

template <int BM, int BN, int BK, int MODE>
rise_status launch_bf16(const PackedGemm& g, hipStream_t s) {
  int tiles_m = g.Mp / BM, tiles_n = g.Np / BN;
  constexpr int NW = BM >= 256 ? kBf16Waves256 : 4;
  hipLaunchKernelGGL((packed_bf16_kernel<BM, BN, BK, MODE, NW>), dim3(tiles_m * tiles_n),
                     dim3(64 * NW), 0, s, g.C, g.ldc, (const uint16_t*)g.Ap,
                     (const uint16_t*)g.Bp, g.M, g.N, g.Kp, g.Mp, g.Np, tiles_m, tiles_n);
  return check_launch("packed_bf16_kernel");
}

template <int MODE>
rise_status launch_kblock(const PackedGemm& g, hipStream_t s) {
  int tiles_m = g.Mp / 256, tiles_n = g.Np / 256;
  hipLaunchKernelGGL(packed_kblock_kernel<MODE>, dim3(tiles_m * tiles_n), dim3(kThreads), 0, s,
                     g.C, g.ldc, g.Ap, g.Bp, g.M, g.N, g.Kp, g.Mp, g.Np, tiles_m, tiles_n);
  return check_launch("packed_kblock_kernel");
}

template <int BM, int BN>
rise_status launch_fp8(const PackedGemm& g, hipStream_t s) {
  int tiles_m = g.Mp / BM, tiles_n = g.Np / BN;
  hipLaunchKernelGGL((packed_fp8_kernel<BM, BN>), dim3(tiles_m * tiles_n), dim3(kThreads), 0, s,
                     g.C, g.ldc, (const uint8_t*)g.Ap, (const uint8_t*)g.Bp, g.M, g.N, g.Kp, g.Mp,
                     g.Np, tiles_m, tiles_n);
  return check_launch("packed_fp8_kernel");
}

}  // namespace

int gemm_lowp_tiles(rise_mode mode, rise_tile* out, int cap) {
  int n = 0;
  for (const auto& r : kTiles)
    if (r.mode == mode) {
      if (out && n < cap) out[n] = r.t;
      n++;
    }
  return n;
}

bool gemm_lowp_tile_supported(rise_mode mode, const rise_tile& t) {
  for (const auto& r : kTiles)
    if (r.mode == mode && r.t.bm == t.bm && r.t.bn == t.bn && r.t.bk == t.bk) return true;
  return false;
}

rise_tile gemm_lowp_default_tile(rise_mode mode, int M, int N, int K) {
  // 256 x 256 when it still gives every CU a tile, else 128 x 128; at 256 x
  // 256 the K-blocked kernel where it is the faster one (measured at 8192^3
  // with preparation: bf16 1.08-1.24 ms against 1.12-1.32 for the row-major
  // 256 x 256 x 64 tile, bf16x3 2.71-2.91 against 3.12-3.18 ms for 256 x 256
  // x 32, bf16x6 5.06 against 6.78 ms for the row-major 256 x 256 x 16 tile,
  // fp8 0.62 against 0.83 ms for 128 x 128)
  long tiles_big = (long)((M + 255) / 256) * ((N + 255) / 256);
  const bool big = tiles_big >= 256;
  switch (mode) {
    case RISE_MODE_BF16: return big ? rise_tile{256, 256, 32} : rise_tile{128, 128, 64};
    case RISE_MODE_BF16X3: return big ? rise_tile{256, 256, 16} : rise_tile{128, 128, 32};
    case RISE_MODE_BF16X6: return big ? rise_tile{256, 256, 16} : rise_tile{128, 128, 16};
    default: return big ? rise_tile{256, 256, 128} : rise_tile{128, 128, 128};
  }
}

size_t gemm_lowp_workspace(int M, int N, int K, rise_mode mode, const rise_tile& t) {
  int64_t Mp = round_up(M, t.bm), Np = round_up(N, t.bn), Kp = round_up(K, t.bk);
  return (size_t)round_up((int64_t)prep_bytes(Mp, Kp, mode), 256) + prep_bytes(Np, Kp, mode);
}

// K-blocked layout (K per block) of the tiles packed_kblock_kernel runs
int packed_kblock(rise_mode mode, const rise_tile& t) {
  if (mode == RISE_MODE_FP8 && t.bm == 256) return KBlock<RISE_MODE_FP8>::elems;
  if (mode == RISE_MODE_BF16 && t.bm == 256 && t.bk == 32) return KBlock<RISE_MODE_BF16>::elems;
  if (mode == RISE_MODE_BF16X3 && t.bm == 256 && t.bk == 16)
    return KBlock<RISE_MODE_BF16X3>::elems;
  if (mode == RISE_MODE_BF16X6 && t.bm == 256 && t.bk == 16)
    return KBlock<RISE_MODE_BF16X6>::elems;
  return 0;
}

rise_status launch_packed_gemm(const PackedGemm& g, const rise_tile& t, hipStream_t s) {
  if (g.kblock != packed_kblock(g.mode, t))
    return fail(RISE_ERR_UNSUPPORTED, "packed gemm: operand layout does not match the tile");
  switch (g.mode) {
    case RISE_MODE_BF16:
      if (t.bm == 256 && t.bk == 32) return launch_kblock<RISE_MODE_BF16>(g, s);
      if (t.bm == 256) return launch_bf16<256, 256, 64, RISE_MODE_BF16>(g, s);
      return launch_bf16<128, 128, 64, RISE_MODE_BF16>(g, s);
    case RISE_MODE_BF16X3:
      if (t.bm == 256 && t.bk == 16) return launch_kblock<RISE_MODE_BF16X3>(g, s);
      if (t.bm == 256) return launch_bf16<256, 256, 32, RISE_MODE_BF16X3>(g, s);
      return launch_bf16<128, 128, 32, RISE_MODE_BF16X3>(g, s);
    case RISE_MODE_BF16X6:
      if (t.bm == 256) return launch_kblock<RISE_MODE_BF16X6>(g, s);
      return launch_bf16<128, 128, 16, RISE_MODE_BF16X6>(g, s);
    case RISE_MODE_FP8:
      if (t.bm == 256) return launch_kblock<RISE_MODE_FP8>(g, s);
      return launch_fp8<128, 128>(g, s);
    default:
      return fail(RISE_ERR_UNSUPPORTED, "packed gemm: mode");
  }
}

rise_status launch_gemm_lowp(const GemmLowpArgs& a, const rise_tile& t, void* ws, hipStream_t s) {
  const int64_t Mp = round_up(a.M, t.bm), Np = round_up(a.N, t.bn), Kp = round_up(a.K, t.bk);
  uint8_t* wsA = (uint8_t*)ws;
  uint8_t* wsB = wsA + round_up((int64_t)prep_bytes(Mp, Kp, a.mode), 256);
  // A: M vectors of length K; B: N vectors of length K (columns of B)
  const int kb = packed_kblock(a.mode, t);
  PrepArgs pa{wsA, Mp, Kp, a.A, a.M, a.K, a.ta ? 1 : a.lda, a.ta ? a.lda : 1, a.mode,
              a.tA == RISE_BF16, kb};
  PrepArgs pb{wsB, Np, Kp, a.B, a.N, a.K, a.tb ? a.ldb : 1, a.tb ? 1 : a.ldb, a.mode,
              a.tB == RISE_BF16, kb};
  rise_status st = launch_prep(pa, s);
  if (st != RISE_OK) return st;
  st = launch_prep(pb, s);
  if (st != RISE_OK) return st;
  PackedGemm g{a.C, a.ldc, wsA, wsB, a.M, a.N, (int)Kp, (int)Mp, (int)Np, a.mode, kb};
  return launch_packed_gemm(g, t, s);
}

}  // namespace rise
