// Operand preparation for the reduced-precision GEMM modes: map(cast) over an
// operand, materialised once (toMem, paper Sec. V-B) in the K-contiguous,
// zero-padded layout the matrix-core kernels read.  B is read through
// transpose here, so the contraction kernels see transpose(B) rows.
//
//   BF16   : bf16(a), round to nearest even
//   BF16X3 : hi = bf16(a), lo = bf16(a - hi)            (a - hi is exact in f32)
//   BF16X6 : a1 = bf16(a), a2 = bf16(a - a1), a3 = bf16(a - a1 - a2)
//   FP8    : per 32-element block along K: e = largest integer with
//            amax * 2^e <= 448 (0 for an all-zero block), q = e4m3(a * 2^e)
//            (round to nearest even), scale byte 127 - e (E8M0 of 2^-e).
//
// A source whose rows are K-contiguous streams straight through (bf16 modes);
// otherwise each workgroup transposes a 64 x 64 (rows x K) tile through LDS so
// that both the read (along whichever source dimension is contiguous) and the
// write (along K) are coalesced.
#include "gemm_lowp.h"

namespace rise {
namespace {

constexpr int kThreads = 256;
constexpr int TR = 64;  // rows per tile
constexpr int TK = 64;  // K per tile

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  // round to nearest even on the f32 bit pattern; NaN stays a quiet NaN
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Four values (|v| <= 448) to E4M3 in one word, lowest byte first, with the
// gfx950 conversion instruction (OCP E4M3: bias 7, no infinities; round to
// nearest even, subnormals below 2^-6 in steps of 2^-9; checked bit for bit
// against the oracle's encodings, subnormals and 448 included)
__device__ __forceinline__ uint32_t e4m3x4(float a, float b, float c, float d) {
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
  return (uint32_t)w;
}

// Largest e with amax * 2^e <= 448 (= 1.75 * 2^8), from the f32 fields of amax;
// 0 for amax = 0; at most 127.
__device__ __forceinline__ int e4m3_block_exp(float amax) {
  uint32_t a = __float_as_uint(amax) & 0x7fffffffu;
  if (a == 0) return 0;
  int ef = (int)(a >> 23);
  if (ef == 0) return 127;  // f32 subnormal amax: any e up to 127 fits
  uint32_t mant = a & 0x7fffffu;
  int e = (mant <= 0x600000u ? 135 : 134) - ef;
  return e > 127 ? 127 : e;
}

// element k of row r in a part of rows_out x k_out (kb = 0) or K-blocked by kb
__device__ __forceinline__ int64_t at(int64_t r, int64_t k, int64_t rows_out, int64_t k_out,
                                      int kb) {
  return kb ? ((k / kb) * rows_out + r) * kb + k % kb : r * k_out + k;
}
// scale byte of 32-element block b of row r (FP8), the same layouts
__device__ __forceinline__ int64_t scale_at(int64_t r, int64_t b, int64_t rows_out,
                                            int64_t k_out, int kb) {
  if (!kb) return r * (k_out / 32) + b;
  const int g = kb / 32;
  return ((b / g) * rows_out + r) * g + b % g;
}

// Thread -> (row, first of 8 consecutive K) for the streaming kernels.  By
// default lanes run along a row (a wave reads 2 KB of one row; its writes are
// one contiguous run, or 64-byte K blocks rows_out * kb apart).  K blocks
// narrower than 64 bytes (kb = 16 bf16 values, rows_out a multiple of 8): a
// wave takes 8 rows x 64 K, 8 lanes per row, and consecutive waves take
// consecutive row groups, so a block's writes from consecutive rows are
// adjacent (256-byte runs) instead of 32-byte pieces (8192^2 bf16x3: 115
// against 207 us; the 64-byte blocks of bf16 and FP8 stream faster along rows,
// 78-82 against 108-113 us).
__device__ __forceinline__ bool narrow_blocks(int kb, int elem_bytes) {
  return kb && kb * elem_bytes < 64;
}
__device__ __forceinline__ bool stream_pos(int64_t t, int64_t rows_out, int64_t k_out, int kb,
                                           int elem_bytes, int64_t& gr, int64_t& gk) {
  if (!narrow_blocks(kb, elem_bytes)) {
    const int64_t chunks = (k_out + 7) / 8;
    gr = t / chunks;
    gk = (t - gr * chunks) * 8;
    return gr < rows_out;
  }
  const int64_t w = t >> 6, groups = rows_out / 8;
  const int l = (int)(t & 63);
  gr = (w % groups) * 8 + l / 8;
  gk = (w / groups) * 64 + (l % 8) * 8;
  return gk < k_out;
}
inline int64_t stream_threads(int64_t rows_out, int64_t k_out, int kb, int elem_bytes) {
  return kb && kb * elem_bytes < 64 ? (rows_out / 8) * ((k_out + 63) / 64) * 64
                                    : rows_out * ((k_out + 7) / 8);
}

template <typename SRC>
__device__ __forceinline__ float load_src(const SRC* p);
template <>
__device__ __forceinline__ float load_src<float>(const float* p) { return *p; }
template <>
__device__ __forceinline__ float load_src<uint16_t>(const uint16_t* p) { return bf16_to_f32(*p); }

// layout: 0 = strided scalar loads, 1 = K contiguous (ld_k == 1) with float4,
// 2 = rows contiguous (ld_r == 1) with float4
template <typename SRC, int MODE, int LAYOUT>
__global__ __launch_bounds__(kThreads) void prep_kernel(void* __restrict__ out, int64_t rows_out,
                                                        int64_t k_out,
                                                        const SRC* __restrict__ src,
                                                        int64_t rows, int64_t K, int64_t ld_r,
                                                        int64_t ld_k, int vec_out, int kb) {
  __shared__ float tile[TR][TK + 1];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * TR;
  const int64_t k0 = (int64_t)blockIdx.y * TK;

  // ---- load the source tile (zeros outside rows x K) ----------------------
  if (LAYOUT == 1) {
#pragma unroll
    for (int p = 0; p < TR * TK / 4 / kThreads; p++) {
      int c = tid + kThreads * p;
      int row = c / (TK / 4), kk = (c % (TK / 4)) * 4;
      int64_t gr = r0 + row, gk = k0 + kk;
      f32x4 v = {0.f, 0.f, 0.f, 0.f};
      if (gr < rows) {
        const float* q = reinterpret_cast<const float*>(src) + gr * ld_r + gk;
        if (gk + 3 < K) {
          v = *reinterpret_cast<const f32x4*>(q);
        } else {
          if (gk + 0 < K) v.x = q[0];
          if (gk + 1 < K) v.y = q[1];
          if (gk + 2 < K) v.z = q[2];
        }
      }
      tile[row][kk + 0] = v.x;
      tile[row][kk + 1] = v.y;
      tile[row][kk + 2] = v.z;
      tile[row][kk + 3] = v.w;
    }
  } else if (LAYOUT == 2) {
#pragma unroll
    for (int p = 0; p < TR * TK / 4 / kThreads; p++) {
      int c = tid + kThreads * p;
      int kk = c / (TR / 4), row = (c % (TR / 4)) * 4;
      int64_t gr = r0 + row, gk = k0 + kk;
      f32x4 v = {0.f, 0.f, 0.f, 0.f};
      if (gk < K) {
        const float* q = reinterpret_cast<const float*>(src) + gk * ld_k + gr;
        if (gr + 3 < rows) {
          v = *reinterpret_cast<const f32x4*>(q);
        } else {
          if (gr + 0 < rows) v.x = q[0];
          if (gr + 1 < rows) v.y = q[1];
          if (gr + 2 < rows) v.z = q[2];
        }
      }
      tile[row + 0][kk] = v.x;
      tile[row + 1][kk] = v.y;
      tile[row + 2][kk] = v.z;
      tile[row + 3][kk] = v.w;
    }
  } else {
    for (int c = tid; c < TR * TK; c += kThreads) {
      int row = c / TK, kk = c % TK;
      int64_t gr = r0 + row, gk = k0 + kk;
      tile[row][kk] = (gr < rows && gk < K) ? load_src<SRC>(src + gr * ld_r + gk * ld_k) : 0.f;
    }
  }
  __syncthreads();

  // ---- convert 16 consecutive K of one row per thread ----------------------
  const int row = tid / 4, kc = (tid % 4) * 16;
  const int64_t gr = r0 + row, gk = k0 + kc;
  if (gr >= rows_out) return;  // (no barrier follows)
  float x[16];
#pragma unroll
  for (int e = 0; e < 16; e++) x[e] = tile[row][kc + e];
  const bool full = gk + 16 <= k_out;

  if (MODE == RISE_MODE_FP8) {
    float amax = 0.f;
#pragma unroll
    for (int e = 0; e < 16; e++) amax = fmaxf(amax, fabsf(x[e]));
    amax = fmaxf(amax, __shfl_xor(amax, 1));  // the 32-element block spans lanes 2j, 2j+1
    const int ex = e4m3_block_exp(amax);
    const float s = __uint_as_float((uint32_t)(127 + ex) << 23);  // 2^ex, ex >= -120
    i32x4 v;
#pragma unroll
    for (int w = 0; w < 4; w++)
      v[w] = (int)e4m3x4(x[4 * w] * s, x[4 * w + 1] * s, x[4 * w + 2] * s, x[4 * w + 3] * s);
    // 16 codes of one row: inside one K block (gk % 16 == 0, kb a multiple of 32)
    uint8_t* o = reinterpret_cast<uint8_t*>(out) + at(gr, gk, rows_out, k_out, kb);
    if (full && vec_out) {
      *reinterpret_cast<i32x4*>(o) = v;
    } else {
      for (int e = 0; e < 16; e++)
        if (gk + e < k_out) o[e] = (uint8_t)((uint32_t)v[e / 4] >> (8 * (e % 4)));
    }
    if ((kc & 31) == 0 && gk < k_out) {
      uint8_t* sp = reinterpret_cast<uint8_t*>(out) + rows_out * k_out;
      sp[scale_at(gr, gk / 32, rows_out, k_out, kb)] = (uint8_t)(127 - ex);
    }
    return;
  }

  constexpr int PARTS = MODE == RISE_MODE_BF16 ? 1 : MODE == RISE_MODE_BF16X3 ? 2 : 3;
  const int64_t plane = rows_out * k_out;
#pragma unroll
  for (int p = 0; p < PARTS; p++) {
    uint16_t h[16];
#pragma unroll
    for (int e = 0; e < 16; e++) {
      h[e] = bf16_rne(x[e]);
      x[e] = x[e] - bf16_to_f32(h[e]);  // exact residual
    }
    uint16_t* o = reinterpret_cast<uint16_t*>(out) + p * plane + at(gr, gk, rows_out, k_out, kb);
    if (full && vec_out) {
      i32x4 v0, v1;
#pragma unroll
      for (int w = 0; w < 4; w++) {
        v0[w] = (int)((uint32_t)h[2 * w] | ((uint32_t)h[2 * w + 1] << 16));
        v1[w] = (int)((uint32_t)h[8 + 2 * w] | ((uint32_t)h[8 + 2 * w + 1] << 16));
      }
      reinterpret_cast<i32x4*>(o)[0] = v0;
      reinterpret_cast<i32x4*>(o)[1] = v1;
    } else {
      for (int e = 0; e < 16; e++)
        if (gk + e < k_out) o[e] = h[e];
    }
  }
}

// Source rows already K-contiguous (ld_k == 1, 16-byte aligned rows): no
// transpose is needed, so the bf16 modes stream without LDS.  Each thread
// converts 8 consecutive K of one row (two 16-byte loads, one 16-byte store
// per part), threads placed by stream_pos.
template <int MODE>
__global__ __launch_bounds__(kThreads) void prep_stream_kernel(
    void* __restrict__ out, int64_t rows_out, int64_t k_out, const float* __restrict__ src,
    int64_t rows, int64_t K, int64_t ld_r, int vec_out, int kb) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  int64_t gr, gk;
  if (!stream_pos(t, rows_out, k_out, kb, 2, gr, gk)) return;
  float x[8];
  if (gr < rows && gk + 8 <= K) {
    const f32x4* q = reinterpret_cast<const f32x4*>(src + gr * ld_r + gk);
    const f32x4 v0 = q[0], v1 = q[1];
    x[0] = v0.x; x[1] = v0.y; x[2] = v0.z; x[3] = v0.w;
    x[4] = v1.x; x[5] = v1.y; x[6] = v1.z; x[7] = v1.w;
  } else {
#pragma unroll
    for (int e = 0; e < 8; e++) x[e] = (gr < rows && gk + e < K) ? src[gr * ld_r + gk + e] : 0.f;
  }
  constexpr int PARTS = MODE == RISE_MODE_BF16 ? 1 : MODE == RISE_MODE_BF16X3 ? 2 : 3;
  const int64_t plane = rows_out * k_out;
#pragma unroll
  for (int p = 0; p < PARTS; p++) {
    uint16_t h[8];
#pragma unroll
    for (int e = 0; e < 8; e++) {
      h[e] = bf16_rne(x[e]);
      x[e] = x[e] - bf16_to_f32(h[e]);  // exact residual
    }
    uint16_t* o = reinterpret_cast<uint16_t*>(out) + p * plane + at(gr, gk, rows_out, k_out, kb);
    if (vec_out && gk + 8 <= k_out) {
      i32x4 v;
#pragma unroll
      for (int w = 0; w < 4; w++) v[w] = (int)((uint32_t)h[2 * w] | ((uint32_t)h[2 * w + 1] << 16));
      *reinterpret_cast<i32x4*>(o) = v;
    } else {
#pragma unroll
      for (int e = 0; e < 8; e++)
        if (gk + e < k_out) o[e] = h[e];
    }
  }
}

// The same for FP8 (k_out a multiple of 32, so a 32-element scale block is the
// 8-value chunks of 4 consecutive lanes of one row): the block's amax is
// combined across those lanes, each lane stores its 8 codes, the block's first
// lane its scale byte.
__global__ __launch_bounds__(kThreads) void prep_stream_fp8_kernel(
    uint8_t* __restrict__ out, int64_t rows_out, int64_t k_out, const float* __restrict__ src,
    int64_t rows, int64_t K, int64_t ld_r, int kb) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  int64_t gr, gk;
  // k_out is a multiple of 32, so whole 4-lane blocks leave together
  if (!stream_pos(t, rows_out, k_out, kb, 1, gr, gk)) return;
  float x[8];
  if (gr < rows && gk + 8 <= K) {
    const f32x4* q = reinterpret_cast<const f32x4*>(src + gr * ld_r + gk);
    const f32x4 v0 = q[0], v1 = q[1];
    x[0] = v0.x; x[1] = v0.y; x[2] = v0.z; x[3] = v0.w;
    x[4] = v1.x; x[5] = v1.y; x[6] = v1.z; x[7] = v1.w;
  } else {
#pragma unroll
    for (int e = 0; e < 8; e++) x[e] = (gr < rows && gk + e < K) ? src[gr * ld_r + gk + e] : 0.f;
  }
  float amax = 0.f;
#pragma unroll
  for (int e = 0; e < 8; e++) amax = fmaxf(amax, fabsf(x[e]));
  amax = fmaxf(amax, __shfl_xor(amax, 1));
  amax = fmaxf(amax, __shfl_xor(amax, 2));
  const int ex = e4m3_block_exp(amax);
  const float sc = __uint_as_float((uint32_t)(127 + ex) << 23);  // 2^ex, ex >= -120
  const uint32_t w0 = e4m3x4(x[0] * sc, x[1] * sc, x[2] * sc, x[3] * sc);
  const uint32_t w1 = e4m3x4(x[4] * sc, x[5] * sc, x[6] * sc, x[7] * sc);
  *reinterpret_cast<uint2*>(out + at(gr, gk, rows_out, k_out, kb)) = uint2{w0, w1};
  if ((gk & 31) == 0) out[rows_out * k_out + scale_at(gr, gk / 32, rows_out, k_out, kb)] = (uint8_t)(127 - ex);
}

template <typename SRC, int MODE>
rise_status launch_mode(const PrepArgs& a, hipStream_t s) {
  dim3 grid((unsigned)((a.rows_out + TR - 1) / TR), (unsigned)((a.k_out + TK - 1) / TK));
  dim3 block(kThreads);
  auto aligned = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  int elem_out = MODE == RISE_MODE_FP8 ? 1 : 2;
  int vec_out = aligned(a.out) && (a.k_out * elem_out) % 16 == 0;
  const SRC* src = reinterpret_cast<const SRC*>(a.src);
  int layout = 0;
  if (sizeof(SRC) == 4 && aligned(a.src)) {
    if (a.ld_k == 1 && a.ld_r % 4 == 0) layout = 1;
    else if (a.ld_r == 1 && a.ld_k % 4 == 0) layout = 2;
  }
  if (layout == 1 && MODE != RISE_MODE_FP8) {
    const int64_t threads = stream_threads(a.rows_out, a.k_out, a.kblock, 2);
    hipLaunchKernelGGL((prep_stream_kernel<MODE>), dim3((unsigned)((threads + kThreads - 1) / kThreads)),
                       block, 0, s, a.out, a.rows_out, a.k_out, reinterpret_cast<const float*>(a.src),
                       a.rows, a.K, a.ld_r, vec_out, a.kblock);
    return check_launch("prep_stream_kernel");
  }
  if (layout == 1 && MODE == RISE_MODE_FP8 && vec_out && a.k_out % 32 == 0) {
    const int64_t threads = stream_threads(a.rows_out, a.k_out, a.kblock, 1);
    hipLaunchKernelGGL(prep_stream_fp8_kernel, dim3((unsigned)((threads + kThreads - 1) / kThreads)),
                       block, 0, s, reinterpret_cast<uint8_t*>(a.out), a.rows_out, a.k_out,
                       reinterpret_cast<const float*>(a.src), a.rows, a.K, a.ld_r, a.kblock);
    return check_launch("prep_stream_fp8_kernel");
  }
  if (layout == 1)
    hipLaunchKernelGGL((prep_kernel<SRC, MODE, 1>), grid, block, 0, s, a.out, a.rows_out, a.k_out,
                       src, a.rows, a.K, a.ld_r, a.ld_k, vec_out, a.kblock);
  else if (layout == 2)
    hipLaunchKernelGGL((prep_kernel<SRC, MODE, 2>), grid, block, 0, s, a.out, a.rows_out, a.k_out,
                       src, a.rows, a.K, a.ld_r, a.ld_k, vec_out, a.kblock);
  else
    hipLaunchKernelGGL((prep_kernel<SRC, MODE, 0>), grid, block, 0, s, a.out, a.rows_out, a.k_out,
                       src, a.rows, a.K, a.ld_r, a.ld_k, vec_out, a.kblock);
  return check_launch("prep_kernel");
}

}  // namespace

int prep_parts(rise_mode mode) {
  switch (mode) {
    case RISE_MODE_BF16: return 1;
    case RISE_MODE_BF16X3: return 2;
    case RISE_MODE_BF16X6: return 3;
    case RISE_MODE_FP8: return 1;
    default: return 0;
  }
}

size_t prep_bytes(int64_t rows_out, int64_t k_out, rise_mode mode) {
  if (mode == RISE_MODE_FP8) return (size_t)(rows_out * k_out + rows_out * (k_out / 32));
  return (size_t)prep_parts(mode) * (size_t)(rows_out * k_out) * 2;
}

rise_status launch_prep(const PrepArgs& a, hipStream_t s) {
  // whole 16-element runs of a thread stay in one block; FP8 scale bytes pair up
  const int kb_unit = a.mode == RISE_MODE_FP8 ? 32 : 16;
  if (a.kblock < 0 || a.kblock % kb_unit || (a.kblock && (a.k_out % a.kblock || a.rows_out % 8)))
    return fail(RISE_ERR_SHAPE,
                "prep: K block must be a multiple of 16 (FP8: 32) dividing k_out, rows_out a "
                "multiple of 8");
  if (a.rows_out == 0 || a.k_out == 0) return RISE_OK;
  if (a.src_bf16) {
    if (a.mode != RISE_MODE_BF16) return fail(RISE_ERR_DTYPE, "prep: bf16 source needs mode BF16");
    return launch_mode<uint16_t, RISE_MODE_BF16>(a, s);
  }
  switch (a.mode) {
    case RISE_MODE_BF16: return launch_mode<float, RISE_MODE_BF16>(a, s);
    case RISE_MODE_BF16X3: return launch_mode<float, RISE_MODE_BF16X3>(a, s);
    case RISE_MODE_BF16X6: return launch_mode<float, RISE_MODE_BF16X6>(a, s);
    case RISE_MODE_FP8: return launch_mode<float, RISE_MODE_FP8>(a, s);
    default: return fail(RISE_ERR_UNSUPPORTED, "prep: mode has no preparation");
  }
}

}  // namespace rise
