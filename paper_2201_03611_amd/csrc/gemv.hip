// Matrix-vector product, the paper's running example (Sec. IV):
//
//   y = A |> map(row => zip(row, x) |> map(*) |> reduce(+, 0))
//
// It reads every element of A once and does one multiply-add per element, so it
// is bound by HBM bandwidth (0.5 flop per byte), not by arithmetic: the kernels
// are organised around coalesced 16-byte loads and enough loads in flight.
//
//   A row-major (the paper's layout, RISE_OP_N): a wavefront owns 4 rows at a
//     time (map over rows -> waves, as the generated kernel's work-items own
//     rows); its lanes stride along the rows in 16-byte chunks (split of the
//     row into lane-sized pieces), each chunk of x is loaded once for the 4
//     rows, and the per-lane partial sums are combined across the wavefront
//     (the reduce, as a tree over the 64 lanes);
//   A read through transpose (RISE_OP_T, A stored K x M): a thread owns 4
//     consecutive outputs and sweeps rows of the stored A with 16-byte loads;
//     K is split over workgroups when there are too few column blocks to fill
//     the GPU, and a second kernel sums the split-K partials in a fixed order.
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <mutex>

#include "common.h"

namespace rise {
namespace {

constexpr int kThreads = 256;
constexpr int kRowsPerWave = 4;
constexpr int kColsPerBlock = kThreads * 4;  // outputs per workgroup (RISE_OP_T)

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <bool VEC>
__global__ __launch_bounds__(kThreads) void gemv_rows(float* __restrict__ y,
                                                      const float* __restrict__ A, int64_t lda,
                                                      const float* __restrict__ x, int M, int K,
                                                      int64_t row_groups) {
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = (int64_t)gridDim.x * (kThreads / 64);
  for (int64_t g = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); g < row_groups;
       g += nwaves) {
    const int r0 = (int)(g * kRowsPerWave);
    const float* rows[kRowsPerWave];
#pragma unroll
    for (int j = 0; j < kRowsPerWave; j++)  // rows past M repeat the last row; never stored
      rows[j] = A + (int64_t)min(r0 + j, M - 1) * lda;
    float acc[kRowsPerWave] = {0.f, 0.f, 0.f, 0.f};
    int k_done = 0;
    if (VEC) {
      const int nchunk = K / 4;
      f32x4 a4[kRowsPerWave];
#pragma unroll
      for (int j = 0; j < kRowsPerWave; j++) a4[j] = f32x4{0.f, 0.f, 0.f, 0.f};
      int c = lane;
      // two chunks per lane per iteration keep more loads in flight
      for (; c + 64 < nchunk; c += 128) {
        const f32x4 x0 = reinterpret_cast<const f32x4*>(x)[c];
        const f32x4 x1 = reinterpret_cast<const f32x4*>(x)[c + 64];
        f32x4 v0[kRowsPerWave], v1[kRowsPerWave];
#pragma unroll
        for (int j = 0; j < kRowsPerWave; j++) {
          v0[j] = reinterpret_cast<const f32x4*>(rows[j])[c];
          v1[j] = reinterpret_cast<const f32x4*>(rows[j])[c + 64];
        }
#pragma unroll
        for (int j = 0; j < kRowsPerWave; j++) {
          a4[j].x = fmaf(v0[j].x, x0.x, a4[j].x);
          a4[j].y = fmaf(v0[j].y, x0.y, a4[j].y);
          a4[j].z = fmaf(v0[j].z, x0.z, a4[j].z);
          a4[j].w = fmaf(v0[j].w, x0.w, a4[j].w);
          a4[j].x = fmaf(v1[j].x, x1.x, a4[j].x);
          a4[j].y = fmaf(v1[j].y, x1.y, a4[j].y);
          a4[j].z = fmaf(v1[j].z, x1.z, a4[j].z);
          a4[j].w = fmaf(v1[j].w, x1.w, a4[j].w);
        }
      }
      for (; c < nchunk; c += 64) {
        const f32x4 x0 = reinterpret_cast<const f32x4*>(x)[c];
#pragma unroll
        for (int j = 0; j < kRowsPerWave; j++) {
          const f32x4 v = reinterpret_cast<const f32x4*>(rows[j])[c];
          a4[j].x = fmaf(v.x, x0.x, a4[j].x);
          a4[j].y = fmaf(v.y, x0.y, a4[j].y);
          a4[j].z = fmaf(v.z, x0.z, a4[j].z);
          a4[j].w = fmaf(v.w, x0.w, a4[j].w);
        }
      }
#pragma unroll
      for (int j = 0; j < kRowsPerWave; j++) acc[j] = (a4[j].x + a4[j].y) + (a4[j].z + a4[j].w);
      k_done = nchunk * 4;
    }
    for (int k = k_done + lane; k < K; k += 64) {  // scalar path / ragged tail
      const float xv = x[k];
#pragma unroll
      for (int j = 0; j < kRowsPerWave; j++) acc[j] = fmaf(rows[j][k], xv, acc[j]);
    }
#pragma unroll
    for (int j = 0; j < kRowsPerWave; j++) {
      const float s = wave_sum(acc[j]);
      if (lane == 0 && r0 + j < M) y[r0 + j] = s;
    }
  }
}

// out[kc * ldo + m] = sum over k in chunk kc of A[k][m] * x[k], added in k order.
// DEEP keeps four rows of loads in flight per thread instead of two (for grids
// too small to hide the latency with more waves); the sums are the same.
template <bool VEC, bool DEEP>
__global__ __launch_bounds__(kThreads) void gemv_cols(float* __restrict__ out, int64_t ldo,
                                                      const float* __restrict__ A, int64_t lda,
                                                      const float* __restrict__ x, int M, int K,
                                                      int mblocks, int kchunk) {
  const int mb = blockIdx.x % mblocks, kc = blockIdx.x / mblocks;
  const int m = mb * kColsPerBlock + threadIdx.x * 4;
  const int k0 = kc * kchunk, k1 = min(K, k0 + kchunk);
  if (m >= M) return;  // no barriers in this kernel
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  if (VEC && m + 3 < M) {
    int k = k0;
    if (DEEP) {
      for (; k + 3 < k1; k += 4) {
        const f32x4 a0 = *reinterpret_cast<const f32x4*>(A + (int64_t)k * lda + m);
        const f32x4 a1 = *reinterpret_cast<const f32x4*>(A + (int64_t)(k + 1) * lda + m);
        const f32x4 a2 = *reinterpret_cast<const f32x4*>(A + (int64_t)(k + 2) * lda + m);
        const f32x4 a3 = *reinterpret_cast<const f32x4*>(A + (int64_t)(k + 3) * lda + m);
        const float x0 = x[k], x1 = x[k + 1], x2 = x[k + 2], x3 = x[k + 3];
        acc.x = fmaf(a0.x, x0, acc.x); acc.y = fmaf(a0.y, x0, acc.y);
        acc.z = fmaf(a0.z, x0, acc.z); acc.w = fmaf(a0.w, x0, acc.w);
        acc.x = fmaf(a1.x, x1, acc.x); acc.y = fmaf(a1.y, x1, acc.y);
        acc.z = fmaf(a1.z, x1, acc.z); acc.w = fmaf(a1.w, x1, acc.w);
        acc.x = fmaf(a2.x, x2, acc.x); acc.y = fmaf(a2.y, x2, acc.y);
        acc.z = fmaf(a2.z, x2, acc.z); acc.w = fmaf(a2.w, x2, acc.w);
        acc.x = fmaf(a3.x, x3, acc.x); acc.y = fmaf(a3.y, x3, acc.y);
        acc.z = fmaf(a3.z, x3, acc.z); acc.w = fmaf(a3.w, x3, acc.w);
      }
    }
    for (; k + 1 < k1; k += 2) {
      const f32x4 a0 = *reinterpret_cast<const f32x4*>(A + (int64_t)k * lda + m);
      const f32x4 a1 = *reinterpret_cast<const f32x4*>(A + (int64_t)(k + 1) * lda + m);
      const float x0 = x[k], x1 = x[k + 1];
      acc.x = fmaf(a0.x, x0, acc.x); acc.y = fmaf(a0.y, x0, acc.y);
      acc.z = fmaf(a0.z, x0, acc.z); acc.w = fmaf(a0.w, x0, acc.w);
      acc.x = fmaf(a1.x, x1, acc.x); acc.y = fmaf(a1.y, x1, acc.y);
      acc.z = fmaf(a1.z, x1, acc.z); acc.w = fmaf(a1.w, x1, acc.w);
    }
    for (; k < k1; k++) {
      const f32x4 a0 = *reinterpret_cast<const f32x4*>(A + (int64_t)k * lda + m);
      const float x0 = x[k];
      acc.x = fmaf(a0.x, x0, acc.x); acc.y = fmaf(a0.y, x0, acc.y);
      acc.z = fmaf(a0.z, x0, acc.z); acc.w = fmaf(a0.w, x0, acc.w);
    }
    *reinterpret_cast<f32x4*>(out + (int64_t)kc * ldo + m) = acc;
    return;
  }
  float a[4] = {0.f, 0.f, 0.f, 0.f};
  for (int k = k0; k < k1; k++) {
    const float x0 = x[k];
#pragma unroll
    for (int q = 0; q < 4; q++)
      if (m + q < M) a[q] = fmaf(A[(int64_t)k * lda + m + q], x0, a[q]);
  }
#pragma unroll
  for (int q = 0; q < 4; q++)
    if (m + q < M) out[(int64_t)kc * ldo + m + q] = a[q];
}

__global__ void gemv_reduce(float* __restrict__ y, const float* __restrict__ part, int M,
                            int nparts) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  // fixed order (part 0 first); the loads of 8 parts are issued together
  float s = 0.f;
  int p = 0;
  for (; p + 8 <= nparts; p += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; u++) v[u] = part[(int64_t)(p + u) * M + m];
#pragma unroll
    for (int u = 0; u < 8; u++) s += v[u];
  }
  for (; p < nparts; p++) s += part[(int64_t)p * M + m];
  y[m] = s;
}

struct ColSplit {
  int mblocks, kchunks, kchunk;
};
ColSplit col_split(int64_t M, int64_t K) {
  ColSplit c;
  c.mblocks = (int)((M + kColsPerBlock - 1) / kColsPerBlock);
  // about 1024 workgroups in all (four per compute unit; measured at 16384^2:
  // 171 us against 202 us with 2048, whose extra partial sums and shorter
  // per-workgroup row sweeps cost more than they hide), chunks of at least 64
  // rows of A
  int64_t want = (1024 + c.mblocks - 1) / c.mblocks;
  int64_t most = std::max<int64_t>(1, (K + 63) / 64);
  c.kchunks = (int)std::max<int64_t>(1, std::min(want, most));
  c.kchunk = (int)((K + c.kchunks - 1) / c.kchunks);
  if (c.kchunk == 0) c.kchunk = 1;
  c.kchunks = (int)std::max<int64_t>(1, (K + c.kchunk - 1) / c.kchunk);
  return c;
}

}  // namespace

size_t gemv_workspace(int64_t M, int64_t K, bool trans) {
  if (!trans || M == 0 || K == 0) return 0;
  const ColSplit c = col_split(M, K);
  return c.kchunks > 1 ? (size_t)c.kchunks * M * 4 : 0;
}

int gemv_parts(int64_t M, int64_t K, bool trans) {
  if (!trans || M == 0 || K == 0) return 1;
  return col_split(M, K).kchunks;
}

rise_status launch_gemv(const GemvArgs& a, void* ws, hipStream_t s) {
  // K = 0 needs no special case: the kernels reduce over an empty range and
  // store the initial value 0
  auto aligned = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  if (!a.trans) {
    const bool vec = aligned(a.A) && aligned(a.x) && a.lda % 4 == 0;
    const int64_t groups = (a.M + kRowsPerWave - 1) / kRowsPerWave;
    const int64_t blocks =
        std::min<int64_t>((groups + 3) / 4, (int64_t)device_cu_count() * 8);
    if (vec)
      hipLaunchKernelGGL(gemv_rows<true>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a.y, a.A,
                         a.lda, a.x, a.M, a.K, groups);
    else
      hipLaunchKernelGGL(gemv_rows<false>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a.y,
                         a.A, a.lda, a.x, a.M, a.K, groups);
    return check_launch("gemv_rows");
  }
  const ColSplit c = col_split(a.M, a.K);
  const bool vec = aligned(a.A) && a.lda % 4 == 0;
  float* out = c.kchunks > 1 ? (float*)ws : a.y;
  const int64_t ldo = a.M;
  const unsigned grid = (unsigned)((int64_t)c.mblocks * c.kchunks);
  // below two workgroups per compute unit, deeper loads per thread (4096^2:
  // 15.5 us against 18.3 us); at 8192^2 and above they measured slower
  const bool deep = (int64_t)grid < 2 * (int64_t)device_cu_count();
  if (vec && deep)
    hipLaunchKernelGGL((gemv_cols<true, true>), dim3(grid), dim3(kThreads), 0, s, out, ldo, a.A,
                       a.lda, a.x, a.M, a.K, c.mblocks, c.kchunk);
  else if (vec)
    hipLaunchKernelGGL((gemv_cols<true, false>), dim3(grid), dim3(kThreads), 0, s, out, ldo,
                       a.A, a.lda, a.x, a.M, a.K, c.mblocks, c.kchunk);
  else
    hipLaunchKernelGGL((gemv_cols<false, false>), dim3(grid), dim3(kThreads), 0, s, out, ldo,
                       a.A, a.lda, a.x, a.M, a.K, c.mblocks, c.kchunk);
  rise_status st = check_launch("gemv_cols");
  if (st != RISE_OK || c.kchunks == 1) return st;
  hipLaunchKernelGGL(gemv_reduce, dim3((unsigned)((a.M + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, a.y, (const float*)ws, a.M, c.kchunks);
  return check_launch("gemv_reduce");
}


// ---------------------------------------------------------------------------
// Fixed scratch for the entry point that allocates nothing (rise_gemv_noalloc).
// The split-K partials of the transposed product go to this file-scope device
// array instead of a caller workspace.  Its size covers every split col_split
// picks: kchunks > 1 only when there are at most 1023 column blocks, and then
// kchunks * M <= ceil(1024 / mblocks) * mblocks * 1024 <= 2046 * 1024 floats.
// Each device holds its own copy for the life of the process; its device
// address is looked up once per device (hipGetSymbolAddress with that device
// current) and only that address is handed to kernels.
// ---------------------------------------------------------------------------
constexpr size_t kGemvScratchBytes = RISE_GEMV_NOALLOC_SCRATCH_BYTES;
static_assert(kGemvScratchBytes >= (size_t)2046 * kColsPerBlock * 4, "scratch below the largest split");
static __device__ __align__(256) unsigned char scratch[kGemvScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::atomic<void*> g_scratch_ptr[kMaxDevices];
std::mutex g_scratch_mu;
}  // namespace

size_t gemv_scratch_bytes() { return kGemvScratchBytes; }

rise_status gemv_scratch(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(RISE_ERR_HIP, "rise_gemv_noalloc: hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) return fail(RISE_ERR_HIP, "rise_gemv_noalloc: device index above 63");
  void* p = g_scratch_ptr[dev].load(std::memory_order_acquire);
  if (!p) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
    if (!p) {
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return fail(RISE_ERR_HIP, std::string("rise_gemv_noalloc: hipGetSymbolAddress(scratch): ") +
                                      hipGetErrorString(e));
      g_scratch_ptr[dev].store(p, std::memory_order_release);
    }
  }
  *out = p;
  return RISE_OK;
}

}  // namespace rise
