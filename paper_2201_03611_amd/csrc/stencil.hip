// 2D stencil: out = in |> pad2D |> slide2D(k, 1) |> map(map(weighted reduce)).
//
// The pattern is HBM-bound (about 6 flop per byte for 5 x 5), so the kernel is
// organised around memory traffic, not arithmetic:
//   pad2D (clamp or zero)  -> index remapping while the halo tile is fetched;
//                             nothing padded is ever stored;
//   slide2D                -> one (TY + 2R) x (TX + 8) halo tile per workgroup,
//                             staged in LDS (toMem(Local), paper Sec. V-B/C) with
//                             coalesced 16-byte loads, so every input element
//                             is fetched from HBM about once;
//   map(map(...))          -> each lane owns 4 adjacent outputs of a row and
//                             walks down TY / 4 rows, keeping the k rows of
//                             its window in registers (each LDS row is read
//                             once per lane, as three 16-byte reads);
//   zip |> map(*) |> reduce -> k*k FMAs per output in registers (fuseReduceMap,
//                             Sec. IV-B), weights in scalar registers;
//   join                   -> 16-byte coalesced stores.
// Square windows of 1, 3, 5 and 7 use this kernel; other odd sizes up to 15
// use a direct per-output kernel.
#include "common.h"

namespace rise {
namespace {

constexpr int kThreads = 256;
constexpr int TX = 256;            // columns per workgroup (64 lanes x 4)
constexpr int TY = 32;             // rows per workgroup (4 waves x 8)
constexpr int RW = TY / 4;         // rows per wave
constexpr int HALO = 4;            // LDS columns left and right of the tile
constexpr int LCOLS = TX + 2 * HALO;
constexpr int LCHUNKS = LCOLS / 4;  // 16-byte chunks per LDS row

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

template <int K, bool VEC>
__global__ __launch_bounds__(kThreads) void stencil2d_tiled(
    float* __restrict__ out, int64_t ld_out, const float* __restrict__ in, int64_t ld_in, int H,
    int W, const float* __restrict__ w, int zero_pad, int tiles_x) {
  constexpr int R = (K - 1) / 2;
  constexpr int ROWS = TY + 2 * R;
  constexpr int TOTAL = ROWS * LCHUNKS;
  constexpr int PER = (TOTAL + kThreads - 1) / kThreads;
  __shared__ f32x4 tile[ROWS][LCHUNKS];

  const int tid = threadIdx.x;
  int lid = xcd_contiguous(blockIdx.x, gridDim.x);
  const int y0 = (lid / tiles_x) * TY;
  const int x0 = (lid % tiles_x) * TX;

  // ---- halo tile: global -> registers -> LDS ------------------------------
  f32x4 st[PER];
#pragma unroll
  for (int p = 0; p < PER; p++) {
    const int c = tid + p * kThreads;
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (c < TOTAL) {
      const int lr = c / LCHUNKS, cc = c - lr * LCHUNKS;
      int gy = y0 - R + lr;
      const int gx = x0 - HALO + cc * 4;
      bool row_ok = true;
      if (gy < 0 || gy >= H) {
        if (zero_pad) row_ok = false;
        gy = clampi(gy, 0, H - 1);
      }
      if (row_ok) {
        const float* rp = in + (int64_t)gy * ld_in;
        if (VEC && gx >= 0 && gx + 3 < W) {
          v = *reinterpret_cast<const f32x4*>(rp + gx);
        } else {
          float e[4];
#pragma unroll
          for (int q = 0; q < 4; q++) {
            int xx = gx + q;
            if (xx < 0 || xx >= W) {
              e[q] = zero_pad ? 0.f : rp[clampi(xx, 0, W - 1)];
            } else {
              e[q] = rp[xx];
            }
          }
          v = f32x4{e[0], e[1], e[2], e[3]};
        }
      }
    }
    st[p] = v;
  }
#pragma unroll
  for (int p = 0; p < PER; p++) {
    const int c = tid + p * kThreads;
    if (c < TOTAL) {
      const int lr = c / LCHUNKS;
      tile[lr][c - lr * LCHUNKS] = st[p];
    }
  }
  __syncthreads();

  // ---- weights (uniform: scalar loads) -----------------------------------
  float wt[K][K];
#pragma unroll
  for (int dy = 0; dy < K; dy++)
#pragma unroll
    for (int dx = 0; dx < K; dx++) wt[dy][dx] = w[dy * K + dx];

  // ---- windows and weighted reduce ----------------------------------------
  const int lane = tid & 63, wave = tid >> 6;
  const int r0 = wave * RW;  // first output row of this wave (tile-local)
  // lane's chunks: LDS chunk `lane` = columns x-4..x-1, lane+1 = x..x+3, lane+2 = x+4..x+7
  float win[RW + 2 * R][12];
#pragma unroll
  for (int j = 0; j < RW + 2 * R; j++) {
    f32x4 c1 = tile[r0 + j][lane + 1];
    win[j][4] = c1.x; win[j][5] = c1.y; win[j][6] = c1.z; win[j][7] = c1.w;
    if (R > 0) {
      f32x4 c0 = tile[r0 + j][lane];
      f32x4 c2 = tile[r0 + j][lane + 2];
      win[j][0] = c0.x; win[j][1] = c0.y; win[j][2] = c0.z; win[j][3] = c0.w;
      win[j][8] = c2.x; win[j][9] = c2.y; win[j][10] = c2.z; win[j][11] = c2.w;
    }
  }
  const int x = x0 + lane * 4;
#pragma unroll
  for (int o = 0; o < RW; o++) {
    float acc[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      float a = 0.f;
#pragma unroll
      for (int dy = 0; dy < K; dy++)
#pragma unroll
        for (int dx = 0; dx < K; dx++) a = fmaf(win[o + dy][4 + q + dx - R], wt[dy][dx], a);
      acc[q] = a;
    }
    const int y = y0 + r0 + o;
    if (y < H) {
      float* op = out + (int64_t)y * ld_out;
      if (VEC && x + 3 < W) {
        *reinterpret_cast<f32x4*>(op + x) = f32x4{acc[0], acc[1], acc[2], acc[3]};
      } else {
#pragma unroll
        for (int q = 0; q < 4; q++)
          if (x + q < W) op[x + q] = acc[q];
      }
    }
  }
}

// Any odd kh x kw up to 15 x 15: one thread per output, reads through the
// caches with clamped or zero-filled indices.
__global__ __launch_bounds__(kThreads) void stencil2d_direct(
    float* __restrict__ out, int64_t ld_out, const float* __restrict__ in, int64_t ld_in, int H,
    int W, const float* __restrict__ w, int kh, int kw, int zero_pad) {
  const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= (int64_t)H * W) return;
  const int y = (int)(idx / W), x = (int)(idx - (int64_t)y * W);
  const int rh = (kh - 1) / 2, rw = (kw - 1) / 2;
  float a = 0.f;
  for (int dy = 0; dy < kh; dy++) {
    int yy = y + dy - rh;
    bool yin = yy >= 0 && yy < H;
    if (!yin && zero_pad) continue;
    yy = clampi(yy, 0, H - 1);
    for (int dx = 0; dx < kw; dx++) {
      int xx = x + dx - rw;
      bool xin = xx >= 0 && xx < W;
      if (!xin && zero_pad) continue;
      xx = clampi(xx, 0, W - 1);
      a = fmaf(in[(int64_t)yy * ld_in + xx], w[dy * kw + dx], a);
    }
  }
  out[(int64_t)y * ld_out + x] = a;
}

template <int K>
rise_status launch_tiled(const StencilArgs& a, bool vec, hipStream_t s) {
  int tiles_x = (a.W + TX - 1) / TX, tiles_y = (a.H + TY - 1) / TY;
  dim3 grid(tiles_x * tiles_y), block(kThreads);
  int zero = a.pad == RISE_PAD_ZERO;
  if (vec)
    hipLaunchKernelGGL((stencil2d_tiled<K, true>), grid, block, 0, s, a.out, a.ld_out, a.in,
                       a.ld_in, a.H, a.W, a.w, zero, tiles_x);
  else
    hipLaunchKernelGGL((stencil2d_tiled<K, false>), grid, block, 0, s, a.out, a.ld_out, a.in,
                       a.ld_in, a.H, a.W, a.w, zero, tiles_x);
  return check_launch("stencil2d_tiled");
}

}  // namespace

rise_status launch_stencil2d(const StencilArgs& a, hipStream_t s) {
  auto aligned = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  bool vec = aligned(a.in) && aligned(a.out) && a.ld_in % 4 == 0 && a.ld_out % 4 == 0;
  if (a.kh == a.kw) {
    switch (a.kh) {
      case 1: return launch_tiled<1>(a, vec, s);
      case 3: return launch_tiled<3>(a, vec, s);
      case 5: return launch_tiled<5>(a, vec, s);
      case 7: return launch_tiled<7>(a, vec, s);
      default: break;
    }
  }
  int64_t n = (int64_t)a.H * a.W;
  dim3 grid((unsigned)((n + kThreads - 1) / kThreads)), block(kThreads);
  hipLaunchKernelGGL(stencil2d_direct, grid, block, 0, s, a.out, a.ld_out, a.in, a.ld_in, a.H,
                     a.W, a.w, a.kh, a.kw, (int)(a.pad == RISE_PAD_ZERO));
  return check_launch("stencil2d_direct");
}

}  // namespace rise
