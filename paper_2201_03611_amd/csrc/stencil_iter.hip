// iterate with a size-preserving body (Sec. VI): `steps` applications of the
// 2D stencil, pad2D |> slide2D |> weighted reduce, each reading the image the
// previous one wrote (a Jacobi-style iteration).
//
// The paper's translation is a double buffer in memory and one loop round per
// application.  That is the fuse = 1 schedule here: one stencil launch per
// step, ping-ponging between two images in the caller's workspace; the first
// launch reads the input and the last writes the output.
//
// fuse = T > 1 runs T steps per launch (temporal blocking).  A workgroup loads
// a 128-column region of the image with a halo of T*r rows and columns, with
// pad2D applied, and keeps the steps in LDS, which is itself a double buffer:
// step t reads one LDS image and writes the other, on a region that shrinks
// by r per side and step, until the last step leaves the output tile
// (128 - 2rT columns by 32 rows), which goes to HBM.  HBM then carries the
// image once per T steps instead of once per step, at the price of the halo
// recomputation.
//
// Padding inside the fused steps: every LDS image holds, at positions outside
// the image, what pad2D would read there (the nearest edge value for clamp, 0
// for zero), so a step is the same unguarded weighted sum everywhere.  After
// each intermediate step, tiles that reach past the image rewrite those
// positions from the freshly computed edge (clamp) or with zeros.
//
// Every output is the sum over dy (outer) and dx (inner) of fma(x, w, acc)
// from 0, the order of the single-step kernels, so fused and unfused
// schedules give identical bits.
#include <stdint.h>

#include <algorithm>

#include "common.h"

namespace rise {
namespace {

constexpr int kThreads = 256;
constexpr int kItW = 128;   // LDS region width: 64 lanes x 2 columns
constexpr int kItTH = 32;   // output rows per tile
constexpr int kItTMax = 4;  // most steps per launch

template <int K>
struct ItCfg {
  static constexpr int R = (K - 1) / 2;
  static constexpr int PITCH = kItW + 2 * R;  // R spare columns each side
  static constexpr int ROWS = kItTH + 2 * R * kItTMax;
  static constexpr int BUF = ROWS * PITCH;
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Input region of one tile, one thread's share: column tid % 128 of rows
// tid / 128, tid / 128 + 2, ...  Every load reads a clamped, always valid
// address (no branches, so the loads stay in flight until the values are
// written to LDS); bit j of `zero` marks values that zero padding replaces.
template <int K>
struct ItRegs {
  static constexpr int N = ItCfg<K>::ROWS / 2;
  static_assert(N <= 32, "zero mask bits");
  float v[N];
  uint32_t zero;
};

template <int K>
__device__ __forceinline__ void it_fetch(ItRegs<K>& st, const float* __restrict__ in,
                                         int64_t ld_in, int H, int W, int zero_pad, int gy0,
                                         int gx0) {
  const int c = threadIdx.x & (kItW - 1), r0 = threadIdx.x >> 7;
  const int gx = gx0 + c, gxc = clampi(gx, 0, W - 1);
  const bool col_in = gx >= 0 && gx < W;
  uint32_t z = 0;
#pragma unroll
  for (int j = 0; j < ItRegs<K>::N; j++) {
    const int gy = gy0 + r0 + 2 * j;
    st.v[j] = in[(int64_t)clampi(gy, 0, H - 1) * ld_in + gxc];
    if (zero_pad && !(col_in && gy >= 0 && gy < H)) z |= 1u << j;
  }
  st.zero = z;
}

template <int K>
__device__ __forceinline__ void it_stash(const ItRegs<K>& st, float* img, int rows) {
  constexpr int R = ItCfg<K>::R, P = ItCfg<K>::PITCH;
  const int c = threadIdx.x & (kItW - 1), r0 = threadIdx.x >> 7;
#pragma unroll
  for (int j = 0; j < ItRegs<K>::N; j++)
    if (r0 + 2 * j < rows) img[(r0 + 2 * j) * P + R + c] = (st.zero >> j) & 1u ? 0.f : st.v[j];
}

// A resident grid: the row-major tile raster is cut into 8 contiguous bands,
// one per XCD (workgroup b runs on XCD b % 8), and workgroup j of an XCD takes
// tiles j, j + per, ... of its band.  While a workgroup runs the steps of one
// tile, the input region of its next tile is already on its way into
// registers.
template <int K>
__global__ __launch_bounds__(kThreads) void stencil_iter_fused(
    float* __restrict__ out, int64_t ld_out, const float* __restrict__ in, int64_t ld_in, int H,
    int W, const float* __restrict__ w, int zero_pad, int steps, int tiles_x, int ntiles,
    int per, int keep_out) {
  using Cfg = ItCfg<K>;
  constexpr int R = Cfg::R, P = Cfg::PITCH;
  __shared__ float lds[2 * Cfg::BUF];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int xcd = blockIdx.x % kNumXcd, jx = blockIdx.x / kNumXcd;
  const int band_end = (int)((int64_t)ntiles * (xcd + 1) / kNumXcd);
  int tile = (int)((int64_t)ntiles * xcd / kNumXcd) + jx;
  if (tile >= band_end) return;  // the whole workgroup leaves before any barrier
  const int RT = R * steps, TW = kItW - 2 * RT, ROWS = kItTH + 2 * RT;

  float wt[K][K];
#pragma unroll
  for (int dy = 0; dy < K; dy++)
#pragma unroll
    for (int dx = 0; dx < K; dx++) wt[dy][dx] = w[dy * K + dx];

  ItRegs<K> st;
  int y0 = (tile / tiles_x) * kItTH, x0 = (tile % tiles_x) * TW;
  it_fetch<K>(st, in, ld_in, H, W, zero_pad, y0 - RT, x0 - RT);
  while (true) {
    const int gy0 = y0 - RT, gx0 = x0 - RT;  // image position of LDS row 0, column 0
    __syncthreads();  // every wave is done reading the previous tile's last image
    // step 0: the input region with pad2D applied (column c at LDS index R + c)
    it_stash<K>(st, lds, ROWS);
    const int next = tile + per;
    const bool more = next < band_end;
    const int ny0 = (next / tiles_x) * kItTH, nx0 = (next % tiles_x) * TW;
    if (more) it_fetch<K>(st, in, ld_in, H, W, zero_pad, ny0 - RT, nx0 - RT);
    const bool border = gy0 < 0 || gy0 + ROWS > H || gx0 < 0 || gx0 + kItW > W;

    int cur = 0;
    for (int t = 1; t <= steps; t++) {
      __syncthreads();
      const float* src = lds + cur * Cfg::BUF;
      float* dst = lds + (cur ^ 1) * Cfg::BUF;
      // rows [R t, ROWS - R t) in blocks of 4; the last block is moved up so
      // that no block leaves the region (overlapping rows are recomputed with
      // the same result).  Every lane computes columns 2 lane, 2 lane + 1 over
      // the full width; columns outside the region come out as garbage that
      // no later step inside the region reads.
      const int lo = R * t, hi = ROWS - R * t, nb = (hi - lo + 3) >> 2;
      for (int b = wave; b < nb; b += kThreads / 64) {
        const int r0 = min(lo + 4 * b, hi - 4);
        float acc[4][2];
#pragma unroll
        for (int o = 0; o < 4; o++) acc[o][0] = acc[o][1] = 0.f;
#pragma unroll
        for (int j = 0; j < 4 + 2 * R; j++) {
          // data columns 2 lane - R .. 2 lane + 1 + R sit at LDS 2 lane .. 2 lane + K
          const float* row = src + (r0 - R + j) * P + 2 * lane;
          float v[K + 1];
#pragma unroll
          for (int e = 0; e < K + 1; e += 2) {
            const float2 p2 = *reinterpret_cast<const float2*>(row + e);
            v[e] = p2.x;
            v[e + 1] = p2.y;
          }
#pragma unroll
          for (int o = 0; o < 4; o++) {
            const int dy = j - o;
            if (dy >= 0 && dy < K) {
#pragma unroll
              for (int q = 0; q < 2; q++)
#pragma unroll
                for (int dx = 0; dx < K; dx++)
                  acc[o][q] = fmaf(v[q + dx], wt[dy][dx], acc[o][q]);
            }
          }
        }
#pragma unroll
        for (int o = 0; o < 4; o++) {
          float* d = dst + (r0 + o) * P + R + 2 * lane;
          d[0] = acc[o][0];
          d[1] = acc[o][1];
        }
      }
      cur ^= 1;
      if (t < steps && border) {
        // restore pad2D's values outside the image inside the new region
        __syncthreads();
        float* img = lds + cur * Cfg::BUF;
        const int n = (hi - lo) * kItW;
        if (zero_pad) {
          for (int i = tid; i < n; i += kThreads) {
            const int r = lo + (i >> 7), c = i & (kItW - 1);
            const int gy = gy0 + r, gx = gx0 + c;
            if (c >= lo && c < kItW - lo && (gy < 0 || gy >= H || gx < 0 || gx >= W))
              img[r * P + R + c] = 0.f;
          }
        } else {
          // columns first (rows inside the image), then whole rows, so corners
          // take the corner value
          for (int i = tid; i < n; i += kThreads) {
            const int r = lo + (i >> 7), c = i & (kItW - 1);
            const int gy = gy0 + r, gx = gx0 + c;
            if (c >= lo && c < kItW - lo && gy >= 0 && gy < H && (gx < 0 || gx >= W))
              img[r * P + R + c] = img[r * P + R + clampi(gx, 0, W - 1) - gx0];
          }
          __syncthreads();
          for (int i = tid; i < n; i += kThreads) {
            const int r = lo + (i >> 7), c = i & (kItW - 1);
            const int gy = gy0 + r;
            if (c >= lo && c < kItW - lo && (gy < 0 || gy >= H))
              img[r * P + R + c] = img[(clampi(gy, 0, H - 1) - gy0) * P + R + c];
          }
        }
      }
    }
    __syncthreads();
    // the output tile: rows RT .. RT + 32, columns RT .. RT + TW of the last image
    const float* img = lds + cur * Cfg::BUF;
    {
      const int c = tid & (kItW - 1), x = x0 + c;
      if (c < TW && x < W) {
#pragma unroll 4
        for (int r = tid >> 7; r < kItTH; r += 2) {
          const int y = y0 + r;
          if (y < H) {
            const float v = img[(RT + r) * P + R + RT + c];
            if (keep_out)  // the next launch reads it: leave it in the caches
              out[(int64_t)y * ld_out + x] = v;
            else
              __builtin_nontemporal_store(v, out + (int64_t)y * ld_out + x);
          }
        }
      }
    }
    if (!more) break;
    tile = next;
    y0 = ny0;
    x0 = nx0;
  }
}

template <int K>
rise_status launch_fused(const StencilArgs& a, int steps, hipStream_t s) {
  const int TW = kItW - 2 * ItCfg<K>::R * steps;
  const int tiles_x = (a.W + TW - 1) / TW, tiles_y = (a.H + kItTH - 1) / kItTH;
  const int64_t ntiles = (int64_t)tiles_x * tiles_y;
  if (ntiles > INT32_MAX) return fail(RISE_ERR_SHAPE, "rise_stencil2d_iterate: too many tiles");
  static const int occ = [] {
    int o = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, stencil_iter_fused<K>, kThreads, 0) !=
            hipSuccess || o < 1)
      o = 1;
    return o;
  }();
  // workgroups per XCD: as many as stay resident, evened out over the band
  const int64_t band = (ntiles + kNumXcd - 1) / kNumXcd;
  const int64_t max_per = std::max<int64_t>(1, (int64_t)occ * device_cu_count() / kNumXcd);
  const int64_t rounds = (band + max_per - 1) / max_per;
  const int per = (int)std::max<int64_t>(1, (band + rounds - 1) / rounds);
  hipLaunchKernelGGL(stencil_iter_fused<K>, dim3(kNumXcd * per), dim3(kThreads), 0, s, a.out,
                     a.ld_out, a.in, a.ld_in, a.H, a.W, a.w, (int)(a.pad == RISE_PAD_ZERO), steps,
                     tiles_x, (int)ntiles, per, (int)a.keep_out);
  return check_launch("stencil_iter_fused");
}

int launches(int64_t steps, int fuse) { return (int)((steps + fuse - 1) / fuse); }

}  // namespace

bool stencil_iterate_fusable(int kh, int kw) { return kh == kw && (kh == 3 || kh == 5); }
int stencil_iterate_max_fuse() { return kItTMax; }

// Measured on MI355X at 4096^2: for 3x3 four fused steps beat one launch per
// step (19 vs 21 us per step); for 5x5 the fused steps are bound by the FMA
// rate (k*k FMAs per pixel and step plus the halo recomputation) and lose to
// one launch per step, which is bound by HBM (36 vs 28 us per step).
int stencil_iterate_default_fuse(int kh, int kw) {
  return kh == 3 && kw == 3 ? kItTMax : 1;
}

size_t stencil_iterate_workspace(int64_t H, int64_t W, int64_t steps, int fuse) {
  if (steps <= 1 || fuse < 1) return 0;
  const int L = launches(steps, fuse);
  const size_t img = ((size_t)H * W * 4 + 255) / 256 * 256;
  return L >= 3 ? 2 * img : L == 2 ? img : 0;
}

rise_status launch_stencil_iterate(const StencilArgs& a, int64_t steps, int fuse, void* ws,
                                   hipStream_t s) {
  if (steps == 0) {
    const hipError_t e = hipMemcpy2DAsync(a.out, a.ld_out * 4, a.in, a.ld_in * 4,
                                          (size_t)a.W * 4, a.H, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess)
      return fail(RISE_ERR_HIP, std::string("rise_stencil2d_iterate: copy: ") + hipGetErrorString(e));
    return RISE_OK;
  }
  const int L = launches(steps, fuse);
  const size_t img = ((size_t)a.H * a.W * 4 + 255) / 256 * 256;
  float* buf[2] = {(float*)ws, (float*)((char*)ws + img)};
  const float* src = a.in;
  int64_t ld_src = a.ld_in;
  for (int i = 0; i < L; i++) {
    const bool last = i == L - 1;
    StencilArgs b = a;
    b.in = src;
    b.ld_in = ld_src;
    b.out = last ? a.out : buf[i & 1];
    b.ld_out = last ? a.ld_out : a.W;
    b.keep_out = !last;  // the next launch reads it
    const int n = (int)std::min<int64_t>(fuse, steps - (int64_t)i * fuse);
    rise_status st;
    if (n == 1)
      st = launch_stencil2d(b, stencil_default_schedule(a.H, a.W, a.kh, a.kw), s);
    else if (a.kh == 3)
      st = launch_fused<3>(b, n, s);
    else
      st = launch_fused<5>(b, n, s);
    if (st != RISE_OK) return st;
    src = b.out;
    ld_src = b.ld_out;
  }
  return RISE_OK;
}

}  // namespace rise
