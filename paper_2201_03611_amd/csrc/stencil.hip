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
// That is the LDS halo-tile schedule.  The streaming schedule below keeps the
// window in registers instead and exchanges neighbours with wavefront shifts;
// the caller picks one through rise_stencil_schedule (both compute the same
// sums in the same order).  Square windows of 1, 3, 5 and 7 use these
// kernels; other odd sizes up to 15 use a direct per-output kernel.
#include <stdint.h>

#include <algorithm>
#include <climits>

#include "async_copy.h"
#include "common.h"
#include "tiles.h"

namespace rise {
namespace {

using tiles::clampi;
using tiles::kThreads;
constexpr int TX = tiles::kStencilTX;  // columns per workgroup / wave strip (64 lanes x 4)

template <int K, bool VEC, int TY, bool NT>
__global__ __launch_bounds__(kThreads) void stencil2d_tiled(
    float* __restrict__ out, int64_t ld_out, const float* __restrict__ in, int64_t ld_in, int H,
    int W, const float* __restrict__ w, int zero_pad, int tiles_x) {
  __shared__ f32x4 lds[tiles::StencilCfg<K, TY>::LDS_CHUNKS];
  const int lid = xcd_contiguous(blockIdx.x, gridDim.x);
  tiles::stencil_lds_tile<K, VEC, TY, NT>(out, ld_out, in, ld_in, H, W, w, zero_pad,
                                      (lid / tiles_x) * TY, (lid % tiles_x) * TX, lds);
}

// Resident-grid pipelined schedule: the LDS halo tile above, but each
// workgroup walks a fixed list of tiles.  Per tile: one barrier, then the
// loads of the next tile are issued into registers, the current tile is
// reduced from one LDS buffer into registers, the next tile is written to the
// other LDS buffer, and only then are the current outputs stored.  The loads
// are thus the oldest vector-memory operations when their data is needed (the
// single vmcnt counter of gfx9 also counts stores), and HBM traffic overlaps
// the k*k FMAs inside every workgroup (with aligned rows the fetch has no
// branches, so no merge point forces an early wait).  The row-major tile raster is cut into 8
// contiguous bands, one per XCD (workgroup b runs on XCD b % 8); workgroup j
// of an XCD takes tiles j, j + per, j + 2 per, ... of its band, so the XCD's
// workgroups sweep the band together and halo rows shared by vertically
// adjacent tiles are read while they are still in that XCD's L2.  Output
// stores are non-temporal.
template <int K, bool VEC, int TY>
__global__ __launch_bounds__(kThreads) void stencil2d_pipe(
    float* __restrict__ out, int64_t ld_out, const float* __restrict__ in, int64_t ld_in, int H,
    int W, const float* __restrict__ w, int zero_pad, int tiles_x, int ntiles, int per) {
  using Cfg = tiles::StencilCfg<K, TY>;
  __shared__ f32x4 lds[2][Cfg::LDS_CHUNKS];
  const int xcd = blockIdx.x % kNumXcd, j = blockIdx.x / kNumXcd;
  const int band_end = (int)((int64_t)ntiles * (xcd + 1) / kNumXcd);
  int t = (int)((int64_t)ntiles * xcd / kNumXcd) + j;
  if (t >= band_end) return;  // the whole workgroup leaves before any barrier

  float wt[K][K];
  tiles::stencil_weights<K>(wt, w);
  tiles::StencilRegs<K, TY> st;
  uint32_t mode = 0;
  const bool whole_chunks = VEC && (W & 3) == 0;  // the branch-free fetch needs W % 4 == 0
  auto fetch = [&](int y0, int x0) {
    if (whole_chunks)
      tiles::stencil_fetch_aligned<K, TY>(st, mode, in, ld_in, H, W, zero_pad, y0, x0);
    else
      tiles::stencil_fetch<K, VEC, TY>(st, in, ld_in, H, W, zero_pad, y0, x0);
  };
  auto stash = [&](f32x4* dst) {
    if (whole_chunks)
      tiles::stencil_stash_aligned<K, TY>(st, mode, dst);
    else
      tiles::stencil_stash<K, TY>(st, dst);
  };
  int y0 = (t / tiles_x) * TY, x0 = (t % tiles_x) * TX;
  fetch(y0, x0);
  stash(lds[0]);
  int buf = 0;
  while (true) {
    __syncthreads();  // lds[buf] is complete; every wave is done with lds[buf ^ 1]
    const int next = t + per;
    const bool more = next < band_end;
    const int ny0 = (next / tiles_x) * TY, nx0 = (next % tiles_x) * TX;
    if (more) fetch(ny0, nx0);
    float res[TY / 4][4];
    tiles::stencil_compute<K, TY>(res, wt, lds[buf]);
    if (more) stash(lds[buf ^ 1]);
    tiles::stencil_store<VEC, TY, true>(out, ld_out, H, W, res, y0, x0);
    if (!more) break;
    t = next;
    y0 = ny0;
    x0 = nx0;
    buf ^= 1;
  }
}

// Asynchronous-copy schedule (aligned rows, W % 4 == 0): the halo tile goes
// from HBM to LDS with global_load_lds (16 bytes per lane, no registers held),
// DIST tiles ahead through a ring of DIST + 1 LDS tiles, so each workgroup
// keeps DIST tiles of loads in flight while it reduces the current one.  pad2D
// is applied in the copy addresses: rows through clamped row addresses (clamp)
// or a page of zeros (zero); columns left or right of the image through the
// zero page (zero) or, for clamp, by replacing those 16-byte chunks with the
// edge element in registers when the window is read.  Every tile issues the same number of
// copies and stores (outputs outside the image go to a dump page), so the
// waits are fixed vmcnt counts.
__device__ __align__(16) float g_stencil_zero_page[4];  // never written: zeros
__device__ __align__(16) float g_stencil_dump_page[4];  // sink of out-of-image stores

__device__ __forceinline__ void st_copy16_to_lds(const void* src, void* lds_base) {
  async::copy16(src, lds_base);
}
template <int N>
__device__ __forceinline__ void st_wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt field is 6 bits");
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
#endif
}
__device__ __forceinline__ void st_wait_lgkmcnt0() {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#endif
}
__device__ __forceinline__ void st_raw_barrier() {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("s_barrier" ::: "memory");
#endif
}

template <int K, int TY, int DIST>
struct AsyncCfg {
  static constexpr int R = (K - 1) / 2;
  static constexpr int ROWS = TY + 2 * R;
  static constexpr int CHUNKS = ROWS * tiles::kLChunks;  // 16-byte chunks of the halo tile
  static constexpr int NI = (CHUNKS + 63) / 64;           // wave copy instructions per tile
  static constexpr int QPW = (NI + 3) / 4;                // per wave (the last wave may have one less)
  static constexpr int NST = TY / 4;                      // 16-byte stores per lane per tile
  static constexpr int NBUF = DIST + 1;
  static constexpr int STAGE = NI * 64;                   // chunks per LDS tile (rounded up)
};

template <int K, int TY, int DIST>
__global__ __launch_bounds__(kThreads) void stencil2d_async(
    float* __restrict__ out, int64_t ld_out, const float* __restrict__ in, int64_t ld_in, int H,
    int W, const float* __restrict__ w, int zero_pad, int tiles_x, int ntiles, int per) {
  using C = AsyncCfg<K, TY, DIST>;
  constexpr int R = C::R, LC = tiles::kLChunks;
  __shared__ f32x4 halo[C::NBUF][C::STAGE];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int xcd = blockIdx.x % kNumXcd, j = blockIdx.x / kNumXcd;
  const int band_end = (int)((int64_t)ntiles * (xcd + 1) / kNumXcd);
  int t = (int)((int64_t)ntiles * xcd / kNumXcd) + j;
  if (t >= band_end) return;  // the whole workgroup leaves before any barrier
  const int last = band_end - 1;

  float wt[K][K];
  tiles::stencil_weights<K>(wt, w);

  auto issue = [&](int tile, int buf) {
    const int y0 = (tile / tiles_x) * TY, x0 = (tile % tiles_x) * TX;
#pragma unroll
    for (int q = 0; q < C::QPW; q++) {
      const int g = wave + 4 * q;
      if (g < C::NI) {
        const int c = g * 64 + lane;
        const void* src = g_stencil_zero_page;
        if (c < C::CHUNKS) {
          const int lr = c / LC, cc = c - lr * LC;
          const int gy = y0 - R + lr, gx = x0 - tiles::kHalo + 4 * cc;
          const bool inside = gy >= 0 && gy < H && gx >= 0 && gx < W;
          if (inside || !zero_pad)
            src = in + (int64_t)clampi(gy, 0, H - 1) * ld_in + clampi(gx, 0, W - 4);
        }
        st_copy16_to_lds(src, &halo[buf][g * 64]);
      }
    }
  };
  const bool full_copies = wave + 4 * (C::QPW - 1) < C::NI;  // wave-uniform copy count

#pragma unroll
  for (int d = 0; d < DIST; d++) issue(min(t + d * per, last), d);
  st_wait_vmcnt<0>();
  int buf = 0;
  while (true) {
    const int next = t + per;
    const bool more = next < band_end;
    const int y0 = (t / tiles_x) * TY, x0 = (t % tiles_x) * TX;
    st_wait_lgkmcnt0();  // this wave's reads of the previous tile are done
    st_raw_barrier();    // every wave's copies into halo[buf] are visible
    // refill the tile reduced in the previous iteration, DIST tiles ahead
    issue(min(t + DIST * per, last), (buf + DIST) % C::NBUF);
    // clamp at the left and right image edges: those chunks were copied from
    // an arbitrary in-image address and are replaced in registers
    const int x = x0 + 4 * lane;
    const bool left = !zero_pad && x0 == 0;
    const int lim = !zero_pad && x0 + TX + tiles::kHalo > W ? W : INT_MAX;
    float res[TY / 4][4];
    tiles::stencil_compute<K, TY, true>(res, wt, halo[buf], left, lim, x);
    // the next tile's copies have landed: younger than them are the copies of
    // DIST - 1 later tiles and the stores of DIST - 1 earlier tiles
    if (full_copies)
      st_wait_vmcnt<(DIST - 1) * (C::QPW + C::NST)>();
    else
      st_wait_vmcnt<(DIST - 1) * (C::QPW - 1 + C::NST)>();
#pragma unroll
    for (int o = 0; o < TY / 4; o++) {
      const int y = y0 + wave * (TY / 4) + o;
      float* dst = (y < H && x < W) ? out + (int64_t)y * ld_out + x : g_stencil_dump_page;
      __builtin_nontemporal_store(f32x4{res[o][0], res[o][1], res[o][2], res[o][3]},
                                  reinterpret_cast<f32x4*>(dst));
    }
    if (!more) break;
    t = next;
    buf = (buf + 1) % C::NBUF;
  }
}

// Streaming schedule: every wave owns one 256-column strip segment of `L`
// output rows and walks down it.  Each input row of the segment (plus the r
// halo rows above and below) is fetched once as one 16-byte chunk per lane;
// the chunks of the neighbouring lanes (columns x-4..x-1 and x+4..x+7) arrive
// through wavefront shifts (DPP wave_shr / wave_shl), and only lanes 0 and 63
// fetch the 4 columns beyond the strip.  Input rows are prefetched P rows
// ahead into registers; the k window rows live in a register ring.  No LDS and
// no barriers: waves run independently, so loads and FMAs of different waves
// overlap freely.
__device__ __forceinline__ float wave_from_left(float v) {  // lane l receives lane l-1
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float wave_from_right(float v) {  // lane l receives lane l+1
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}

template <bool VEC>
__device__ __forceinline__ f32x4 load_chunk4(const float* __restrict__ in, int64_t ld_in, int H,
                                             int W, int gy, int gx, int zero_pad) {
  // 4 consecutive elements of padded row gy starting at padded column gx
  if (gy < 0 || gy >= H) {
    if (zero_pad) return f32x4{0.f, 0.f, 0.f, 0.f};
    gy = clampi(gy, 0, H - 1);
  }
  const float* rp = in + (int64_t)gy * ld_in;
  if (VEC && gx >= 0 && gx + 3 < W) return *reinterpret_cast<const f32x4*>(rp + gx);
  float e[4];
#pragma unroll
  for (int q = 0; q < 4; q++) {
    int xx = gx + q;
    if (xx < 0 || xx >= W)
      e[q] = zero_pad ? 0.f : rp[clampi(xx, 0, W - 1)];
    else
      e[q] = rp[xx];
  }
  return f32x4{e[0], e[1], e[2], e[3]};
}

template <int K, bool VEC, int L>
__global__ __launch_bounds__(kThreads) void stencil2d_stream(
    float* __restrict__ out, int64_t ld_out, const float* __restrict__ in, int64_t ld_in, int H,
    int W, const float* __restrict__ w, int zero_pad, int segs, int tasks) {
  constexpr int R = (K - 1) / 2;
  constexpr int P = K >= 4 ? K : K * ((4 + K - 1) / K);  // prefetch depth, a multiple of K
  constexpr int NIN = L + 2 * R;                          // input rows consumed per segment

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int task = xcd_contiguous(blockIdx.x, gridDim.x) * 4 + wave;
  if (task >= tasks) return;  // whole wave leaves; no barriers in this kernel
  const int strip = task / segs, seg = task - strip * segs;
  const int x0 = strip * TX, x = x0 + 4 * lane;
  const int ys = seg * L;
  const int edge_x = lane == 0 ? x0 - 4 : x0 + TX;  // used by lanes 0 and 63 only
  const bool edge_lane = lane == 0 || lane == 63;

  float wt[K][K];
#pragma unroll
  for (int dy = 0; dy < K; dy++)
#pragma unroll
    for (int dx = 0; dx < K; dx++) wt[dy][dx] = w[dy * K + dx];

  f32x4 raw[P], edge[P];
  float win[K][12];
#pragma unroll
  for (int p = 0; p < P; p++) edge[p] = f32x4{0.f, 0.f, 0.f, 0.f};

  auto fetch = [&](int t, int slot) {  // input row t of the segment = padded row ys - R + t
    const int gy = ys - R + t;
    raw[slot] = load_chunk4<VEC>(in, ld_in, H, W, gy, x, zero_pad);
    if (edge_lane) edge[slot] = load_chunk4<VEC>(in, ld_in, H, W, gy, edge_x, zero_pad);
  };

#pragma unroll
  for (int p = 0; p < P; p++)
    if (p < NIN) fetch(p, p);

  for (int t0 = 0; t0 < NIN; t0 += P) {
#pragma unroll
    for (int p = 0; p < P; p++) {
      const int t = t0 + p;
      if (t >= NIN) break;
      // expand input row t into its window slot: [x-4..x-1 | x..x+3 | x+4..x+7]
      float* row = win[p % K];
      const f32x4 c = raw[p];
      const f32x4 e = edge[p];
      row[4] = c.x; row[5] = c.y; row[6] = c.z; row[7] = c.w;
      if (R > 0) {
        float l0 = wave_from_left(c.x), l1 = wave_from_left(c.y);
        float l2 = wave_from_left(c.z), l3 = wave_from_left(c.w);
        float r0 = wave_from_right(c.x), r1 = wave_from_right(c.y);
        float r2 = wave_from_right(c.z), r3 = wave_from_right(c.w);
        if (lane == 0) { l0 = e.x; l1 = e.y; l2 = e.z; l3 = e.w; }
        if (lane == 63) { r0 = e.x; r1 = e.y; r2 = e.z; r3 = e.w; }
        row[0] = l0; row[1] = l1; row[2] = l2; row[3] = l3;
        row[8] = r0; row[9] = r1; row[10] = r2; row[11] = r3;
      }
      if (t + P < NIN) fetch(t + P, p);
      if (t >= 2 * R) {
        const int y = ys + t - 2 * R;
        if (y < H) {
          float acc[4];
#pragma unroll
          for (int q = 0; q < 4; q++) {
            float a = 0.f;
#pragma unroll
            for (int dy = 0; dy < K; dy++)
#pragma unroll
              for (int dx = 0; dx < K; dx++)
                a = fmaf(win[(p + K - 2 * R + dy) % K][4 + q + dx - R], wt[dy][dx], a);
            acc[q] = a;
          }
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

template <int K, bool VEC, int TY>
rise_status launch_tiled(const StencilArgs& a, hipStream_t s) {
  int tiles_x = (a.W + TX - 1) / TX, tiles_y = (a.H + TY - 1) / TY;
  if (a.keep_out)
    hipLaunchKernelGGL((stencil2d_tiled<K, VEC, TY, false>), dim3(tiles_x * tiles_y),
                       dim3(kThreads), 0, s, a.out, a.ld_out, a.in, a.ld_in, a.H, a.W, a.w,
                       (int)(a.pad == RISE_PAD_ZERO), tiles_x);
  else
    hipLaunchKernelGGL((stencil2d_tiled<K, VEC, TY, true>), dim3(tiles_x * tiles_y),
                       dim3(kThreads), 0, s, a.out, a.ld_out, a.in, a.ld_in, a.H, a.W, a.w,
                       (int)(a.pad == RISE_PAD_ZERO), tiles_x);
  return check_launch("stencil2d_tiled");
}

// Workgroups per XCD for the pipelined schedule: as many as stay resident
// (occupancy x CUs / 8), then evened out so that every workgroup of a band
// gets the same number of tiles, give or take one.
template <int K, bool VEC, int TY>
rise_status launch_pipe(const StencilArgs& a, hipStream_t s) {
  const int tiles_x = (a.W + TX - 1) / TX, tiles_y = (a.H + TY - 1) / TY;
  const int64_t ntiles = (int64_t)tiles_x * tiles_y;
  if (ntiles > INT32_MAX) return fail(RISE_ERR_SHAPE, "rise_stencil2d: too many tiles");
  // resident workgroups per CU (a property of the kernel on gfx950)
  static const int occ = [] {
    int o = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, stencil2d_pipe<K, VEC, TY>, kThreads, 0) !=
            hipSuccess || o < 1)
      o = 1;
    return o;
  }();
  const int64_t band = (ntiles + kNumXcd - 1) / kNumXcd;
  const int64_t max_per = std::max<int64_t>(1, (int64_t)occ * device_cu_count() / kNumXcd);
  const int64_t rounds = (band + max_per - 1) / max_per;
  const int per = (int)std::max<int64_t>(1, (band + rounds - 1) / rounds);
  hipLaunchKernelGGL((stencil2d_pipe<K, VEC, TY>), dim3(kNumXcd * per), dim3(kThreads), 0, s,
                     a.out, a.ld_out, a.in, a.ld_in, a.H, a.W, a.w, (int)(a.pad == RISE_PAD_ZERO),
                     tiles_x, (int)ntiles, per);
  return check_launch("stencil2d_pipe");
}

template <int K, int TY>
rise_status launch_async(const StencilArgs& a, hipStream_t s) {
  constexpr int DIST = 2;
  const int tiles_x = (a.W + TX - 1) / TX, tiles_y = (a.H + TY - 1) / TY;
  const int64_t ntiles = (int64_t)tiles_x * tiles_y;
  if (ntiles > INT32_MAX) return fail(RISE_ERR_SHAPE, "rise_stencil2d: too many tiles");
  static const int occ = [] {
    int o = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, stencil2d_async<K, TY, DIST>, kThreads,
                                                     0) != hipSuccess || o < 1)
      o = 1;
    return o;
  }();
  const int64_t band = (ntiles + kNumXcd - 1) / kNumXcd;
  const int64_t max_per = std::max<int64_t>(1, (int64_t)occ * device_cu_count() / kNumXcd);
  const int64_t rounds = (band + max_per - 1) / max_per;
  const int per = (int)std::max<int64_t>(1, (band + rounds - 1) / rounds);
  hipLaunchKernelGGL((stencil2d_async<K, TY, DIST>), dim3(kNumXcd * per), dim3(kThreads), 0, s,
                     a.out, a.ld_out, a.in, a.ld_in, a.H, a.W, a.w, (int)(a.pad == RISE_PAD_ZERO),
                     tiles_x, (int)ntiles, per);
  return check_launch("stencil2d_async");
}

template <int K, bool VEC, int L>
rise_status launch_stream(const StencilArgs& a, hipStream_t s) {
  int strips = (a.W + TX - 1) / TX, segs = (a.H + L - 1) / L;
  int tasks = strips * segs;
  hipLaunchKernelGGL((stencil2d_stream<K, VEC, L>), dim3((tasks + 3) / 4), dim3(kThreads), 0, s,
                     a.out, a.ld_out, a.in, a.ld_in, a.H, a.W, a.w, (int)(a.pad == RISE_PAD_ZERO),
                     segs, tasks);
  return check_launch("stencil2d_stream");
}

template <int K, bool VEC>
rise_status launch_k(const StencilArgs& a, const rise_stencil_schedule& sc, hipStream_t s) {
  if (sc.variant == RISE_STENCIL_LDS_TILE) {
    if (sc.rows == 8) return launch_tiled<K, VEC, 8>(a, s);
    if (sc.rows == 16) return launch_tiled<K, VEC, 16>(a, s);
    if (sc.rows == 32) return launch_tiled<K, VEC, 32>(a, s);
  } else if (sc.variant == RISE_STENCIL_LDS_PIPE) {
    if (sc.rows == 8) return launch_pipe<K, VEC, 8>(a, s);
    if (sc.rows == 16) return launch_pipe<K, VEC, 16>(a, s);
    if (sc.rows == 32) return launch_pipe<K, VEC, 32>(a, s);
  } else if (sc.variant == RISE_STENCIL_ASYNC) {
    // whole 16-byte chunks only; other images take the LDS tile of the same rows
    if (!VEC || (a.W & 3) != 0) return launch_tiled<K, VEC, 16>(a, s);
    if (sc.rows == 8) return launch_async<K, 8>(a, s);
    if (sc.rows == 16) return launch_async<K, 16>(a, s);
  } else {
    if (sc.rows == 16) return launch_stream<K, VEC, 16>(a, s);
    if (sc.rows == 32) return launch_stream<K, VEC, 32>(a, s);
    if (sc.rows == 64) return launch_stream<K, VEC, 64>(a, s);
    if (sc.rows == 128) return launch_stream<K, VEC, 128>(a, s);
  }
  return fail(RISE_ERR_UNSUPPORTED, "rise_stencil2d: schedule rows");
}

const rise_stencil_schedule kSchedules[] = {
    {RISE_STENCIL_LDS_TILE, 8},  {RISE_STENCIL_LDS_TILE, 16}, {RISE_STENCIL_LDS_TILE, 32},
    {RISE_STENCIL_STREAM, 16},   {RISE_STENCIL_STREAM, 32},   {RISE_STENCIL_STREAM, 64},
    {RISE_STENCIL_STREAM, 128},  {RISE_STENCIL_LDS_PIPE, 8},  {RISE_STENCIL_LDS_PIPE, 16},
    {RISE_STENCIL_LDS_PIPE, 32}, {RISE_STENCIL_ASYNC, 8},    {RISE_STENCIL_ASYNC, 16}};

}  // namespace

int stencil_schedules(rise_stencil_schedule* out, int cap) {
  int n = (int)(sizeof(kSchedules) / sizeof(kSchedules[0]));
  for (int i = 0; out && i < n && i < cap; i++) out[i] = kSchedules[i];
  return n;
}

bool stencil_schedule_supported(const rise_stencil_schedule& sc) {
  for (const auto& k : kSchedules)
    if (k.variant == sc.variant && k.rows == sc.rows) return true;
  return false;
}

rise_stencil_schedule stencil_default_schedule(int H, int W, int kh, int kw) {
  // measured on 4096^2: the 8-row LDS tile (64 VGPRs, eight waves per SIMD) is
  // fastest for 3x3 and 5x5, the 16-row tile for 7x7
  return rise_stencil_schedule{RISE_STENCIL_LDS_TILE, kh <= 5 && kw <= 5 ? 8 : 16};
}

rise_status launch_stencil2d(const StencilArgs& a, const rise_stencil_schedule& sc,
                             hipStream_t s) {
  auto aligned = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  bool vec = aligned(a.in) && aligned(a.out) && a.ld_in % 4 == 0 && a.ld_out % 4 == 0;
  if (a.kh == a.kw) {
    switch (a.kh) {
      case 1: return vec ? launch_k<1, true>(a, sc, s) : launch_k<1, false>(a, sc, s);
      case 3: return vec ? launch_k<3, true>(a, sc, s) : launch_k<3, false>(a, sc, s);
      case 5: return vec ? launch_k<5, true>(a, sc, s) : launch_k<5, false>(a, sc, s);
      case 7: return vec ? launch_k<7, true>(a, sc, s) : launch_k<7, false>(a, sc, s);
      default: break;
    }
  }
  int64_t n = (int64_t)a.H * a.W;
  dim3 grid((unsigned)((n + kThreads - 1) / kThreads)), block(kThreads);
  hipLaunchKernelGGL(stencil2d_direct, grid, block, 0, s, a.out, a.ld_out, a.in, a.ld_in, a.H,
                     a.W, a.w, a.kh, a.kw, (int)(a.pad == RISE_PAD_ZERO));
  return check_launch("stencil2d_direct");
}


// ===========================================================================
// Adjoint of the stencil (backward).
//
// dIn: the stencil is linear in its input, out = S in, and dIn = S^T dOut.
//   zero pad:  S^T is the stencil with the window rotated by 180 degrees applied
//              to dOut with zero padding (a window element at offset (dy, dx)
//              becomes the element at (-dy, -dx));
//   clamp pad: the same everywhere except the first/last row and column, which
//              also collect the contributions clamped onto them:
//              dIn[p] = sum_d w[d] sum { dOut[o] : clamp(o + d - r) = p },
//              evaluated separately per dimension.
// dW:  dW[dy][dx] = sum over outputs (y, x) of dOut[y][x] * window(y, x)[dy][dx],
//      a reduction over all pixels: per-wave partial sums (streaming the input
//      like the forward kernel) then one deterministic reduction.
// ===========================================================================
namespace {

__global__ void rotate180_kernel(float* __restrict__ dst, const float* __restrict__ w, int n) {
  int t = threadIdx.x + blockIdx.x * blockDim.x;
  if (t < n) dst[t] = w[n - 1 - t];
}

// o range of {o in [0, N) : clamp(o + d - r, 0, N - 1) == p}
__device__ __forceinline__ void clamp_preimage(int p, int d, int r, int N, int& lo, int& hi) {
  const int exact = p - d + r;
  lo = (p == 0) ? 0 : exact;
  hi = (p == N - 1) ? N - 1 : exact;
  if (lo < 0) lo = 0;
  if (hi > N - 1) hi = N - 1;
}

__global__ __launch_bounds__(kThreads) void adjoint_clamp_border(
    float* __restrict__ din, int64_t ld_din, const float* __restrict__ dout, int64_t ld_dout,
    int H, int W, const float* __restrict__ w, int kh, int kw) {
  // border pixels: row 0, row H-1, then column 0 and column W-1 of rows 1..H-2
  const int n_top = W, n_bot = H > 1 ? W : 0, n_mid = H > 2 ? H - 2 : 0;
  const int n_side = W > 1 ? 2 * n_mid : n_mid;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int py, px;
  if (i < n_top) {
    py = 0; px = i;
  } else if ((i -= n_top) < n_bot) {
    py = H - 1; px = i;
  } else if ((i -= n_bot) < n_side) {
    py = 1 + (i % n_mid);
    px = (i < n_mid) ? 0 : W - 1;
  } else {
    return;
  }
  const int rh = (kh - 1) / 2, rw = (kw - 1) / 2;
  float acc = 0.f;
  for (int dy = 0; dy < kh; dy++) {
    int ylo, yhi;
    clamp_preimage(py, dy, rh, H, ylo, yhi);
    for (int dx = 0; dx < kw; dx++) {
      int xlo, xhi;
      clamp_preimage(px, dx, rw, W, xlo, xhi);
      float s = 0.f;
      for (int oy = ylo; oy <= yhi; oy++)
        for (int ox = xlo; ox <= xhi; ox++) s += dout[(int64_t)oy * ld_dout + ox];
      acc = fmaf(w[dy * kw + dx], s, acc);
    }
  }
  din[(int64_t)py * ld_din + px] = acc;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Per-wave partial sums of dW over one 256-column strip segment of L output rows.
template <int K, bool VEC, int L>
__global__ __launch_bounds__(kThreads) void stencil_dw_stream(
    float* __restrict__ partial, const float* __restrict__ dout, int64_t ld_dout,
    const float* __restrict__ in, int64_t ld_in, int H, int W, int zero_pad, int segs,
    int tasks) {
  constexpr int R = (K - 1) / 2;
  constexpr int P = K >= 4 ? K : K * ((4 + K - 1) / K);
  constexpr int NIN = L + 2 * R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int task = xcd_contiguous(blockIdx.x, gridDim.x) * 4 + wave;
  if (task >= tasks) return;
  const int strip = task / segs, seg = task - strip * segs;
  const int x0 = strip * TX, x = x0 + 4 * lane;
  const int ys = seg * L;
  const int edge_x = lane == 0 ? x0 - 4 : x0 + TX;
  const bool edge_lane = lane == 0 || lane == 63;

  f32x4 raw[P], edge[P], grad[P];
  float win[K][12];
  float acc[K][K];
#pragma unroll
  for (int p = 0; p < P; p++) edge[p] = grad[p] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int dy = 0; dy < K; dy++)
#pragma unroll
    for (int dx = 0; dx < K; dx++) acc[dy][dx] = 0.f;

  // dOut chunk of output row o (zero outside the image: those outputs do not exist)
  auto fetch_grad = [&](int o) -> f32x4 {
    const int y = ys + o;
    if (o < 0 || o >= L || y >= H) return f32x4{0.f, 0.f, 0.f, 0.f};
    const float* rp = dout + (int64_t)y * ld_dout;
    if (VEC && x + 3 < W) return *reinterpret_cast<const f32x4*>(rp + x);
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (x + 0 < W) v.x = rp[x + 0];
    if (x + 1 < W) v.y = rp[x + 1];
    if (x + 2 < W) v.z = rp[x + 2];
    if (x + 3 < W) v.w = rp[x + 3];
    return v;
  };
  auto fetch = [&](int t, int slot) {
    const int gy = ys - R + t;
    raw[slot] = load_chunk4<VEC>(in, ld_in, H, W, gy, x, zero_pad);
    if (edge_lane) edge[slot] = load_chunk4<VEC>(in, ld_in, H, W, gy, edge_x, zero_pad);
    grad[slot] = fetch_grad(t - 2 * R);  // the output row this input row completes
  };

#pragma unroll
  for (int p = 0; p < P; p++)
    if (p < NIN) fetch(p, p);

  for (int t0 = 0; t0 < NIN; t0 += P) {
#pragma unroll
    for (int p = 0; p < P; p++) {
      const int t = t0 + p;
      if (t >= NIN) break;
      float* row = win[p % K];
      const f32x4 c = raw[p];
      const f32x4 e = edge[p];
      const f32x4 g = grad[p];
      row[4] = c.x; row[5] = c.y; row[6] = c.z; row[7] = c.w;
      if (R > 0) {
        float l0 = wave_from_left(c.x), l1 = wave_from_left(c.y);
        float l2 = wave_from_left(c.z), l3 = wave_from_left(c.w);
        float r0 = wave_from_right(c.x), r1 = wave_from_right(c.y);
        float r2 = wave_from_right(c.z), r3 = wave_from_right(c.w);
        if (lane == 0) { l0 = e.x; l1 = e.y; l2 = e.z; l3 = e.w; }
        if (lane == 63) { r0 = e.x; r1 = e.y; r2 = e.z; r3 = e.w; }
        row[0] = l0; row[1] = l1; row[2] = l2; row[3] = l3;
        row[8] = r0; row[9] = r1; row[10] = r2; row[11] = r3;
      }
      if (t + P < NIN) fetch(t + P, p);
      if (t >= 2 * R) {
        const float gq[4] = {g.x, g.y, g.z, g.w};
#pragma unroll
        for (int dy = 0; dy < K; dy++)
#pragma unroll
          for (int dx = 0; dx < K; dx++) {
            float a = acc[dy][dx];
#pragma unroll
            for (int q = 0; q < 4; q++)
              a = fmaf(gq[q], win[(p + K - 2 * R + dy) % K][4 + q + dx - R], a);
            acc[dy][dx] = a;
          }
      }
    }
  }
#pragma unroll
  for (int dy = 0; dy < K; dy++)
#pragma unroll
    for (int dx = 0; dx < K; dx++) {
      float v = wave_sum(acc[dy][dx]);
      if (lane == 0) partial[(int64_t)task * K * K + dy * K + dx] = v;
    }
}

// Any odd kh x kw: block (chunk, tap) sums dOut * window over a chunk of pixels.
__global__ __launch_bounds__(kThreads) void stencil_dw_direct(
    float* __restrict__ partial, const float* __restrict__ dout, int64_t ld_dout,
    const float* __restrict__ in, int64_t ld_in, int H, int W, int kh, int kw, int zero_pad,
    int chunk) {
  const int tap = blockIdx.y, dy = tap / kw, dx = tap - dy * kw;
  const int rh = (kh - 1) / 2, rw = (kw - 1) / 2;
  const int64_t n = (int64_t)H * W;
  const int64_t p0 = (int64_t)blockIdx.x * chunk;
  float acc = 0.f;
  for (int64_t i = p0 + threadIdx.x; i < p0 + chunk && i < n; i += kThreads) {
    const int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
    int yy = y + dy - rh, xx = x + dx - rw;
    const bool inside = yy >= 0 && yy < H && xx >= 0 && xx < W;
    if (!inside && zero_pad) continue;
    yy = clampi(yy, 0, H - 1);
    xx = clampi(xx, 0, W - 1);
    acc = fmaf(dout[(int64_t)y * ld_dout + x], in[(int64_t)yy * ld_in + xx], acc);
  }
  __shared__ float red[kThreads / 64];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int q = 0; q < kThreads / 64; q++) s += red[q];
    partial[(int64_t)blockIdx.x * gridDim.y + tap] = s;
  }
}

// dW[t] = sum over parts of partial[part][t] (one block per tap, fixed order).
__global__ __launch_bounds__(kThreads) void reduce_partials(float* __restrict__ dW,
                                                            const float* __restrict__ partial,
                                                            int parts, int taps) {
  const int t = blockIdx.x;
  float acc = 0.f;
  for (int p = threadIdx.x; p < parts; p += kThreads) acc += partial[(int64_t)p * taps + t];
  __shared__ float red[kThreads / 64];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int q = 0; q < kThreads / 64; q++) s += red[q];
    dW[t] = s;
  }
}

constexpr int kDwRows = 32;       // output rows per wave in the streaming dW kernel
constexpr int kDwChunk = 65536;   // pixels per block in the direct dW kernel

bool dw_streaming(int kh, int kw) { return kh == kw && (kh == 1 || kh == 3 || kh == 5 || kh == 7); }

int64_t dw_parts(int H, int W, int kh, int kw) {
  if (dw_streaming(kh, kw)) {
    int64_t strips = (W + TX - 1) / TX, segs = (H + kDwRows - 1) / kDwRows;
    return strips * segs;
  }
  return ((int64_t)H * W + kDwChunk - 1) / kDwChunk;
}

template <int K, bool VEC>
rise_status launch_dw_stream(float* partial, const StencilBwdArgs& a, hipStream_t s) {
  int strips = (a.W + TX - 1) / TX, segs = (a.H + kDwRows - 1) / kDwRows;
  int tasks = strips * segs;
  hipLaunchKernelGGL((stencil_dw_stream<K, VEC, kDwRows>), dim3((tasks + 3) / 4), dim3(kThreads),
                     0, s, partial, a.dout, a.ld_dout, a.in, a.ld_in, a.H, a.W,
                     (int)(a.pad == RISE_PAD_ZERO), segs, tasks);
  return check_launch("stencil_dw_stream");
}

}  // namespace

size_t stencil_backward_workspace(int H, int W, int kh, int kw) {
  size_t rot = 256;  // rotated weights (kh * kw <= 225 floats = 900 bytes, rounded below)
  rot = ((size_t)kh * kw * 4 + 255) / 256 * 256;
  size_t part = (size_t)dw_parts(H, W, kh, kw) * kh * kw * 4;
  return rot + part;
}

rise_status launch_stencil2d_backward(const StencilBwdArgs& a, void* ws, hipStream_t s) {
  const int taps = a.kh * a.kw;
  float* rot = (float*)ws;
  float* partial = (float*)((char*)ws + ((size_t)taps * 4 + 255) / 256 * 256);
  rise_status st = RISE_OK;
  if (a.din) {
    hipLaunchKernelGGL(rotate180_kernel, dim3(1), dim3(256), 0, s, rot, a.w, taps);
    if ((st = check_launch("rotate180_kernel")) != RISE_OK) return st;
    StencilArgs f{a.din, a.ld_din, a.dout, a.ld_dout, a.H, a.W, rot, a.kh, a.kw, RISE_PAD_ZERO};
    st = launch_stencil2d(f, stencil_default_schedule(a.H, a.W, a.kh, a.kw), s);
    if (st != RISE_OK) return st;
    if (a.pad == RISE_PAD_CLAMP) {
      int n = a.W + (a.H > 1 ? a.W : 0) + (a.H > 2 ? (a.W > 1 ? 2 : 1) * (a.H - 2) : 0);
      hipLaunchKernelGGL(adjoint_clamp_border, dim3((n + kThreads - 1) / kThreads),
                         dim3(kThreads), 0, s, a.din, a.ld_din, a.dout, a.ld_dout, a.H, a.W,
                         a.w, a.kh, a.kw);
      if ((st = check_launch("adjoint_clamp_border")) != RISE_OK) return st;
    }
  }
  if (a.dw) {
    const int64_t parts = dw_parts(a.H, a.W, a.kh, a.kw);
    auto aligned = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
    bool vec = aligned(a.in) && aligned(a.dout) && a.ld_in % 4 == 0 && a.ld_dout % 4 == 0;
    if (dw_streaming(a.kh, a.kw)) {
      switch (a.kh) {
        case 1: st = vec ? launch_dw_stream<1, true>(partial, a, s) : launch_dw_stream<1, false>(partial, a, s); break;
        case 3: st = vec ? launch_dw_stream<3, true>(partial, a, s) : launch_dw_stream<3, false>(partial, a, s); break;
        case 5: st = vec ? launch_dw_stream<5, true>(partial, a, s) : launch_dw_stream<5, false>(partial, a, s); break;
        default: st = vec ? launch_dw_stream<7, true>(partial, a, s) : launch_dw_stream<7, false>(partial, a, s); break;
      }
    } else {
      hipLaunchKernelGGL(stencil_dw_direct, dim3((unsigned)parts, (unsigned)taps), dim3(kThreads),
                         0, s, partial, a.dout, a.ld_dout, a.in, a.ld_in, a.H, a.W, a.kh, a.kw,
                         (int)(a.pad == RISE_PAD_ZERO), kDwChunk);
      st = check_launch("stencil_dw_direct");
    }
    if (st != RISE_OK) return st;
    hipLaunchKernelGGL(reduce_partials, dim3(taps), dim3(kThreads), 0, s, a.dw, partial,
                       (int)parts, taps);
    if ((st = check_launch("reduce_partials")) != RISE_OK) return st;
  }
  return RISE_OK;
}

}  // namespace rise
