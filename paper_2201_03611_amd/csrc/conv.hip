// Multi-channel stencil layer (a "convolution" layer): NHWC bfloat16 activations,
// FP32 weights rounded to bfloat16 for the matrix cores, FP32 accumulation.
//
//   out[b][y][x][co] = reduce(+, 0) over ci of
//                      stencil(pad2D(in[b][.][.][ci]), w[co][ci])     (3 x 3 window)
//
// is a contraction over K = (tap, ci) = 9 * Cin for every output pixel, i.e. an
// implicit GEMM with M = pixels and N = Cout: the window gather (pad2D |>
// slide2D) is an index view into an LDS halo tile, never materialised in HBM.
//
// Forward (and dIn, which is the same kernel on dOut with the window rotated by
// 180 degrees and the channel roles swapped): out^T = W' X with the prepared
// weights as the A operand (held in registers for the whole persistent
// workgroup) and the pixels of an LDS halo ring as the B operand; the halo is
// copied asynchronously a few tiles ahead (see conv3x3_fwd below).
// dW (the gradient of the weights) contracts over pixels instead: per tile the
// dOut tile and the input halo are staged transposed (pixels contiguous, one
// copy per horizontal tap offset so every fragment read is aligned), each
// workgroup accumulates its share of dW^T in registers, and a fixed-order
// reduction over workgroups finishes it.
#include <stdint.h>

#include <algorithm>

#include "async_copy.h"
#include "common.h"
#include "conv.h"

namespace rise {
namespace {

constexpr int kThreads = 256;
constexpr int TXP = 64;              // output pixels per row of a tile
constexpr int HC = TXP + 2;          // halo columns
constexpr int TAPS = 9;

__device__ __forceinline__ uint16_t f32_to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Two floats to two bf16 (round to nearest even) in one 32-bit word, low half
// first: one v_cvt_pk_bf16_f32 on gfx950.
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{lo, hi}, bf16x2_t));
}

// dst[o][tap * I + i] = bf16(weight), with
//   forward : o = co, i = ci, weight = w[co][ci][tap]
//   adjoint : o = ci, i = co, weight = w[co][ci][8 - tap]   (180-degree rotation)
__global__ void conv_prep_weights(uint16_t* __restrict__ dst, uint16_t* __restrict__ zero_page,
                                  const float* __restrict__ w, int Cout, int Cin, int adjoint) {
  if (blockIdx.x == 0 && threadIdx.x < 128) zero_page[threadIdx.x] = 0;  // 256 bytes
  const int n = Cout * Cin * TAPS;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const int co = e / (Cin * TAPS), rem = e - co * Cin * TAPS, ci = rem / TAPS, tap = rem % TAPS;
    const uint16_t v = f32_to_bf16(w[e]);
    if (!adjoint)
      dst[(int64_t)co * TAPS * Cin + tap * Cin + ci] = v;
    else
      dst[(int64_t)ci * TAPS * Cout + (TAPS - 1 - tap) * Cout + co] = v;
  }
}

// chunk k of weight row o -> LDS chunk index; rows are padded to KCP chunks (a
// multiple of 8, KCP = 8 mod 16 for the shapes here) so the XOR stays inside the
// row, and the key (o / 2) spreads 16 consecutive rows over 16 slots
template <int KCP>
__device__ __forceinline__ int wslot(int o, int k) {
  static_assert(KCP % 8 == 0, "padded row");
  return o * KCP + (k ^ ((o >> 1) & 7));
}

// Asynchronous global -> LDS copy of 16 bytes per lane (gfx950
// global_load_lds_dwordx4: lane i's bytes land at lds_base + 16 i), its wait,
// and a barrier without the workgroup fence (a fence would also wait for the
// copies in flight).  The instruction text exists only in the device pass.
__device__ __forceinline__ void copy16_to_lds(const void* src, void* lds_base) {
  async::copy16(src, lds_base);
}
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

// Forward layer (and dIn with the adjoint weights): out^T = W' . X as an
// implicit GEMM with M = Cout (the prepared weights, A operand), N = pixels
// (B operand, gathered from the LDS halo: pad2D |> slide2D as an index view)
// and K = 9 * Cin.
//   * persistent workgroups of 4 waves; a wave owns one cout block of 32 and
//     NPB blocks of 32 pixels of one tile row; its weight fragments for every
//     k-step stay in registers for the whole kernel (36 x 16 bytes per lane
//     for 64 input channels), so only pixels are read from LDS;
//   * a tile is TYF rows x 64 pixels of one image (TYF = 1 for 64 output
//     channels, 2 for 32); its (TYF+2) x 66 halo is copied global -> LDS
//     asynchronously into a ring of NBUF buffers, NBUF - 1 tiles ahead of the
//     one being reduced; out-of-image halo pixels are fetched from a zeroed
//     256-byte page (zero padding) or from the clamped pixel;
//   * the waits count instructions: every tile issues the same copies (the
//     tail re-copies the band's last tile into a free buffer) and the same
//     stores (out-of-image outputs go to a 256-byte dump page), so "the copies
//     of tile i+1 have landed" is a fixed vmcnt;
//   * halo pixels sit at an odd pitch of CH + 1 16-byte chunks (one chunk of
//     padding per pixel, filled from the zero page), so the 16 pixels a lane
//     group reads at one chunk hit 16 distinct bank slots, and every fragment
//     read of a row is one base register plus an immediate offset (a swizzle
//     would cost address arithmetic per read);
//   * the D layout gives each lane 4 consecutive output channels of a pixel
//     per register group: rounded to bf16 and stored as 8 bytes.
template <int CI, int CO>
struct FwdCfg {
  static constexpr int CH = CI / 8;                 // 16-byte chunks per pixel
  static constexpr int NCB = CO / 32;               // cout blocks
  static constexpr int NPB = 1;                     // pixel blocks per wave (registers)
  static constexpr int WPR = NCB * (2 / NPB);       // waves per tile row
  static constexpr int RPW = WPR == 4 ? 2 : 1;      // rows each wave computes, one after the other
  static constexpr int TYF = 4 / WPR * RPW;         // tile rows
  static constexpr int KS = TAPS * CI / 16;         // k-steps of 16
  static constexpr int PITCH = CH + 1;             // chunks per halo pixel (odd)
  static constexpr int SLOTS = (TYF + 2) * HC * PITCH; // halo chunks
  static constexpr int NQ = (SLOTS + 63) / 64;      // wave-sized copies per tile
  static constexpr int QPW = (NQ + 3) / 4;          // copies per wave (at most)
  static constexpr int NBUF = RPW > 1 ? 2 : 3;      // halo ring (two taller tiles fit 2 per CU)
  static constexpr int XPF = CI == 64 ? 3 : 4;      // fragment lookahead (k-steps)
  static_assert(WPR * TYF == 4 * RPW, "four waves per tile");
};

template <int CI, int CO>
__global__ __launch_bounds__(kThreads, 2) void conv3x3_fwd(
    uint16_t* __restrict__ out, const uint16_t* __restrict__ in,
    const uint16_t* __restrict__ wp, const uint16_t* __restrict__ zero_page,
    uint16_t* __restrict__ dump_page, int B, int H, int W, int zero_pad, int tiles_x, int tiles_y,
    int ntiles, int per) {
  using F = FwdCfg<CI, CO>;
  constexpr int CH = F::CH, NPB = F::NPB, NCB = F::NCB, KS = F::KS, NQ = F::NQ, QPW = F::QPW;
  constexpr int TYF = F::TYF, NBUF = F::NBUF, DIST = NBUF - 1;
  constexpr int RPW = F::RPW;
  constexpr int NST = 4 * NPB * RPW;  // stores per wave per tile
  __shared__ i32x4 halo[NBUF][NQ * 64];  // padded to whole copies; the tail is never read

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int il = lane & 31, kh = lane >> 5;
  const int wrow = wave / F::WPR, rem = wave % F::WPR;
  const int wcb = rem % NCB, wpb = rem / NCB;

  const int xcd = blockIdx.x % kNumXcd, jb = blockIdx.x / kNumXcd;
  const int band_end = (int)((int64_t)ntiles * (xcd + 1) / kNumXcd);
  int t = (int)((int64_t)ntiles * xcd / kNumXcd) + jb;
  if (t >= band_end) return;  // the whole workgroup leaves before any barrier

  // weight fragments: lane (il, kh) holds w'[wcb*32 + il][16 ks + 8 kh .. +8]
  bf16x8 wf[KS];
  {
    const uint16_t* wr = wp + (int64_t)(wcb * 32 + il) * (TAPS * CI) + 8 * kh;
#pragma unroll
    for (int ks = 0; ks < KS; ks++) wf[ks] = *reinterpret_cast<const bf16x8*>(wr + 16 * ks);
  }
  // copy geometry of this lane: copy q of this wave fills slot (wave + 4 q) *
  // 64 + lane = pixel p, chunk c, packed as (halo row << 16 | halo column << 8
  // | chunk), -1 for a pixel's padding chunk and past the halo (recomputed per
  // tile rather than held: it costs a few VALU per copy and no registers
  // across the k loop)
  auto geo = [&](int q) {
    const int g = wave + 4 * q, sl = g * 64 + lane;
    if (g >= NQ || sl >= F::SLOTS) return -1;
    const int p = sl / F::PITCH, c = sl % F::PITCH;
    if (c == CH) return -1;
    return ((p / HC) << 16) | ((p % HC) << 8) | c;
  };
  auto coords = [&](int tt, int& b, int& y0, int& x0) {
    const int per_img = tiles_x * tiles_y;
    b = tt / per_img;
    const int r = tt - b * per_img;
    y0 = (r / tiles_x) * TYF;
    x0 = (r % tiles_x) * TXP;
  };
  const bool offs_fit = (int64_t)(TYF + 2) * W * CI < ((int64_t)1 << 31);
  auto issue = [&](int tt, int buf) {
    int b, y0, x0;
    coords(tt, b, y0, x0);
    const uint16_t* img = in + (int64_t)b * H * W * CI;
    if (offs_fit && y0 >= 1 && y0 + TYF + 1 <= H && x0 >= 1 && x0 + TXP + 1 <= W) {
      // interior tile (no clamping): every copy reads the halo's first pixel
      // plus an offset given by the copy geometry
      const uint16_t* base = img + ((int64_t)(y0 - 1) * W + (x0 - 1)) * CI;
#pragma unroll
      for (int q = 0; q < QPW; q++) {
        const int g = wave + 4 * q;
        if (g < NQ) {
          const int gq = geo(q);
          const int off = ((gq >> 16) * W + ((gq >> 8) & 255)) * CI + (gq & 255) * 8;
          copy16_to_lds(gq >= 0 ? (const void*)(base + off) : zero_page, &halo[buf][g * 64]);
        }
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < QPW; q++) {
      const int g = wave + 4 * q;
      if (g < NQ) {
        const int gq = geo(q);
        const void* src = zero_page;
        if (gq >= 0) {
          int gy = y0 - 1 + (gq >> 16), gx = x0 - 1 + ((gq >> 8) & 255);
          const bool inside = gy >= 0 && gy < H && gx >= 0 && gx < W;
          if (inside || !zero_pad) {
            gy = gy < 0 ? 0 : (gy >= H ? H - 1 : gy);
            gx = gx < 0 ? 0 : (gx >= W ? W - 1 : gx);
            src = img + ((int64_t)gy * W + gx) * CI + (gq & 255) * 8;
          }
        }
        copy16_to_lds(src, &halo[buf][g * 64]);
      }
    }
  };

  // the copies of one tile by this wave (wave-uniform)
  const bool full_copies = wave + 4 * (QPW - 1) < NQ;
  const int last = band_end - 1;
#pragma unroll
  for (int d = 0; d < DIST; d++) issue(min(t + d * per, last), d);
  wait_vmcnt<0>();  // the first tiles' copies (and the weight loads) have landed
  int buf = 0;
  while (true) {
    const int next = t + per;
    const bool more = next < band_end;
    wait_lgkmcnt0();  // this wave's reads of the previous buffer are done
    raw_barrier();    // every wave's copies into halo[buf] are visible
    // refill the buffer reduced in the previous iteration, DIST tiles ahead
    issue(min(t + DIST * per, last), (buf + DIST) % NBUF);

    // the wave's rows of the tile, one after the other (same registers)
#pragma unroll 1
    for (int rr = 0; rr < RPW; rr++) {
      f32x16 acc[NPB];
#pragma unroll
      for (int pb = 0; pb < NPB; pb++)
#pragma unroll
        for (int r = 0; r < 16; r++) acc[pb][r] = 0.f;
      // pixel fragments are read XPF k-steps ahead of their MFMA (a ring of
      // XPF + 1 register slots): one MFMA per k-step is shorter than the LDS
      // latency, so a one-step lookahead would stall every step
      constexpr int XPF = F::XPF;
      bf16x8 xf[XPF + 1][NPB];
      auto read_x = [&](int ks, int slot) {
        const int tap = ks / (CI / 16), c16 = ks % (CI / 16);
        const int dy = tap / 3, dx = tap % 3;
#pragma unroll
        for (int pb = 0; pb < NPB; pb++) {
          const int p = (wrow * RPW + rr + dy) * HC + 32 * (wpb * NPB + pb) + il + dx;
          xf[slot][pb] = __builtin_bit_cast(bf16x8, halo[buf][p * F::PITCH + 2 * c16 + kh]);
        }
      };
#pragma unroll
      for (int ks = 0; ks < XPF && ks < KS; ks++) read_x(ks, ks);
#pragma unroll
      for (int ks = 0; ks < KS; ks++) {
        if (ks + XPF < KS) read_x(ks + XPF, (ks + XPF) % (XPF + 1));
#pragma unroll
        for (int pb = 0; pb < NPB; pb++)
          acc[pb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[ks], xf[ks % (XPF + 1)][pb], acc[pb],
                                                            0, 0, 0);
#pragma unroll
        for (int pb = 0; pb < NPB; pb++) {
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
        }
      }

      int b, y0, x0;
      coords(t, b, y0, x0);
      const int y = y0 + wrow * RPW + rr;
#pragma unroll
      for (int pb = 0; pb < NPB; pb++) {
        const int x = x0 + 32 * (wpb * NPB + pb) + il;
        uint16_t* dst = (y < H && x < W)
                            ? out + (((int64_t)b * H + y) * W + x) * CO + wcb * 32 + 4 * kh
                            : dump_page + 4 * kh;
#pragma unroll
        for (int g = 0; g < 4; g++) {
          const uint32_t lo = pack_bf16x2(acc[pb][4 * g], acc[pb][4 * g + 1]);
          const uint32_t hi = pack_bf16x2(acc[pb][4 * g + 2], acc[pb][4 * g + 3]);
          *reinterpret_cast<uint2*>(dst + 8 * g) = uint2{lo, hi};
        }
      }
    }
    // the next tile's copies have landed: younger than them are the copies of
    // DIST - 1 later tiles and the stores of the DIST latest tiles (this one's included)
    if (full_copies)
      wait_vmcnt<DIST * NST + (DIST - 1) * QPW>();
    else
      wait_vmcnt<DIST * NST + (DIST - 1) * (QPW - 1)>();
    if (!more) break;
    t = next;
    buf = (buf + 1) % NBUF;
  }
}

// ---------------------------------------------------------------------------
// dW: each workgroup accumulates dW^T restricted to its tiles.
//   dWt[o][tap * CI + ci] = sum over pixels of dOut[px][o] * in[px shifted by tap][ci]
// Tile: 2 rows x 64 pixels.  M = CO (lane rows), N = 9*CI (lane columns),
// K = the tile's 128 pixels, 8 consecutive pixels of one row per lane.
// The tiles sit in LDS as stored (NHWC: a pixel's channels contiguous, rows
// padded by 16 bytes) and the MFMA fragments, which need 8 consecutive pixels
// of one channel per lane, are read with the gfx950 LDS transpose read
// ds_read_b64_tr_b16.  Within each group of 16 lanes it takes the 16 addresses
// as a 16 x 4 block of 16-bit values M[s][e] (lane s supplies the 4 values at
// its address) and returns M[4 j + i / 4][i % 4] as element j of lane i.  With
// source lane s = 4 j + q pointing at channels c0 + 4 q .. + 3 of pixel k0 + j,
// lane i receives channel c0 + i at pixels k0 .. k0 + 3.  One copy of the
// input halo then serves all three tap columns (a tap column is a shift of
// the pixel address).
// ---------------------------------------------------------------------------
constexpr int WTY = 2;               // rows per dW tile
constexpr int WHR = WTY + 2;         // halo rows

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) s16x4 lds_s16x4;

// 4 consecutive pixels of one channel per lane (see above); p points at the
// 16-bit value this lane supplies as a source.
__device__ __forceinline__ s16x4 read_tr16(const uint16_t* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)p);
#else
  return s16x4{0, 0, 0, 0};
#endif
}

template <int CI, int CO>
__global__ __launch_bounds__(kThreads) void conv3x3_dw(
    float* __restrict__ partial, const uint16_t* __restrict__ dout,
    const uint16_t* __restrict__ in, int B, int H, int W, int zero_pad, int tiles_x,
    int tiles_y, int ntiles) {
  // dW^T is CO x 9 CI in 32 x 32 blocks: row blocks mb (output channels), column
  // blocks nb (tap, input channel).  Wave w owns column blocks w, w + 4, ... for
  // every row block, so each input fragment it reads feeds CO / 32 MFMAs
  constexpr int MB = CO / 32;                         // row blocks
  constexpr int NBC = TAPS * CI / 32;                 // column blocks
  constexpr int PER_WAVE = (NBC + 3) / 4;             // column blocks per wave (at most)
  static_assert(CI % 32 == 0 && CO % 32 == 0, "channel counts");
  constexpr int PXT = WTY * TXP;                      // pixels per tile (128)
  constexpr int GS = CO + 8;                          // dOut pixel stride (16-bit values)
  constexpr int XS = CI + 8;                          // input pixel stride
  __shared__ __attribute__((aligned(16))) uint16_t go[PXT * GS];       // [pixel][o]
  __shared__ __attribute__((aligned(16))) uint16_t xs[WHR * HC * XS];  // [row][column][ci]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int il = lane & 31, kh = lane >> 5;
  // transpose-read source coordinates of this lane: pixel offset and channel offset
  const int grp16 = lane >> 4, i16 = lane & 15;
  const int src_px = 8 * (grp16 >> 1) + (i16 >> 2);   // + 4 for the second read
  const int src_ch = 16 * (grp16 & 1) + 4 * (i16 & 3);
  // Workgroup b runs on XCD b % 8; a workgroup walks a contiguous run of tiles,
  // in which vertically neighbouring tiles (two shared halo rows) follow each other.
  const int run = (ntiles + gridDim.x - 1) / gridDim.x;
  const int t0 = blockIdx.x * run, t_end = min(ntiles, t0 + run);
  f32x16 acc[PER_WAVE][MB];
#pragma unroll
  for (int q = 0; q < PER_WAVE; q++)
#pragma unroll
    for (int m = 0; m < MB; m++)
#pragma unroll
      for (int r = 0; r < 16; r++) acc[q][m][r] = 0.f;

  // All 16-byte loads of a tile are issued together (clamped addresses; a flag
  // says which values padding zeroes), one tile ahead: they are in flight
  // while the current tile's MFMAs run.
  constexpr int NGC = PXT * (CO / 8);                 // dOut chunks
  constexpr int NXC = WHR * HC * (CI / 8);            // input halo chunks
  constexpr int NG = NGC / kThreads;
  constexpr int NX = (NXC + kThreads - 1) / kThreads;
  static_assert(NGC % kThreads == 0 && NG + NX <= 32, "chunks per thread");
  i32x4 gv[NG], xv[NX];
  uint32_t zero = 0;
  auto fetch = [&](int t) {
    const int b = t / (tiles_x * tiles_y);
    const int rem = t - b * tiles_x * tiles_y;
    const int ty = rem % tiles_y, tx = rem / tiles_y;
    const int y0 = ty * WTY, x0 = tx * TXP;
    const uint16_t* img = in + (int64_t)b * H * W * CI;
    const uint16_t* g = dout + (int64_t)b * H * W * CO;
    zero = 0;
#pragma unroll
    for (int i = 0; i < NG; i++) {
      const int c = tid + i * kThreads, p = c / (CO / 8), ch = c - p * (CO / 8);
      const int gy = y0 + p / TXP, gx = x0 + p % TXP;
      const int gyc = gy >= H ? H - 1 : gy, gxc = gx >= W ? W - 1 : gx;
      gv[i] = reinterpret_cast<const i32x4*>(g + ((int64_t)gyc * W + gxc) * CO)[ch];
      if (gy >= H || gx >= W) zero |= 1u << i;  // outputs outside the image do not exist
    }
#pragma unroll
    for (int i = 0; i < NX; i++) {
      const int c = min(tid + i * kThreads, NXC - 1), hp = c / (CI / 8), ch = c - hp * (CI / 8);
      const int hr = hp / HC, hc = hp - hr * HC;
      const int gy = y0 - 1 + hr, gx = x0 - 1 + hc;
      const int gyc = gy < 0 ? 0 : (gy >= H ? H - 1 : gy), gxc = gx < 0 ? 0 : (gx >= W ? W - 1 : gx);
      xv[i] = reinterpret_cast<const i32x4*>(img + ((int64_t)gyc * W + gxc) * CI)[ch];
      const bool inside = gy >= 0 && gy < H && gx >= 0 && gx < W;
      if (zero_pad && !inside) zero |= 1u << (NG + i);
    }
  };
  if (t0 < t_end) fetch(t0);
  for (int t = t0; t < t_end; t++) {
    __syncthreads();  // every wave is done reading the previous tile
    const i32x4 z4 = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < NG; i++) {
      const int c = tid + i * kThreads, p = c / (CO / 8), ch = c - p * (CO / 8);
      *reinterpret_cast<i32x4*>(&go[p * GS + 8 * ch]) = (zero >> i) & 1u ? z4 : gv[i];
    }
#pragma unroll
    for (int i = 0; i < NX; i++) {
      const int c = tid + i * kThreads;
      if (c < NXC) {
        const int hp = c / (CI / 8), ch = c - hp * (CI / 8);
        *reinterpret_cast<i32x4*>(&xs[hp * XS + 8 * ch]) = (zero >> (NG + i)) & 1u ? z4 : xv[i];
      }
    }
    if (t + 1 < t_end) fetch(t + 1);
    __syncthreads();
    // K loop over the tile's pixels: 16 per step, rows r = 0..WTY-1, 64 pixels each
#pragma unroll
    for (int ks = 0; ks < PXT / 16; ks++) {
      const int r = (16 * ks) / TXP;
      const int pb = (16 * ks) % TXP + src_px;  // this lane's source pixel in row r
      bf16x8 av[MB];
#pragma unroll
      for (int m = 0; m < MB; m++) {
        const uint16_t* pa = &go[(r * TXP + pb) * GS + 32 * m + src_ch];
        const s16x4 lo = read_tr16(pa), hi = read_tr16(pa + 4 * GS);
        av[m] = __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
      }
#pragma unroll
      for (int q = 0; q < PER_WAVE; q++) {
        const int nb = wave + 4 * q;
        if (nb >= NBC) break;  // wave-uniform
        const int n0 = 32 * nb;  // n = tap * CI + ci
        const int tap = n0 / CI, c0 = n0 - tap * CI;
        const int dy = tap / 3, dx = tap - dy * 3;
        const uint16_t* pbv = &xs[((r + dy) * HC + pb + dx) * XS + c0 + src_ch];
        const s16x4 lo = read_tr16(pbv), hi = read_tr16(pbv + 4 * XS);
        const bf16x8 bv =
            __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
#pragma unroll
        for (int m = 0; m < MB; m++)
          acc[q][m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[m], bv, acc[q][m], 0, 0, 0);
      }
    }
  }
  // partial[block][o][n] of dW^T
  float* dst = partial + (int64_t)blockIdx.x * CO * TAPS * CI;
#pragma unroll
  for (int q = 0; q < PER_WAVE; q++) {
    const int nb = wave + 4 * q;
    if (nb >= NBC) break;
#pragma unroll
    for (int m = 0; m < MB; m++)
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int o = 32 * m + 8 * (r >> 2) + 4 * kh + (r & 3);
        const int n = 32 * nb + il;
        dst[(int64_t)o * TAPS * CI + n] = acc[q][m][r];
      }
  }
}

// dW[co][ci][tap] = sum over blocks of partial[block][co][tap * CI + ci] (fixed order)
__global__ __launch_bounds__(kThreads) void conv_dw_reduce(float* __restrict__ dw,
                                                           const float* __restrict__ partial,
                                                           int blocks, int CO, int CI) {
  const int n = CO * TAPS * CI;
  const int e = blockIdx.x * kThreads + threadIdx.x;
  if (e >= n) return;
  // the sum runs in block order; the loads of 8 blocks are issued together
  float s = 0.f;
  int q = 0;
  for (; q + 8 <= blocks; q += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; u++) v[u] = partial[(int64_t)(q + u) * n + e];
#pragma unroll
    for (int u = 0; u < 8; u++) s += v[u];
  }
  for (; q < blocks; q++) s += partial[(int64_t)q * n + e];
  const int o = e / (TAPS * CI), rem = e - o * TAPS * CI, tap = rem / CI, ci = rem - tap * CI;
  dw[((int64_t)o * CI + ci) * TAPS + tap] = s;
}

// Persistent workgroups of the dW kernel (each walks a contiguous run of tiles).
int dw_blocks(int B, int H, int W) {
  int64_t tiles = (int64_t)B * ((H + WTY - 1) / WTY) * ((W + TXP - 1) / TXP);
  int64_t blocks = 256 * 2;  // two workgroups per CU on 256 CUs
  return (int)(tiles < blocks ? tiles : blocks);
}

template <int CI, int CO>
rise_status launch_fwd(uint16_t* out, const uint16_t* in, const uint16_t* wp,
                       const uint16_t* zero_page, uint16_t* dump_page, int B, int H, int W,
                       int zero, hipStream_t s) {
  constexpr int TYF = FwdCfg<CI, CO>::TYF;
  const int tiles_x = (W + TXP - 1) / TXP, tiles_y = (H + TYF - 1) / TYF;
  const int64_t ntiles = (int64_t)B * tiles_x * tiles_y;
  if (ntiles > INT32_MAX) return fail(RISE_ERR_SHAPE, "conv: too many tiles");
  // workgroups per XCD: as many as stay resident, evened out over the band
  static const int occ = [] {
    int o = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, conv3x3_fwd<CI, CO>, kThreads, 0) !=
            hipSuccess || o < 1)
      o = 1;
    return o;
  }();
  const int64_t band = (ntiles + kNumXcd - 1) / kNumXcd;
  const int64_t max_per = std::max<int64_t>(1, (int64_t)occ * device_cu_count() / kNumXcd);
  const int64_t rounds = (band + max_per - 1) / max_per;
  const int per = (int)std::max<int64_t>(1, (band + rounds - 1) / rounds);
  hipLaunchKernelGGL((conv3x3_fwd<CI, CO>), dim3(kNumXcd * per), dim3(kThreads), 0, s, out, in,
                     wp, zero_page, dump_page, B, H, W, zero, tiles_x, tiles_y, (int)ntiles, per);
  return check_launch("conv3x3_fwd");
}

template <int CI, int CO>
rise_status launch_dw(float* partial, const uint16_t* dout, const uint16_t* in, int B, int H,
                      int W, int zero, hipStream_t s) {
  const int tiles_x = (W + TXP - 1) / TXP, tiles_y = (H + WTY - 1) / WTY;
  const int ntiles = B * tiles_x * tiles_y;
  const int grid = dw_blocks(B, H, W);
  hipLaunchKernelGGL((conv3x3_dw<CI, CO>), dim3(grid), dim3(kThreads), 0, s, partial, dout, in, B,
                     H, W, zero, tiles_x, tiles_y, ntiles);
  return check_launch("conv3x3_dw");
}

rise_status fwd_dispatch(uint16_t* out, const uint16_t* in, const uint16_t* wp, void* pages,
                         int B, int CI, int CO, int H, int W, int zero, hipStream_t s) {
  const uint16_t* zero_page = (const uint16_t*)pages;
  uint16_t* dump_page = (uint16_t*)((char*)pages + 256);
#define RISE_CONV_CASE(I, O) \
  if (CI == I && CO == O)    \
    return launch_fwd<I, O>(out, in, wp, zero_page, dump_page, B, H, W, zero, s);
  RISE_CONV_CASE(16, 32) RISE_CONV_CASE(16, 64) RISE_CONV_CASE(32, 32)
  RISE_CONV_CASE(32, 64) RISE_CONV_CASE(64, 32) RISE_CONV_CASE(64, 64)
#undef RISE_CONV_CASE
  return fail(RISE_ERR_UNSUPPORTED, "conv: channel counts");
}

rise_status dw_dispatch(float* partial, const uint16_t* dout, const uint16_t* in, int B, int CI,
                        int CO, int H, int W, int zero, hipStream_t s) {
  if (CI == 32 && CO == 32) return launch_dw<32, 32>(partial, dout, in, B, H, W, zero, s);
  if (CI == 32 && CO == 64) return launch_dw<32, 64>(partial, dout, in, B, H, W, zero, s);
  if (CI == 64 && CO == 32) return launch_dw<64, 32>(partial, dout, in, B, H, W, zero, s);
  if (CI == 64 && CO == 64) return launch_dw<64, 64>(partial, dout, in, B, H, W, zero, s);
  return fail(RISE_ERR_UNSUPPORTED, "conv backward: channel counts");
}

size_t round256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

bool conv_supported(int Cin, int Cout, int kh, int kw, bool backward) {
  if (kh != 3 || kw != 3) return false;
  bool fwd_ok = (Cin == 16 || Cin == 32 || Cin == 64) && (Cout == 32 || Cout == 64);
  if (!backward) return fwd_ok;
  // backward runs the forward kernel with the roles of Cin and Cout swapped (dIn) and the
  // dW kernel
  bool din_ok = (Cout == 16 || Cout == 32 || Cout == 64) && (Cin == 32 || Cin == 64);
  bool dw_ok = (Cin == 32 || Cin == 64) && (Cout == 32 || Cout == 64);
  return din_ok && dw_ok;
}

// workspace: [prepared bf16 weights | 256-byte zero page | 256-byte dump page |
//             dW partials (backward)]
size_t conv_forward_workspace(int Cin, int Cout) {
  return round256((size_t)Cout * TAPS * Cin * 2) + 512;
}

size_t conv_backward_workspace(int B, int Cin, int Cout, int H, int W) {
  return conv_forward_workspace(Cin, Cout) + (size_t)dw_blocks(B, H, W) * Cout * TAPS * Cin * 4;
}

rise_status launch_conv2d(const ConvArgs& a, void* ws, hipStream_t s) {
  uint16_t* wp = (uint16_t*)ws;
  uint16_t* zp = (uint16_t*)((char*)ws + round256((size_t)a.Cout * TAPS * a.Cin * 2));
  hipLaunchKernelGGL(conv_prep_weights, dim3(64), dim3(kThreads), 0, s, wp, zp, a.w, a.Cout, a.Cin,
                     0);
  rise_status st = check_launch("conv_prep_weights");
  if (st != RISE_OK) return st;
  return fwd_dispatch(a.out, a.in, wp, zp, a.B, a.Cin, a.Cout, a.H, a.W, a.zero_pad, s);
}

rise_status launch_conv2d_backward(const ConvBwdArgs& a, void* ws, hipStream_t s) {
  uint16_t* wp = (uint16_t*)ws;
  uint16_t* zp = (uint16_t*)((char*)ws + round256((size_t)a.Cout * TAPS * a.Cin * 2));
  float* partial = (float*)((char*)ws + conv_forward_workspace(a.Cin, a.Cout));
  rise_status st = RISE_OK;
  if (a.din) {
    // dIn = the layer with dOut as input, channel roles swapped and the window rotated
    hipLaunchKernelGGL(conv_prep_weights, dim3(64), dim3(kThreads), 0, s, wp, zp, a.w, a.Cout,
                       a.Cin, 1);
    if ((st = check_launch("conv_prep_weights")) != RISE_OK) return st;
    st = fwd_dispatch(a.din, a.dout, wp, zp, a.B, a.Cout, a.Cin, a.H, a.W, 1, s);
    if (st != RISE_OK) return st;
  }
  if (a.dw) {
    st = dw_dispatch(partial, a.dout, a.in, a.B, a.Cin, a.Cout, a.H, a.W, a.zero_pad, s);
    if (st != RISE_OK) return st;
    const int n = a.Cout * TAPS * a.Cin;
    hipLaunchKernelGGL(conv_dw_reduce, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                       a.dw, partial, dw_blocks(a.B, a.H, a.W), a.Cout, a.Cin);
    if ((st = check_launch("conv_dw_reduce")) != RISE_OK) return st;
  }
  return RISE_OK;
}

}  // namespace rise
