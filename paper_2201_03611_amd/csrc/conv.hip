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
// 180 degrees and the channel roles swapped):
//   * persistent workgroups; the whole prepared weight matrix [Cout][9*Cin]
//     (bf16, 73.7 KB for 64 -> 64) is loaded into LDS once per workgroup;
//   * a tile is 4 rows x 64 pixels of one image: its (4+2) x (64+2) halo is
//     staged in LDS with 16-byte chunks XOR-swizzled by pixel so that the 32
//     pixels a half-wave reads hit distinct banks;
//   * wave w computes row w of the tile: 64 pixels x Cout with
//     v_mfma_f32_32x32x16_bf16, 8 consecutive input channels per lane;
//   * the FP32 result is rounded to bf16 and staged through LDS for 16-byte
//     coalesced NHWC stores.
// dW (the gradient of the weights) contracts over pixels instead: per tile the
// dOut tile and the input halo are staged transposed (pixels contiguous, one
// copy per horizontal tap offset so every fragment read is aligned), each
// workgroup accumulates its share of dW^T in registers, and a fixed-order
// reduction over workgroups finishes it.
#include "common.h"
#include "conv.h"

namespace rise {
namespace {

constexpr int kThreads = 256;
constexpr int TY = 4;                // output rows per forward tile (one per wave)
constexpr int TXP = 64;              // output pixels per row of a tile
constexpr int HR = TY + 2;           // halo rows
constexpr int HC = TXP + 2;          // halo columns
constexpr int TAPS = 9;

__device__ __forceinline__ uint16_t f32_to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// dst[o][tap * I + i] = bf16(weight), with
//   forward : o = co, i = ci, weight = w[co][ci][tap]
//   adjoint : o = ci, i = co, weight = w[co][ci][8 - tap]   (180-degree rotation)
__global__ void conv_prep_weights(uint16_t* __restrict__ dst, const float* __restrict__ w, int Cout,
                                  int Cin, int adjoint) {
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

// 16-byte chunk c of halo pixel p (CH chunks per pixel) -> LDS chunk index.  A
// 16-lane group of ds_read_b128 is served from one 256-byte line (64 banks): the
// XOR key changes every 16/CH pixels so 16 consecutive pixels at one logical
// chunk use 16 distinct slots.
template <int CH>
__device__ __forceinline__ int halo_slot(int p, int c) {
  return p * CH + (c ^ ((p / (16 / CH)) % CH));
}
// chunk k of weight row o -> LDS chunk index; rows are padded to KCP chunks (a
// multiple of 8, KCP = 8 mod 16 for the shapes here) so the XOR stays inside the
// row, and the key (o / 2) spreads 16 consecutive rows over 16 slots
template <int KCP>
__device__ __forceinline__ int wslot(int o, int k) {
  static_assert(KCP % 8 == 0, "padded row");
  return o * KCP + (k ^ ((o >> 1) & 7));
}

template <int CI, int CO>
__global__ __launch_bounds__(kThreads, 1) void conv3x3_fwd(
    uint16_t* __restrict__ out, const uint16_t* __restrict__ in,
    const uint16_t* __restrict__ wp, int B, int H, int W, int zero_pad, int tiles_x,
    int tiles_y, int ntiles) {
  constexpr int CH = CI / 8;            // 16-byte chunks per halo pixel
  constexpr int KC = TAPS * CI / 8;     // 16-byte chunks per weight row
  constexpr int KCP = (KC + 7) / 8 * 8; // padded row in LDS
  constexpr int NJ = CO / 32;           // 32-wide output-channel blocks
  constexpr int HALO_CHUNKS = HR * HC * CH;
  constexpr int STAGE_CHUNKS = TY * TXP * CO / 8;
  constexpr int BUF = HALO_CHUNKS > STAGE_CHUNKS ? HALO_CHUNKS : STAGE_CHUNKS;
  static_assert(CI % 16 == 0 && CO % 32 == 0, "channel counts");
  __shared__ i32x4 wl[CO * KCP];
  __shared__ i32x4 buf[BUF];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int il = lane & 31, kh = lane >> 5;

  for (int c = tid; c < CO * KC; c += kThreads) {
    const int o = c / KC, k = c - o * KC;
    wl[wslot<KCP>(o, k)] = reinterpret_cast<const i32x4*>(wp)[c];
  }

  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int b = t / (tiles_x * tiles_y);
    const int rem = t - b * tiles_x * tiles_y;
    const int ty = rem % tiles_y, tx = rem / tiles_y;  // walk down a column of tiles
    const int y0 = ty * TY, x0 = tx * TXP;
    const uint16_t* img = in + (int64_t)b * H * W * CI;
    __syncthreads();  // previous tile's staging reads (and the weight stores) are done

    for (int c = tid; c < HALO_CHUNKS; c += kThreads) {
      const int p = c / CH, ch = c - p * CH;
      const int hr = p / HC, hc = p - hr * HC;
      int gy = y0 - 1 + hr, gx = x0 - 1 + hc;
      i32x4 v = {0, 0, 0, 0};
      const bool inside = gy >= 0 && gy < H && gx >= 0 && gx < W;
      if (inside || !zero_pad) {
        gy = gy < 0 ? 0 : (gy >= H ? H - 1 : gy);
        gx = gx < 0 ? 0 : (gx >= W ? W - 1 : gx);
        v = reinterpret_cast<const i32x4*>(img + ((int64_t)gy * W + gx) * CI)[ch];
      }
      buf[halo_slot<CH>(p, ch)] = v;
    }
    __syncthreads();

    f32x16 acc[2][NJ];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
      for (int j = 0; j < NJ; j++)
#pragma unroll
        for (int r = 0; r < 16; r++) acc[i][j][r] = 0.f;

#pragma unroll 1
    for (int tap = 0; tap < TAPS; tap++) {
      const int dy = tap / 3, dx = tap - dy * 3;
#pragma unroll
      for (int c16 = 0; c16 < CI / 16; c16++) {
        const int ch = 2 * c16 + kh;
        bf16x8 a[2], bb[NJ];
#pragma unroll
        for (int i = 0; i < 2; i++) {
          const int p = (wave + dy) * HC + 32 * i + il + dx;
          a[i] = __builtin_bit_cast(bf16x8, buf[halo_slot<CH>(p, ch)]);
        }
#pragma unroll
        for (int j = 0; j < NJ; j++)
          bb[j] = __builtin_bit_cast(bf16x8, wl[wslot<KCP>(32 * j + il, tap * CH + ch)]);
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
          for (int j = 0; j < NJ; j++)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], bb[j], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();  // halo no longer read: reuse it as the output staging area

    uint16_t* stage = reinterpret_cast<uint16_t*>(buf);
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
      for (int j = 0; j < NJ; j++)
#pragma unroll
        for (int r = 0; r < 16; r++) {
          const int px = 32 * i + 8 * (r >> 2) + 4 * kh + (r & 3);
          stage[(wave * TXP + px) * CO + 32 * j + il] = f32_to_bf16(acc[i][j][r]);
        }
    __syncthreads();
    uint16_t* dst = out + (int64_t)b * H * W * CO;
    for (int c = tid; c < STAGE_CHUNKS; c += kThreads) {
      const int p = c / (CO / 8), ch = c - p * (CO / 8);
      const int ry = p / TXP, rx = p - ry * TXP;
      const int gy = y0 + ry, gx = x0 + rx;
      if (gy < H && gx < W)
        reinterpret_cast<i32x4*>(dst + ((int64_t)gy * W + gx) * CO)[ch] = buf[c];
    }
  }
}

// ---------------------------------------------------------------------------
// dW: each workgroup accumulates dW^T restricted to its tiles.
//   dWt[o][tap * CI + ci] = sum over pixels of dOut[px][o] * in[px shifted by tap][ci]
// Tile: 2 rows x 64 pixels.  M = CO (lane rows), N = 9*CI (lane columns),
// K = the tile's 128 pixels, 8 consecutive pixels of one row per lane.
// ---------------------------------------------------------------------------
constexpr int WTY = 2;               // rows per dW tile
constexpr int WHR = WTY + 2;         // halo rows

template <int CI, int CO>
__global__ __launch_bounds__(kThreads, 1) void conv3x3_dw(
    float* __restrict__ partial, const uint16_t* __restrict__ dout,
    const uint16_t* __restrict__ in, int B, int H, int W, int zero_pad, int tiles_x,
    int tiles_y, int ntiles) {
  constexpr int NBLK = (CO / 32) * (TAPS * CI / 32);  // 32 x 32 blocks of dW^T
  constexpr int PER_WAVE = (NBLK + 3) / 4;            // wave w owns blocks w, w + 4, ...
  static_assert(CI % 32 == 0 && CO % 32 == 0, "channel counts");
  constexpr int PXT = WTY * TXP;                      // pixels per tile (128)
  // dOut tile transposed: go[o * GP + p], p = r * TXP + x; input halo transposed and
  // shifted: xs[(dx * CI + ci) * XP + hr * TXP + p] = in[row hr][pixel p + dx - 1][ci].
  // The per-channel strides GP and XP are odd multiples of 16 bytes, so the 32
  // channels a half-wave reads fall in distinct bank groups.
  constexpr int GP = PXT + 8;
  constexpr int XP = WHR * TXP + 8;
  __shared__ __attribute__((aligned(16))) uint16_t go[CO * GP];
  __shared__ __attribute__((aligned(16))) uint16_t xs[3 * CI * XP];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int il = lane & 31, kh = lane >> 5;
  f32x16 acc[PER_WAVE];
#pragma unroll
  for (int q = 0; q < PER_WAVE; q++)
#pragma unroll
    for (int r = 0; r < 16; r++) acc[q][r] = 0.f;

  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int b = t / (tiles_x * tiles_y);
    const int rem = t - b * tiles_x * tiles_y;
    const int ty = rem % tiles_y, tx = rem / tiles_y;
    const int y0 = ty * WTY, x0 = tx * TXP;
    const uint16_t* img = in + (int64_t)b * H * W * CI;
    const uint16_t* g = dout + (int64_t)b * H * W * CO;
    __syncthreads();
    // dOut tile -> go[o][p] (zero outside the image: those outputs do not exist)
    for (int c = tid; c < PXT * CO / 8; c += kThreads) {
      const int p = c / (CO / 8), ch = c - p * (CO / 8);
      const int gy = y0 + p / TXP, gx = x0 + p % TXP;
      i32x4 v = {0, 0, 0, 0};
      if (gy < H && gx < W) v = reinterpret_cast<const i32x4*>(g + ((int64_t)gy * W + gx) * CO)[ch];
      const uint16_t* e = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
      for (int q = 0; q < 8; q++) go[(ch * 8 + q) * GP + p] = e[q];
    }
    // input halo -> three shifted transposed copies
    for (int c = tid; c < WHR * HC * (CI / 8); c += kThreads) {
      const int hp = c / (CI / 8), ch = c - hp * (CI / 8);
      const int hr = hp / HC, hc = hp - hr * HC;
      int gy = y0 - 1 + hr, gx = x0 - 1 + hc;
      i32x4 v = {0, 0, 0, 0};
      const bool inside = gy >= 0 && gy < H && gx >= 0 && gx < W;
      if (inside || !zero_pad) {
        gy = gy < 0 ? 0 : (gy >= H ? H - 1 : gy);
        gx = gx < 0 ? 0 : (gx >= W ? W - 1 : gx);
        v = reinterpret_cast<const i32x4*>(img + ((int64_t)gy * W + gx) * CI)[ch];
      }
      const uint16_t* e = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
      for (int dx = 0; dx < 3; dx++) {
        const int p = hc - dx;  // output pixel whose tap dx reads this halo column
        if (p >= 0 && p < TXP) {
#pragma unroll
          for (int q = 0; q < 8; q++)
            xs[(dx * CI + ch * 8 + q) * XP + hr * TXP + p] = e[q];
        }
      }
    }
    __syncthreads();
    // K loop over the tile's pixels: 8 per lane, rows r = 0..WTY-1, 64 pixels each
#pragma unroll
    for (int ks = 0; ks < PXT / 16; ks++) {
      const int r = (16 * ks) / TXP;
      const int p0 = (16 * ks) % TXP + 8 * kh;
#pragma unroll
      for (int q = 0; q < PER_WAVE; q++) {
        const int blk = wave + 4 * q;
        if (blk >= NBLK) break;  // wave-uniform
        const int mb = blk % (CO / 32), nb = blk / (CO / 32);
        const int o = 32 * mb + il;
        const int n = 32 * nb + il;  // n = tap * CI + ci
        const int tap = n / CI, ci = n - tap * CI;
        const int dy = tap / 3, dx = tap - dy * 3;
        const bf16x8 av =
            __builtin_bit_cast(bf16x8, *reinterpret_cast<const i32x4*>(&go[o * GP + r * TXP + p0]));
        const bf16x8 bv = __builtin_bit_cast(
            bf16x8, *reinterpret_cast<const i32x4*>(&xs[(dx * CI + ci) * XP + (r + dy) * TXP + p0]));
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[q], 0, 0, 0);
      }
    }
  }
  // partial[block][o][n] of dW^T
  float* dst = partial + (int64_t)blockIdx.x * CO * TAPS * CI;
#pragma unroll
  for (int q = 0; q < PER_WAVE; q++) {
    const int blk = wave + 4 * q;
    if (blk >= NBLK) break;
    const int mb = blk % (CO / 32), nb = blk / (CO / 32);
#pragma unroll
    for (int r = 0; r < 16; r++) {
      const int o = 32 * mb + 8 * (r >> 2) + 4 * kh + (r & 3);
      const int n = 32 * nb + il;
      dst[(int64_t)o * TAPS * CI + n] = acc[q][r];
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
  float s = 0.f;
  for (int q = 0; q < blocks; q++) s += partial[(int64_t)q * n + e];
  const int o = e / (TAPS * CI), rem = e - o * TAPS * CI, tap = rem / CI, ci = rem - tap * CI;
  dw[((int64_t)o * CI + ci) * TAPS + tap] = s;
}

int dw_blocks(int B, int H, int W) {
  int64_t tiles = (int64_t)B * ((H + WTY - 1) / WTY) * ((W + TXP - 1) / TXP);
  int64_t blocks = 256 * 2;  // two waves of persistent workgroups over 256 CUs
  return (int)(tiles < blocks ? tiles : blocks);
}

template <int CI, int CO>
rise_status launch_fwd(uint16_t* out, const uint16_t* in, const uint16_t* wp, int B, int H, int W,
                       int zero, hipStream_t s) {
  const int tiles_x = (W + TXP - 1) / TXP, tiles_y = (H + TY - 1) / TY;
  const int ntiles = B * tiles_x * tiles_y;
  const int grid = ntiles < 256 ? ntiles : 256;
  hipLaunchKernelGGL((conv3x3_fwd<CI, CO>), dim3(grid), dim3(kThreads), 0, s, out, in, wp, B, H, W,
                     zero, tiles_x, tiles_y, ntiles);
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

rise_status fwd_dispatch(uint16_t* out, const uint16_t* in, const uint16_t* wp, int B, int CI,
                         int CO, int H, int W, int zero, hipStream_t s) {
#define RISE_CONV_CASE(I, O) \
  if (CI == I && CO == O) return launch_fwd<I, O>(out, in, wp, B, H, W, zero, s);
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

size_t conv_forward_workspace(int Cin, int Cout) { return round256((size_t)Cout * TAPS * Cin * 2); }

size_t conv_backward_workspace(int B, int Cin, int Cout, int H, int W) {
  return round256((size_t)Cout * TAPS * Cin * 2) +
         (size_t)dw_blocks(B, H, W) * Cout * TAPS * Cin * 4;
}

rise_status launch_conv2d(const ConvArgs& a, void* ws, hipStream_t s) {
  uint16_t* wp = (uint16_t*)ws;
  hipLaunchKernelGGL(conv_prep_weights, dim3(64), dim3(kThreads), 0, s, wp, a.w, a.Cout, a.Cin, 0);
  rise_status st = check_launch("conv_prep_weights");
  if (st != RISE_OK) return st;
  return fwd_dispatch(a.out, a.in, wp, a.B, a.Cin, a.Cout, a.H, a.W, a.zero_pad, s);
}

rise_status launch_conv2d_backward(const ConvBwdArgs& a, void* ws, hipStream_t s) {
  uint16_t* wp = (uint16_t*)ws;
  float* partial = (float*)((char*)ws + round256((size_t)a.Cout * TAPS * a.Cin * 2));
  rise_status st = RISE_OK;
  if (a.din) {
    // dIn = the layer with dOut as input, channel roles swapped and the window rotated
    hipLaunchKernelGGL(conv_prep_weights, dim3(64), dim3(kThreads), 0, s, wp, a.w, a.Cout, a.Cin,
                       1);
    if ((st = check_launch("conv_prep_weights")) != RISE_OK) return st;
    st = fwd_dispatch(a.din, a.dout, wp, a.B, a.Cout, a.Cin, a.H, a.W, 1, s);
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
