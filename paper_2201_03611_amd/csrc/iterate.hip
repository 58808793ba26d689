// iterate with the tree-reduction body (Sec. VI):
//
//   iterate(n, m, k, split(n) |> map(reduce(+, 0)), arr)
//
// turns n^k * m values into m: each of the k rounds replaces every group of n
// neighbours by their left-fold sum from 0.  The paper compiles iterate into a
// double buffer in memory that the rounds ping-pong through.  Here one kernel
// launch (a "pass") runs as many consecutive rounds as fit one workgroup: the
// workgroup loads a chunk of up to 8192 values that covers whole groups of
// n^L inputs, runs the L rounds in LDS (itself a double buffer: two regions
// that swap source and destination every round) and stores one value per
// group.  Only the pass outputs go through HBM, ping-ponging between the two
// halves of the caller's workspace; the first pass reads the input and the
// last writes the output, as the paper's swap/done commands arrange.
//
// Every round adds in exactly the order the definition gives (left fold from
// 0 within each group, groups independent), so the result is the one a
// sequential float implementation of the program produces, bit for bit.
// Work is one add per input value: the passes are bound by HBM reads.
#include <stdint.h>

#include <algorithm>

#include "common.h"

namespace rise {
namespace {

constexpr int kThreads = 256;
constexpr int kChunk = 8192;              // values per workgroup and pass
constexpr int kVecPerThread = kChunk / 4 / kThreads;
constexpr int kRegionB = kChunk;          // second LDS region (round outputs <= kChunk / 2)
constexpr int kLdsFloats = kChunk + kChunk / 2;

// Word address in LDS of logical index e: the low 6 bits (the bank, 64 banks
// of 4 bytes) are XORed with the folded higher 6-bit groups.  Lanes that read
// with any power-of-two stride then hit 64 different banks.
__device__ __forceinline__ int swz(int e) { return e ^ (((e >> 6) ^ (e >> 12)) & 63); }

// Left fold from 0 over r consecutive values held by one thread; r is 1, 2 or
// 4 (the rounds that fit inside one 16-byte load), n is 2 or 4 when r > 1.
__device__ __forceinline__ void fold_in_regs(float (&v)[4], int n, int r) {
  if (r == 1) return;
  if (n == 2) {  // one round: (0+a)+b pairs; a second round when r == 4
    v[0] = (0.f + v[0]) + v[1];
    v[1] = (0.f + v[2]) + v[3];
    if (r == 4) v[0] = (0.f + v[0]) + v[1];
    return;
  }
  v[0] = (((0.f + v[0]) + v[1]) + v[2]) + v[3];  // n == 4, r == 4
}

// One pass: groups g0 .. g0+q-1 of G = n^L inputs each; rounds 1..a run in
// registers (R = n^a values per register fold), rounds a+1..L in LDS.
__global__ __launch_bounds__(kThreads) void iterate_sum_pass(
    float* __restrict__ dst, const float* __restrict__ src, int64_t len_out, int n, int L,
    int G, int q, int a, int R, int vec) {
  __shared__ float lds[kLdsFloats];
  const int tid = threadIdx.x;
  const int64_t g0 = (int64_t)blockIdx.x * q;
  const int qv = (int)(len_out - g0 < q ? len_out - g0 : q);
  const int C = qv * G;  // values present in this chunk
  const float* s = src + g0 * G;
  if (vec) {
    const int nv = C / 4, per = 4 / R;
    float4 x[kVecPerThread];
#pragma unroll
    for (int i = 0; i < kVecPerThread; i++) {
      const int v = tid + i * kThreads;
      x[i] = v < nv ? reinterpret_cast<const float4*>(s)[v] : float4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int i = 0; i < kVecPerThread; i++) {
      const int v = tid + i * kThreads;
      if (v < nv) {
        float r[4] = {x[i].x, x[i].y, x[i].z, x[i].w};
        fold_in_regs(r, n, R);
        for (int c = 0; c < per; c++) lds[swz(v * per + c)] = r[c];
      }
    }
    // a chunk of C = 4*nv + t values (t < 4, a multiple of R): fold the tail
    const int tail = (C - nv * 4) / R;
    if (tid < tail) {
      float r[4] = {0.f, 0.f, 0.f, 0.f};
      for (int c = 0; c < R; c++) r[c] = s[nv * 4 + tid * R + c];
      fold_in_regs(r, n, R);
      lds[swz(nv * per + tid)] = r[0];
    }
  } else {  // unaligned chunk: plain loads, every round in LDS (R == 1)
    float x[kChunk / kThreads];
#pragma unroll
    for (int i = 0; i < kChunk / kThreads; i++) {
      const int e = tid + i * kThreads;
      x[i] = e < C ? s[e] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < kChunk / kThreads; i++) {
      const int e = tid + i * kThreads;
      if (e < C) lds[swz(e)] = x[i];
    }
  }
  int len = C / R, from = 0, to = kRegionB;
  for (int round = a; round < L; round++) {
    __syncthreads();
    const int lo = len / n;
    for (int o = tid; o < lo; o += kThreads) {
      const int b = from + o * n;
      float acc = 0.f;
      for (int j = 0; j < n; j++) acc = acc + lds[swz(b + j)];
      lds[swz(to + o)] = acc;
    }
    len = lo;
    const int t = from;
    from = to;
    to = t;
  }
  __syncthreads();
  for (int o = tid; o < qv; o += kThreads) dst[g0 + o] = lds[swz(from + o)];
}

// The N values of one group from a 4-byte-aligned address, in loads of up to
// 16 bytes that need only 4-byte alignment (N = 3: one 12-byte load).
typedef float f32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));
typedef float f32x3_a4 __attribute__((ext_vector_type(3), aligned(4)));
typedef float f32x2_a4 __attribute__((ext_vector_type(2), aligned(4)));
template <int N>
__device__ __forceinline__ void load_group(float (&v)[N], const float* p) {
#pragma unroll
  for (int j = 0; j + 4 <= N; j += 4) {
    const f32x4_a4 t = *reinterpret_cast<const f32x4_a4*>(p + j);
    v[j] = t.x;
    v[j + 1] = t.y;
    v[j + 2] = t.z;
    v[j + 3] = t.w;
  }
  constexpr int j = N / 4 * 4;
  if constexpr (N - j == 3) {
    const f32x3_a4 t = *reinterpret_cast<const f32x3_a4*>(p + j);
    v[j] = t.x;
    v[j + 1] = t.y;
    v[j + 2] = t.z;
  } else if constexpr (N - j == 2) {
    const f32x2_a4 t = *reinterpret_cast<const f32x2_a4*>(p + j);
    v[j] = t.x;
    v[j + 1] = t.y;
  } else if constexpr (N - j == 1) {
    v[j] = p[j];
  }
}

// Fan-ins 3 to 8, passes of at least one round: the first round runs in
// registers straight from the loads, each thread folding whole groups of N
// neighbours, so LDS holds one value per group (never the raw chunk) and the
// later rounds run there as in iterate_sum_pass.  With an aligned chunk a
// thread loads a unit of the fewest consecutive groups that stays 16-byte
// aligned (one group for N = 4 and 8, two for 6, four for odd N) with 16-byte
// loads; the groups past the last whole unit, unaligned chunks and every chunk
// for N = 6 (whose two-group units measured slower) load group by group in
// 4-byte-aligned loads of up to 16 bytes.  The LDS tile is a sixth of
// iterate_sum_pass's or less, so eight workgroups share a CU instead of three
// and their loads overlap the other workgroups' LDS rounds.  The sums are the
// same left folds from 0, in the same order.
template <int N>
__global__ __launch_bounds__(kThreads) void iterate_sum_pass_first(
    float* __restrict__ dst, const float* __restrict__ src, int64_t len_out, int L, int G, int q,
    int vec) {
  constexpr int kA = (kChunk / N + 63) / 64 * 64;      // round-1 outputs (whole swizzle blocks)
  constexpr int kB = (kChunk / N / N + 63) / 64 * 64;  // round-2 outputs
  __shared__ float lds[kA + kB];
  const int tid = threadIdx.x;
  const int64_t g0 = (int64_t)blockIdx.x * q;
  const int qv = (int)(len_out - g0 < q ? len_out - g0 : q);
  const int C1 = qv * (G / N);  // groups of the first round in this chunk
  const float* s = src + g0 * G;
  if (vec) {
    constexpr int UG = N % 4 == 0 ? 1 : N % 2 == 0 ? 2 : 4;  // groups per 16-byte-aligned unit
    constexpr int UV = UG * N / 4;                           // 16-byte loads per unit
    constexpr int kU = (kChunk / N / UG + kThreads - 1) / kThreads;  // units per thread
    const int nu = C1 / UG;
    float4 x[kU][UV];
#pragma unroll
    for (int i = 0; i < kU; i++) {
      const int u = tid + i * kThreads;
#pragma unroll
      for (int j = 0; j < UV; j++)
        x[i][j] = u < nu ? reinterpret_cast<const float4*>(s)[(int64_t)u * UV + j]
                         : float4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int i = 0; i < kU; i++) {
      const int u = tid + i * kThreads;
      if (u < nu) {
        float f[4 * UV];
#pragma unroll
        for (int j = 0; j < UV; j++) {
          f[4 * j] = x[i][j].x;
          f[4 * j + 1] = x[i][j].y;
          f[4 * j + 2] = x[i][j].z;
          f[4 * j + 3] = x[i][j].w;
        }
#pragma unroll
        for (int g = 0; g < UG; g++) {
          float acc = 0.f;
#pragma unroll
          for (int j = 0; j < N; j++) acc = acc + f[g * N + j];
          lds[swz(UG * u + g)] = acc;
        }
      }
    }
    const int o = UG * nu + tid;  // groups past the last whole unit
    if (o < C1) {
      float acc = 0.f;
#pragma unroll
      for (int j = 0; j < N; j++) acc = acc + s[(int64_t)o * N + j];
      lds[swz(o)] = acc;
    }
  } else {
    constexpr int kGr = (kChunk / N + kThreads - 1) / kThreads;  // groups per thread
    float x[kGr][N];
#pragma unroll
    for (int i = 0; i < kGr; i++) {
      const int o = tid + i * kThreads;
      if (o < C1) {
        load_group<N>(x[i], s + (int64_t)o * N);
      } else {
#pragma unroll
        for (int j = 0; j < N; j++) x[i][j] = 0.f;
      }
    }
#pragma unroll
    for (int i = 0; i < kGr; i++) {
      const int o = tid + i * kThreads;
      if (o < C1) {
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < N; j++) acc = acc + x[i][j];
        lds[swz(o)] = acc;
      }
    }
  }
  int len = C1, from = 0, to = kA;
  for (int round = 1; round < L; round++) {
    __syncthreads();
    const int lo = len / N;
    for (int o = tid; o < lo; o += kThreads) {
      const int b = from + o * N;
      float acc = 0.f;
#pragma unroll
      for (int j = 0; j < N; j++) acc = acc + lds[swz(b + j)];
      lds[swz(to + o)] = acc;
    }
    len = lo;
    const int t = from;
    from = to;
    to = t;
  }
  __syncthreads();
  for (int o = tid; o < qv; o += kThreads) dst[g0 + o] = lds[swz(from + o)];
}

// Binary tree (n = 2), 16-byte aligned chunk, L >= 2 rounds: rounds 1-2 fold
// each 16-byte load in registers; the next rounds pair neighbouring lanes of a
// wavefront (lanes hold consecutive positions, so an exchange with lane t ^ 2^j
// is exactly the neighbour pairing of the next round); past 64 positions one
// value per wavefront and load goes through LDS and a single wavefront runs the
// remaining rounds the same way.  One barrier in all, and a few hundred bytes
// of LDS, so many workgroups share a CU and keep loads in flight.
__device__ __forceinline__ float pair_round(float v, int off) {
  // the lower lane of each pair holds the left operand: (0 + lower) + upper
  return (0.f + v) + __shfl_xor(v, off, 64);
}

__global__ __launch_bounds__(kThreads) void iterate_sum_pass_bin(
    float* __restrict__ dst, const float* __restrict__ src, int64_t len_out, int L, int q) {
  __shared__ float part[kChunk / 256];
  const int tid = threadIdx.x, lane = tid & 63;
  const int64_t g0 = (int64_t)blockIdx.x * q;
  const int qv = (int)(len_out - g0 < q ? len_out - g0 : q);
  const int nv = (qv << L) >> 2;  // 16-byte loads present (G = 2^L is a multiple of 4)
  const float4* s = reinterpret_cast<const float4*>(src + (g0 << L));
  float4 x[kVecPerThread];
#pragma unroll
  for (int i = 0; i < kVecPerThread; i++) {
    const int p = tid + i * kThreads;
    x[i] = p < nv ? s[p] : float4{0.f, 0.f, 0.f, 0.f};
  }
  float v[kVecPerThread];
#pragma unroll
  for (int i = 0; i < kVecPerThread; i++) {
    const float a = (0.f + x[i].x) + x[i].y, b = (0.f + x[i].z) + x[i].w;
    v[i] = (0.f + a) + b;
  }
  // positions beyond the chunk hold zeros and only ever pair with each other:
  // the chunk is a whole number of groups, and every round pairs inside a group
  const int sh = L - 2 < 6 ? L - 2 : 6;
  for (int j = 0; j < sh; j++) {
#pragma unroll
    for (int i = 0; i < kVecPerThread; i++) v[i] = pair_round(v[i], 1 << j);
  }
  if (L - 2 <= 6) {
#pragma unroll
    for (int i = 0; i < kVecPerThread; i++) {
      const int p = tid + i * kThreads;
      if (p < nv && (lane & ((1 << sh) - 1)) == 0) dst[g0 + (p >> sh)] = v[i];
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < kVecPerThread; i++) {
    const int p = tid + i * kThreads;
    if (lane == 0 && p < nv) part[p >> 6] = v[i];
  }
  __syncthreads();
  if (tid >= 64) return;
  const int cnt = nv >> 6, r = L - 8;  // cnt <= 32 positions left, r <= 5 rounds
  float w = lane < cnt ? part[lane] : 0.f;
  for (int j = 0; j < r; j++) w = pair_round(w, 1 << j);
  if (lane < cnt && (lane & ((1 << r) - 1)) == 0) dst[g0 + (lane >> r)] = w;
}

struct Pass {
  int L, G, q, a, R;
  int64_t len_in, len_out, blocks;
};

// Rounds per pass: as many as keep one group inside a chunk.  n == 1 rounds are
// all alike (each adds 0), so one is run for any k >= 1.
int plan(int64_t n, int64_t m, int64_t k, Pass* out, int cap) {
  if (n == 1 && k > 1) k = 1;
  int64_t len = m;
  for (int64_t i = 0; i < k; i++) len *= n;
  int np = 0;
  int64_t left = k;
  do {
    Pass p{};
    int64_t G = 1;
    int L = 0;
    while (L < left && G * n <= kChunk) {
      G *= n;
      L++;
    }
    if (n == 1) L = (int)left;  // G stays 1
    p.L = L;
    p.G = (int)G;
    p.len_in = len;
    p.len_out = len / G;
    // a round writes at most half a chunk into the second LDS region, except
    // for n == 1, whose round keeps every value: its chunk is half as long
    const int64_t fit = n == 1 ? kChunk / 2 : kChunk / G;
    p.q = (int)std::max<int64_t>(1, std::min<int64_t>(fit, p.len_out));
    p.blocks = (p.len_out + p.q - 1) / p.q;
    const int regs = n == 2 ? 2 : n == 4 ? 1 : 0;
    p.a = std::min(regs, L);
    p.R = 1;
    for (int i = 0; i < p.a; i++) p.R *= (int)n;
    if (np == cap) return -1;
    out[np++] = p;
    len = p.len_out;
    left -= L;
  } while (left > 0);
  return np;
}

constexpr int kMaxPasses = 64;

}  // namespace

int iterate_max_fan_in() { return kChunk; }

size_t iterate_sum_workspace(int64_t n, int64_t m, int64_t k) {
  Pass ps[kMaxPasses];
  const int np = plan(n, m, k, ps, kMaxPasses);
  if (np <= 1) return 0;
  const size_t half = ((size_t)ps[0].len_out * 4 + 255) / 256 * 256;
  return 2 * half;
}

int iterate_sum_rounds(int64_t n, int64_t m, int64_t k, int32_t* rounds, int cap) {
  Pass ps[kMaxPasses];
  const int np = plan(n, m, k, ps, kMaxPasses);
  for (int i = 0; rounds && i < np && i < cap; i++) rounds[i] = ps[i].L;
  return np;
}

rise_status launch_iterate_sum(float* out, const float* in, int64_t n, int64_t m, int64_t k,
                               void* ws, hipStream_t s) {
  Pass ps[kMaxPasses];
  const int np = plan(n, m, k, ps, kMaxPasses);
  if (np < 1) return fail(RISE_ERR_SHAPE, "rise_iterate_sum: no pass plan for these sizes");
  const size_t half = ((size_t)ps[0].len_out * 4 + 255) / 256 * 256;
  float* buf[2] = {(float*)ws, (float*)((char*)ws + half)};
  const float* src = in;
  for (int i = 0; i < np; i++) {
    const Pass& p = ps[i];
    float* dst = i == np - 1 ? out : buf[i & 1];
    // the chunk of every workgroup starts 16-byte aligned when q*G is a
    // multiple of 4 and the source is
    const bool vec = ((uintptr_t)src & 15) == 0 && ((int64_t)p.q * p.G) % 4 == 0;
    const int a = vec ? p.a : 0, R = vec ? p.R : 1;
    const dim3 grid((unsigned)p.blocks), block(kThreads);
    const int v = vec ? 1 : 0;
    if (n == 2 && vec && p.L >= 2)
      hipLaunchKernelGGL(iterate_sum_pass_bin, grid, block, 0, s, dst, src, p.len_out, p.L, p.q);
    else if (p.L < 1)  // k = 0: a copy
      hipLaunchKernelGGL(iterate_sum_pass, grid, block, 0, s, dst, src, p.len_out, (int)n, p.L,
                         p.G, p.q, a, R, v);
    else if (n == 3)
      hipLaunchKernelGGL(iterate_sum_pass_first<3>, grid, block, 0, s, dst, src, p.len_out, p.L,
                         p.G, p.q, v);
    else if (n == 4)
      hipLaunchKernelGGL(iterate_sum_pass_first<4>, grid, block, 0, s, dst, src, p.len_out, p.L,
                         p.G, p.q, v);
    else if (n == 5)
      hipLaunchKernelGGL(iterate_sum_pass_first<5>, grid, block, 0, s, dst, src, p.len_out, p.L,
                         p.G, p.q, v);
    else if (n == 6)  // a group per 16 + 8-byte load pair beats units of two groups
      hipLaunchKernelGGL(iterate_sum_pass_first<6>, grid, block, 0, s, dst, src, p.len_out, p.L,
                         p.G, p.q, 0);
    else if (n == 7)
      hipLaunchKernelGGL(iterate_sum_pass_first<7>, grid, block, 0, s, dst, src, p.len_out, p.L,
                         p.G, p.q, v);
    else if (n == 8)
      hipLaunchKernelGGL(iterate_sum_pass_first<8>, grid, block, 0, s, dst, src, p.len_out, p.L,
                         p.G, p.q, v);
    else
      hipLaunchKernelGGL(iterate_sum_pass, dim3((unsigned)p.blocks), dim3(kThreads), 0, s, dst,
                         src, p.len_out, (int)n, p.L, p.G, p.q, a, R, vec ? 1 : 0);
    rise_status st = check_launch("iterate_sum_pass");
    if (st != RISE_OK) return st;
    src = dst;
  }
  return RISE_OK;
}

}  // namespace rise
