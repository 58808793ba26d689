// Batched form: many GEMMs and stencils of uneven sizes in one persistent launch.
//
// The batch is the outer map of the patterns: every (problem, output tile) pair
// is an independent work item (distinct output acceptors, paper Sec. V-C), so
// the items can run in any order.  The host builds a table of problem
// descriptors and the work items, picks a tile shape for every GEMM from a
// measured cost table, and captures one graph of persistent kernels, one per
// class of tile, each with the registers and occupancy its tile needs:
//   [reset counter] -> [GEMM tiles] -> [stencil tiles, one kernel per window
//   side and load width present]
// In the GEMM kernel every workgroup repeatedly takes the next item (largest
// estimated cost first) with one atomic add and runs the matching tile function
// (tiles.h); the stencil tiles of one class cost the same, so the stencil
// kernels walk their item list round-robin without a counter.  A batch costs
// one graph launch instead of one launch per problem.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "batched.h"
#include "tiles.h"

namespace rise {
namespace {

using tiles::kThreads;

// tile kinds of the persistent kernel
enum Kind : int {
  F32_64x64_N, F32_64x64_T, F32_128x64_N, F32_128x64_T, F32_64x128_N, F32_64x128_T,
  F32_128x128_N, F32_128x128_T,
  BF16_64x64_N, BF16_64x64_T, BF16_128x128_N, BF16_128x128_T,
  STENCIL_1, STENCIL_3, STENCIL_5, STENCIL_7,                   // 16-byte vector paths
  STENCIL_1S, STENCIL_3S, STENCIL_5S, STENCIL_7S,               // any alignment / ld
  NUM_KINDS
};
struct KindShape {
  int bm, bn, bk;
};
// The GEMM kernel keeps the FP32 slabs 16 deep (LDS for several resident
// workgroups); its tile kinds are separate, non-inlined functions with their
// own register allocation.  Stencil tiles are 8 output rows x 256 columns for
// windows up to 5 x 5 and 16 rows for 7 x 7, the one-problem kernel's choice.
constexpr int kF32BK = 16;
constexpr int kBf16BK = 64;  // bf16 slab depth: 64 k per barrier
constexpr int kGemmOccupancy = 2;
constexpr int stencil_rows(int k) { return k <= 5 ? 8 : 16; }
const KindShape kShape[NUM_KINDS] = {
    {64, 64, kF32BK}, {64, 64, kF32BK}, {128, 64, kF32BK}, {128, 64, kF32BK},
    {64, 128, kF32BK}, {64, 128, kF32BK}, {128, 128, kF32BK}, {128, 128, kF32BK},
    {64, 64, kBf16BK}, {64, 64, kBf16BK}, {128, 128, kBf16BK}, {128, 128, kBf16BK},
    {stencil_rows(1), 256, 0}, {stencil_rows(3), 256, 0}, {stencil_rows(5), 256, 0},
    {stencil_rows(7), 256, 0},  {stencil_rows(1), 256, 0}, {stencil_rows(3), 256, 0},
    {stencil_rows(5), 256, 0},  {stencil_rows(7), 256, 0}};
constexpr int kStencilClasses = NUM_KINDS - STENCIL_1;  // side x load width

struct Desc {  // one problem; device addresses as integers (see gptr)
  uint64_t out;
  uint64_t a;      // GEMM A / stencil input
  uint64_t b;      // GEMM B / stencil weights
  int64_t lda, ldb, ldc;  // stencil: lda = ld_in, ldc = ld_out
  int M, N, K;            // stencil: M = H, N = W, K = window side
  int kind;
  int tiles_n;            // tiles along N (GEMM) or along W (stencil)
  int zero_pad;
  int pad_;
};
struct Item {
  int desc, tile;
};

constexpr int cmax(int a, int b) { return a > b ? a : b; }
// FP32 tiles of problems whose storage allows it (tiles::f32_async_eligible)
// run the asynchronous-ring schedule with this many slabs in flight
constexpr int kF32Stages = 3;
// the largest GEMM tile of any kind
constexpr int kGemmLdsBytes =
    cmax(cmax(cmax(4 * tiles::F32Cfg<128, 128, kF32BK, false, false>::LDS_FLOATS,
                   4 * tiles::F32Cfg<128, 128, kF32BK, false, true>::LDS_FLOATS),
              16 * tiles::F32AsyncCfg<128, 128, kF32Stages>::LDS_CHUNKS),
         16 * tiles::Bf16Cfg<128, 128, kBf16BK>::LDS_CHUNKS);
static_assert(kGemmLdsBytes * kGemmOccupancy <= 160 * 1024, "LDS of the resident workgroups");

// A descriptor address as a pointer into global memory: built from the integer
// through the global address space, so the compiler uses global (not flat)
// memory instructions even in the separately compiled item functions.
template <typename T>
__device__ __forceinline__ T* gptr(uint64_t v) {
  return (T*)((__attribute__((address_space(1))) T*)v);
}

template <int BM, int BN, bool TB>
__device__ __noinline__ void item_f32(const Desc& d, int tm, int tn, char* lds) {
  const float* A = gptr<const float>(d.a);
  const float* B = gptr<const float>(d.b);
  float* C = gptr<float>(d.out);
  if (tiles::f32_async_eligible(A, d.lda, B, d.ldb, d.M, d.N, d.K, false, TB))
    tiles::gemm_f32_async_tile<BM, BN, kF32Stages, false, TB>(
        C, d.ldc, A, d.lda, B, d.ldb, d.M, d.N, d.K, tm * BM, tn * BN,
        reinterpret_cast<f32x4*>(lds));
  else
    tiles::gemm_f32_tile<BM, BN, kF32BK, false, TB, true>(C, d.ldc, A, d.lda, B, d.ldb, d.M, d.N,
                                                          d.K, tm * BM, tn * BN,
                                                          reinterpret_cast<float*>(lds));
}
template <int BM, int BN, bool TB>
__device__ __noinline__ void item_bf16(const Desc& d, int tm, int tn, char* lds) {
  tiles::gemm_bf16_tile<BM, BN, kBf16BK, TB>(gptr<float>(d.out), d.ldc, gptr<const uint16_t>(d.a),
                                        d.lda, gptr<const uint16_t>(d.b), d.ldb, d.M, d.N, d.K,
                                        tm * BM, tn * BN, reinterpret_cast<i32x4*>(lds));
}
__device__ __forceinline__ void run_gemm_item(const Desc& d, int tile, char* lds) {
  const int tm = tile / d.tiles_n, tn = tile - tm * d.tiles_n;
  switch (d.kind) {
    case F32_64x64_N: item_f32<64, 64, false>(d, tm, tn, lds); break;
    case F32_64x64_T: item_f32<64, 64, true>(d, tm, tn, lds); break;
    case F32_128x64_N: item_f32<128, 64, false>(d, tm, tn, lds); break;
    case F32_128x64_T: item_f32<128, 64, true>(d, tm, tn, lds); break;
    case F32_64x128_N: item_f32<64, 128, false>(d, tm, tn, lds); break;
    case F32_64x128_T: item_f32<64, 128, true>(d, tm, tn, lds); break;
    case F32_128x128_N: item_f32<128, 128, false>(d, tm, tn, lds); break;
    case F32_128x128_T: item_f32<128, 128, true>(d, tm, tn, lds); break;
    case BF16_64x64_N: item_bf16<64, 64, false>(d, tm, tn, lds); break;
    case BF16_64x64_T: item_bf16<64, 64, true>(d, tm, tn, lds); break;
    case BF16_128x128_N: item_bf16<128, 128, false>(d, tm, tn, lds); break;
    case BF16_128x128_T: item_bf16<128, 128, true>(d, tm, tn, lds); break;
    default: break;
  }
}

__global__ void reset_counter(int* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

// Every workgroup takes items until the list is exhausted; the exit condition
// (item >= n_items) is reached by every workgroup because the counter only grows.
// The index of the following item is requested (thread 0, one atomic) while the
// current item runs, so the atomic's round trip is off the critical path.
__global__ __launch_bounds__(kThreads, kGemmOccupancy) void batched_gemm_kernel(
    const Desc* __restrict__ descs, const Item* __restrict__ items, int n_items, int* counter) {
  __shared__ __attribute__((aligned(16))) char lds[kGemmLdsBytes];
  __shared__ int next;
  if (threadIdx.x == 0) next = atomicAdd(counter, 1);
  __syncthreads();
  int it = next;
  for (;;) {
    __syncthreads();  // every thread has read `next` before it is overwritten
    if (it >= n_items) break;
    int pre = 0;
    if (threadIdx.x == 0) pre = atomicAdd(counter, 1);  // the following item
    const Item item = items[it];
    run_gemm_item(descs[item.desc], item.tile, lds);
    if (threadIdx.x == 0) next = pre;
    __syncthreads();  // the LDS buffer is free for the next item; `next` is visible
    it = next;
  }
}

// Stencil tiles of one window side and load width: workgroup b runs items b,
// b + grid, b + 2 grid, ... (the items of a class cost the same).  The plans
// launch one workgroup per item: the hardware then keeps every CU at the
// occupancy below with a new tile's loads in flight as soon as one finishes,
// which a resident grid walking its items in turn did not (the 512 + 256
// batch: 2.53 -> 2.48 ms FP32, 1.50 -> 1.44 ms bf16).
// resident workgroups per CU: as many as the tile's registers allow without
// spilling; the window of 5 x 5 and 7 x 7 tiles streams through registers a
// row at a time (44-49 and 75-80 VGPRs with the item loop, against 78-83 and
// 143-151 holding the whole window), and 7 x 7 is held to six by its 23 KB of LDS
constexpr int stencil_occupancy(int k) { return k <= 5 ? 8 : 6; }

template <int K, bool VEC>
__global__ __launch_bounds__(kThreads, stencil_occupancy(K)) void batched_stencil_kernel(const Desc* __restrict__ descs,
                                                                   const Item* __restrict__ items,
                                                                   int n_items) {
  constexpr int TY = stencil_rows(K);
  __shared__ f32x4 lds[tiles::StencilCfg<K, TY>::LDS_CHUNKS];
  for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
    // the item and its descriptor are the same for every lane: scalar registers
    const int desc = __builtin_amdgcn_readfirstlane(items[i].desc);
    const int tile = __builtin_amdgcn_readfirstlane(items[i].tile);
    const Desc& d = descs[desc];
    const int tm = tile / d.tiles_n, tn = tile - tm * d.tiles_n;
    tiles::stencil_lds_tile<K, VEC, TY, true, true, (K >= 5)>(
        gptr<float>(d.out), d.ldc, gptr<const float>(d.a), d.lda, d.M, d.N, gptr<const float>(d.b),
        d.zero_pad, tm * TY, tn * tiles::kStencilTX, lds);
    __syncthreads();  // every wave is done with the LDS tile before the next item fills it
  }
}

template <int K, bool VEC>
const void* stencil_kernel_ptr() {
  return reinterpret_cast<const void*>(&batched_stencil_kernel<K, VEC>);
}
// class c = kind - STENCIL_1: sides 1, 3, 5, 7 with 16-byte loads, then scalar
const void* stencil_class_kernel(int c) {
  switch (c) {
    case 0: return stencil_kernel_ptr<1, true>();
    case 1: return stencil_kernel_ptr<3, true>();
    case 2: return stencil_kernel_ptr<5, true>();
    case 3: return stencil_kernel_ptr<7, true>();
    case 4: return stencil_kernel_ptr<1, false>();
    case 5: return stencil_kernel_ptr<3, false>();
    case 6: return stencil_kernel_ptr<5, false>();
    default: return stencil_kernel_ptr<7, false>();
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

// Cost model of one tile: a + b * K microseconds (GEMM), a (stencil); measured
// per kind by rise_autotune_batched and read from its table.  The built-in
// values below were measured on an MI355X with that routine.
struct Cost {
  double a, b;
};
Cost g_default_cost[NUM_KINDS] = {
    {1.0, 0.0040}, {1.0, 0.0042}, {1.2, 0.0068}, {1.2, 0.0070}, {1.2, 0.0068}, {1.2, 0.0070},
    {1.5, 0.0125}, {1.5, 0.0128}, {1.0, 0.0014}, {1.0, 0.0016}, {1.5, 0.0040}, {1.5, 0.0044},
    {1.0, 0.0},    {1.5, 0.0},    {2.0, 0.0},    {2.5, 0.0},
    {1.5, 0.0},    {2.0, 0.0},    {2.5, 0.0},    {3.0, 0.0}};

const char* kKindNames[NUM_KINDS] = {
    "f32_64x64_N", "f32_64x64_T", "f32_128x64_N", "f32_128x64_T", "f32_64x128_N",
    "f32_64x128_T", "f32_128x128_N", "f32_128x128_T", "bf16_64x64_N", "bf16_64x64_T",
    "bf16_128x128_N", "bf16_128x128_T", "stencil_1", "stencil_3", "stencil_5", "stencil_7",
    "stencil_1_scalar", "stencil_3_scalar", "stencil_5_scalar", "stencil_7_scalar"};

bool load_costs(const char* path, Cost* cost) {
  for (int k = 0; k < NUM_KINDS; k++) cost[k] = g_default_cost[k];
  if (!path) return true;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char name[64];
  double a, b;
  while (fscanf(f, "%63s %lf %lf", name, &a, &b) == 3) {
    for (int k = 0; k < NUM_KINDS; k++)
      if (std::string(name) == kKindNames[k]) cost[k] = Cost{a, b};
  }
  fclose(f);
  return true;
}

int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

double gemm_cost(const Cost* cost, int kind, int M, int N, int K) {
  const KindShape& s = kShape[kind];
  return (double)ceil_div(M, s.bm) * ceil_div(N, s.bn) * (cost[kind].a + cost[kind].b * K);
}

int pick_gemm_kind(const Cost* cost, int dtype, int opB, int M, int N, int K, int forced) {
  if (forced >= 0) return forced;
  const int t = opB == RISE_OP_T ? 1 : 0;
  int best = -1;
  double best_c = 0;
  const int first = dtype == RISE_F32 ? F32_64x64_N : BF16_64x64_N;
  const int last = dtype == RISE_F32 ? F32_128x128_T : BF16_128x128_T;
  for (int k = first + t; k <= last; k += 2) {
    double c = gemm_cost(cost, k, M, N, K);
    if (best < 0 || c < best_c) best = k, best_c = c;
  }
  return best;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

rise_status check_gemm_problem(const rise_gemm_problem& p, int i) {
  auto where = [&](const char* w) { return std::string("batched gemm ") + std::to_string(i) + ": " + w; };
  if (p.M < 0 || p.N < 0 || p.K < 0 || p.M >= (1LL << 31) || p.N >= (1LL << 31) || p.K >= (1LL << 31))
    return fail(RISE_ERR_SHAPE, where("sizes"));
  if (p.dtype != RISE_F32 && p.dtype != RISE_BF16) return fail(RISE_ERR_DTYPE, where("dtype"));
  if (p.opB != RISE_OP_N && p.opB != RISE_OP_T) return fail(RISE_ERR_UNSUPPORTED, where("opB"));
  if (p.M == 0 || p.N == 0) return RISE_OK;
  if (!p.C || (p.K > 0 && (!p.A || !p.B))) return fail(RISE_ERR_NULL, where("NULL pointer"));
  const int64_t bc = p.opB == RISE_OP_N ? p.N : p.K;
  if (p.ldc < p.N || (p.K > 0 && (p.lda < p.K || p.ldb < bc))) return fail(RISE_ERR_SHAPE, where("ld"));
  const int q = p.dtype == RISE_F32 ? 4 : 8;  // elements per 16 bytes
  if (p.K > 0 && (!aligned16(p.A) || !aligned16(p.B) || p.lda % q || p.ldb % q))
    return fail(RISE_ERR_UNSUPPORTED, where("A, B must be 16-byte aligned with lda, ldb multiples "
                                            "of 16 bytes"));
  if (p.dtype == RISE_BF16 && (p.K % 8 || (p.opB == RISE_OP_N && p.N % 8)))
    return fail(RISE_ERR_UNSUPPORTED, where("bf16 needs K (and N when B is K x N) multiples of 8"));
  const int64_t esz = p.dtype == RISE_F32 ? 4 : 2;
  auto span = [](const void* ptr, int64_t rows, int64_t cols, int64_t ld, int64_t e) {
    uintptr_t lo = (uintptr_t)ptr;
    return std::make_pair(lo, lo + (uintptr_t)(((rows - 1) * ld + cols) * e));
  };
  auto rc = span(p.C, p.M, p.N, p.ldc, 4);
  if (p.K > 0) {
    auto ra = span(p.A, p.M, p.K, p.lda, esz);
    auto rb = span(p.B, p.opB == RISE_OP_N ? p.K : p.N, bc, p.ldb, esz);
    auto ov = [](std::pair<uintptr_t, uintptr_t> x, std::pair<uintptr_t, uintptr_t> y) {
      return x.first < y.second && y.first < x.second;
    };
    if (ov(rc, ra) || ov(rc, rb)) return fail(RISE_ERR_ALIAS, where("C overlaps A or B"));
  }
  return RISE_OK;
}

rise_status check_stencil_problem(const rise_stencil_problem& p, int i) {
  auto where = [&](const char* w) { return std::string("batched stencil ") + std::to_string(i) + ": " + w; };
  if (p.H < 0 || p.W < 0 || p.H >= (1LL << 31) || p.W >= (1LL << 31))
    return fail(RISE_ERR_SHAPE, where("sizes"));
  if (p.k != 1 && p.k != 3 && p.k != 5 && p.k != 7)
    return fail(RISE_ERR_UNSUPPORTED, where("window side must be 1, 3, 5 or 7"));
  if (p.pad != RISE_PAD_CLAMP && p.pad != RISE_PAD_ZERO) return fail(RISE_ERR_UNSUPPORTED, where("pad"));
  if (p.H == 0 || p.W == 0) return RISE_OK;
  if (!p.out || !p.in || !p.w) return fail(RISE_ERR_NULL, where("NULL pointer"));
  if (p.ld_in < p.W || p.ld_out < p.W) return fail(RISE_ERR_SHAPE, where("ld"));
  uintptr_t olo = (uintptr_t)p.out, ohi = olo + (uintptr_t)(((p.H - 1) * p.ld_out + p.W) * 4);
  uintptr_t ilo = (uintptr_t)p.in, ihi = ilo + (uintptr_t)(((p.H - 1) * p.ld_in + p.W) * 4);
  uintptr_t wlo = (uintptr_t)p.w, whi = wlo + (uintptr_t)(p.k * p.k * 4);
  if ((olo < ihi && ilo < ohi) || (olo < whi && wlo < ohi))
    return fail(RISE_ERR_ALIAS, where("out overlaps in or w"));
  return RISE_OK;
}

}  // namespace

// one kernel of a plan: items [first, first + count) of the item list;
// cls = -1 is the GEMM kernel, else the stencil class (kind - STENCIL_1)
struct Launch {
  int cls, first, count, grid;
};

struct PlanImpl {
  Desc* d_desc = nullptr;
  Item* d_items = nullptr;
  int* d_counter = nullptr;
  int n_items = 0;
  std::vector<Launch> launches;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int> kinds;  // chosen kind per problem (GEMMs first, then stencils)
  double est_us = 0;
};

namespace {
// [reset counter] -> the plan's kernels, in order on one stream; the first
// launch error, if any
hipError_t enqueue(const PlanImpl* p, hipStream_t s) {
  hipLaunchKernelGGL(reset_counter, dim3(1), dim3(64), 0, s, p->d_counter);
  hipError_t e = hipGetLastError();
  for (const Launch& l : p->launches) {
    if (e != hipSuccess) break;
    const Item* items = p->d_items + l.first;
    if (l.cls < 0) {
      hipLaunchKernelGGL(batched_gemm_kernel, dim3(l.grid), dim3(kThreads), 0, s, p->d_desc, items,
                         l.count, p->d_counter);
      e = hipGetLastError();
    } else {
      void* args[] = {(void*)&p->d_desc, (void*)&items, (void*)&l.count};
      e = hipLaunchKernel(stencil_class_kernel(l.cls), dim3(l.grid), dim3(kThreads), args, 0, s);
    }
  }
  return e;
}
}  // namespace

rise_status plan_build(PlanImpl** out, const rise_gemm_problem* g, int ng,
                       const rise_stencil_problem* st, int ns, const char* tune_path,
                       int forced_kind, hipStream_t stream) {
  *out = nullptr;
  if (ng < 0 || ns < 0) return fail(RISE_ERR_SHAPE, "rise_plan_create: negative count");
  if ((ng > 0 && !g) || (ns > 0 && !st)) return fail(RISE_ERR_NULL, "rise_plan_create: NULL list");
  for (int i = 0; i < ng; i++) {
    rise_status s = check_gemm_problem(g[i], i);
    if (s != RISE_OK) return s;
  }
  for (int i = 0; i < ns; i++) {
    rise_status s = check_stencil_problem(st[i], i);
    if (s != RISE_OK) return s;
  }
  Cost cost[NUM_KINDS];
  if (!load_costs(tune_path, cost)) return fail(RISE_ERR_UNSUPPORTED, "rise_plan_create: cannot read tune table");

  std::vector<Desc> descs;
  std::vector<double> unit;  // estimated microseconds per tile of each problem
  std::vector<int> ntile;
  auto plan = new PlanImpl();
  for (int i = 0; i < ng; i++) {
    const rise_gemm_problem& p = g[i];
    const int kind = pick_gemm_kind(cost, p.dtype, p.opB, (int)p.M, (int)p.N, (int)p.K,
                                    forced_kind);
    plan->kinds.push_back(kind);
    const KindShape& s = kShape[kind];
    Desc d{(uint64_t)(uintptr_t)p.C, (uint64_t)(uintptr_t)p.A, (uint64_t)(uintptr_t)p.B, p.lda,
           p.ldb, p.ldc, (int)p.M, (int)p.N, (int)p.K, kind, ceil_div(p.N, s.bn), 0, 0};
    descs.push_back(d);
    ntile.push_back((p.M == 0 || p.N == 0) ? 0 : ceil_div(p.M, s.bm) * d.tiles_n);
    unit.push_back(cost[kind].a + cost[kind].b * p.K);
  }
  for (int i = 0; i < ns; i++) {
    const rise_stencil_problem& p = st[i];
    const bool vec = aligned16(p.in) && aligned16(p.out) && p.ld_in % 4 == 0 && p.ld_out % 4 == 0;
    const int kind = forced_kind >= STENCIL_1 ? forced_kind
                                              : (vec ? STENCIL_1 : STENCIL_1S) + (p.k - 1) / 2;
    plan->kinds.push_back(kind);
    Desc d{(uint64_t)(uintptr_t)p.out, (uint64_t)(uintptr_t)p.in, (uint64_t)(uintptr_t)p.w,
           p.ld_in, 0, p.ld_out, (int)p.H, (int)p.W, p.k, kind,
           ceil_div(p.W, tiles::kStencilTX), p.pad == RISE_PAD_ZERO, 0};
    descs.push_back(d);
    ntile.push_back((p.H == 0 || p.W == 0) ? 0 : ceil_div(p.H, kShape[kind].bm) * d.tiles_n);
    unit.push_back(cost[kind].a);
  }
  // GEMM tiles in longest-processing-time order (largest estimated cost first,
  // so the tail of the GEMM kernel is made of the cheapest tiles), then the
  // stencil tiles grouped by class (window side, load width), each group one
  // kernel.
  std::vector<int> order(descs.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return unit[x] > unit[y]; });
  std::vector<Item> items;
  for (int d : order) {
    plan->est_us += unit[d] * ntile[d];
    if (descs[d].kind < STENCIL_1)
      for (int t = 0; t < ntile[d]; t++) items.push_back(Item{d, t});
  }
  const int n_gemm_items = (int)items.size();
  int stencil_first[kStencilClasses], stencil_count[kStencilClasses];
  for (int c = 0; c < kStencilClasses; c++) {
    stencil_first[c] = (int)items.size();
    for (int d : order)
      if (descs[d].kind == STENCIL_1 + c)
        for (int t = 0; t < ntile[d]; t++) items.push_back(Item{d, t});
    stencil_count[c] = (int)items.size() - stencil_first[c];
  }
  plan->n_items = (int)items.size();

  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  if (n_gemm_items > 0)
    plan->launches.push_back(
        Launch{-1, 0, n_gemm_items, std::max(1, std::min(n_gemm_items, kGemmOccupancy * cus))});
  for (int c = 0; c < kStencilClasses; c++)
    if (stencil_count[c] > 0)  // one workgroup per item
      plan->launches.push_back(Launch{c, stencil_first[c], stencil_count[c], stencil_count[c]});

  hipError_t e = hipSuccess;
  const size_t nd = std::max<size_t>(descs.size(), 1), ni = std::max<size_t>(items.size(), 1);
  if ((e = hipMalloc(&plan->d_desc, nd * sizeof(Desc))) != hipSuccess ||
      (e = hipMalloc(&plan->d_items, ni * sizeof(Item))) != hipSuccess ||
      (e = hipMalloc(&plan->d_counter, 256)) != hipSuccess) {
    rise_plan_free(plan);
    return fail(RISE_ERR_HIP, std::string("rise_plan_create: ") + hipGetErrorString(e));
  }
  if ((!descs.empty() &&
       (e = hipMemcpy(plan->d_desc, descs.data(), descs.size() * sizeof(Desc), hipMemcpyHostToDevice)) != hipSuccess) ||
      (!items.empty() &&
       (e = hipMemcpy(plan->d_items, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice)) != hipSuccess)) {
    rise_plan_free(plan);
    return fail(RISE_ERR_HIP, std::string("rise_plan_create: ") + hipGetErrorString(e));
  }
  // capture the plan's kernels on a private stream
  hipStream_t cap;
  if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess) {
    rise_plan_free(plan);
    return fail(RISE_ERR_HIP, std::string("rise_plan_create: ") + hipGetErrorString(e));
  }
  e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const hipError_t le = enqueue(plan, cap);
    e = hipStreamEndCapture(cap, &plan->graph);
    if (e == hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cap);
  if (e != hipSuccess) {
    rise_plan_free(plan);
    return fail(RISE_ERR_HIP, std::string("rise_plan_create: graph: ") + hipGetErrorString(e));
  }
  (void)stream;
  *out = plan;
  return RISE_OK;
}

rise_status plan_launch(PlanImpl* p, hipStream_t s) {
  hipError_t e = hipGraphLaunch(p->exec, s);
  if (e != hipSuccess) return fail(RISE_ERR_HIP, std::string("rise_plan_launch: ") + hipGetErrorString(e));
  return RISE_OK;
}

rise_status plan_launch_direct(PlanImpl* p, hipStream_t s) {
  const hipError_t e = enqueue(p, s);
  if (e != hipSuccess)
    return fail(RISE_ERR_HIP, std::string("rise_plan_launch_direct: ") + hipGetErrorString(e));
  return RISE_OK;
}

void rise_plan_free(PlanImpl* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->d_desc) (void)hipFree(p->d_desc);
  if (p->d_items) (void)hipFree(p->d_items);
  if (p->d_counter) (void)hipFree(p->d_counter);
  delete p;
}

int plan_items(const PlanImpl* p) { return p->n_items; }
// workgroups of the plan's first kernel (a plan of one tile class has one)
int plan_grid(const PlanImpl* p) { return p->launches.empty() ? 1 : p->launches[0].grid; }
double plan_estimate(const PlanImpl* p) { return p->est_us; }
int plan_kind(const PlanImpl* p, int i) { return i >= 0 && i < (int)p->kinds.size() ? p->kinds[i] : -1; }
const char* kind_name(int k) { return k >= 0 && k < NUM_KINDS ? kKindNames[k] : ""; }
int num_kinds() { return NUM_KINDS; }
int kind_is_stencil(int k) { return k >= STENCIL_1; }
int kind_stencil_side(int k) { return 1 + 2 * ((k - STENCIL_1) % 4); }
int kind_dtype(int k) { return k >= BF16_64x64_N && k <= BF16_128x128_T ? RISE_BF16 : RISE_F32; }
int kind_opb(int k) { return k < STENCIL_1 ? (k & 1) : -1; }
rise_tile kind_tile(int k) {
  if (k < 0 || k >= STENCIL_1) return rise_tile{0, 0, 0};
  return rise_tile{kShape[k].bm, kShape[k].bn, kShape[k].bk};
}

}  // namespace rise
