// Batched form: many GEMMs and stencils of uneven sizes in one persistent launch.
//
// The batch is the outer map of the patterns: every (problem, output tile) pair
// is an independent work item (distinct output acceptors, paper Sec. V-C), so
// the items can run in any order.  The host builds a table of problem
// descriptors and a flat list of work items sorted by estimated cost (largest
// first), picks a tile shape for every GEMM from a measured cost table, and
// captures  [reset counter] -> [persistent kernel]  in a HIP graph.  Every
// persistent workgroup repeatedly takes the next item with one atomic add and
// runs the matching tile function (tiles.h) on a shared LDS buffer, so a batch
// costs one launch instead of one per problem.
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
// Three resident workgroups per CU: the many small tiles of a batch are
// latency-bound, and more workgroups in flight hide that latency.  For the
// LDS to allow it (a third of 160 KB per workgroup) the FP32 slabs here are 16
// deep, not the 32 of the one-problem kernels.  The GEMM tile kinds are
// separate, non-inlined functions with their own register allocation, so the
// kernel's 168 registers need to hold only the stencil tiles (measured on the
// 512 GEMM + 256 stencil batch: 3.8 ms against 4.6 ms with two workgroups per
// CU and every kind inlined).
constexpr int kF32BK = 16;
constexpr int kOccupancy = 3;
const KindShape kShape[NUM_KINDS] = {
    {64, 64, kF32BK}, {64, 64, kF32BK}, {128, 64, kF32BK}, {128, 64, kF32BK},
    {64, 128, kF32BK}, {64, 128, kF32BK}, {128, 128, kF32BK}, {128, 128, kF32BK},
    {64, 64, 32}, {64, 64, 32}, {128, 128, 32}, {128, 128, 32},
    {16, 256, 0}, {16, 256, 0}, {16, 256, 0}, {16, 256, 0},
    {16, 256, 0}, {16, 256, 0}, {16, 256, 0}, {16, 256, 0}};
constexpr int kStencilRows = 16;

struct Desc {  // one problem
  float* out;
  const void* a;   // GEMM A / stencil input
  const void* b;   // GEMM B / stencil weights
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
// the largest tile of any kind
constexpr int kLdsBytes =
    cmax(cmax(4 * tiles::F32Cfg<128, 128, kF32BK, false, false>::LDS_FLOATS,
              4 * tiles::F32Cfg<128, 128, kF32BK, false, true>::LDS_FLOATS),
         cmax(16 * tiles::Bf16Cfg<128, 128, 32>::LDS_CHUNKS,
              16 * tiles::StencilCfg<7, kStencilRows>::LDS_CHUNKS));
static_assert(kLdsBytes * kOccupancy <= 160 * 1024, "LDS of the resident workgroups");

template <int BM, int BN, bool TB>
__device__ __noinline__ void item_f32(const Desc& d, int tm, int tn, char* lds) {
  tiles::gemm_f32_tile<BM, BN, kF32BK, false, TB, true>(
      d.out, d.ldc, reinterpret_cast<const float*>(d.a), d.lda,
      reinterpret_cast<const float*>(d.b), d.ldb, d.M, d.N, d.K, tm * BM, tn * BN,
      reinterpret_cast<float*>(lds));
}
template <int BM, int BN, bool TB>
__device__ __noinline__ void item_bf16(const Desc& d, int tm, int tn, char* lds) {
  tiles::gemm_bf16_tile<BM, BN, 32, TB>(d.out, d.ldc, reinterpret_cast<const uint16_t*>(d.a),
                                        d.lda, reinterpret_cast<const uint16_t*>(d.b), d.ldb, d.M,
                                        d.N, d.K, tm * BM, tn * BN, reinterpret_cast<i32x4*>(lds));
}
template <int K, bool VEC>
__device__ __forceinline__ void item_stencil(const Desc& d, int tm, int tn, char* lds) {
  tiles::stencil_lds_tile<K, VEC, kStencilRows>(
      d.out, d.ldc, reinterpret_cast<const float*>(d.a), d.lda, d.M, d.N,
      reinterpret_cast<const float*>(d.b), d.zero_pad, tm * kStencilRows, tn * tiles::kStencilTX,
      reinterpret_cast<f32x4*>(lds));
}

__device__ __forceinline__ void run_item(const Desc& d, int tile, char* lds) {
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
    case STENCIL_1: item_stencil<1, true>(d, tm, tn, lds); break;
    case STENCIL_3: item_stencil<3, true>(d, tm, tn, lds); break;
    case STENCIL_5: item_stencil<5, true>(d, tm, tn, lds); break;
    case STENCIL_7: item_stencil<7, true>(d, tm, tn, lds); break;
    case STENCIL_1S: item_stencil<1, false>(d, tm, tn, lds); break;
    case STENCIL_3S: item_stencil<3, false>(d, tm, tn, lds); break;
    case STENCIL_5S: item_stencil<5, false>(d, tm, tn, lds); break;
    case STENCIL_7S: item_stencil<7, false>(d, tm, tn, lds); break;
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
__global__ __launch_bounds__(kThreads, kOccupancy) void batched_kernel(const Desc* __restrict__ descs,
                                                              const Item* __restrict__ items,
                                                              int n_items, int* counter) {
  __shared__ __attribute__((aligned(16))) char lds[kLdsBytes];
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
    run_item(descs[item.desc], item.tile, lds);
    if (threadIdx.x == 0) next = pre;
    __syncthreads();  // the LDS buffer is free for the next item; `next` is visible
    it = next;
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

struct PlanImpl {
  Desc* d_desc = nullptr;
  Item* d_items = nullptr;
  int* d_counter = nullptr;
  int n_items = 0, grid = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int> kinds;  // chosen kind per problem (GEMMs first, then stencils)
  double est_us = 0;
};

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
    Desc d{p.C, p.A, p.B, p.lda, p.ldb, p.ldc, (int)p.M, (int)p.N, (int)p.K, kind,
           ceil_div(p.N, s.bn), 0, 0};
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
    Desc d{p.out, p.in, p.w, p.ld_in, 0, p.ld_out, (int)p.H, (int)p.W, p.k, kind,
           ceil_div(p.W, tiles::kStencilTX), p.pad == RISE_PAD_ZERO, 0};
    descs.push_back(d);
    ntile.push_back((p.H == 0 || p.W == 0) ? 0 : ceil_div(p.H, kStencilRows) * d.tiles_n);
    unit.push_back(cost[kind].a);
  }
  // Each class (matrix-core-bound GEMM tiles, HBM-bound stencil tiles) in
  // longest-processing-time order, so the tail of the launch is made of the
  // cheapest items; the two lists are then merged in proportion to their
  // estimated time, so that at any moment both kinds of tile are in flight and
  // the stencils' memory traffic overlaps the GEMMs' arithmetic.
  std::vector<int> order(descs.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return unit[x] > unit[y]; });
  std::vector<Item> cls[2];
  std::vector<double> cls_us[2];
  double total[2] = {0.0, 0.0};
  for (int d : order) {
    const int c = descs[d].kind >= STENCIL_1 ? 1 : 0;
    plan->est_us += unit[d] * ntile[d];
    total[c] += unit[d] * ntile[d];
    for (int t = 0; t < ntile[d]; t++) {
      cls[c].push_back(Item{d, t});
      cls_us[c].push_back(unit[d]);
    }
  }
  std::vector<Item> items;
  items.reserve(cls[0].size() + cls[1].size());
  size_t next[2] = {0, 0};
  double done[2] = {0.0, 0.0};
  while (next[0] < cls[0].size() || next[1] < cls[1].size()) {
    int c;
    if (next[0] >= cls[0].size()) c = 1;
    else if (next[1] >= cls[1].size()) c = 0;
    else c = done[0] / total[0] <= done[1] / total[1] ? 0 : 1;
    items.push_back(cls[c][next[c]]);
    done[c] += cls_us[c][next[c]];
    next[c]++;
  }
  plan->n_items = (int)items.size();

  int dev = 0, cus = 256;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  plan->grid = std::max(1, std::min(plan->n_items, kOccupancy * cus));

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
  // capture [reset counter] -> [persistent kernel] on a private stream
  hipStream_t cap;
  if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess) {
    rise_plan_free(plan);
    return fail(RISE_ERR_HIP, std::string("rise_plan_create: ") + hipGetErrorString(e));
  }
  e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(reset_counter, dim3(1), dim3(64), 0, cap, plan->d_counter);
    if (plan->n_items > 0)
      hipLaunchKernelGGL(batched_kernel, dim3(plan->grid), dim3(kThreads), 0, cap, plan->d_desc,
                         plan->d_items, plan->n_items, plan->d_counter);
    e = hipStreamEndCapture(cap, &plan->graph);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
  hipStreamDestroy(cap);
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
  hipLaunchKernelGGL(reset_counter, dim3(1), dim3(64), 0, s, p->d_counter);
  if (p->n_items > 0)
    hipLaunchKernelGGL(batched_kernel, dim3(p->grid), dim3(kThreads), 0, s, p->d_desc, p->d_items,
                       p->n_items, p->d_counter);
  return check_launch("batched_kernel");
}

void rise_plan_free(PlanImpl* p) {
  if (!p) return;
  if (p->exec) hipGraphExecDestroy(p->exec);
  if (p->graph) hipGraphDestroy(p->graph);
  if (p->d_desc) hipFree(p->d_desc);
  if (p->d_items) hipFree(p->d_items);
  if (p->d_counter) hipFree(p->d_counter);
  delete p;
}

int plan_items(const PlanImpl* p) { return p->n_items; }
int plan_grid(const PlanImpl* p) { return p->grid; }
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
