// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "rise.h"

namespace rise {

// ---------------------------------------------------------------------------
// error reporting (thread-local message behind rise_last_error)
// ---------------------------------------------------------------------------
rise_status fail(rise_status s, const std::string& msg);
void clear_error();
rise_status check_launch(const char* what);
// compute units of the current device (cached per device)
int device_cu_count();

// ---------------------------------------------------------------------------
// vector types of the gfx950 matrix-core builtins
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;
constexpr int kNumXcd = 8;  // MI355X: 8 accelerator complex dies, 32 CUs each

// Workgroups are dispatched round-robin over the XCDs (block b runs on XCD
// b % 8).  Remap so that each XCD receives a contiguous range of logical tile
// ids, which then share that XCD's L2.
__device__ __forceinline__ int xcd_contiguous(int bid, int nblocks) {
  if (nblocks % kNumXcd != 0) return bid;
  return (bid % kNumXcd) * (nblocks / kNumXcd) + bid / kNumXcd;
}

// Logical tile id -> (tile row, tile col), visiting `group` tile rows
// column by column so concurrently running tiles share A and B panels.
__device__ __forceinline__ void grouped_tile(int lid, int tiles_m, int tiles_n, int group,
                                             int& tm, int& tn) {
  int per_group = group * tiles_n;
  int g = lid / per_group;
  int first = g * group;
  int gs = tiles_m - first < group ? tiles_m - first : group;
  int in = lid - g * per_group;
  tm = first + in % gs;
  tn = in / gs;
}

// ---------------------------------------------------------------------------
// kernel launchers (each validates nothing; the API layer did)
// ---------------------------------------------------------------------------
struct GemmF32Args {
  float* C;
  int64_t ldc;
  const float* A;
  int64_t lda;
  const float* B;
  int64_t ldb;
  int M, N, K;
  bool ta, tb;
};
bool gemm_f32_tile_supported(const rise_tile& t);
rise_tile gemm_f32_default_tile(int M, int N, int K);
int gemm_f32_tiles(rise_tile* out, int cap);
rise_status launch_gemm_f32(const GemmF32Args& a, const rise_tile& t, hipStream_t s);

struct StencilArgs {
  float* out;
  int64_t ld_out;
  const float* in;
  int64_t ld_in;
  int H, W;
  const float* w;
  int kh, kw;
  int pad;  // rise_pad
  bool keep_out = false;  // the output is read again next (normal, not non-temporal, stores)
};
int stencil_schedules(rise_stencil_schedule* out, int cap);
bool stencil_schedule_supported(const rise_stencil_schedule& sc);
rise_stencil_schedule stencil_default_schedule(int H, int W, int kh, int kw);
rise_status launch_stencil2d(const StencilArgs& a, const rise_stencil_schedule& sc, hipStream_t s);

struct StencilBwdArgs {
  float* din;  // may be null
  int64_t ld_din;
  float* dw;   // may be null
  const float* dout;
  int64_t ld_dout;
  const float* in;
  int64_t ld_in;
  int H, W;
  const float* w;
  int kh, kw;
  int pad;
};
size_t stencil_backward_workspace(int H, int W, int kh, int kw);

// ---------------------------------------------------------------------------
// matrix-vector product (gemv.hip)
// ---------------------------------------------------------------------------
struct GemvArgs {
  float* y;
  const float* A;
  int64_t lda;
  bool trans;  // A stored K x M, read through transpose
  const float* x;
  int M, K;
};
size_t gemv_workspace(int64_t M, int64_t K, bool trans);
int gemv_parts(int64_t M, int64_t K, bool trans);
rise_status launch_gemv(const GemvArgs& a, void* ws, hipStream_t s);
// the fixed per-device scratch of rise_gemv_noalloc: its size, and its device
// address on the current device (looked up on the first call per device)
size_t gemv_scratch_bytes();
rise_status gemv_scratch(void** out);
rise_status launch_stencil2d_backward(const StencilBwdArgs& a, void* ws, hipStream_t s);

// ---------------------------------------------------------------------------
// iterated stencil (stencil_iter.hip)
// ---------------------------------------------------------------------------
bool stencil_iterate_fusable(int kh, int kw);
int stencil_iterate_max_fuse();
int stencil_iterate_default_fuse(int kh, int kw);
size_t stencil_iterate_workspace(int64_t H, int64_t W, int64_t steps, int fuse);
rise_status launch_stencil_iterate(const StencilArgs& a, int64_t steps, int fuse, void* ws,
                                   hipStream_t s);

// ---------------------------------------------------------------------------
// iterate with the tree-reduction body (iterate.hip)
// ---------------------------------------------------------------------------
int iterate_max_fan_in();
size_t iterate_sum_workspace(int64_t n, int64_t m, int64_t k);
int iterate_sum_rounds(int64_t n, int64_t m, int64_t k, int32_t* rounds, int cap);
rise_status launch_iterate_sum(float* out, const float* in, int64_t n, int64_t m, int64_t k,
                               void* ws, hipStream_t s);

}  // namespace rise
