// C ABI entry points: argument validation (before anything is enqueued) and
// dispatch to the kernels.  Every rejected call names its reason through
// rise_last_error(); nothing is chosen silently.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <string>

#include "common.h"
#include "batched.h"
#include "conv.h"
#include "gemm_lowp.h"
#include "tune.h"

namespace rise {

static thread_local std::string g_last_error;

rise_status fail(rise_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

void clear_error() { g_last_error.clear(); }

rise_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(RISE_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return RISE_OK;
}

int device_cu_count() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  if (dev >= 0 && dev < 64) {
    int v = cache[dev].load(std::memory_order_relaxed);
    if (v > 0) return v;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  if (dev >= 0 && dev < 64) cache[dev].store(cus, std::memory_order_relaxed);
  return cus;
}

namespace {

constexpr int64_t kDimLimit = (int64_t)1 << 31;

struct Range {
  uintptr_t lo, hi;  // [lo, hi)
};

// Byte range touched by a rows x cols row-major array with leading dimension ld.
Range span(const void* p, int64_t rows, int64_t cols, int64_t ld, int64_t esize) {
  if (rows <= 0 || cols <= 0) return Range{0, 0};
  uintptr_t lo = (uintptr_t)p;
  return Range{lo, lo + (uintptr_t)(((rows - 1) * ld + cols) * esize)};
}

bool overlaps(Range a, Range b) {
  if (a.lo == a.hi || b.lo == b.hi) return false;
  return a.lo < b.hi && b.lo < a.hi;
}

bool dim_ok(int64_t v) { return v >= 0 && v < kDimLimit; }

// The tile a GEMM runs when the caller passes none: the tune cache's entry for
// these sizes and mode on this device, else the built-in default of the mode.
rise_tile chosen_gemm_tile(int64_t M, int64_t N, int64_t K, rise_mode mode) {
  rise_tile t;
  if (M > 0 && N > 0 && K > 0 && tune_lookup_gemm(M, N, K, (int)mode, &t) &&
      (mode == RISE_MODE_F32 ? gemm_f32_tile_supported(t) : gemm_lowp_tile_supported(mode, t)))
    return t;
  return mode == RISE_MODE_F32 ? gemm_f32_default_tile((int)M, (int)N, (int)K)
                               : gemm_lowp_default_tile(mode, (int)M, (int)N, (int)K);
}

// The schedule a stencil runs when the caller passes none (tune cache, else default).
rise_stencil_schedule chosen_stencil_schedule(int64_t H, int64_t W, int kh, int kw) {
  rise_stencil_schedule sc;
  if (kh == kw && H > 0 && W > 0 && tune_lookup_stencil(H, W, kh, &sc) &&
      stencil_schedule_supported(sc))
    return sc;
  return stencil_default_schedule((int)H, (int)W, kh, kw);
}

}  // namespace
}  // namespace rise

using namespace rise;

extern "C" {

const char* rise_status_string(rise_status s) {
  switch (s) {
    case RISE_OK: return "ok";
    case RISE_ERR_NULL: return "null pointer";
    case RISE_ERR_SHAPE: return "invalid shape or leading dimension";
    case RISE_ERR_ALIAS: return "output overlaps an input";
    case RISE_ERR_DTYPE: return "element type and mode have no kernel";
    case RISE_ERR_UNSUPPORTED: return "unsupported argument";
    case RISE_ERR_WORKSPACE: return "workspace missing or too small";
    case RISE_ERR_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

const char* rise_last_error(void) { return g_last_error.c_str(); }

int32_t rise_gemm_tiles(rise_mode mode, rise_tile* out, int32_t cap) {
  if (mode == RISE_MODE_F32) return gemm_f32_tiles(out, cap);
  return gemm_lowp_tiles(mode, out, cap);
}

rise_status rise_gemm_default_tile(int64_t M, int64_t N, int64_t K, rise_mode mode,
                                   rise_tile* out) {
  clear_error();
  if (!dim_ok(M) || !dim_ok(N) || !dim_ok(K))
    return fail(RISE_ERR_SHAPE, "rise_gemm_default_tile: sizes must be in [0, 2^31)");
  if (mode < RISE_MODE_F32 || mode > RISE_MODE_FP8)
    return fail(RISE_ERR_UNSUPPORTED, "rise_gemm_default_tile: unknown mode");
  if (!out) return fail(RISE_ERR_NULL, "rise_gemm_default_tile: out is NULL");
  *out = chosen_gemm_tile(M, N, K, mode);
  return RISE_OK;
}

size_t rise_gemm_workspace(int64_t M, int64_t N, int64_t K, rise_mode mode,
                           const rise_tile* tile) {
  if (mode == RISE_MODE_F32) return 0;
  if (!dim_ok(M) || !dim_ok(N) || !dim_ok(K)) return 0;
  rise_tile t = tile ? *tile : chosen_gemm_tile(M, N, K, mode);
  return gemm_lowp_workspace((int)M, (int)N, (int)K, mode, t);
}

rise_status rise_gemm(float* C, int64_t ldc, const void* A, rise_dtype tA, int64_t lda,
                      rise_op opA, const void* B, rise_dtype tB, int64_t ldb, rise_op opB,
                      int64_t M, int64_t N, int64_t K, rise_mode mode, const rise_tile* tile,
                      void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (!dim_ok(M) || !dim_ok(N) || !dim_ok(K))
    return fail(RISE_ERR_SHAPE, "rise_gemm: sizes must be in [0, 2^31)");
  if (opA != RISE_OP_N && opA != RISE_OP_T) return fail(RISE_ERR_UNSUPPORTED, "rise_gemm: opA");
  if (opB != RISE_OP_N && opB != RISE_OP_T) return fail(RISE_ERR_UNSUPPORTED, "rise_gemm: opB");
  if (mode < RISE_MODE_F32 || mode > RISE_MODE_FP8)
    return fail(RISE_ERR_UNSUPPORTED, "rise_gemm: unknown mode");
  if (tA != RISE_F32 && tA != RISE_BF16) return fail(RISE_ERR_DTYPE, "rise_gemm: tA");
  if (tB != RISE_F32 && tB != RISE_BF16) return fail(RISE_ERR_DTYPE, "rise_gemm: tB");
  if (M == 0 || N == 0) return RISE_OK;
  if (!C) return fail(RISE_ERR_NULL, "rise_gemm: C is NULL");
  if (ldc < N) return fail(RISE_ERR_SHAPE, "rise_gemm: ldc < N");
  // stored shapes of A and B
  const int64_t ar = opA == RISE_OP_N ? M : K, ac = opA == RISE_OP_N ? K : M;
  const int64_t br = opB == RISE_OP_N ? K : N, bc = opB == RISE_OP_N ? N : K;
  if (K > 0) {
    if (!A || !B) return fail(RISE_ERR_NULL, "rise_gemm: A or B is NULL");
    if (lda < ac) return fail(RISE_ERR_SHAPE, "rise_gemm: lda below the stored row length");
    if (ldb < bc) return fail(RISE_ERR_SHAPE, "rise_gemm: ldb below the stored row length");
  }
  const int64_t ea = tA == RISE_F32 ? 4 : 2, eb = tB == RISE_F32 ? 4 : 2;
  Range rc = span(C, M, N, ldc, 4);
  if (K > 0 && (overlaps(rc, span(A, ar, ac, lda, ea)) || overlaps(rc, span(B, br, bc, ldb, eb))))
    return fail(RISE_ERR_ALIAS, "rise_gemm: C overlaps A or B");

  if (mode == RISE_MODE_F32) {
    if (tA != RISE_F32 || tB != RISE_F32)
      return fail(RISE_ERR_DTYPE, "rise_gemm: mode F32 needs FP32 operands");
    rise_tile t = tile ? *tile : chosen_gemm_tile(M, N, K, mode);
    if (!gemm_f32_tile_supported(t))
      return fail(RISE_ERR_UNSUPPORTED, "rise_gemm: tile not supported for mode F32");
    GemmF32Args a{C, ldc, (const float*)A, lda, (const float*)B, ldb, (int)M, (int)N, (int)K,
                  opA == RISE_OP_T, opB == RISE_OP_T};
    return launch_gemm_f32(a, t, (hipStream_t)stream);
  }

  if (mode != RISE_MODE_BF16 && (tA != RISE_F32 || tB != RISE_F32))
    return fail(RISE_ERR_DTYPE, "rise_gemm: split and FP8 modes need FP32 operands");
  rise_tile t = tile ? *tile : chosen_gemm_tile(M, N, K, mode);
  if (!gemm_lowp_tile_supported(mode, t))
    return fail(RISE_ERR_UNSUPPORTED, "rise_gemm: tile not supported for this mode");
  size_t need = gemm_lowp_workspace((int)M, (int)N, (int)K, mode, t);
  if (need > 0 && (!ws || ws_bytes < need))
    return fail(RISE_ERR_WORKSPACE, "rise_gemm: workspace below rise_gemm_workspace()");
  if (need > 0 && ((uintptr_t)ws & 255))
    return fail(RISE_ERR_WORKSPACE, "rise_gemm: workspace must be 256-byte aligned");
  if (need > 0) {
    Range rw{(uintptr_t)ws, (uintptr_t)ws + need};
    if (overlaps(rw, rc) || (K > 0 && (overlaps(rw, span(A, ar, ac, lda, ea)) ||
                                       overlaps(rw, span(B, br, bc, ldb, eb)))))
      return fail(RISE_ERR_ALIAS, "rise_gemm: workspace overlaps C, A or B");
  }
  GemmLowpArgs a{C, ldc, A, tA, lda, opA == RISE_OP_T, B, tB, ldb, opB == RISE_OP_T,
                 (int)M, (int)N, (int)K, mode};
  return launch_gemm_lowp(a, t, ws, (hipStream_t)stream);
}

size_t rise_prep_bytes(int64_t rows_out, int64_t k_out, rise_mode mode) {
  if (rows_out < 0 || k_out < 0) return 0;
  return prep_bytes(rows_out, k_out, mode);
}

rise_status rise_prep_operand(void* out, int64_t rows_out, int64_t k_out, const float* src,
                              int64_t rows, int64_t K, int64_t ld_r, int64_t ld_k,
                              rise_mode mode, void* stream) {
  clear_error();
  if (mode != RISE_MODE_BF16 && mode != RISE_MODE_BF16X3 && mode != RISE_MODE_BF16X6 &&
      mode != RISE_MODE_FP8)
    return fail(RISE_ERR_UNSUPPORTED, "rise_prep_operand: mode has no preparation");
  if (!dim_ok(rows) || !dim_ok(K) || !dim_ok(rows_out) || !dim_ok(k_out))
    return fail(RISE_ERR_SHAPE, "rise_prep_operand: sizes must be in [0, 2^31)");
  if (rows_out < rows || k_out < K)
    return fail(RISE_ERR_SHAPE, "rise_prep_operand: destination smaller than the source");
  if (mode == RISE_MODE_FP8 && k_out % 32 != 0)
    return fail(RISE_ERR_SHAPE, "rise_prep_operand: FP8 needs k_out a multiple of 32");
  if (ld_r < 0 || ld_k < 0) return fail(RISE_ERR_SHAPE, "rise_prep_operand: negative stride");
  if (rows_out == 0 || k_out == 0) return RISE_OK;
  if (!out) return fail(RISE_ERR_NULL, "rise_prep_operand: out is NULL");
  if (rows > 0 && K > 0) {
    if (!src) return fail(RISE_ERR_NULL, "rise_prep_operand: src is NULL");
    uintptr_t lo = (uintptr_t)src;
    uintptr_t hi = lo + (uintptr_t)(((rows - 1) * ld_r + (K - 1) * ld_k + 1) * 4);
    Range ro{(uintptr_t)out, (uintptr_t)out + prep_bytes(rows_out, k_out, mode)};
    if (overlaps(ro, Range{lo, hi})) return fail(RISE_ERR_ALIAS, "rise_prep_operand: overlap");
  }
  PrepArgs a{out, rows_out, k_out, src, rows, K, ld_r, ld_k, mode};
  return launch_prep(a, (hipStream_t)stream);
}

int32_t rise_stencil_schedules(rise_stencil_schedule* out, int32_t cap) {
  return stencil_schedules(out, cap);
}

rise_status rise_stencil2d_default_schedule(int64_t H, int64_t W, int32_t kh, int32_t kw,
                                            rise_stencil_schedule* out) {
  clear_error();
  if (!dim_ok(H) || !dim_ok(W))
    return fail(RISE_ERR_SHAPE, "rise_stencil2d_default_schedule: sizes must be in [0, 2^31)");
  if (kh <= 0 || kw <= 0 || kh % 2 == 0 || kw % 2 == 0 || kh > 15 || kw > 15)
    return fail(RISE_ERR_UNSUPPORTED,
                "rise_stencil2d_default_schedule: window sides must be odd and <= 15");
  if (!out) return fail(RISE_ERR_NULL, "rise_stencil2d_default_schedule: out is NULL");
  const bool scheduled = kh == kw && (kh == 1 || kh == 3 || kh == 5 || kh == 7);
  *out = scheduled ? chosen_stencil_schedule(H, W, kh, kw) : rise_stencil_schedule{-1, 0};
  return RISE_OK;
}

rise_status rise_stencil2d(float* out, int64_t ld_out, const float* in, int64_t ld_in,
                           int64_t H, int64_t W, const float* w, int32_t kh, int32_t kw,
                           rise_pad pad, const rise_stencil_schedule* sched, void* stream) {
  clear_error();
  if (!dim_ok(H) || !dim_ok(W) || H * W >= kDimLimit * 2)
    return fail(RISE_ERR_SHAPE, "rise_stencil2d: sizes must be in [0, 2^31)");
  if (kh <= 0 || kw <= 0 || kh % 2 == 0 || kw % 2 == 0 || kh > 15 || kw > 15)
    return fail(RISE_ERR_UNSUPPORTED, "rise_stencil2d: window sides must be odd and <= 15");
  if (pad != RISE_PAD_CLAMP && pad != RISE_PAD_ZERO)
    return fail(RISE_ERR_UNSUPPORTED, "rise_stencil2d: unknown pad mode");
  if (H == 0 || W == 0) return RISE_OK;
  if (!out || !in || !w) return fail(RISE_ERR_NULL, "rise_stencil2d: NULL pointer");
  if (ld_in < W || ld_out < W) return fail(RISE_ERR_SHAPE, "rise_stencil2d: ld below W");
  Range ro = span(out, H, W, ld_out, 4);
  if (overlaps(ro, span(in, H, W, ld_in, 4)) || overlaps(ro, span(w, kh, kw, kw, 4)))
    return fail(RISE_ERR_ALIAS, "rise_stencil2d: out overlaps in or w");
  rise_stencil_schedule sc = sched ? *sched : chosen_stencil_schedule(H, W, kh, kw);
  if (!stencil_schedule_supported(sc))
    return fail(RISE_ERR_UNSUPPORTED, "rise_stencil2d: unknown schedule");
  StencilArgs a{out, ld_out, in, ld_in, (int)H, (int)W, w, kh, kw, (int)pad};
  return launch_stencil2d(a, sc, (hipStream_t)stream);
}

int32_t rise_stencil2d_iterate_max_fuse(void) { return stencil_iterate_max_fuse(); }

// the fuse a call runs with, or -1 when the request has no schedule
static int iterate_fuse(int32_t kh, int32_t kw, int32_t fuse) {
  if (fuse == 0) return stencil_iterate_default_fuse(kh, kw);
  if (fuse == 1) return 1;
  if (fuse < 0 || fuse > stencil_iterate_max_fuse() || !stencil_iterate_fusable(kh, kw))
    return -1;
  return fuse;
}

int32_t rise_stencil2d_iterate_default_fuse(int32_t kh, int32_t kw) {
  return stencil_iterate_default_fuse(kh, kw);
}

size_t rise_stencil2d_iterate_workspace(int64_t H, int64_t W, int32_t kh, int32_t kw,
                                        int64_t steps, int32_t fuse) {
  const int f = iterate_fuse(kh, kw, fuse);
  if (!dim_ok(H) || !dim_ok(W) || steps < 0 || f < 0) return 0;
  return stencil_iterate_workspace(H, W, steps, f);
}

rise_status rise_stencil2d_iterate(float* out, int64_t ld_out, const float* in, int64_t ld_in,
                                   int64_t H, int64_t W, const float* w, int32_t kh, int32_t kw,
                                   rise_pad pad, int64_t steps, int32_t fuse, void* ws,
                                   size_t ws_bytes, void* stream) {
  clear_error();
  if (!dim_ok(H) || !dim_ok(W) || H * W >= kDimLimit * 2)
    return fail(RISE_ERR_SHAPE, "rise_stencil2d_iterate: sizes must be in [0, 2^31)");
  if (steps < 0 || steps >= kDimLimit)
    return fail(RISE_ERR_SHAPE, "rise_stencil2d_iterate: steps must be in [0, 2^31)");
  if (kh <= 0 || kw <= 0 || kh % 2 == 0 || kw % 2 == 0 || kh > 15 || kw > 15)
    return fail(RISE_ERR_UNSUPPORTED, "rise_stencil2d_iterate: window sides must be odd and <= 15");
  if (pad != RISE_PAD_CLAMP && pad != RISE_PAD_ZERO)
    return fail(RISE_ERR_UNSUPPORTED, "rise_stencil2d_iterate: unknown pad mode");
  const int f = iterate_fuse(kh, kw, fuse);
  if (f < 0)
    return fail(RISE_ERR_UNSUPPORTED,
                "rise_stencil2d_iterate: fuse > 1 needs a square 3x3 or 5x5 window and at most "
                "rise_stencil2d_iterate_max_fuse() steps");
  if (H == 0 || W == 0) return RISE_OK;
  if (!out || !in || !w) return fail(RISE_ERR_NULL, "rise_stencil2d_iterate: NULL pointer");
  if (ld_in < W || ld_out < W) return fail(RISE_ERR_SHAPE, "rise_stencil2d_iterate: ld below W");
  const Range ro = span(out, H, W, ld_out, 4), ri = span(in, H, W, ld_in, 4),
              rw = span(w, kh, kw, kw, 4);
  if (overlaps(ro, ri) || overlaps(ro, rw))
    return fail(RISE_ERR_ALIAS, "rise_stencil2d_iterate: out overlaps in or w");
  const size_t need = stencil_iterate_workspace(H, W, steps, f);
  if (need > 0) {
    if (!ws || ws_bytes < need)
      return fail(RISE_ERR_WORKSPACE,
                  "rise_stencil2d_iterate: workspace below rise_stencil2d_iterate_workspace()");
    if ((uintptr_t)ws & 255)
      return fail(RISE_ERR_WORKSPACE, "rise_stencil2d_iterate: workspace must be 256-byte aligned");
    const Range rs{(uintptr_t)ws, (uintptr_t)ws + need};
    if (overlaps(rs, ro) || overlaps(rs, ri) || overlaps(rs, rw))
      return fail(RISE_ERR_ALIAS, "rise_stencil2d_iterate: workspace overlaps out, in or w");
  }
  StencilArgs a{out, ld_out, in, ld_in, (int)H, (int)W, w, kh, kw, (int)pad};
  return launch_stencil_iterate(a, steps, f, ws, (hipStream_t)stream);
}

int32_t rise_gemv_parts(int64_t M, int64_t K, rise_op opA) {
  if (!dim_ok(M) || !dim_ok(K) || (opA != RISE_OP_N && opA != RISE_OP_T)) return 0;
  return gemv_parts(M, K, opA == RISE_OP_T);
}

size_t rise_gemv_workspace(int64_t M, int64_t K, rise_op opA) {
  if (!dim_ok(M) || !dim_ok(K) || (opA != RISE_OP_N && opA != RISE_OP_T)) return 0;
  const size_t b = gemv_workspace(M, K, opA == RISE_OP_T);
  return (b + 255) / 256 * 256;
}

// argument checks shared by rise_gemv and rise_gemv_noalloc (everything but
// the workspace); RISE_OK with *noop set when M = 0
static rise_status check_gemv(const char* who, float* y, const float* A, int64_t lda, rise_op opA,
                              const float* x, int64_t M, int64_t K, bool* noop) {
  const std::string w(who);
  *noop = false;
  if (!dim_ok(M) || !dim_ok(K)) return fail(RISE_ERR_SHAPE, w + ": sizes must be in [0, 2^31)");
  if (opA != RISE_OP_N && opA != RISE_OP_T) return fail(RISE_ERR_UNSUPPORTED, w + ": opA");
  if (M == 0) {
    *noop = true;
    return RISE_OK;
  }
  if (!y) return fail(RISE_ERR_NULL, w + ": y is NULL");
  const int64_t ar = opA == RISE_OP_N ? M : K, ac = opA == RISE_OP_N ? K : M;
  const Range ry = span(y, 1, M, M, 4);
  if (K > 0) {
    if (!A || !x) return fail(RISE_ERR_NULL, w + ": A or x is NULL");
    if (lda < ac) return fail(RISE_ERR_SHAPE, w + ": lda below the stored row length");
    if (overlaps(ry, span(A, ar, ac, lda, 4)) || overlaps(ry, span(x, 1, K, K, 4)))
      return fail(RISE_ERR_ALIAS, w + ": y overlaps A or x");
  }
  return RISE_OK;
}

rise_status rise_gemv(float* y, const float* A, int64_t lda, rise_op opA, const float* x,
                      int64_t M, int64_t K, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  bool noop = false;
  rise_status st = check_gemv("rise_gemv", y, A, lda, opA, x, M, K, &noop);
  if (st != RISE_OK || noop) return st;
  const int64_t ar = opA == RISE_OP_N ? M : K, ac = opA == RISE_OP_N ? K : M;
  const Range ry = span(y, 1, M, M, 4);
  const size_t need = gemv_workspace(M, K, opA == RISE_OP_T);
  if (need > 0) {
    if (!ws || ws_bytes < need)
      return fail(RISE_ERR_WORKSPACE, "rise_gemv: workspace below rise_gemv_workspace()");
    if ((uintptr_t)ws & 255)
      return fail(RISE_ERR_WORKSPACE, "rise_gemv: workspace must be 256-byte aligned");
    const Range rw{(uintptr_t)ws, (uintptr_t)ws + need};
    if (overlaps(rw, ry) || overlaps(rw, span(A, ar, ac, lda, 4)) ||
        overlaps(rw, span(x, 1, K, K, 4)))
      return fail(RISE_ERR_ALIAS, "rise_gemv: workspace overlaps y, A or x");
  }
  GemvArgs a{y, A, lda, opA == RISE_OP_T, x, (int)M, (int)K};
  return launch_gemv(a, ws, (hipStream_t)stream);
}

rise_status rise_gemv_noalloc(float* y, const float* A, int64_t lda, rise_op opA, const float* x,
                              int64_t M, int64_t K, void* stream) {
  clear_error();
  bool noop = false;
  rise_status st = check_gemv("rise_gemv_noalloc", y, A, lda, opA, x, M, K, &noop);
  if (st != RISE_OK || noop) return st;
  const size_t need = gemv_workspace(M, K, opA == RISE_OP_T);
  if (need > gemv_scratch_bytes())
    return fail(RISE_ERR_WORKSPACE, "rise_gemv_noalloc: split-K partials (" + std::to_string(need) +
                                        " bytes) exceed the fixed scratch of " +
                                        std::to_string(gemv_scratch_bytes()) + " bytes");
  void* scratch = nullptr;
  if (need > 0) {
    st = gemv_scratch(&scratch);
    if (st != RISE_OK) return st;
  }
  GemvArgs a{y, A, lda, opA == RISE_OP_T, x, (int)M, (int)K};
  return launch_gemv(a, scratch, (hipStream_t)stream);
}

// n^k * m when it is below 2^40, else -1
static int64_t iterate_len(int64_t n, int64_t m, int64_t k) {
  const int64_t lim = (int64_t)1 << 40;
  if (n < 1 || m < 0 || k < 0 || m >= lim) return -1;
  if (n == 1) return m;
  int64_t v = m;
  for (int64_t i = 0; i < k && v > 0; i++) {
    if (v > (lim - 1) / n) return -1;
    v *= n;
  }
  return v;
}

size_t rise_iterate_sum_workspace(int64_t n, int64_t m, int64_t k) {
  if (iterate_len(n, m, k) < 0 || n > iterate_max_fan_in() || m == 0) return 0;
  return iterate_sum_workspace(n, m, k);
}

int32_t rise_iterate_sum_passes(int64_t n, int64_t m, int64_t k, int32_t* rounds,
                                int32_t cap) {
  if (iterate_len(n, m, k) < 0 || n > iterate_max_fan_in() || m == 0) return 0;
  return iterate_sum_rounds(n, m, k, rounds, cap < 0 ? 0 : cap);
}

rise_status rise_iterate_sum(float* out, const float* in, int64_t n, int64_t m, int64_t k,
                             void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (n < 1 || k < 0 || m < 0)
    return fail(RISE_ERR_SHAPE, "rise_iterate_sum: needs n >= 1, m >= 0, k >= 0");
  if (n > iterate_max_fan_in())
    return fail(RISE_ERR_UNSUPPORTED, "rise_iterate_sum: fan-in n above 8192");
  const int64_t len = iterate_len(n, m, k);
  if (len < 0) return fail(RISE_ERR_SHAPE, "rise_iterate_sum: n^k * m must be below 2^40");
  if (m == 0) return RISE_OK;
  if (!out || !in) return fail(RISE_ERR_NULL, "rise_iterate_sum: out or in is NULL");
  const Range ro = span(out, 1, m, m, 4), ri = span(in, 1, len, len, 4);
  if (overlaps(ro, ri)) return fail(RISE_ERR_ALIAS, "rise_iterate_sum: out overlaps in");
  const size_t need = iterate_sum_workspace(n, m, k);
  if (need > 0) {
    if (!ws || ws_bytes < need)
      return fail(RISE_ERR_WORKSPACE, "rise_iterate_sum: workspace below rise_iterate_sum_workspace()");
    if ((uintptr_t)ws & 255)
      return fail(RISE_ERR_WORKSPACE, "rise_iterate_sum: workspace must be 256-byte aligned");
    const Range rw{(uintptr_t)ws, (uintptr_t)ws + need};
    if (overlaps(rw, ro) || overlaps(rw, ri))
      return fail(RISE_ERR_ALIAS, "rise_iterate_sum: workspace overlaps out or in");
  }
  return launch_iterate_sum(out, in, n, m, k, ws, (hipStream_t)stream);
}

size_t rise_gemm_backward_workspace(int64_t M, int64_t N, int64_t K, rise_mode mode) {
  size_t a = rise_gemm_workspace(M, K, N, mode, nullptr);  // dA: M x K, reduction over N
  size_t b = rise_gemm_workspace(K, N, M, mode, nullptr);  // dB: K x N, reduction over M
  return a > b ? a : b;
}

rise_status rise_gemm_backward(float* dA, int64_t ldda, float* dB, int64_t lddb, const float* dC,
                               int64_t lddc, const float* A, int64_t lda, const float* B,
                               int64_t ldb, int64_t M, int64_t N, int64_t K, rise_mode mode,
                               void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (!dim_ok(M) || !dim_ok(N) || !dim_ok(K))
    return fail(RISE_ERR_SHAPE, "rise_gemm_backward: sizes must be in [0, 2^31)");
  if (dA && dB) {
    if (overlaps(span(dA, M, K, ldda, 4), span(dB, K, N, lddb, 4)))
      return fail(RISE_ERR_ALIAS, "rise_gemm_backward: dA overlaps dB");
  }
  // Every output is checked against every input, not only against the inputs of
  // its own product: dA is written before the dB product reads A, and the
  // workspace is rewritten by each product's operand preparation.
  Range rc = span(dC, M, N, lddc, 4), ra = span(A, M, K, lda, 4), rb = span(B, K, N, ldb, 4);
  const Range rda = dA ? span(dA, M, K, ldda, 4) : Range{0, 0};
  const Range rdb = dB ? span(dB, K, N, lddb, 4) : Range{0, 0};
  if (overlaps(rda, rc) || overlaps(rda, ra) || overlaps(rda, rb))
    return fail(RISE_ERR_ALIAS, "rise_gemm_backward: dA overlaps an input");
  if (overlaps(rdb, rc) || overlaps(rdb, ra) || overlaps(rdb, rb))
    return fail(RISE_ERR_ALIAS, "rise_gemm_backward: dB overlaps an input");
  if (ws && ws_bytes > 0) {
    const Range rw{(uintptr_t)ws, (uintptr_t)ws + ws_bytes};
    if (overlaps(rw, rda) || overlaps(rw, rdb) || overlaps(rw, rc) || overlaps(rw, ra) ||
        overlaps(rw, rb))
      return fail(RISE_ERR_ALIAS, "rise_gemm_backward: workspace overlaps an operand");
  }
  rise_status st = RISE_OK;
  if (dA) {  // dA (M x K) = dC (M x N) . transpose(B), B stored K x N
    st = rise_gemm(dA, ldda, dC, RISE_F32, lddc, RISE_OP_N, B, RISE_F32, ldb, RISE_OP_T, M, K, N,
                   mode, nullptr, ws, ws_bytes, stream);
    if (st != RISE_OK) return st;
  }
  if (dB) {  // dB (K x N) = transpose(A) . dC, A stored M x K
    st = rise_gemm(dB, lddb, A, RISE_F32, lda, RISE_OP_T, dC, RISE_F32, lddc, RISE_OP_N, K, N, M,
                   mode, nullptr, ws, ws_bytes, stream);
  }
  return st;
}

size_t rise_stencil2d_backward_workspace(int64_t H, int64_t W, int32_t kh, int32_t kw) {
  if (!dim_ok(H) || !dim_ok(W) || kh <= 0 || kw <= 0 || kh > 15 || kw > 15) return 0;
  return stencil_backward_workspace((int)H, (int)W, kh, kw);
}

rise_status rise_stencil2d_backward(float* dIn, int64_t ld_din, float* dW, const float* dOut,
                                    int64_t ld_dout, const float* in, int64_t ld_in, int64_t H,
                                    int64_t W, const float* w, int32_t kh, int32_t kw,
                                    rise_pad pad, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (!dim_ok(H) || !dim_ok(W))
    return fail(RISE_ERR_SHAPE, "rise_stencil2d_backward: sizes must be in [0, 2^31)");
  if (kh <= 0 || kw <= 0 || kh % 2 == 0 || kw % 2 == 0 || kh > 15 || kw > 15)
    return fail(RISE_ERR_UNSUPPORTED, "rise_stencil2d_backward: window sides must be odd, <= 15");
  if (pad != RISE_PAD_CLAMP && pad != RISE_PAD_ZERO)
    return fail(RISE_ERR_UNSUPPORTED, "rise_stencil2d_backward: unknown pad mode");
  if (!dIn && !dW) return RISE_OK;
  if (H == 0 || W == 0) {
    if (dW) return fail(RISE_ERR_SHAPE, "rise_stencil2d_backward: dW of an empty image");
    return RISE_OK;
  }
  if (!dOut) return fail(RISE_ERR_NULL, "rise_stencil2d_backward: dOut is NULL");
  if (dIn && !w) return fail(RISE_ERR_NULL, "rise_stencil2d_backward: w is NULL");
  if (dW && !in) return fail(RISE_ERR_NULL, "rise_stencil2d_backward: in is NULL");
  if (ld_dout < W || (dIn && ld_din < W) || (dW && ld_in < W))
    return fail(RISE_ERR_SHAPE, "rise_stencil2d_backward: ld below W");
  size_t need = stencil_backward_workspace((int)H, (int)W, kh, kw);
  if (!ws || ws_bytes < need)
    return fail(RISE_ERR_WORKSPACE, "rise_stencil2d_backward: workspace too small");
  if ((uintptr_t)ws & 255)
    return fail(RISE_ERR_WORKSPACE, "rise_stencil2d_backward: workspace must be 256-byte aligned");
  Range rws{(uintptr_t)ws, (uintptr_t)ws + need};
  Range rg = span(dOut, H, W, ld_dout, 4);
  Range rin = dW ? span(in, H, W, ld_in, 4) : Range{0, 0};
  Range rwt = dIn ? span(w, kh, kw, kw, 4) : Range{0, 0};
  Range rdi = dIn ? span(dIn, H, W, ld_din, 4) : Range{0, 0};
  Range rdw = dW ? span(dW, kh, kw, kw, 4) : Range{0, 0};
  for (Range o : {rdi, rdw, rws})
    for (Range i : {rg, rin, rwt})
      if (overlaps(o, i)) return fail(RISE_ERR_ALIAS, "rise_stencil2d_backward: output overlaps input");
  if (overlaps(rdi, rdw) || overlaps(rdi, rws) || overlaps(rdw, rws))
    return fail(RISE_ERR_ALIAS, "rise_stencil2d_backward: outputs overlap");
  StencilBwdArgs a{dIn, ld_din, dW, dOut, ld_dout, in, ld_in, (int)H, (int)W, w, kh, kw, (int)pad};
  return launch_stencil2d_backward(a, ws, (hipStream_t)stream);
}

namespace {
bool conv_dims_ok(int64_t B, int64_t Cin, int64_t Cout, int64_t H, int64_t W) {
  return B >= 0 && H >= 0 && W >= 0 && dim_ok(B * H * W) && Cin > 0 && Cout > 0;
}
bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }
}  // namespace

size_t rise_conv2d_workspace(int32_t Cin, int32_t Cout) {
  if (Cin <= 0 || Cout <= 0) return 0;
  return conv_forward_workspace(Cin, Cout);
}

rise_status rise_conv2d(uint16_t* out, const uint16_t* in, const float* w, int32_t B, int32_t Cin,
                        int32_t Cout, int32_t H, int32_t W, int32_t kh, int32_t kw, rise_pad pad,
                        void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (!conv_dims_ok(B, Cin, Cout, H, W)) return fail(RISE_ERR_SHAPE, "rise_conv2d: sizes");
  if (pad != RISE_PAD_CLAMP && pad != RISE_PAD_ZERO)
    return fail(RISE_ERR_UNSUPPORTED, "rise_conv2d: unknown pad mode");
  if (!conv_supported(Cin, Cout, kh, kw, false))
    return fail(RISE_ERR_UNSUPPORTED, "rise_conv2d: needs a 3x3 window, Cin in {16,32,64}, "
                                      "Cout in {32,64}");
  if (B == 0 || H == 0 || W == 0) return RISE_OK;
  if (!out || !in || !w) return fail(RISE_ERR_NULL, "rise_conv2d: NULL pointer");
  if (!aligned16(out) || !aligned16(in))
    return fail(RISE_ERR_SHAPE, "rise_conv2d: activations must be 16-byte aligned");
  size_t need = conv_forward_workspace(Cin, Cout);
  if (!ws || ws_bytes < need) return fail(RISE_ERR_WORKSPACE, "rise_conv2d: workspace too small");
  if ((uintptr_t)ws & 255) return fail(RISE_ERR_WORKSPACE, "rise_conv2d: workspace alignment");
  const int64_t px = (int64_t)B * H * W;
  Range ro{(uintptr_t)out, (uintptr_t)out + (uintptr_t)(px * Cout * 2)};
  Range ri{(uintptr_t)in, (uintptr_t)in + (uintptr_t)(px * Cin * 2)};
  Range rw{(uintptr_t)w, (uintptr_t)w + (uintptr_t)Cout * Cin * 9 * 4};
  Range rs{(uintptr_t)ws, (uintptr_t)ws + need};
  if (overlaps(ro, ri) || overlaps(ro, rw) || overlaps(ro, rs) || overlaps(rs, ri) ||
      overlaps(rs, rw))
    return fail(RISE_ERR_ALIAS, "rise_conv2d: output or workspace overlaps an input");
  ConvArgs a{out, in, w, B, Cin, Cout, H, W, pad == RISE_PAD_ZERO};
  return launch_conv2d(a, ws, (hipStream_t)stream);
}

size_t rise_conv2d_backward_workspace(int32_t B, int32_t Cin, int32_t Cout, int32_t H, int32_t W) {
  if (!conv_dims_ok(B, Cin, Cout, H, W)) return 0;
  return conv_backward_workspace(B, Cin, Cout, H, W);
}

rise_status rise_conv2d_backward(uint16_t* dIn, float* dW, const uint16_t* dOut,
                                 const uint16_t* in, const float* w, int32_t B, int32_t Cin,
                                 int32_t Cout, int32_t H, int32_t W, int32_t kh, int32_t kw,
                                 rise_pad pad, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (!conv_dims_ok(B, Cin, Cout, H, W)) return fail(RISE_ERR_SHAPE, "rise_conv2d_backward: sizes");
  if (pad != RISE_PAD_CLAMP && pad != RISE_PAD_ZERO)
    return fail(RISE_ERR_UNSUPPORTED, "rise_conv2d_backward: unknown pad mode");
  if (!conv_supported(Cin, Cout, kh, kw, true))
    return fail(RISE_ERR_UNSUPPORTED, "rise_conv2d_backward: needs a 3x3 window, Cin and Cout "
                                      "in {32,64}");
  if (dIn && pad != RISE_PAD_ZERO)
    return fail(RISE_ERR_UNSUPPORTED, "rise_conv2d_backward: dIn is implemented for zero padding");
  if (!dIn && !dW) return RISE_OK;
  if (B == 0 || H == 0 || W == 0) {
    if (dW) return fail(RISE_ERR_SHAPE, "rise_conv2d_backward: dW of an empty batch");
    return RISE_OK;
  }
  if (!dOut || (dIn && !w) || (dW && !in)) return fail(RISE_ERR_NULL, "rise_conv2d_backward: NULL");
  if (!aligned16(dOut) || (dIn && !aligned16(dIn)) || (dW && !aligned16(in)))
    return fail(RISE_ERR_SHAPE, "rise_conv2d_backward: activations must be 16-byte aligned");
  size_t need = conv_backward_workspace(B, Cin, Cout, H, W);
  if (!ws || ws_bytes < need)
    return fail(RISE_ERR_WORKSPACE, "rise_conv2d_backward: workspace too small");
  if ((uintptr_t)ws & 255)
    return fail(RISE_ERR_WORKSPACE, "rise_conv2d_backward: workspace alignment");
  const int64_t px = (int64_t)B * H * W;
  Range rdi = dIn ? Range{(uintptr_t)dIn, (uintptr_t)dIn + (uintptr_t)(px * Cin * 2)} : Range{0, 0};
  Range rdw = dW ? Range{(uintptr_t)dW, (uintptr_t)dW + (uintptr_t)Cout * Cin * 9 * 4} : Range{0, 0};
  Range rs{(uintptr_t)ws, (uintptr_t)ws + need};
  Range rg{(uintptr_t)dOut, (uintptr_t)dOut + (uintptr_t)(px * Cout * 2)};
  Range rin = dW ? Range{(uintptr_t)in, (uintptr_t)in + (uintptr_t)(px * Cin * 2)} : Range{0, 0};
  Range rwt = dIn ? Range{(uintptr_t)w, (uintptr_t)w + (uintptr_t)Cout * Cin * 9 * 4} : Range{0, 0};
  for (Range o : {rdi, rdw, rs})
    for (Range i : {rg, rin, rwt})
      if (overlaps(o, i)) return fail(RISE_ERR_ALIAS, "rise_conv2d_backward: output overlaps input");
  if (overlaps(rdi, rdw) || overlaps(rdi, rs) || overlaps(rdw, rs))
    return fail(RISE_ERR_ALIAS, "rise_conv2d_backward: outputs overlap");
  ConvBwdArgs a{dIn, dW, dOut, in, w, B, Cin, Cout, H, W, pad == RISE_PAD_ZERO};
  return launch_conv2d_backward(a, ws, (hipStream_t)stream);
}

struct rise_plan {
  rise::PlanImpl* impl;
};

rise_status rise_plan_create(rise_plan** plan, const rise_gemm_problem* gemms, int32_t n_gemm,
                             const rise_stencil_problem* stencils, int32_t n_stencil,
                             const char* tune_table, void* stream) {
  clear_error();
  if (!plan) return fail(RISE_ERR_NULL, "rise_plan_create: plan is NULL");
  *plan = nullptr;
  PlanImpl* impl = nullptr;
  rise_status st = plan_build(&impl, gemms, n_gemm, stencils, n_stencil, tune_table, -1,
                              (hipStream_t)stream);
  if (st != RISE_OK) return st;
  *plan = new rise_plan{impl};
  return RISE_OK;
}

rise_status rise_plan_launch(rise_plan* plan, void* stream) {
  clear_error();
  if (!plan || !plan->impl) return fail(RISE_ERR_NULL, "rise_plan_launch: plan is NULL");
  return plan_launch(plan->impl, (hipStream_t)stream);
}

rise_status rise_plan_launch_direct(rise_plan* plan, void* stream) {
  clear_error();
  if (!plan || !plan->impl) return fail(RISE_ERR_NULL, "rise_plan_launch_direct: plan is NULL");
  return plan_launch_direct(plan->impl, (hipStream_t)stream);
}

rise_status rise_plan_destroy(rise_plan* plan) {
  clear_error();
  if (!plan) return RISE_OK;
  rise_plan_free(plan->impl);
  delete plan;
  return RISE_OK;
}

int32_t rise_plan_items(const rise_plan* plan) {
  return plan && plan->impl ? plan_items(plan->impl) : 0;
}

rise_status rise_plan_tile(const rise_plan* plan, int32_t problem, rise_tile* tile) {
  clear_error();
  if (!plan || !plan->impl || !tile) return fail(RISE_ERR_NULL, "rise_plan_tile: NULL");
  const int k = plan_kind(plan->impl, problem);
  if (k < 0) return fail(RISE_ERR_SHAPE, "rise_plan_tile: problem index outside the plan");
  if (kind_is_stencil(k)) return fail(RISE_ERR_SHAPE, "rise_plan_tile: not a GEMM problem");
  *tile = kind_tile(k);
  return RISE_OK;
}

static rise_status run_once(const rise_gemm_problem* g, int ng, const rise_stencil_problem* s,
                            int ns, void* stream) {
  rise_plan* plan = nullptr;
  rise_status st = rise_plan_create(&plan, g, ng, s, ns, nullptr, stream);
  if (st != RISE_OK) return st;
  st = rise_plan_launch(plan, stream);
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  rise_plan_destroy(plan);
  if (st == RISE_OK && e != hipSuccess)
    st = fail(RISE_ERR_HIP, std::string("batched: ") + hipGetErrorString(e));
  return st;
}

rise_status rise_gemm_batched(const rise_gemm_problem* gemms, int32_t n, void* stream) {
  return run_once(gemms, n, nullptr, 0, stream);
}

rise_status rise_stencil2d_batched(const rise_stencil_problem* stencils, int32_t n,
                                   void* stream) {
  return run_once(nullptr, 0, stencils, n, stream);
}

rise_status rise_autotune_batched(const char* table_path, void* stream) {
  clear_error();
  if (!table_path) return fail(RISE_ERR_NULL, "rise_autotune_batched: table_path is NULL");
  hipStream_t s = (hipStream_t)stream;
  const int n = 4096;
  void *A = nullptr, *B = nullptr, *C = nullptr, *w = nullptr;
  hipError_t e;
  if ((e = hipMalloc(&A, (size_t)n * n * 4)) != hipSuccess || (e = hipMalloc(&B, (size_t)n * n * 4)) != hipSuccess ||
      (e = hipMalloc(&C, (size_t)n * n * 4)) != hipSuccess || (e = hipMalloc(&w, 256)) != hipSuccess) {
    hipFree(A); hipFree(B); hipFree(C); hipFree(w);
    return fail(RISE_ERR_HIP, std::string("rise_autotune_batched: ") + hipGetErrorString(e));
  }
  hipMemsetAsync(A, 0, (size_t)n * n * 4, s);
  hipMemsetAsync(B, 0, (size_t)n * n * 4, s);
  hipMemsetAsync(w, 0, 256, s);
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  FILE* f = fopen(table_path, "w");
  if (!f) {
    hipFree(A); hipFree(B); hipFree(C); hipFree(w);
    return fail(RISE_ERR_UNSUPPORTED, "rise_autotune_batched: cannot write the table");
  }
  rise_status st = RISE_OK;
  // time one plan (graph launches) and return the cost of one item slot in us:
  // total time x concurrent workgroups / items
  auto measure = [&](const rise_gemm_problem* g, const rise_stencil_problem* sp, int kind,
                     double* per_item) -> rise_status {
    PlanImpl* p = nullptr;
    rise_status r = plan_build(&p, g, g ? 1 : 0, sp, sp ? 1 : 0, nullptr, kind, s);
    if (r != RISE_OK) return r;
    plan_launch(p, s);  // warm-up
    hipEventRecord(e0, s);
    const int reps = 5;
    for (int i = 0; i < reps; i++) plan_launch(p, s);
    hipEventRecord(e1, s);
    hipEventSynchronize(e1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    *per_item = (double)ms * 1e3 / reps * plan_grid(p) / std::max(1, plan_items(p));
    rise_plan_free(p);
    return RISE_OK;
  };
  for (int k = 0; k < num_kinds() && st == RISE_OK; k++) {
    if (kind_is_stencil(k)) {
      const int side = kind_stencil_side(k);
      rise_stencil_problem sp{(float*)C, (const float*)A, (const float*)w, n, n, n, n, side,
                              RISE_PAD_CLAMP};
      double t = 0;
      st = measure(nullptr, &sp, k, &t);
      fprintf(f, "%s %.6f %.8f\n", kind_name(k), t, 0.0);
    } else {
      double t1 = 0, t2 = 0;
      const int K1 = 128, K2 = 1024;
      rise_gemm_problem g1{(float*)C, A, B, n, n, K1, K1, kind_opb(k) ? K1 : n, n,
                           kind_dtype(k), kind_opb(k)};
      rise_gemm_problem g2{(float*)C, A, B, n, n, K2, K2, kind_opb(k) ? K2 : n, n,
                           kind_dtype(k), kind_opb(k)};
      st = measure(&g1, nullptr, k, &t1);
      if (st == RISE_OK) st = measure(&g2, nullptr, k, &t2);
      const double b = (t2 - t1) / (K2 - K1), a = t1 - b * K1;
      fprintf(f, "%s %.6f %.8f\n", kind_name(k), a, b);
    }
  }
  fclose(f);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(A); hipFree(B); hipFree(C); hipFree(w);
  return st;
}

}  // extern "C"
