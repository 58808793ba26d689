// Reduced-precision GEMM modes (BF16, split BF16, FP8): operand preparation
// and the packed matrix-core kernels.
#pragma once

#include "common.h"

namespace rise {

// ---- operand preparation --------------------------------------------------
struct PrepArgs {
  void* out;
  int64_t rows_out, k_out;
  const void* src;  // float (or bf16 bits when src_bf16)
  int64_t rows, K, ld_r, ld_k;
  rise_mode mode;
  bool src_bf16 = false;
  // 0: each part is rows_out x k_out, K contiguous.  kblock > 0 (a multiple of
  // 16, of 32 for FP8, dividing k_out): K-blocked, K block b of row r holds
  // kblock consecutive elements at (b * rows_out + r) * kblock, so one block of
  // consecutive rows is contiguous; FP8 scale bytes likewise in groups of
  // kblock / 32.
  int kblock = 0;
};
int prep_parts(rise_mode mode);
size_t prep_bytes(int64_t rows_out, int64_t k_out, rise_mode mode);
rise_status launch_prep(const PrepArgs& a, hipStream_t s);

// ---- packed kernels ---------------------------------------------------------
struct GemmLowpArgs {
  float* C;
  int64_t ldc;
  const void* A;
  rise_dtype tA;
  int64_t lda;
  bool ta;
  const void* B;
  rise_dtype tB;
  int64_t ldb;
  bool tb;
  int M, N, K;
  rise_mode mode;
};
int gemm_lowp_tiles(rise_mode mode, rise_tile* out, int cap);
bool gemm_lowp_tile_supported(rise_mode mode, const rise_tile& t);
rise_tile gemm_lowp_default_tile(rise_mode mode, int M, int N, int K);
size_t gemm_lowp_workspace(int M, int N, int K, rise_mode mode, const rise_tile& t);
rise_status launch_gemm_lowp(const GemmLowpArgs& a, const rise_tile& t, void* ws, hipStream_t s);

// Packed operands already prepared in the layout launch_prep writes: A parts
// Mp x Kp, B parts Np x Kp (B read as transpose(B) rows), Kp a multiple of the
// tile's bk, Mp and Np multiples of bm and bn; K-blocked by kblock when
// packed_kblock(mode, tile) is nonzero.
struct PackedGemm {
  float* C;
  int64_t ldc;
  const void* Ap;  // parts planes of Mp x Kp (FP8: bytes, then the scale plane)
  const void* Bp;
  int M, N, Kp, Mp, Np;
  rise_mode mode;
  int kblock = 0;
};
int packed_kblock(rise_mode mode, const rise_tile& t);
rise_status launch_packed_gemm(const PackedGemm& g, const rise_tile& t, hipStream_t s);

}  // namespace rise
