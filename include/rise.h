/*
 * rise.h -- C ABI of the MI355X (gfx950) library for the dense data-parallel
 * patterns of RISE ("RISE & Shine: Language-Oriented Compiler Design",
 * arXiv 2201.03611): the matrix product map(map(reduce . zip)) and the 2D
 * stencil pad2D |> slide2D |> weighted reduce.
 *
 * Conventions shared by every entry point
 *  - Outputs come first, then sizes, then inputs, mirroring the generated
 *    kernel signature of the paper (Sec. V, OpenCL listing: restrict output,
 *    sizes, restrict const inputs) and its dependent-function sizes-before-
 *    arrays order (Sec. IV, matrix-vector program).
 *  - The caller owns every buffer.  Array pointers are device pointers unless a
 *    comment says otherwise.  The library allocates no device memory on these
 *    paths; scratch space is passed in (`ws`, `ws_bytes`) and its size comes from
 *    the matching *_workspace query.
 *  - Outputs must not overlap inputs (the kernels' pointers are restrict).
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL is the null
 *    stream).  Inputs must stay valid until the stream reaches the call.
 *  - Nothing is chosen implicitly (Sec. V-B: a program whose memory choice is
 *    missing is rejected, not completed by the compiler): an argument the
 *    library has no kernel for is rejected with a status, and nothing is
 *    enqueued.  rise_last_error() returns a thread-local description.
 *  - Row-major storage everywhere; ld* are leading dimensions in elements.
 *  - Sizes are int64_t; each dimension must be below 2^31.
 */
#ifndef RISE_H
#define RISE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RISE_OK = 0,
  RISE_ERR_NULL = 1,        /* a required pointer is NULL                         */
  RISE_ERR_SHAPE = 2,       /* negative size, ld below the row length, size limit */
  RISE_ERR_ALIAS = 3,       /* an output overlaps an input                        */
  RISE_ERR_DTYPE = 4,       /* element type / mode combination has no kernel      */
  RISE_ERR_UNSUPPORTED = 5, /* even or oversized window, unknown tile or mode     */
  RISE_ERR_WORKSPACE = 6,   /* workspace missing or too small                     */
  RISE_ERR_HIP = 7          /* the HIP runtime reported an error                  */
} rise_status;

/* storage element types of GEMM operands */
typedef enum { RISE_F32 = 0, RISE_BF16 = 1 } rise_dtype;

/* arithmetic of the GEMM contraction (always FP32 accumulation and FP32 C):
 *  F32    : FP32 operands on the FP32 matrix cores
 *  BF16   : operands rounded to bfloat16 (round to nearest even)
 *  BF16X3 : each FP32 operand split a = hi + lo (hi = bf16(a), lo = bf16(a - hi));
 *           C = Ah Bh + Ah Bl + Al Bh
 *  BF16X6 : three-way split a = a1 + a2 + a3; the six products Ai Bj, i + j <= 4
 *  FP8    : OCP E4M3 operands, one power-of-two scale per 32 consecutive K
 *           elements of each row of A and each column of B                     */
typedef enum {
  RISE_MODE_F32 = 0,
  RISE_MODE_BF16 = 1,
  RISE_MODE_BF16X3 = 2,
  RISE_MODE_BF16X6 = 3,
  RISE_MODE_FP8 = 4
} rise_mode;

/* how an operand is read: as stored, or through transpose (a view, no copy) */
typedef enum { RISE_OP_N = 0, RISE_OP_T = 1 } rise_op;

/* boundary of pad2D: replicate the nearest edge element, or the constant 0 */
typedef enum { RISE_PAD_CLAMP = 0, RISE_PAD_ZERO = 1 } rise_pad;

/* An explicit schedule for one GEMM: the tile sizes produced by splitJoinMap
 * on the two maps (bm, bn) and by split on the reduction (bk).  The paper keeps
 * such choices outside the program, supplied by a strategy (Sec. IV-B/C); here
 * the caller passes one or NULL, and NULL takes the tune cache's choice for
 * these sizes and mode (rise_autotune_gemm below) or, without one, the
 * library's default for the mode.  rise_gemm_tiles() lists the supported ones. */
typedef struct {
  int32_t bm, bn, bk;
} rise_tile;

const char* rise_status_string(rise_status s);

/* Thread-local text of the last error raised on this thread ("" if none). */
const char* rise_last_error(void);

/* Number of supported tiles for `mode`; if `out` is non-NULL, up to `cap` of
 * them are written there.  Host-only, enqueues nothing. */
int32_t rise_gemm_tiles(rise_mode mode, rise_tile* out, int32_t cap);

/* The strategy rise_gemm applies when its `tile` argument is NULL: writes to
 * *out the tile the library picks for these sizes and mode -- the tune cache's
 * entry for them on the current device if there is one, else the built-in
 * default (Sec. IV-B/C leave that choice to a strategy outside the program;
 * this reports it).  Host-only, enqueues nothing.  Errors: sizes outside
 * [0, 2^31) (RISE_ERR_SHAPE), an unknown mode (RISE_ERR_UNSUPPORTED), out NULL
 * (RISE_ERR_NULL); *out is then left unchanged. */
rise_status rise_gemm_default_tile(int64_t M, int64_t N, int64_t K, rise_mode mode,
                                   rise_tile* out);

/* ------------------------------------------------------------------------ */
/* GEMM                                                                     */
/* ------------------------------------------------------------------------ */

/* Bytes of workspace rise_gemm needs for these sizes, mode and tile (NULL =
 * the tile rise_gemm_default_tile reports).  0 for RISE_MODE_F32, which reads
 * its operands in place. */
size_t rise_gemm_workspace(int64_t M, int64_t N, int64_t K, rise_mode mode,
                           const rise_tile* tile);

/* C = A . B  (M x N, FP32, leading dimension ldc), with
 *   A: M x K, read from storage of type tA through opA
 *      (RISE_OP_N: stored M x K, element (i,k) at A[i*lda + k];
 *       RISE_OP_T: stored K x M, element (i,k) at A[k*lda + i])
 *   B: K x N, read through opB the same way (RISE_OP_T: stored N x K).
 * Semantics: C = A |> map(aRow => transpose(B) |> map(bCol =>
 *   zip(aRow, bCol) |> map(*) |> reduce(+, 0))), the paper's matrix-vector
 * program (Sec. IV, running example) mapped over the columns of B, evaluated
 * in the arithmetic of `mode`.  K = 0 writes C = 0 (reduce of an empty array is
 * its initial value); M = 0 or N = 0 is a successful no-op.
 * Types: mode F32 needs tA = tB = RISE_F32; BF16 accepts RISE_F32 (rounded)
 * or RISE_BF16 operands; BF16X3, BF16X6 and FP8 need RISE_F32 operands.
 * Workspace: at least rise_gemm_workspace(M, N, K, mode, tile) bytes, 256-byte
 * aligned; it holds the prepared operands and is overwritten. */
rise_status rise_gemm(float* C, int64_t ldc, const void* A, rise_dtype tA, int64_t lda,
                      rise_op opA, const void* B, rise_dtype tB, int64_t ldb, rise_op opB,
                      int64_t M, int64_t N, int64_t K, rise_mode mode, const rise_tile* tile,
                      void* ws, size_t ws_bytes, void* stream);

/* Matrix-vector product, the paper's running example (Sec. IV):
 *   y = A |> map(row => zip(row, x) |> map(*) |> reduce(+, 0))
 * y: M floats (device); A: M x K FP32 read through opA (RISE_OP_N: stored
 * M x K row-major, element (i,k) at A[i*lda + k], the layout of the paper's
 * generated kernel; RISE_OP_T: stored K x M, element (i,k) at A[k*lda + i]);
 * x: K floats.  FP32 arithmetic, the reduction order is the library's (any
 * order is a correct reduce).  K = 0 writes y = 0; M = 0 is a no-op.
 * Workspace: rise_gemv_workspace(M, K, opA) bytes (0 for RISE_OP_N; split-K
 * partials for RISE_OP_T), 256-byte aligned; ws may be NULL when that is 0.
 * Errors: NULL pointers, negative or too large sizes, lda below the stored
 * row length, y overlapping A or x, a short, misaligned or overlapping
 * workspace return a status and enqueue nothing. */
size_t rise_gemv_workspace(int64_t M, int64_t K, rise_op opA);
rise_status rise_gemv(float* y, const float* A, int64_t lda, rise_op opA, const float* x,
                      int64_t M, int64_t K, void* ws, size_t ws_bytes, void* stream);

/* The schedule rise_gemv runs for these sizes: the number of slices the
 * reduction over K is split into (1 = one kernel writes y; more = each slice's
 * partial sums go to the workspace and a second kernel adds them in slice
 * order).  Always 1 for RISE_OP_N.  Host-only; 0 for invalid sizes or opA. */
int32_t rise_gemv_parts(int64_t M, int64_t K, rise_op opA);

/* rise_gemv without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, arithmetic, results and errors as
 * rise_gemv; the split-K partials of RISE_OP_T go to a fixed scratch array of
 * RISE_GEMV_NOALLOC_SCRATCH_BYTES inside the library (one per device, held until
 * the process ends; its device address is looked up on the first call on each
 * device, with that device current).  The stream must belong to the current
 * device.  The library allocates nothing on this path.  A split needing more
 * than the scratch returns RISE_ERR_WORKSPACE and enqueues nothing (the
 * library's splits never do: at most 2046 * 1024 floats).  Every call on one
 * device shares that device's scratch, so calls that overlap in time on one
 * device (different streams, or different threads without ordering) race and
 * may return wrong sums; calls ordered on one stream are safe.  The scratch
 * needs no clearing: every partial a call reads, that call wrote. */
#define RISE_GEMV_NOALLOC_SCRATCH_BYTES ((size_t)8 << 20)
rise_status rise_gemv_noalloc(float* y, const float* A, int64_t lda, rise_op opA, const float* x,
                              int64_t M, int64_t K, void* stream);

/* iterate (Sec. VI) with the tree-reduction body:
 *   out = iterate(n, m, k, split(n) |> map(reduce(+, 0)), in)
 * in: n^k * m floats (device), out: m floats (device).  Each of the k rounds
 * replaces every group of n neighbouring values by their sum, a left fold from
 * 0 in FP32 in index order; the rounds run in exactly that order, so out is
 * bit-identical to a sequential float evaluation of the program (out[j] is the
 * tree sum of in[j*n^k .. (j+1)*n^k)).  k = 0 copies m values; n = 1 adds 0 to
 * every value (k rounds of it equal one); m = 0 is a no-op.
 * Limits: 1 <= n <= 8192 (one group of a round is summed inside one
 * workgroup), k >= 0, n^k * m < 2^40.
 * Workspace: rise_iterate_sum_workspace(n, m, k) bytes, 256-byte aligned (the
 * double buffer between kernel passes; 0 when one pass covers all rounds, and
 * ws may then be NULL).
 * Errors: NULL pointers, sizes outside the limits, out overlapping in, a
 * short, misaligned or overlapping workspace return a status and enqueue
 * nothing. */
size_t rise_iterate_sum_workspace(int64_t n, int64_t m, int64_t k);
rise_status rise_iterate_sum(float* out, const float* in, int64_t n, int64_t m, int64_t k,
                             void* ws, size_t ws_bytes, void* stream);

/* How rise_iterate_sum compiles iterate (Sec. VI) for these sizes: returns the
 * number of kernel passes (each runs several rounds inside LDS; consecutive
 * passes ping-pong through the workspace halves) and writes the rounds of
 * each pass to rounds[0 .. min(passes, cap)) when rounds is non-NULL.  For
 * n > 1 the rounds add up to k; n = 1 runs one round.  Host-only; 0 when the
 * sizes are outside rise_iterate_sum's limits or m = 0. */
int32_t rise_iterate_sum_passes(int64_t n, int64_t m, int64_t k, int32_t* rounds, int32_t cap);

/* Gradients of L(C) with C = A . B (A: M x K, B: K x N, row-major FP32):
 *   dA = dC . transpose(B)   (M x K)     dB = transpose(A) . dC   (K x N)
 * written as two GEMMs that read transpose views of the stored operands (no
 * copies), in the arithmetic of `mode`.  Either of dA, dB may be NULL (skipped).
 * Workspace: rise_gemm_backward_workspace(M, N, K, mode) bytes, 256-byte aligned.
 * The transpose view is the paper-silent primitive read as swapping two
 * dimensions; the gradient of the bilinear map follows from its definition. */
size_t rise_gemm_backward_workspace(int64_t M, int64_t N, int64_t K, rise_mode mode);
rise_status rise_gemm_backward(float* dA, int64_t ldda, float* dB, int64_t lddb, const float* dC,
                               int64_t lddc, const float* A, int64_t lda, const float* B,
                               int64_t ldb, int64_t M, int64_t N, int64_t K, rise_mode mode,
                               void* ws, size_t ws_bytes, void* stream);

/* Operand preparation of a reduced-precision mode (the map(cast) the mode's
 * contraction consumes; map fusion, Sec. IV-B, lets it run as its own pass).
 * The source holds `rows` vectors of length K; element k of vector r is
 * src[r*ld_r + k*ld_k] (A row-major M x K: ld_r = lda, ld_k = 1; B row-major
 * K x N: ld_r = 1, ld_k = ldb).  The destination holds `parts` planes (1 for
 * BF16 and FP8, 2 for BF16X3, 3 for BF16X6), each rows_out x k_out,
 * row-major, rows_out >= rows, k_out >= K; entries beyond (rows, K) are
 * written as zero.  BF16 modes store bfloat16 bit patterns (2 bytes); FP8
 * stores E4M3 bytes, followed by a scale plane of rows_out x (k_out / 32)
 * E8M0 bytes (the dequantisation factor 2^(byte - 127) of each 32-element
 * block; k_out must be a multiple of 32).  Bytes written:
 * rise_prep_bytes(rows_out, k_out, mode). */
size_t rise_prep_bytes(int64_t rows_out, int64_t k_out, rise_mode mode);
rise_status rise_prep_operand(void* out, int64_t rows_out, int64_t k_out, const float* src,
                              int64_t rows, int64_t K, int64_t ld_r, int64_t ld_k,
                              rise_mode mode, void* stream);

/* ------------------------------------------------------------------------ */
/* 2D stencil                                                               */
/* ------------------------------------------------------------------------ */

/* How the stencil is scheduled (the choice the paper leaves to an explicit
 * strategy, Sec. IV-B/C; both schedules compute the same sums in the same order):
 *  RISE_STENCIL_LDS_TILE: each workgroup stages a halo tile of `rows` output
 *    rows x 256 columns in LDS (toMem(Local), Sec. V-B), then each lane reduces
 *    4 adjacent outputs per row from it;
 *  RISE_STENCIL_STREAM: each wavefront walks down a 256-column strip segment of
 *    `rows` output rows, keeps the window rows in registers and receives its
 *    neighbours' columns through wavefront shifts;
 *  RISE_STENCIL_LDS_PIPE: the LDS halo tile of RISE_STENCIL_LDS_TILE, run by a
 *    resident grid (a few workgroups per compute unit) in which each workgroup
 *    walks a fixed list of tiles and fetches tile i+1 into registers while it
 *    reduces tile i from a double-buffered LDS tile, so HBM traffic and the
 *    k*k FMAs overlap inside every workgroup.
 *  RISE_STENCIL_ASYNC: the LDS halo tile filled by asynchronous global -> LDS
 *    copies two tiles ahead through a ring of three LDS tiles (no registers
 *    hold data in flight), on a resident grid; for 16-byte aligned rows with
 *    W % 4 == 0 (other images run RISE_STENCIL_LDS_TILE with 16 rows).
 * rise_stencil_schedules() lists the supported (variant, rows) pairs. */
typedef enum {
  RISE_STENCIL_LDS_TILE = 0,
  RISE_STENCIL_STREAM = 1,
  RISE_STENCIL_LDS_PIPE = 2,
  RISE_STENCIL_ASYNC = 3
} rise_stencil_variant;
typedef struct {
  int32_t variant; /* rise_stencil_variant */
  int32_t rows;
} rise_stencil_schedule;

/* Number of supported schedules; up to `cap` are written to `out` if non-NULL.
 * Host-only. */
int32_t rise_stencil_schedules(rise_stencil_schedule* out, int32_t cap);

/* The schedule rise_stencil2d runs when its `sched` argument is NULL, written
 * to *out (a strategy's choice, Sec. IV-B/C, reported): the tune cache's entry
 * for (H, W, k) on the current device if there is one, else the default.  Windows other than
 * square 1, 3, 5 and 7 run the direct per-output kernel, reported as
 * variant -1, rows 0.  Host-only, enqueues nothing.  Errors: sizes outside
 * [0, 2^31) (RISE_ERR_SHAPE), even or oversized window sides
 * (RISE_ERR_UNSUPPORTED), out NULL (RISE_ERR_NULL). */
rise_status rise_stencil2d_default_schedule(int64_t H, int64_t W, int32_t kh, int32_t kw,
                                            rise_stencil_schedule* out);

/* out = in |> pad2D(pad) |> slide2D(kh x kw, 1)
 *          |> map(map(win => zip(join(win), join(w)) |> map(*) |> reduce(+, 0)))
 * in: H x W FP32 (ld_in), out: H x W FP32 (ld_out), w: kh x kw FP32 weights,
 * row-major, device memory.  Window element (dy, dx) of output (y, x) is
 * input (y + dy - (kh-1)/2, x + dx - (kw-1)/2) (cross-correlation), outside
 * the image either the nearest edge element (clamp) or 0 (zero).  kh and kw
 * must be odd and at most 15; square 1, 3, 5 and 7 windows run the scheduled
 * kernels, other sizes a direct per-output kernel that ignores `sched`.
 * sched = NULL takes the library default.  H = 0 or W = 0 is a no-op. */
rise_status rise_stencil2d(float* out, int64_t ld_out, const float* in, int64_t ld_in,
                           int64_t H, int64_t W, const float* w, int32_t kh, int32_t kw,
                           rise_pad pad, const rise_stencil_schedule* sched, void* stream);


/* iterate (Sec. VI) with the stencil as a size-preserving body:
 *   out = in |> stencil |> stencil |> ... (`steps` times)
 * each application being rise_stencil2d(w, kh, kw, pad) of the previous image
 * (steps = 0 copies in to out).  in, out: H x W FP32 (ld_in, ld_out), w as for
 * rise_stencil2d; out must not overlap in.
 * fuse selects the schedule, the number of steps one kernel launch runs:
 *   1  one stencil launch per step through a double buffer of two H x W images
 *      in the workspace (the paper's translation of iterate);
 *   2 .. rise_stencil2d_iterate_max_fuse(): that many steps per launch, kept
 *      in an LDS double buffer with a halo of fuse*(k-1)/2 (square 3x3 and
 *      5x5 windows only; others return RISE_ERR_UNSUPPORTED);
 *   0  the library default: 4 for 3x3 windows, 1 otherwise (for 5x5 the
 *      fused steps are bound by the FMA rate and measured slower than one
 *      HBM-bound launch per step).
 * The last launch runs the remaining steps.  All schedules give identical
 * results (each output is the same FP32 sum in the same order).
 * Workspace: rise_stencil2d_iterate_workspace(H, W, kh, kw, steps, fuse) bytes,
 * 256-byte aligned (0, one or two dense H x W images).  Errors as for
 * rise_stencil2d, plus steps < 0, an unknown fuse, and a short, misaligned or
 * overlapping workspace. */
int32_t rise_stencil2d_iterate_max_fuse(void);
/* The steps per launch that fuse = 0 selects for this window (host-only). */
int32_t rise_stencil2d_iterate_default_fuse(int32_t kh, int32_t kw);
size_t rise_stencil2d_iterate_workspace(int64_t H, int64_t W, int32_t kh, int32_t kw,
                                        int64_t steps, int32_t fuse);
rise_status rise_stencil2d_iterate(float* out, int64_t ld_out, const float* in, int64_t ld_in,
                                   int64_t H, int64_t W, const float* w, int32_t kh, int32_t kw,
                                   rise_pad pad, int64_t steps, int32_t fuse, void* ws,
                                   size_t ws_bytes, void* stream);

/* Gradients of L(out) with out = rise_stencil2d(in, w) (same sizes, window and
 * padding), given dOut (H x W):
 *   dIn = S^T dOut, the adjoint of pad2D |> slide2D |> weighted reduce: with
 *         zero padding the stencil of dOut with the 180-degree rotated window,
 *         with clamp padding the same plus, on the first/last row and column,
 *         every contribution the clamp mapped onto them;
 *   dW[dy][dx] = sum over (y, x) of dOut[y][x] * window(y, x)[dy][dx].
 * Either dIn or dW may be NULL (skipped); `in` is read only for dW and `w`
 * only for dIn.  FP32, row-major, device memory.  Workspace:
 * rise_stencil2d_backward_workspace(H, W, kh, kw) bytes, 256-byte aligned
 * (rotated window and per-strip partial sums; dW is reduced in a fixed order,
 * so results are deterministic). */
size_t rise_stencil2d_backward_workspace(int64_t H, int64_t W, int32_t kh, int32_t kw);
rise_status rise_stencil2d_backward(float* dIn, int64_t ld_din, float* dW, const float* dOut,
                                    int64_t ld_dout, const float* in, int64_t ld_in, int64_t H,
                                    int64_t W, const float* w, int32_t kh, int32_t kw,
                                    rise_pad pad, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Multi-channel stencil layer (convolution layer), NHWC bfloat16           */
/* ------------------------------------------------------------------------ */

/* out[b][y][x][co] = reduce(+, 0) over ci of
 *     stencil(pad2D(in[b][.][.][ci]), w[co][ci])
 * i.e. the 2D stencil above (cross-correlation order) summed over input
 * channels (the multi-channel reading of the stencil pattern; the paper defines
 * no convolution layer).  in: B x H x W x Cin and out: B x H x W x Cout are
 * bfloat16 bit patterns (NHWC, 16-byte aligned); w: Cout x Cin x kh x kw FP32,
 * rounded to bfloat16 (nearest even) for the matrix cores; FP32 accumulation,
 * output rounded to bfloat16.  Supported: kh = kw = 3, Cin in {16, 32, 64},
 * Cout in {32, 64}; other shapes return RISE_ERR_UNSUPPORTED.  Workspace:
 * rise_conv2d_workspace(Cin, Cout) bytes (the prepared weights). */
size_t rise_conv2d_workspace(int32_t Cin, int32_t Cout);
rise_status rise_conv2d(uint16_t* out, const uint16_t* in, const float* w, int32_t B, int32_t Cin,
                        int32_t Cout, int32_t H, int32_t W, int32_t kh, int32_t kw, rise_pad pad,
                        void* ws, size_t ws_bytes, void* stream);

/* Gradients of L(out), out = rise_conv2d(in, w), given dOut (B x H x W x Cout,
 * bfloat16 NHWC):
 *   dIn (B x H x W x Cin, bfloat16) = the layer applied to dOut with the channel
 *       roles swapped and the window rotated by 180 degrees (the adjoint of zero
 *       padding; clamp padding is rejected when dIn is requested);
 *   dW  (Cout x Cin x 3 x 3, FP32) = sum over (b, y, x) of
 *       dOut[b][y][x][co] * window_ci(b, y, x)[dy][dx], reduced in a fixed order.
 * Either output may be NULL.  Supported: Cin and Cout in {32, 64}, kh = kw = 3.
 * Workspace: rise_conv2d_backward_workspace(B, Cin, Cout, H, W) bytes. */
size_t rise_conv2d_backward_workspace(int32_t B, int32_t Cin, int32_t Cout, int32_t H, int32_t W);
rise_status rise_conv2d_backward(uint16_t* dIn, float* dW, const uint16_t* dOut,
                                 const uint16_t* in, const float* w, int32_t B, int32_t Cin,
                                 int32_t Cout, int32_t H, int32_t W, int32_t kh, int32_t kw,
                                 rise_pad pad, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Autotuning: the strategy search (Sec. IV-B/C keep tile sizes and the      */
/* mapping of maps onto the hardware outside the program, as an explicit    */
/* strategy that a user or a search supplies)                               */
/* ------------------------------------------------------------------------ */

/* Time every supported tile of `mode` (rise_gemm_tiles) on an M x N x K product
 * of row-major FP32 operands (opA = opB = RISE_OP_N) on the current device and
 * record the fastest in the text cache file `cache_path`, keyed by (M, N, K,
 * mode, GPU architecture name such as "gfx950"); an entry of the same key is
 * replaced, other entries are kept.  Allocates (and frees) device memory for
 * the operands and the workspace and synchronises `stream`: not for the hot
 * path.  Errors: cache_path NULL (RISE_ERR_NULL), sizes outside [1, 2^31) or
 * operands above 16 GiB (RISE_ERR_SHAPE), an unknown mode or an unwritable
 * file (RISE_ERR_UNSUPPORTED), no device or a HIP failure (RISE_ERR_HIP). */
rise_status rise_autotune_gemm(const char* cache_path, int64_t M, int64_t N, int64_t K,
                               rise_mode mode, void* stream);

/* The same for the stencil: times every schedule of rise_stencil_schedules()
 * on an H x W FP32 image with a k x k window (k in {1, 3, 5, 7}, clamp
 * padding) and records the fastest under (H, W, k, architecture).  Errors as
 * for rise_autotune_gemm (another k: RISE_ERR_UNSUPPORTED). */
rise_status rise_autotune_stencil(const char* cache_path, int64_t H, int64_t W, int32_t k,
                                  void* stream);

/* The cache file that tile = NULL / sched = NULL consult (rise_gemm,
 * rise_gemm_workspace, rise_gemm_default_tile, rise_gemm_backward,
 * rise_stencil2d, rise_stencil2d_default_schedule).  The file is read now and
 * again after each autotune call that writes it; NULL or "" disables the
 * cache.  Until this is called the library uses the file named by the
 * RISE_TUNE_CACHE environment variable, if set.  A missing file is an empty
 * cache.  Process-wide; the file format is one line per entry:
 *   gemm <arch> <M> <N> <K> <mode> <bm> <bn> <bk> <microseconds>
 *   stencil <arch> <H> <W> <k> <variant> <rows> <microseconds>
 * Changing the cache between a workspace query and the call can change the
 * tile and so the workspace needed; rise_gemm then fails with
 * RISE_ERR_WORKSPACE rather than overrun. */
rise_status rise_set_tune_cache(const char* path);

/* ------------------------------------------------------------------------ */
/* Measured ceilings (the denominators of the roofline fractions beside the  */
/* spec-sheet peaks; they compute nothing of the patterns)                   */
/* ------------------------------------------------------------------------ */

/* A streaming device copy of `bytes` (a multiple of 16; 16-byte aligned,
 * non-overlapping device buffers): one 16-byte load and store per thread,
 * workgroup b copying the 4 KB block b in one pass.  Timed over >= 2 GiB it
 * gives the HBM bandwidth a kernel can reach (read + write bytes / time). */
rise_status rise_ceiling_copy(void* dst, const void* src, size_t bytes, void* stream);

/* Back-to-back matrix instructions on every SIMD (four waves per SIMD, four
 * independent accumulators per wave), `iters` rounds: mode RISE_MODE_F32 runs
 * v_mfma_f32_32x32x2_f32, RISE_MODE_BF16 v_mfma_f32_32x32x16_bf16, RISE_MODE_FP8
 * the scaled v_mfma_scale_f32_32x32x64_f8f6f4.  *flops receives the flops the
 * launch issues (host value, set before the call returns); timing the launch
 * gives the matrix-core rate.  sink: device floats, at least
 * rise_ceiling_mfma_sink_floats() of them (one value per lane is written so
 * the loop is not removed).  Errors: NULL pointers, iters outside [1, 2^32],
 * a short sink, another mode. */
size_t rise_ceiling_mfma_sink_floats(void);
rise_status rise_ceiling_mfma(rise_mode mode, int64_t iters, float* sink, size_t sink_floats,
                              double* flops, void* stream);

/* ------------------------------------------------------------------------ */
/* Batched form: many problems, one persistent launch                        */
/* ------------------------------------------------------------------------ */

/* One GEMM of a batch: C (M x N, FP32, ldc) = A (M x K, row-major, lda) . B,
 * B stored K x N (opB = RISE_OP_N) or N x K (RISE_OP_T), ldb; A and B of type
 * dtype (RISE_F32, or RISE_BF16 with FP32 accumulation).  Batched operands must
 * be 16-byte aligned with lda, ldb multiples of 16 bytes; bf16 also needs K (and
 * N when opB = RISE_OP_N) multiples of 8. */
typedef struct {
  float* C;
  const void* A;
  const void* B;
  int64_t M, N, K, lda, ldb, ldc;
  int32_t dtype; /* rise_dtype */
  int32_t opB;   /* rise_op */
} rise_gemm_problem;

/* One stencil of a batch: as rise_stencil2d with a square window of side k in
 * {1, 3, 5, 7} (16-byte vector loads when both images are 16-byte aligned with
 * ld_in, ld_out multiples of 4, scalar loads otherwise). */
typedef struct {
  float* out;
  const float* in;
  const float* w;
  int64_t H, W, ld_in, ld_out;
  int32_t k;
  int32_t pad; /* rise_pad */
} rise_stencil_problem;

/* A plan owns the device copy of the problem descriptors, the work-item list
 * (every output tile of every problem, GEMM tiles largest estimated cost first)
 * and a HIP graph of  [reset the work counter] -> [one persistent GEMM kernel,
 * whose workgroups take tiles from the counter until none are left] -> [one
 * stencil kernel per window side and load width, one workgroup per tile].
 * Launches of one plan share its work counter, so they must not overlap:
 * issue them on one stream, or order them with events.  The batch is the
 * outer map of the patterns: its items write distinct outputs, so any order
 * is correct (distinct output acceptors, paper Sec. V-C).  GEMM tile shapes
 * come from a per-tile cost table (tune_table: a file written by
 * rise_autotune_batched, or NULL for the built-in MI355X table).  plan_create
 * allocates device memory and synchronises; it is not meant for the hot path.
 * The problems' buffers must stay valid for every launch of the plan. */
typedef struct rise_plan rise_plan;
rise_status rise_plan_create(rise_plan** plan, const rise_gemm_problem* gemms, int32_t n_gemm,
                             const rise_stencil_problem* stencils, int32_t n_stencil,
                             const char* tune_table, void* stream);
/* One launch of the captured graph on `stream`. */
rise_status rise_plan_launch(rise_plan* plan, void* stream);
/* The same kernels launched directly (no graph), for comparison. */
rise_status rise_plan_launch_direct(rise_plan* plan, void* stream);
rise_status rise_plan_destroy(rise_plan* plan);
/* Number of work items; the tile (bm, bn, bk) chosen for GEMM `problem`. */
int32_t rise_plan_items(const rise_plan* plan);
rise_status rise_plan_tile(const rise_plan* plan, int32_t problem, rise_tile* tile);

/* Create a plan, launch it once, wait for `stream`, destroy the plan. */
rise_status rise_gemm_batched(const rise_gemm_problem* gemms, int32_t n, void* stream);
rise_status rise_stencil2d_batched(const rise_stencil_problem* stencils, int32_t n,
                                   void* stream);

/* Measure the per-tile cost of every tile kind of the persistent kernel on the
 * current device (a + b * K microseconds per GEMM tile, a per stencil tile) and
 * write the table to `table_path` (text, one "name a b" line per kind).  Uses
 * about 400 MB of temporary device memory; synchronises. */
rise_status rise_autotune_batched(const char* table_path, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RISE_H */
