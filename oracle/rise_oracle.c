/*
 * rise_oracle.c -- the oracle: a plain, slow, CPU-only interpreter of the RISE
 * pattern semantics that the dense GEMM and 2D-stencil kernels implement.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The GPU library shares
 * no source, header, table or helper with it, and neither links the other.
 *
 * What it computes (paper: "RISE & Shine", arXiv 2201.03611):
 *   - map, reduce, zip: the data-parallel primitives of Sec. IV-A (listing of
 *     RISE primitives).  reduce is evaluated as reduceSeq, i.e. a left fold
 *     from index 0 into an accumulator initialised with init (the continuation
 *     translation of reduceSeq in Sec. V-C).
 *   - split, join, idx: the DPIA functional primitives of Sec. V-A.  They are
 *     index remappings ("views", Sec. V-C), never materialised here.
 *   - transpose, slide, pad (clamp or zero): not defined in the paper; they get
 *     their standard readings (transpose swaps two dimensions; slide(sz, sp)
 *     gives windows of sz elements starting every sp; pad repeats the edge
 *     element (clamp) or adds zeros) and are also pure index views.
 *   - GEMM is the paper's matrix-vector program (Sec. IV, running example)
 *     mapped over the columns of B:
 *       C = A |> map(aRow => transpose(B) |> map(bCol =>
 *                 zip(aRow, bCol) |> map(*) |> reduce(+, 0)))
 *   - the 2D stencil is pad2D |> slide2D(k, 1) |> map(map(weighted reduce)).
 *   - gradients are the adjoints of these bilinear maps, written from their
 *     definitions (scatter through the same views; reduce over outputs).
 *   - iterate (Sec. VI) with the tree-reduction body split(n) |> map(reduce(+, 0)):
 *     k applications, each one turning an array of l*n values into l sums of n
 *     neighbours, passed between two temporaries as newDoubleBuffer does.
 *   - operand preparation of the reduced-precision GEMM modes (bf16 rounding,
 *     hi/lo splitting, FP8 E4M3 with power-of-two block scales) written from
 *     the number formats' definitions in exact arithmetic.
 *
 * Arithmetic: every value is widened to double (exact for f32, bf16 and fp8
 * inputs); products of two f32 values are exact in double; sums are left folds
 * in double.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------- */
/* status codes (mirrored by oracle/__init__.py)                          */
/* ---------------------------------------------------------------------- */
enum {
  OR_OK = 0,
  OR_ERR_SHAPE = 1,     /* a type-level size equality does not hold        */
  OR_ERR_ARG = 2,       /* an argument is outside what the definition covers */
  OR_ERR_RANK = 3       /* a view would exceed the supported rank          */
};

/* element encodings of leaf arrays */
enum { EL_F32 = 0, EL_F64 = 1, EL_BF16 = 2 };

/* padding modes */
enum { PAD_CLAMP = 0, PAD_ZERO = 1 };

/* ---------------------------------------------------------------------- */
/* views: an array is a shape plus an index function                      */
/* ---------------------------------------------------------------------- */
#define RMAX 6

enum { OP_LEAF, OP_IDX, OP_SPLIT, OP_JOIN, OP_TRANSPOSE, OP_SLIDE, OP_PAD };

typedef struct view view;
struct view {
  int op;
  int rank;
  int64_t shape[RMAX];
  /* leaf */
  const void* data;
  int elem;
  int64_t stride[RMAX];
  /* derived: `op` applied at dimension `axis` of `inner` */
  const view* inner;
  int axis;
  int64_t p, q;   /* op parameters (see the constructors) */
  int mode;       /* pad mode */
  int bad;        /* set when the construction violated the op's type */
};

static double bf16_bits_to_double(uint16_t b) {
  uint32_t u = ((uint32_t)b) << 16;
  float f;
  memcpy(&f, &u, 4);
  return (double)f;
}

static double leaf_read(const view* v, int64_t off) {
  switch (v->elem) {
    case EL_F32: return (double)((const float*)v->data)[off];
    case EL_F64: return ((const double*)v->data)[off];
    default: return bf16_bits_to_double(((const uint16_t*)v->data)[off]);
  }
}

static view v_leaf(const void* data, int elem, int rank, const int64_t* shape,
                   const int64_t* stride) {
  view v;
  memset(&v, 0, sizeof v);
  v.op = OP_LEAF;
  v.rank = rank;
  v.data = data;
  v.elem = elem;
  for (int d = 0; d < rank; d++) {
    v.shape[d] = shape[d];
    v.stride[d] = stride[d];
  }
  return v;
}

static view v_derived(const view* in, int op, int axis) {
  view v;
  memset(&v, 0, sizeof v);
  v.op = op;
  v.inner = in;
  v.axis = axis;
  v.bad = in->bad || axis < 0 || axis >= in->rank;
  return v;
}

/* idx(i, xs) at dimension axis: removes that dimension. */
static view v_idx(const view* in, int axis, int64_t i) {
  view v = v_derived(in, OP_IDX, axis);
  if (v.bad) return v;
  v.p = i;
  v.rank = in->rank - 1;
  if (i < 0 || i >= in->shape[axis]) v.bad = 1;
  for (int d = 0, s = 0; d < in->rank; d++)
    if (d != axis) v.shape[s++] = in->shape[d];
  return v;
}

/* split(n): Array[n*m, t] -> Array[m, Array[n, t]] at dimension axis. */
static view v_split(const view* in, int axis, int64_t n) {
  view v = v_derived(in, OP_SPLIT, axis);
  if (v.bad) return v;
  if (in->rank + 1 > RMAX || n <= 0 || in->shape[axis] % n != 0) {
    v.bad = 1;
    return v;
  }
  v.p = n;
  v.rank = in->rank + 1;
  for (int d = 0; d < axis; d++) v.shape[d] = in->shape[d];
  v.shape[axis] = in->shape[axis] / n;
  v.shape[axis + 1] = n;
  for (int d = axis + 1; d < in->rank; d++) v.shape[d + 1] = in->shape[d];
  return v;
}

/* join: Array[n, Array[m, t]] -> Array[n*m, t] at dimensions (axis, axis+1). */
static view v_join(const view* in, int axis) {
  view v = v_derived(in, OP_JOIN, axis);
  if (v.bad) return v;
  if (axis + 1 >= in->rank) {
    v.bad = 1;
    return v;
  }
  v.p = in->shape[axis + 1];
  v.rank = in->rank - 1;
  for (int d = 0; d < axis; d++) v.shape[d] = in->shape[d];
  v.shape[axis] = in->shape[axis] * in->shape[axis + 1];
  for (int d = axis + 2; d < in->rank; d++) v.shape[d - 1] = in->shape[d];
  return v;
}

/* transpose: swaps dimensions axis and axis+1. */
static view v_transpose(const view* in, int axis) {
  view v = v_derived(in, OP_TRANSPOSE, axis);
  if (v.bad) return v;
  if (axis + 1 >= in->rank) {
    v.bad = 1;
    return v;
  }
  v.rank = in->rank;
  for (int d = 0; d < in->rank; d++) v.shape[d] = in->shape[d];
  v.shape[axis] = in->shape[axis + 1];
  v.shape[axis + 1] = in->shape[axis];
  return v;
}

/* slide(sz, sp): Array[N, t] -> Array[(N - sz)/sp + 1, Array[sz, t]],
 * window w holds elements w*sp .. w*sp + sz - 1. */
static view v_slide(const view* in, int axis, int64_t sz, int64_t sp) {
  view v = v_derived(in, OP_SLIDE, axis);
  if (v.bad) return v;
  int64_t N = in->shape[axis];
  if (in->rank + 1 > RMAX || sz <= 0 || sp <= 0 || N < sz || (N - sz) % sp != 0) {
    v.bad = 1;
    return v;
  }
  v.p = sz;
  v.q = sp;
  v.rank = in->rank + 1;
  for (int d = 0; d < axis; d++) v.shape[d] = in->shape[d];
  v.shape[axis] = (N - sz) / sp + 1;
  v.shape[axis + 1] = sz;
  for (int d = axis + 1; d < in->rank; d++) v.shape[d + 1] = in->shape[d];
  return v;
}

/* pad(l, r): Array[N, t] -> Array[l + N + r, t]; element i reads i - l inside,
 * outside it reads the nearest edge element (clamp) or the constant 0 (zero). */
static view v_pad(const view* in, int axis, int64_t l, int64_t r, int mode) {
  view v = v_derived(in, OP_PAD, axis);
  if (v.bad) return v;
  if (l < 0 || r < 0 || (mode != PAD_CLAMP && mode != PAD_ZERO) ||
      (mode == PAD_CLAMP && in->shape[axis] == 0)) {
    v.bad = 1;
    return v;
  }
  v.p = l;
  v.q = r;
  v.mode = mode;
  v.rank = in->rank;
  for (int d = 0; d < in->rank; d++) v.shape[d] = in->shape[d];
  v.shape[axis] = l + in->shape[axis] + r;
  return v;
}

/* Translate an index of v into an index of v->inner.  Returns 0 when the
 * element is a zero-padding element (it has no source). */
static int step_index(const view* v, const int64_t* idx, int64_t* t) {
  const view* in = v->inner;
  int a = v->axis;
  switch (v->op) {
    case OP_IDX:
      for (int d = 0, s = 0; d < in->rank; d++) t[d] = (d == a) ? v->p : idx[s++];
      return 1;
    case OP_SPLIT:
      for (int d = 0; d < a; d++) t[d] = idx[d];
      t[a] = idx[a] * v->p + idx[a + 1];
      for (int d = a + 1; d < in->rank; d++) t[d] = idx[d + 1];
      return 1;
    case OP_JOIN:
      for (int d = 0; d < a; d++) t[d] = idx[d];
      t[a] = idx[a] / v->p;
      t[a + 1] = idx[a] % v->p;
      for (int d = a + 2; d < in->rank; d++) t[d] = idx[d - 1];
      return 1;
    case OP_TRANSPOSE:
      for (int d = 0; d < in->rank; d++) t[d] = idx[d];
      t[a] = idx[a + 1];
      t[a + 1] = idx[a];
      return 1;
    case OP_SLIDE:
      for (int d = 0; d < a; d++) t[d] = idx[d];
      t[a] = idx[a] * v->q + idx[a + 1];
      for (int d = a + 1; d < in->rank; d++) t[d] = idx[d + 1];
      return 1;
    case OP_PAD: {
      for (int d = 0; d < in->rank; d++) t[d] = idx[d];
      int64_t i = idx[a] - v->p, n = in->shape[a];
      if (i < 0 || i >= n) {
        if (v->mode == PAD_ZERO) return 0;
        i = i < 0 ? 0 : n - 1;
      }
      t[a] = i;
      return 1;
    }
    default:
      return 0;
  }
}

/* Offset of the leaf element an index of v reads, or -1 for a zero-pad element. */
static int64_t view_source(const view* v, const int64_t* idx) {
  int64_t buf[2][RMAX];
  const int64_t* cur = idx;
  int which = 0;
  while (v->op != OP_LEAF) {
    if (!step_index(v, cur, buf[which])) return -1;
    cur = buf[which];
    which ^= 1;
    v = v->inner;
  }
  int64_t off = 0;
  for (int d = 0; d < v->rank; d++) off += cur[d] * v->stride[d];
  return off;
}

static const view* view_leaf(const view* v) {
  while (v->op != OP_LEAF) v = v->inner;
  return v;
}

static double view_at(const view* v, const int64_t* idx) {
  int64_t off = view_source(v, idx);
  return off < 0 ? 0.0 : leaf_read(view_leaf(v), off);
}

/* ---------------------------------------------------------------------- */
/* expressions                                                            */
/* ---------------------------------------------------------------------- */

/* zip(a, b) |> map(fst * snd) |> reduce(+, init): a left fold from index 0
 * (reduceSeq).  zip requires equal lengths; callers check that. */
static double zip_mul_reduce(const view* a, const view* b, double init) {
  double acc = init;
  for (int64_t i = 0; i < a->shape[0]; i++) acc = acc + view_at(a, &i) * view_at(b, &i);
  return acc;
}

static int oracle_threads_used = 1;

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int oracle_last_threads(void) { return oracle_threads_used; }

/* Threads for the following calls (n >= 1); returns the previous setting. */
int oracle_set_threads(int n) {
#ifdef _OPENMP
  int prev = omp_get_max_threads();
  if (n >= 1) omp_set_num_threads(n);
  return prev;
#else
  (void)n;
  return 1;
#endif
}

static void note_threads(void) {
#ifdef _OPENMP
#pragma omp parallel
  {
#pragma omp single
    oracle_threads_used = omp_get_num_threads();
  }
#else
  oracle_threads_used = 1;
#endif
}

/* A stored matrix seen as its logical M x K (or K x N) array: op 0 reads it as
 * stored (rows x cols, row-major with leading dimension ld), op 1 reads the
 * stored cols x rows array through transpose. */
static view stored_matrix(const void* p, int elem, int64_t rows, int64_t cols, int64_t ld,
                          int op, view* storage) {
  int64_t shape[2], stride[2] = {ld, 1};
  if (op == 0) {
    shape[0] = rows;
    shape[1] = cols;
    *storage = v_leaf(p, elem, 2, shape, stride);
    return *storage;
  }
  shape[0] = cols;
  shape[1] = rows;
  *storage = v_leaf(p, elem, 2, shape, stride);
  return v_transpose(storage, 0);
}

/* ---------------------------------------------------------------------- */
/* GEMM                                                                   */
/* ---------------------------------------------------------------------- */

/* C[i][j] (row-major, leading dimension ldc) for A: M x K, B: K x N, each read
 * through op (0 = as stored, 1 = transpose of the stored array).
 *   C = A |> map(aRow => transpose(B) |> map(bCol =>
 *         zip(aRow, bCol) |> map(*) |> reduce(+, 0)))
 * K = 0 gives C = 0 (reduce of an empty array is its init). */
int oracle_gemm(double* C, int64_t ldc, const void* A, int elemA, int64_t lda, int opA,
                const void* B, int elemB, int64_t ldb, int opB, int64_t M, int64_t N,
                int64_t K) {
  if (M < 0 || N < 0 || K < 0 || ldc < N) return OR_ERR_ARG;
  view As, Bs;
  view Av = stored_matrix(A, elemA, M, K, lda, opA, &As);
  view Bv = stored_matrix(B, elemB, K, N, ldb, opB, &Bs);
  view Bt = v_transpose(&Bv, 0); /* columns of B are the rows of transpose(B) */
  if (Av.bad || Bt.bad) return OR_ERR_SHAPE;
  note_threads();
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < M; i++) {
    view aRow = v_idx(&Av, 0, i);
    for (int64_t j = 0; j < N; j++) {
      view bCol = v_idx(&Bt, 0, j);
      C[i * ldc + j] = zip_mul_reduce(&aRow, &bCol, 0.0);
    }
  }
  return OR_OK;
}

/* The same definition evaluated only at the listed (rows[s], cols[s]). */
int oracle_gemm_sampled(double* out, const int64_t* rows, const int64_t* cols, int64_t count,
                        const void* A, int elemA, int64_t lda, int opA, const void* B,
                        int elemB, int64_t ldb, int opB, int64_t M, int64_t N, int64_t K) {
  view As, Bs;
  view Av = stored_matrix(A, elemA, M, K, lda, opA, &As);
  view Bv = stored_matrix(B, elemB, K, N, ldb, opB, &Bs);
  view Bt = v_transpose(&Bv, 0);
  if (Av.bad || Bt.bad) return OR_ERR_SHAPE;
  for (int64_t s = 0; s < count; s++)
    if (rows[s] < 0 || rows[s] >= M || cols[s] < 0 || cols[s] >= N) return OR_ERR_ARG;
  note_threads();
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t s = 0; s < count; s++) {
    view aRow = v_idx(&Av, 0, rows[s]);
    view bCol = v_idx(&Bt, 0, cols[s]);
    out[s] = zip_mul_reduce(&aRow, &bCol, 0.0);
  }
  return OR_OK;
}

/* The tiled form reached by splitJoinMap on both maps and split on the
 * reduction (Sec. IV-B rewrite rules):
 *   A |> split(mt) |> map(aT => transpose(B) |> split(nt) |> map(bT =>
 *     zip(aT |> map(split(kt)) |> transpose, bT |> map(split(kt)) |> transpose)
 *       |> reduceSeq((acc, (aK, bK)) => acc + aK . transpose(bK), 0)))
 *   |> join the tile grid back into M x N.
 * Requires mt | M, nt | N, kt | K (split's type).  Used to check the law that
 * the tiled and untiled programs agree. */
int oracle_gemm_tiled(double* C, int64_t ldc, const void* A, int elemA, int64_t lda, int opA,
                      const void* B, int elemB, int64_t ldb, int opB, int64_t M, int64_t N,
                      int64_t K, int64_t mt, int64_t nt, int64_t kt) {
  if (mt <= 0 || nt <= 0 || kt <= 0) return OR_ERR_ARG;
  view As, Bs;
  view Av = stored_matrix(A, elemA, M, K, lda, opA, &As);
  view Bv = stored_matrix(B, elemB, K, N, ldb, opB, &Bs);
  view Bt = v_transpose(&Bv, 0);
  view Atiles = v_split(&Av, 0, mt);  /* (M/mt, mt, K) */
  view Btiles = v_split(&Bt, 0, nt);  /* (N/nt, nt, K) */
  if (Atiles.bad || Btiles.bad || K % kt != 0) return OR_ERR_SHAPE;
  int64_t tm = M / mt, tn = N / nt;
  note_threads();
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
  for (int64_t ti = 0; ti < tm; ti++) {
    for (int64_t tj = 0; tj < tn; tj++) {
      view aT = v_idx(&Atiles, 0, ti);        /* (mt, K) */
      view bT = v_idx(&Btiles, 0, tj);        /* (nt, K) */
      view aS = v_split(&aT, 1, kt);          /* (mt, K/kt, kt) */
      view bS = v_split(&bT, 1, kt);          /* (nt, K/kt, kt) */
      view aK = v_transpose(&aS, 0);          /* (K/kt, mt, kt) */
      view bK = v_transpose(&bS, 0);          /* (K/kt, nt, kt) */
      double* acc = (double*)calloc((size_t)(mt * nt), sizeof(double));
      for (int64_t s = 0; s < K / kt; s++) {  /* reduceSeq over k-tiles */
        view a_s = v_idx(&aK, 0, s);          /* (mt, kt) */
        view b_s = v_idx(&bK, 0, s);          /* (nt, kt) */
        for (int64_t i = 0; i < mt; i++) {
          view ar = v_idx(&a_s, 0, i);
          for (int64_t j = 0; j < nt; j++) {
            view br = v_idx(&b_s, 0, j);
            acc[i * nt + j] = zip_mul_reduce(&ar, &br, acc[i * nt + j]);
          }
        }
      }
      /* join . join: tile (ti, tj), element (i, j) lands at (ti*mt + i, tj*nt + j) */
      for (int64_t i = 0; i < mt; i++)
        for (int64_t j = 0; j < nt; j++) C[(ti * mt + i) * ldc + tj * nt + j] = acc[i * nt + j];
      free(acc);
    }
  }
  return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* 2D stencil                                                             */
/* ---------------------------------------------------------------------- */

/* The windows of an image plane: pad2D(r) |> slide2D(k, 1), shape (H, W, kh, kw).
 *   pad2D     = map(pad(rw, rw)) |> pad(rh, rh)
 *   slide2D   = map(slide(kw, 1)) |> slide(kh, 1) |> map(transpose)
 * `chain` must hold 5 views; the last one is returned. */
static const view* stencil_windows(const view* plane, int kh, int kw, int mode, view* chain) {
  int64_t rh = (kh - 1) / 2, rw = (kw - 1) / 2;
  chain[0] = v_pad(plane, 1, rw, rw, mode);      /* map(pad)            */
  chain[1] = v_pad(&chain[0], 0, rh, rh, mode);  /* pad                 */
  chain[2] = v_slide(&chain[1], 1, kw, 1);       /* map(slide): (H+2rh, W, kw) */
  chain[3] = v_slide(&chain[2], 0, kh, 1);       /* slide: (H, kh, W, kw)      */
  chain[4] = v_transpose(&chain[3], 1);          /* map(transpose): (H, W, kh, kw) */
  return &chain[4];
}

static int check_kernel(int kh, int kw, int mode) {
  if (kh <= 0 || kw <= 0 || kh % 2 == 0 || kw % 2 == 0) return OR_ERR_ARG;
  if (mode != PAD_CLAMP && mode != PAD_ZERO) return OR_ERR_ARG;
  return OR_OK;
}

/* out (H x W, row-major) = in |> pad2D |> slide2D(k, 1)
 *     |> map(map(win => zip(join(win), join(w)) |> map(*) |> reduce(+, 0)))
 * Cross-correlation order: window element (dy, dx) meets weight w[dy][dx]. */
int oracle_stencil2d(double* out, const void* in, int elem, int64_t ld_in, int64_t H, int64_t W,
                     const float* w, int kh, int kw, int mode) {
  int rc = check_kernel(kh, kw, mode);
  if (rc) return rc;
  if (H < 0 || W < 0 || ld_in < W) return OR_ERR_ARG;
  if (H == 0 || W == 0) return OR_OK;
  int64_t shape[2] = {H, W}, stride[2] = {ld_in, 1};
  view img = v_leaf(in, elem, 2, shape, stride);
  view chain[5];
  const view* win = stencil_windows(&img, kh, kw, mode, chain);
  int64_t wshape[2] = {kh, kw}, wstride[2] = {kw, 1};
  view wv = v_leaf(w, EL_F32, 2, wshape, wstride);
  view wj = v_join(&wv, 0);
  if (win->bad || wj.bad) return OR_ERR_SHAPE;
  note_threads();
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t y = 0; y < H; y++) {
    view row = v_idx(win, 0, y);
    for (int64_t x = 0; x < W; x++) {
      view wnd = v_idx(&row, 0, x);  /* (kh, kw) */
      view wndj = v_join(&wnd, 0);   /* (kh*kw)  */
      out[y * W + x] = zip_mul_reduce(&wndj, &wj, 0.0);
    }
  }
  return OR_OK;
}

/* Gradients of L = <G, stencil(in, w)> with G = dOut (H x W):
 *   dIn[p]  = sum over (y, x, dy, dx) whose window element reads leaf p of
 *             w[dy][dx] * dOut[y][x]   (the adjoint of pad2D |> slide2D)
 *   dW[dy][dx] = sum over (y, x) of dOut[y][x] * window(y, x)[dy][dx]
 * dIn has the layout of in (leading dimension ld_in); either output may be NULL. */
int oracle_stencil2d_backward(double* dIn, double* dW, const float* dOut, const void* in,
                              int elem, int64_t ld_in, int64_t H, int64_t W, const float* w,
                              int kh, int kw, int mode) {
  int rc = check_kernel(kh, kw, mode);
  if (rc) return rc;
  if (H < 0 || W < 0 || ld_in < W) return OR_ERR_ARG;
  if (dIn)
    for (int64_t y = 0; y < H; y++)
      for (int64_t x = 0; x < W; x++) dIn[y * ld_in + x] = 0.0;
  if (dW)
    for (int t = 0; t < kh * kw; t++) dW[t] = 0.0;
  if (H == 0 || W == 0) return OR_OK;
  int64_t shape[2] = {H, W}, stride[2] = {ld_in, 1};
  view img = v_leaf(in, elem, 2, shape, stride);
  view chain[5];
  const view* win = stencil_windows(&img, kh, kw, mode, chain);
  if (win->bad) return OR_ERR_SHAPE;
  note_threads();
  if (dIn) {
    for (int64_t y = 0; y < H; y++)
      for (int64_t x = 0; x < W; x++) {
        double g = (double)dOut[y * W + x];
        for (int64_t dy = 0; dy < kh; dy++)
          for (int64_t dx = 0; dx < kw; dx++) {
            int64_t idx[4] = {y, x, dy, dx};
            int64_t p = view_source(win, idx);
            if (p >= 0) dIn[p] = dIn[p] + (double)w[dy * kw + dx] * g;
          }
      }
  }
  if (dW) {
#pragma omp parallel for schedule(static, 1)
    for (int t = 0; t < kh * kw; t++) {
      int64_t dy = t / kw, dx = t % kw;
      double acc = 0.0;
      for (int64_t y = 0; y < H; y++)
        for (int64_t x = 0; x < W; x++) {
          int64_t idx[4] = {y, x, dy, dx};
          acc = acc + (double)dOut[y * W + x] * view_at(win, idx);
        }
      dW[t] = acc;
    }
  }
  return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Multi-channel stencil layer (convolution), NHWC activations            */
/* ---------------------------------------------------------------------- */

/* out[b][y][x][co] = reduce(+, 0) over ci of
 *     stencil(pad2D(in[b][.][.][ci]), weights[co][ci])
 * in: B x H x W x Cin (NHWC, elem), weights: Cout x Cin x kh x kw (f32),
 * out: B x H x W x Cout (double). */
int oracle_conv2d(double* out, const void* in, int elem, const float* wts, int64_t B,
                  int64_t Cin, int64_t Cout, int64_t H, int64_t W, int kh, int kw, int mode) {
  int rc = check_kernel(kh, kw, mode);
  if (rc) return rc;
  if (B < 0 || Cin < 0 || Cout < 0 || H < 0 || W < 0) return OR_ERR_ARG;
  int64_t shape[4] = {B, H, W, Cin}, stride[4] = {H * W * Cin, W * Cin, Cin, 1};
  view x4 = v_leaf(in, elem, 4, shape, stride);
  int64_t wshape[4] = {Cout, Cin, kh, kw}, wstride[4] = {Cin * kh * kw, kh * kw, kw, 1};
  view w4 = v_leaf(wts, EL_F32, 4, wshape, wstride);
  note_threads();
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
  for (int64_t b = 0; b < B; b++)
    for (int64_t y = 0; y < H; y++) {
      view img_b = v_idx(&x4, 0, b); /* (H, W, Cin) */
      for (int64_t x = 0; x < W; x++)
        for (int64_t co = 0; co < Cout; co++) {
          view w_co = v_idx(&w4, 0, co); /* (Cin, kh, kw) */
          double acc = 0.0;
          for (int64_t ci = 0; ci < Cin; ci++) {
            view plane = v_idx(&img_b, 2, ci); /* (H, W) */
            view chain[5];
            const view* win = stencil_windows(&plane, kh, kw, mode, chain);
            view wy = v_idx(win, 0, y);
            view wnd = v_idx(&wy, 0, x);
            view wndj = v_join(&wnd, 0);
            view wk = v_idx(&w_co, 0, ci);
            view wkj = v_join(&wk, 0);
            acc = acc + zip_mul_reduce(&wndj, &wkj, 0.0);
          }
          out[((b * H + y) * W + x) * Cout + co] = acc;
        }
    }
  return OR_OK;
}

/* Gradients of L = <G, conv(in, w)> with G = dOut (B x H x W x Cout, f32):
 *   dIn  (B x H x W x Cin): adjoint scatter through the window views;
 *   dW   (Cout x Cin x kh x kw): sum over (b, y, x) of dOut * window.
 * Either output may be NULL. */
int oracle_conv2d_backward(double* dIn, double* dW, const float* dOut, const void* in, int elem,
                           const float* wts, int64_t B, int64_t Cin, int64_t Cout, int64_t H,
                           int64_t W, int kh, int kw, int mode) {
  int rc = check_kernel(kh, kw, mode);
  if (rc) return rc;
  int64_t shape[4] = {B, H, W, Cin}, stride[4] = {H * W * Cin, W * Cin, Cin, 1};
  view x4 = v_leaf(in, elem, 4, shape, stride);
  int64_t nx = B * H * W * Cin;
  if (dIn)
    for (int64_t i = 0; i < nx; i++) dIn[i] = 0.0;
  note_threads();
  if (dIn) {
    /* parallel over (b, ci): each pair owns a disjoint set of dIn elements */
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int64_t b = 0; b < B; b++)
      for (int64_t ci = 0; ci < Cin; ci++) {
        view img_b = v_idx(&x4, 0, b);
        view plane = v_idx(&img_b, 2, ci);
        view chain[5];
        const view* win = stencil_windows(&plane, kh, kw, mode, chain);
        for (int64_t y = 0; y < H; y++)
          for (int64_t x = 0; x < W; x++)
            for (int64_t co = 0; co < Cout; co++) {
              double g = (double)dOut[((b * H + y) * W + x) * Cout + co];
              for (int64_t dy = 0; dy < kh; dy++)
                for (int64_t dx = 0; dx < kw; dx++) {
                  int64_t idx[4] = {y, x, dy, dx};
                  int64_t p = view_source(win, idx);
                  if (p >= 0) {
                    double wv = (double)wts[((co * Cin + ci) * kh + dy) * kw + dx];
                    dIn[p] = dIn[p] + wv * g;
                  }
                }
            }
      }
  }
  if (dW) {
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int64_t co = 0; co < Cout; co++)
      for (int64_t ci = 0; ci < Cin; ci++) {
        for (int64_t t = 0; t < kh * kw; t++) {
          int64_t dy = t / kw, dx = t % kw;
          double acc = 0.0;
          for (int64_t b = 0; b < B; b++) {
            view img_b = v_idx(&x4, 0, b);
            view plane = v_idx(&img_b, 2, ci);
            view chain[5];
            const view* win = stencil_windows(&plane, kh, kw, mode, chain);
            for (int64_t y = 0; y < H; y++)
              for (int64_t x = 0; x < W; x++) {
                int64_t idx[4] = {y, x, dy, dx};
                acc = acc + (double)dOut[((b * H + y) * W + x) * Cout + co] * view_at(win, idx);
              }
          }
          dW[(co * Cin + ci) * kh * kw + t] = acc;
        }
      }
  }
  return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Generic view evaluation (for the pattern-law tests)                    */
/* ---------------------------------------------------------------------- */

/* Materialise a composed view of a rank-`rank` f64 array.  ops is a list of
 * n_ops records of 5 int64: {op, axis, p, q, mode} with op one of
 *   1 idx(p)  2 split(p)  3 join  4 transpose  5 slide(p=sz, q=sp)
 *   6 pad(l=p, r=q, mode)
 * out_shape (RMAX entries) receives the result shape; out receives the
 * elements in row-major order if out_cap is large enough. */
int oracle_view_eval(double* out, int64_t out_cap, int64_t* out_rank, int64_t* out_shape,
                     const double* data, int rank, const int64_t* shape, const int64_t* ops,
                     int n_ops) {
  if (rank <= 0 || rank > RMAX || n_ops < 0 || n_ops > 32) return OR_ERR_ARG;
  int64_t stride[RMAX];
  stride[rank - 1] = 1;
  for (int d = rank - 2; d >= 0; d--) stride[d] = stride[d + 1] * shape[d + 1];
  view chain[33];
  chain[0] = v_leaf(data, EL_F64, rank, shape, stride);
  for (int k = 0; k < n_ops; k++) {
    const int64_t* o = ops + 5 * k;
    const view* in = &chain[k];
    int axis = (int)o[1];
    switch (o[0]) {
      case 1: chain[k + 1] = v_idx(in, axis, o[2]); break;
      case 2: chain[k + 1] = v_split(in, axis, o[2]); break;
      case 3: chain[k + 1] = v_join(in, axis); break;
      case 4: chain[k + 1] = v_transpose(in, axis); break;
      case 5: chain[k + 1] = v_slide(in, axis, o[2], o[3]); break;
      case 6: chain[k + 1] = v_pad(in, axis, o[2], o[3], (int)o[4]); break;
      default: return OR_ERR_ARG;
    }
    if (chain[k + 1].bad) return OR_ERR_SHAPE;
  }
  const view* v = &chain[n_ops];
  *out_rank = v->rank;
  int64_t total = 1;
  for (int d = 0; d < v->rank; d++) {
    out_shape[d] = v->shape[d];
    total *= v->shape[d];
  }
  if (total > out_cap) return OR_ERR_ARG;
  int64_t idx[RMAX];
  for (int64_t e = 0; e < total; e++) {
    int64_t rem = e;
    for (int d = v->rank - 1; d >= 0; d--) {
      idx[d] = v->shape[d] ? rem % v->shape[d] : 0;
      rem = v->shape[d] ? rem / v->shape[d] : 0;
    }
    out[e] = view_at(v, idx);
  }
  return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Operand preparation of the reduced-precision GEMM modes                */
/* ---------------------------------------------------------------------- */

/* Round x to the nearest value with `p` significant bits and minimum exponent
 * `emin` (values below 2^emin use the fixed quantum 2^(emin - p + 1)), ties to
 * even.  nearbyint rounds half to even under the default rounding mode. */
static double round_sig(double x, int p, int emin) {
  if (x == 0.0 || !isfinite(x)) return x;
  int e;
  frexp(x, &e); /* x = f * 2^e, 0.5 <= |f| < 1, so the leading bit has weight 2^(e-1) */
  int lead = e - 1;
  if (lead < emin) lead = emin;
  double quantum = ldexp(1.0, lead - (p - 1));
  return nearbyint(x / quantum) * quantum;
}

/* bfloat16: 8 significant bits, exponent range of f32 (min normal 2^-126). */
double oracle_round_bf16(double x) { return round_sig(x, 8, -126); }

/* Encode a value that is exactly representable in bfloat16 as its 16 bits
 * (the upper half of the f32 encoding, which is exact for such values). */
static uint16_t bf16_encode(double v) {
  float f = (float)v;
  uint32_t u;
  memcpy(&u, &f, 4);
  return (uint16_t)(u >> 16);
}

/* map(cast) to bf16, round to nearest even.  out holds bf16 bit patterns. */
void oracle_quant_bf16(uint16_t* out, const float* in, int64_t n) {
  for (int64_t i = 0; i < n; i++) out[i] = bf16_encode(oracle_round_bf16((double)in[i]));
}

/* hi = bf16(a), lo = bf16(a - hi). */
void oracle_split_bf16(uint16_t* hi, uint16_t* lo, const float* in, int64_t n) {
  for (int64_t i = 0; i < n; i++) {
    double a = (double)in[i];
    double h = oracle_round_bf16(a);
    double l = oracle_round_bf16(a - h);
    hi[i] = bf16_encode(h);
    lo[i] = bf16_encode(l);
  }
}

/* three-way split: a1 = bf16(a), a2 = bf16(a - a1), a3 = bf16(a - a1 - a2). */
void oracle_split3_bf16(uint16_t* p1, uint16_t* p2, uint16_t* p3, const float* in, int64_t n) {
  for (int64_t i = 0; i < n; i++) {
    double a = (double)in[i];
    double x1 = oracle_round_bf16(a);
    double x2 = oracle_round_bf16(a - x1);
    double x3 = oracle_round_bf16(a - x1 - x2);
    p1[i] = bf16_encode(x1);
    p2[i] = bf16_encode(x2);
    p3[i] = bf16_encode(x3);
  }
}

/* OCP FP8 E4M3 ("E4M3FN"): 4 significant bits, min normal 2^-6, subnormal
 * quantum 2^-9, largest finite 448, no infinities.  Round to nearest even,
 * saturating at +-448. */
double oracle_round_e4m3(double x) {
  double r = round_sig(x, 4, -6);
  if (r > 448.0) r = 448.0;
  if (r < -448.0) r = -448.0;
  return r;
}

/* Encode a representable E4M3 value: sign | exponent (bias 7) | 3 mantissa bits. */
static uint8_t e4m3_encode(double v) {
  uint8_t s = (v < 0.0 || (v == 0.0 && signbit(v))) ? 0x80 : 0x00;
  double a = fabs(v);
  if (a == 0.0) return s;
  if (a < ldexp(1.0, -6)) { /* subnormal: value = m * 2^-9 */
    return (uint8_t)(s | (uint8_t)(a / ldexp(1.0, -9)));
  }
  int e;
  double f = frexp(a, &e); /* a = f * 2^e, f in [0.5, 1) */
  int unb = e - 1;         /* a = (2f) * 2^(e-1), 2f in [1, 2) */
  int mant = (int)((2.0 * f - 1.0) * 8.0);
  return (uint8_t)(s | (uint8_t)((unb + 7) << 3) | (uint8_t)mant);
}

/* Scale exponent of a block: the largest integer e with amax * 2^e <= 448
 * (e = 0 when amax = 0), limited to [-127, 127] so that 2^-e is an E8M0 scale.
 * Written from amax = f * 2^E (f in [0.5, 1)) and 448 = 0.875 * 2^9. */
int oracle_e4m3_block_exponent(double amax) {
  if (amax == 0.0) return 0;
  int E;
  double f = frexp(amax, &E);
  int e = (f <= 0.875) ? 9 - E : 8 - E;
  if (e > 127) e = 127;
  if (e < -127) e = -127;
  return e;
}

/* FP8 E4M3 operand with one power-of-two scale per block of `blk` consecutive
 * elements along K.  The operand is `rows` vectors of length K; vector r's
 * element k is src[r * ld_r + k * ld_k] (so a row-major M x K A uses
 * ld_r = lda, ld_k = 1, and a row-major K x N B uses ld_r = 1, ld_k = ldb).
 * Outputs: q[r * K + k] = E4M3 byte of src * 2^e, and
 *          scale[r * nblk + b] = E8M0 byte (127 - e) of the dequantisation
 *          factor 2^-e, nblk = ceil(K / blk).
 * A partial last block is scaled by its own amax. */
int oracle_quant_e4m3_blocks(uint8_t* q, uint8_t* scale, const float* src, int64_t rows,
                             int64_t K, int64_t ld_r, int64_t ld_k, int64_t blk) {
  if (blk <= 0 || rows < 0 || K < 0) return OR_ERR_ARG;
  int64_t nblk = (K + blk - 1) / blk;
  for (int64_t r = 0; r < rows; r++)
    for (int64_t b = 0; b < nblk; b++) {
      int64_t k0 = b * blk, k1 = k0 + blk < K ? k0 + blk : K;
      double amax = 0.0;
      for (int64_t k = k0; k < k1; k++) {
        double a = fabs((double)src[r * ld_r + k * ld_k]);
        if (a > amax) amax = a;
      }
      int e = oracle_e4m3_block_exponent(amax);
      scale[r * nblk + b] = (uint8_t)(127 - e);
      for (int64_t k = k0; k < k1; k++) {
        double v = ldexp((double)src[r * ld_r + k * ld_k], e);
        q[r * K + k] = e4m3_encode(oracle_round_e4m3(v));
      }
    }
  return OR_OK;
}

/* Decode helpers used to build the dequantised operands. */
double oracle_e4m3_decode(uint8_t b) {
  int s = b >> 7, ex = (b >> 3) & 15, m = b & 7;
  double v;
  if (ex == 15 && m == 7) return NAN;
  if (ex == 0)
    v = ldexp((double)m, -9);
  else
    v = ldexp(1.0 + m / 8.0, ex - 7);
  return s ? -v : v;
}

/* Precision modes of the GEMM (same numbering as the GPU library's modes). */
enum { MODE_F32 = 0, MODE_BF16 = 1, MODE_BF16X3 = 2, MODE_BF16X6 = 3, MODE_FP8 = 4 };

/* The value each mode's arithmetic defines, evaluated exactly enough (double):
 *   F32:    A B
 *   BF16:   bf16(A) bf16(B)
 *   BF16X3: Ah Bh + Ah Bl + Al Bh          (hi/lo split of each operand)
 *   BF16X6: sum of A_i B_j over i + j <= 4 (three-way split, 6 products)
 *   FP8:    sum over K-blocks of (qA 2^-eA)(qB 2^-eB)  (E4M3, blocks of 32)
 * A: M x K row-major (lda), B: K x N row-major (ldb), C: M x N row-major.
 * Either the full C (rows == NULL) or the listed samples are produced. */
int oracle_gemm_mode(double* C, const int64_t* rows, const int64_t* cols, int64_t count,
                     const float* A, int64_t lda, const float* B, int64_t ldb, int64_t M,
                     int64_t N, int64_t K, int mode) {
  if (M < 0 || N < 0 || K < 0) return OR_ERR_ARG;
  int nparts = (mode == MODE_F32) ? 1 : (mode == MODE_BF16) ? 1 : (mode == MODE_BF16X3) ? 2
             : (mode == MODE_BF16X6) ? 3 : (mode == MODE_FP8) ? 1 : -1;
  if (nparts < 0) return OR_ERR_ARG;
  /* dequantised operand parts as doubles: Ap[p] is M x K, Bp[p] is K x N */
  double* Ap[3] = {0, 0, 0};
  double* Bp[3] = {0, 0, 0};
  for (int p = 0; p < nparts; p++) {
    Ap[p] = (double*)malloc(sizeof(double) * (size_t)(M * K > 0 ? M * K : 1));
    Bp[p] = (double*)malloc(sizeof(double) * (size_t)(K * N > 0 ? K * N : 1));
  }
  if (mode == MODE_FP8) {
    const int64_t blk = 32;
    int64_t nb = (K + blk - 1) / blk;
    uint8_t* qa = (uint8_t*)malloc((size_t)(M * K + 1));
    uint8_t* sa = (uint8_t*)malloc((size_t)(M * nb + 1));
    uint8_t* qb = (uint8_t*)malloc((size_t)(N * K + 1));
    uint8_t* sb = (uint8_t*)malloc((size_t)(N * nb + 1));
    oracle_quant_e4m3_blocks(qa, sa, A, M, K, lda, 1, blk);
    oracle_quant_e4m3_blocks(qb, sb, B, N, K, 1, ldb, blk);
    for (int64_t i = 0; i < M; i++)
      for (int64_t k = 0; k < K; k++)
        Ap[0][i * K + k] = ldexp(oracle_e4m3_decode(qa[i * K + k]), (int)sa[i * nb + k / blk] - 127);
    for (int64_t j = 0; j < N; j++)
      for (int64_t k = 0; k < K; k++)
        Bp[0][k * N + j] = ldexp(oracle_e4m3_decode(qb[j * K + k]), (int)sb[j * nb + k / blk] - 127);
    free(qa); free(sa); free(qb); free(sb);
  } else {
    for (int64_t i = 0; i < M; i++)
      for (int64_t k = 0; k < K; k++) {
        double a = (double)A[i * lda + k], rem = a;
        for (int p = 0; p < nparts; p++) {
          double part = (mode == MODE_F32) ? rem : oracle_round_bf16(rem);
          Ap[p][i * K + k] = part;
          rem = rem - part;
        }
      }
    for (int64_t k = 0; k < K; k++)
      for (int64_t j = 0; j < N; j++) {
        double b = (double)B[k * ldb + j], rem = b;
        for (int p = 0; p < nparts; p++) {
          double part = (mode == MODE_F32) ? rem : oracle_round_bf16(rem);
          Bp[p][k * N + j] = part;
          rem = rem - part;
        }
      }
  }
  /* products kept: parts (pa, pb) with pa + pb <= nparts - 1 for the split modes
   * (hi/lo: (0,0) (0,1) (1,0); three-way: i + j <= 2 in 0-based part indices) */
  int64_t nout = rows ? count : M * N;
  for (int64_t s = 0; s < nout; s++) C[s] = 0.0;
  int rc = OR_OK;
  double* tmp = (double*)malloc(sizeof(double) * (size_t)(nout > 0 ? nout : 1));
  for (int pa = 0; pa < nparts && rc == OR_OK; pa++)
    for (int pb = 0; pb < nparts && rc == OR_OK; pb++) {
      if (pa + pb > nparts - 1) continue;
      if (rows)
        rc = oracle_gemm_sampled(tmp, rows, cols, count, Ap[pa], EL_F64, K, 0, Bp[pb], EL_F64, N,
                                 0, M, N, K);
      else
        rc = oracle_gemm(tmp, N, Ap[pa], EL_F64, K, 0, Bp[pb], EL_F64, N, 0, M, N, K);
      for (int64_t s = 0; s < nout; s++) C[s] = C[s] + tmp[s];
    }
  free(tmp);
  for (int p = 0; p < nparts; p++) {
    free(Ap[p]);
    free(Bp[p]);
  }
  return rc;
}

/* ---------------------------------------------------------------------- */
/* iterate: the tree reduction of Sec. VI                                 */
/* ---------------------------------------------------------------------- */

/* iterate(n, m, k, body, arr) with body = split(n) |> map(reduce(+, 0)):
 * arr holds n^k * m values; iteration i (0-based) reads the n^(k-i) * m values
 * the previous one produced and writes n^(k-i-1) * m values, value j being the
 * left fold from 0 of elements j*n .. j*n+n-1.  Two temporaries of n^k * m
 * values take turns as the source and the destination (newDoubleBuffer); the
 * first iteration reads arr and the last writes out.  k = 0 leaves arr as it is
 * (out = arr).
 *
 * binary32 = 0: the values and every sum are doubles (exact widening of the
 * float input).  binary32 = 1: the values and every sum are floats, so each
 * addition rounds to binary32 in the order written here, the same order in
 * which a float implementation of this program rounds. */
static int64_t ipow_checked(int64_t n, int64_t k, int64_t m) {
  /* n^k * m, or -1 when it exceeds 2^62 */
  int64_t v = m;
  for (int64_t i = 0; i < k; i++) {
    if (n != 0 && v > ((int64_t)1 << 62) / n) return -1;
    v *= n;
  }
  return v;
}

int oracle_iterate_sum(double* out, const float* in, int64_t n, int64_t m, int64_t k,
                       int binary32) {
  if (n < 1 || m < 0 || k < 0) return OR_ERR_ARG;
  int64_t total = ipow_checked(n, k, m);
  if (total < 0) return OR_ERR_SHAPE;
  if (k == 0) {
    for (int64_t j = 0; j < m; j++) out[j] = (double)in[j];
    return OR_OK;
  }
  size_t cap = (size_t)(total > 0 ? total : 1);
  if (binary32) {
    float* buf[2] = {(float*)malloc(cap * sizeof(float)), (float*)malloc(cap * sizeof(float))};
    if (!buf[0] || !buf[1]) {
      free(buf[0]);
      free(buf[1]);
      return OR_ERR_ARG;
    }
    const float* src = in;
    int64_t len = total;
    for (int64_t i = 0; i < k; i++) {
      int64_t l = len / n;
      float* dst = buf[i & 1];
      for (int64_t j = 0; j < l; j++) {
        float acc = 0.0f;
        for (int64_t t = 0; t < n; t++) acc = acc + src[j * n + t];
        dst[j] = acc;
      }
      src = dst;
      len = l;
    }
    for (int64_t j = 0; j < m; j++) out[j] = (double)src[j];
    free(buf[0]);
    free(buf[1]);
    return OR_OK;
  }
  double* buf[2] = {(double*)malloc(cap * sizeof(double)), (double*)malloc(cap * sizeof(double))};
  if (!buf[0] || !buf[1]) {
    free(buf[0]);
    free(buf[1]);
    return OR_ERR_ARG;
  }
  int64_t len = total;
  /* the first iteration reads the float input, later ones the temporaries */
  for (int64_t j = 0; j < len / n; j++) {
    double acc = 0.0;
    for (int64_t t = 0; t < n; t++) acc = acc + (double)in[j * n + t];
    buf[0][j] = acc;
  }
  len /= n;
  for (int64_t i = 1; i < k; i++) {
    int64_t l = len / n;
    const double* src = buf[(i - 1) & 1];
    double* dst = buf[i & 1];
    for (int64_t j = 0; j < l; j++) {
      double acc = 0.0;
      for (int64_t t = 0; t < n; t++) acc = acc + src[j * n + t];
      dst[j] = acc;
    }
    len = l;
  }
  for (int64_t j = 0; j < m; j++) out[j] = buf[(k - 1) & 1][j];
  free(buf[0]);
  free(buf[1]);
  return OR_OK;
}
