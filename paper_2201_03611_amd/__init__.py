"""Python binding of librise.so: MI355X kernels for the dense RISE patterns.

Functions named rise_* mirror the C ABI (include/rise.h) one to one: they only
marshal torch tensors (device memory) and the current HIP stream into the
library call and raise RiseError on a non-OK status.  Every step of the
computation runs in the library's HIP kernels.  The convenience wrappers
(gemm, stencil2d, ...) allocate outputs and workspaces with torch and then
call the same entry points.
"""
import ctypes

import torch

from . import _lib
from ._lib import (RISE_BF16, RISE_F32, RISE_MODE_BF16, RISE_MODE_BF16X3, RISE_MODE_BF16X6,
                   RISE_MODE_F32, RISE_MODE_FP8, RISE_OP_N, RISE_OP_T, RISE_PAD_CLAMP,
                   RISE_PAD_ZERO, RISE_STENCIL_ASYNC, RISE_STENCIL_LDS_PIPE, RISE_STENCIL_LDS_TILE,
                   RISE_STENCIL_STREAM,
                   RiseGemmProblem,
                   RiseStencilProblem, RiseStencilSchedule, RiseTile)

lib = _lib.load()

MODES = {"f32": RISE_MODE_F32, "bf16": RISE_MODE_BF16, "bf16x3": RISE_MODE_BF16X3,
         "bf16x6": RISE_MODE_BF16X6, "fp8": RISE_MODE_FP8}
PADS = {"clamp": RISE_PAD_CLAMP, "zero": RISE_PAD_ZERO}


class RiseError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = lib.rise_last_error().decode()
        super().__init__(f"{where}: {_lib.STATUS_NAMES.get(status, status)} ({msg})")


def _check(status, where):
    if status != _lib.RISE_OK:
        raise RiseError(status, where)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _mode(m):
    return MODES[m] if isinstance(m, str) else int(m)


def _tile(t):
    if t is None:
        return None
    return ctypes.byref(RiseTile(*t))


def _dtype(t):
    if t.dtype == torch.float32:
        return RISE_F32
    if t.dtype == torch.bfloat16:
        return RISE_BF16
    raise TypeError(f"GEMM operands are float32 or bfloat16, got {t.dtype}")


def _require_cuda(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("librise works on device tensors only")


def _require_dtype(t, dtype, what):
    if t is not None and t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")


def _on_stream(fn):
    """Run a convenience wrapper with `stream` as torch's current stream, so that
    its input copies, its output and workspace allocations and the library call
    all belong to that stream (the caching allocator then cannot hand the
    workspace to another allocation while the kernel still reads it)."""
    import functools

    @functools.wraps(fn)
    def wrapper(*args, stream=None, **kwargs):
        if stream is None:
            return fn(*args, **kwargs)
        with torch.cuda.stream(stream):
            return fn(*args, **kwargs)

    return wrapper


# ---------------------------------------------------------------------------
# one-to-one entry points
# ---------------------------------------------------------------------------
def rise_gemm_tiles(mode):
    m = _mode(mode)
    n = lib.rise_gemm_tiles(m, None, 0)
    arr = (RiseTile * max(n, 1))()
    lib.rise_gemm_tiles(m, arr, n)
    return [(arr[i].bm, arr[i].bn, arr[i].bk) for i in range(n)]


def rise_gemm_default_tile(M, N, K, mode="f32"):
    """The tile rise_gemm runs with tile=None, as (bm, bn, bk)."""
    t = RiseTile()
    _check(lib.rise_gemm_default_tile(M, N, K, _mode(mode), ctypes.byref(t)),
           "rise_gemm_default_tile")
    return (t.bm, t.bn, t.bk)


def rise_gemm_workspace(M, N, K, mode, tile=None):
    return int(lib.rise_gemm_workspace(M, N, K, _mode(mode), _tile(tile)))


def rise_gemm(C, A, B, M, N, K, *, lda, ldb, ldc, opA=RISE_OP_N, opB=RISE_OP_N, mode="f32",
              tile=None, ws=None, stream=None):
    """C (M x N, float32) = A . B; A, B device tensors read through opA / opB."""
    _require_cuda(C, A, B, ws)
    ws_bytes = ws.numel() * ws.element_size() if ws is not None else 0
    st = lib.rise_gemm(_ptr(C), ldc, _ptr(A), _dtype(A), lda, opA, _ptr(B), _dtype(B), ldb, opB,
                       M, N, K, _mode(mode), _tile(tile), _ptr(ws), ws_bytes, _stream(stream))
    _check(st, "rise_gemm")


def rise_gemv_workspace(M, K, opA=RISE_OP_N):
    return int(lib.rise_gemv_workspace(M, K, opA))


def rise_gemv_parts(M, K, opA=RISE_OP_N):
    return int(lib.rise_gemv_parts(M, K, opA))


def rise_gemv(y, A, x, M, K, *, lda, opA=RISE_OP_N, ws=None, stream=None):
    """y (M floats) = A . x, A read through opA (the paper's matrix-vector program)."""
    _require_cuda(y, A, x, ws)
    ws_bytes = ws.numel() * ws.element_size() if ws is not None else 0
    st = lib.rise_gemv(_ptr(y), _ptr(A), lda, opA, _ptr(x), M, K, _ptr(ws), ws_bytes,
                       _stream(stream))
    _check(st, "rise_gemv")


def rise_gemv_noalloc(y, A, x, M, K, *, lda, opA=RISE_OP_N, stream=None):
    """rise_gemv with the split-K partials in the library's fixed per-device
    scratch: no workspace argument, nothing allocated."""
    _require_cuda(y, A, x)
    st = lib.rise_gemv_noalloc(_ptr(y), _ptr(A), lda, opA, _ptr(x), M, K, _stream(stream))
    _check(st, "rise_gemv_noalloc")


RISE_GEMV_NOALLOC_SCRATCH_BYTES = 8 << 20


def rise_iterate_sum_workspace(n, m, k):
    return int(lib.rise_iterate_sum_workspace(n, m, k))


def rise_iterate_sum_passes(n, m, k):
    """Rounds run by each kernel pass of rise_iterate_sum ([] for invalid sizes)."""
    np_ = lib.rise_iterate_sum_passes(n, m, k, None, 0)
    arr = (ctypes.c_int32 * max(np_, 1))()
    lib.rise_iterate_sum_passes(n, m, k, arr, np_)
    return [int(arr[i]) for i in range(np_)]


def rise_iterate_sum(out, x, n, m, k, *, ws=None, stream=None):
    """out (m floats) = iterate(n, m, k, split(n) |> map(reduce(+, 0)), x) (Sec. VI)."""
    _require_cuda(out, x, ws)
    ws_bytes = ws.numel() * ws.element_size() if ws is not None else 0
    st = lib.rise_iterate_sum(_ptr(out), _ptr(x), n, m, k, _ptr(ws), ws_bytes, _stream(stream))
    _check(st, "rise_iterate_sum")


def rise_gemm_backward_workspace(M, N, K, mode):
    return int(lib.rise_gemm_backward_workspace(M, N, K, _mode(mode)))


def rise_gemm_backward(dA, dB, dC, A, B, M, N, K, *, ldda, lddb, lddc, lda, ldb, mode="f32",
                       ws=None, stream=None):
    _require_cuda(dA, dB, dC, A, B, ws)
    ws_bytes = ws.numel() * ws.element_size() if ws is not None else 0
    st = lib.rise_gemm_backward(_ptr(dA), ldda, _ptr(dB), lddb, _ptr(dC), lddc, _ptr(A), lda,
                                _ptr(B), ldb, M, N, K, _mode(mode), _ptr(ws), ws_bytes,
                                _stream(stream))
    _check(st, "rise_gemm_backward")


def rise_prep_bytes(rows_out, k_out, mode):
    return int(lib.rise_prep_bytes(rows_out, k_out, _mode(mode)))


def rise_prep_operand(out, rows_out, k_out, src, rows, K, ld_r, ld_k, mode, stream=None):
    _require_cuda(out, src)
    st = lib.rise_prep_operand(_ptr(out), rows_out, k_out, _ptr(src), rows, K, ld_r, ld_k,
                               _mode(mode), _stream(stream))
    _check(st, "rise_prep_operand")


SCHEDULES = {"lds": RISE_STENCIL_LDS_TILE, "stream": RISE_STENCIL_STREAM,
             "lds_pipe": RISE_STENCIL_LDS_PIPE, "async": RISE_STENCIL_ASYNC}


def rise_stencil_schedules():
    n = lib.rise_stencil_schedules(None, 0)
    arr = (RiseStencilSchedule * max(n, 1))()
    lib.rise_stencil_schedules(arr, n)
    names = {v: k for k, v in SCHEDULES.items()}
    return [(names[arr[i].variant], arr[i].rows) for i in range(n)]


def rise_stencil2d_default_schedule(H, W, kh, kw):
    """The schedule rise_stencil2d runs with schedule=None, as (name, rows);
    ("direct", 0) for windows the scheduled kernels do not cover."""
    sc = RiseStencilSchedule()
    _check(lib.rise_stencil2d_default_schedule(H, W, kh, kw, ctypes.byref(sc)),
           "rise_stencil2d_default_schedule")
    if sc.variant < 0:
        return ("direct", 0)
    names = {v: k for k, v in SCHEDULES.items()}
    return (names[sc.variant], sc.rows)


def _sched(sc):
    if sc is None:
        return None
    v, rows = sc
    return ctypes.byref(RiseStencilSchedule(SCHEDULES[v] if isinstance(v, str) else int(v), rows))


def rise_stencil2d(out, inp, w, H, W, *, ld_out, ld_in, kh, kw, pad="clamp", schedule=None,
                   stream=None):
    _require_cuda(out, inp, w)
    p = PADS[pad] if isinstance(pad, str) else int(pad)
    st = lib.rise_stencil2d(_ptr(out), ld_out, _ptr(inp), ld_in, H, W, _ptr(w), kh, kw, p,
                            _sched(schedule), _stream(stream))
    _check(st, "rise_stencil2d")


def rise_stencil2d_iterate_max_fuse():
    return int(lib.rise_stencil2d_iterate_max_fuse())


def rise_stencil2d_iterate_default_fuse(kh, kw):
    return int(lib.rise_stencil2d_iterate_default_fuse(kh, kw))


def rise_stencil2d_iterate_workspace(H, W, kh, kw, steps, fuse=0):
    return int(lib.rise_stencil2d_iterate_workspace(H, W, kh, kw, steps, fuse))


def rise_stencil2d_iterate(out, inp, w, H, W, *, ld_out, ld_in, kh, kw, steps, pad="clamp",
                           fuse=0, ws=None, stream=None):
    """`steps` applications of the stencil (iterate, Sec. VI); fuse = steps per launch."""
    _require_cuda(out, inp, w, ws)
    p = PADS[pad] if isinstance(pad, str) else int(pad)
    ws_bytes = ws.numel() * ws.element_size() if ws is not None else 0
    st = lib.rise_stencil2d_iterate(_ptr(out), ld_out, _ptr(inp), ld_in, H, W, _ptr(w), kh, kw, p,
                                    steps, fuse, _ptr(ws), ws_bytes, _stream(stream))
    _check(st, "rise_stencil2d_iterate")


def rise_stencil2d_backward_workspace(H, W, kh, kw):
    return int(lib.rise_stencil2d_backward_workspace(H, W, kh, kw))


def rise_stencil2d_backward(dIn, dW, dOut, inp, w, H, W, *, ld_din, ld_dout, ld_in, kh, kw,
                            pad="clamp", ws=None, stream=None):
    _require_cuda(dIn, dW, dOut, inp, w, ws)
    p = PADS[pad] if isinstance(pad, str) else int(pad)
    ws_bytes = ws.numel() * ws.element_size() if ws is not None else 0
    st = lib.rise_stencil2d_backward(_ptr(dIn), ld_din, _ptr(dW), _ptr(dOut), ld_dout, _ptr(inp),
                                     ld_in, H, W, _ptr(w), kh, kw, p, _ptr(ws), ws_bytes,
                                     _stream(stream))
    _check(st, "rise_stencil2d_backward")


def rise_conv2d_workspace(Cin, Cout):
    return int(lib.rise_conv2d_workspace(Cin, Cout))


def rise_conv2d(out, inp, w, B, Cin, Cout, H, W, *, kh=3, kw=3, pad="zero", ws=None, stream=None):
    """out, inp: bfloat16 NHWC device tensors; w: Cout x Cin x kh x kw float32."""
    _require_cuda(out, inp, w, ws)
    p = PADS[pad] if isinstance(pad, str) else int(pad)
    ws_bytes = ws.numel() * ws.element_size() if ws is not None else 0
    st = lib.rise_conv2d(_ptr(out), _ptr(inp), _ptr(w), B, Cin, Cout, H, W, kh, kw, p, _ptr(ws),
                         ws_bytes, _stream(stream))
    _check(st, "rise_conv2d")


def rise_conv2d_backward_workspace(B, Cin, Cout, H, W):
    return int(lib.rise_conv2d_backward_workspace(B, Cin, Cout, H, W))


def rise_conv2d_backward(dIn, dW, dOut, inp, w, B, Cin, Cout, H, W, *, kh=3, kw=3, pad="zero",
                         ws=None, stream=None):
    _require_cuda(dIn, dW, dOut, inp, w, ws)
    p = PADS[pad] if isinstance(pad, str) else int(pad)
    ws_bytes = ws.numel() * ws.element_size() if ws is not None else 0
    st = lib.rise_conv2d_backward(_ptr(dIn), _ptr(dW), _ptr(dOut), _ptr(inp), _ptr(w), B, Cin,
                                  Cout, H, W, kh, kw, p, _ptr(ws), ws_bytes, _stream(stream))
    _check(st, "rise_conv2d_backward")


def rise_plan_create(gemms, n_gemm, stencils, n_stencil, tune_table=None, stream=None):
    """gemms / stencils: ctypes arrays of RiseGemmProblem / RiseStencilProblem."""
    plan = ctypes.c_void_p()
    tt = tune_table.encode() if tune_table else None
    st = lib.rise_plan_create(ctypes.byref(plan), gemms if n_gemm else None, n_gemm,
                              stencils if n_stencil else None, n_stencil, tt, _stream(stream))
    _check(st, "rise_plan_create")
    return plan


def rise_plan_launch(plan, stream=None):
    _check(lib.rise_plan_launch(plan, _stream(stream)), "rise_plan_launch")


def rise_plan_launch_direct(plan, stream=None):
    _check(lib.rise_plan_launch_direct(plan, _stream(stream)), "rise_plan_launch_direct")


def rise_plan_destroy(plan):
    _check(lib.rise_plan_destroy(plan), "rise_plan_destroy")


def rise_plan_items(plan):
    return int(lib.rise_plan_items(plan))


def rise_plan_tile(plan, problem):
    t = RiseTile()
    _check(lib.rise_plan_tile(plan, problem, ctypes.byref(t)), "rise_plan_tile")
    return (t.bm, t.bn, t.bk)


def rise_gemm_batched(gemms, n, stream=None):
    _check(lib.rise_gemm_batched(gemms, n, _stream(stream)), "rise_gemm_batched")


def rise_stencil2d_batched(stencils, n, stream=None):
    _check(lib.rise_stencil2d_batched(stencils, n, _stream(stream)), "rise_stencil2d_batched")


def rise_autotune_batched(table_path, stream=None):
    _check(lib.rise_autotune_batched(table_path.encode(), _stream(stream)),
           "rise_autotune_batched")


def rise_autotune_gemm(cache_path, M, N, K, mode="f32", stream=None):
    """Time every tile of `mode` at M x N x K and record the fastest in cache_path."""
    _check(lib.rise_autotune_gemm(cache_path.encode(), M, N, K, _mode(mode), _stream(stream)),
           "rise_autotune_gemm")


def rise_autotune_stencil(cache_path, H, W, k, stream=None):
    """Time every stencil schedule at H x W, k x k and record the fastest in cache_path."""
    _check(lib.rise_autotune_stencil(cache_path.encode(), H, W, k, _stream(stream)),
           "rise_autotune_stencil")


def rise_set_tune_cache(path):
    """The cache file that tile=None / schedule=None consult (None disables it)."""
    _check(lib.rise_set_tune_cache(path.encode() if path else None), "rise_set_tune_cache")


def rise_ceiling_copy(dst, src, stream=None):
    """Streaming copy of src into dst (device tensors of equal byte size)."""
    _require_cuda(dst, src)
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < n:
        raise ValueError("dst is smaller than src")
    _check(lib.rise_ceiling_copy(_ptr(dst), _ptr(src), n, _stream(stream)), "rise_ceiling_copy")


def rise_ceiling_mfma_sink_floats():
    return int(lib.rise_ceiling_mfma_sink_floats())


def rise_ceiling_mfma(mode, iters, sink, stream=None):
    """Back-to-back matrix instructions of `mode` ("f32", "bf16" or "fp8") on every
    SIMD; returns the flops the launch issues (time it to get the rate)."""
    _require_cuda(sink)
    _require_dtype(sink, torch.float32, "sink")
    fl = ctypes.c_double()
    _check(lib.rise_ceiling_mfma(_mode(mode), iters, _ptr(sink), sink.numel(), ctypes.byref(fl),
                                 _stream(stream)), "rise_ceiling_mfma")
    return fl.value


class Plan:
    """Owning wrapper of a rise_plan (problem arrays are kept alive with it)."""

    def __init__(self, gemms, n_gemm, stencils, n_stencil, tune_table=None, stream=None):
        self._keep = (gemms, stencils)
        self.handle = rise_plan_create(gemms, n_gemm, stencils, n_stencil, tune_table, stream)

    def launch(self, stream=None):
        rise_plan_launch(self.handle, stream)

    def launch_direct(self, stream=None):
        rise_plan_launch_direct(self.handle, stream)

    def items(self):
        return rise_plan_items(self.handle)

    def tile(self, problem):
        return rise_plan_tile(self.handle, problem)

    def destroy(self):
        if self.handle is not None:
            rise_plan_destroy(self.handle)
            self.handle = None


# ---------------------------------------------------------------------------
# convenience wrappers
# ---------------------------------------------------------------------------
@_on_stream
def gemm(A, B, *, transA=False, transB=False, mode="f32", tile=None, out=None, ws=None):
    """Logical A (M x K) times logical B (K x N); transA means A is stored K x M.
    A and B are float32, or bfloat16 for mode "bf16"."""
    for t, nm in ((A, "A"), (B, "B")):
        if t.dtype not in (torch.float32, torch.bfloat16):
            raise TypeError(f"{nm} must be float32 or bfloat16, got {t.dtype}")
    _require_cuda(A, B)
    A = A.contiguous()
    B = B.contiguous()
    M, K = (A.shape[1], A.shape[0]) if transA else A.shape
    K2, N = (B.shape[1], B.shape[0]) if transB else B.shape
    if K != K2:
        raise ValueError(f"inner sizes differ: {K} vs {K2}")
    if out is None:
        out = torch.empty((M, N), device=A.device, dtype=torch.float32)
    need = rise_gemm_workspace(M, N, K, mode, tile)
    if need and ws is None:
        ws = torch.empty(need, device=A.device, dtype=torch.uint8)
    rise_gemm(out, A, B, M, N, K, lda=A.shape[1], ldb=B.shape[1], ldc=out.stride(0),
              opA=RISE_OP_T if transA else RISE_OP_N, opB=RISE_OP_T if transB else RISE_OP_N,
              mode=mode, tile=tile, ws=ws)
    return out


@_on_stream
def gemv(A, x, *, transA=False, out=None):
    """y = A . x for a 2-D float32 device tensor A (read transposed if transA) and a
    vector x; allocates y and the workspace with torch."""
    _require_dtype(A, torch.float32, "A")
    _require_dtype(x, torch.float32, "x")
    _require_cuda(A, x)
    A = A.contiguous()
    x = x.contiguous().reshape(-1)
    M, K = (A.shape[1], A.shape[0]) if transA else A.shape
    op = RISE_OP_T if transA else RISE_OP_N
    y = out if out is not None else torch.empty(M, device=A.device, dtype=torch.float32)
    n = rise_gemv_workspace(M, K, op)
    ws = torch.empty(n, device=A.device, dtype=torch.uint8) if n else None
    if x.numel() != K:
        raise ValueError(f"x has {x.numel()} values, A has {K} columns")
    rise_gemv(y, A, x, M, K, lda=A.stride(0), opA=op, ws=ws)
    return y


@_on_stream
def stencil2d_iterate(img, w, steps, pad="clamp", fuse=0, out=None):
    """`steps` applications of the 2D stencil to a float32 device image; allocates
    the output and the double-buffer workspace with torch."""
    _require_dtype(img, torch.float32, "img")
    _require_cuda(img)  # the small weight array may come from the host; it is copied over
    img = img.contiguous()
    w = w.contiguous().to(device=img.device, dtype=torch.float32)
    H, W = img.shape
    kh, kw = w.shape
    if out is None:
        out = torch.empty((H, W), device=img.device, dtype=torch.float32)
    need = rise_stencil2d_iterate_workspace(H, W, kh, kw, steps, fuse)
    ws = torch.empty(need, device=img.device, dtype=torch.uint8) if need else None
    rise_stencil2d_iterate(out, img, w, H, W, ld_out=out.stride(0), ld_in=W, kh=kh, kw=kw,
                           steps=steps, pad=pad, fuse=fuse, ws=ws)
    return out


@_on_stream
def iterate_sum(x, n, k, *, out=None):
    """Tree reduction of a float32 device tensor by iterate (Sec. VI): k rounds of
    summing groups of n neighbours; x.numel() must be n^k * m, returns m values."""
    _require_dtype(x, torch.float32, "x")
    _require_cuda(x)
    x = x.contiguous().reshape(-1)
    G = int(n) ** int(k)
    if x.numel() % G:
        raise ValueError(f"{x.numel()} values are not a multiple of n^k = {G}")
    m = x.numel() // G
    y = out if out is not None else torch.empty(m, device=x.device, dtype=torch.float32)
    need = rise_iterate_sum_workspace(n, m, k)
    ws = torch.empty(need, device=x.device, dtype=torch.uint8) if need else None
    rise_iterate_sum(y, x, n, m, k, ws=ws)
    return y


@_on_stream
def stencil2d(img, w, pad="clamp", out=None, schedule=None):
    _require_dtype(img, torch.float32, "img")
    _require_cuda(img)  # the small weight array may come from the host; it is copied over
    img = img.contiguous()
    w = w.contiguous().to(device=img.device, dtype=torch.float32)
    H, W = img.shape
    kh, kw = w.shape
    if out is None:
        out = torch.empty((H, W), device=img.device, dtype=torch.float32)
    rise_stencil2d(out, img, w, H, W, ld_out=out.stride(0), ld_in=img.stride(0), kh=kh, kw=kw,
                   pad=pad, schedule=schedule)
    return out


@_on_stream
def prep_operand(src, mode, *, rows, K, ld_r, ld_k, rows_out=None, k_out=None):
    _require_dtype(src, torch.float32, "src")
    _require_cuda(src)
    rows_out = rows if rows_out is None else rows_out
    k_out = K if k_out is None else k_out
    out = torch.empty(rise_prep_bytes(rows_out, k_out, mode), device=src.device,
                      dtype=torch.uint8)
    rise_prep_operand(out, rows_out, k_out, src, rows, K, ld_r, ld_k, mode)
    return out


@_on_stream
def gemm_backward(dC, A, B, *, mode="f32", need_dA=True, need_dB=True):
    """(dA, dB) of C = A . B for row-major FP32 A (M x K), B (K x N), dC (M x N)."""
    for t, nm in ((dC, "dC"), (A, "A"), (B, "B")):
        _require_dtype(t, torch.float32, nm)
    _require_cuda(dC, A, B)
    dC, A, B = dC.contiguous(), A.contiguous(), B.contiguous()
    M, K = A.shape
    N = B.shape[1]
    dA = torch.empty((M, K), device=A.device, dtype=torch.float32) if need_dA else None
    dB = torch.empty((K, N), device=A.device, dtype=torch.float32) if need_dB else None
    need = rise_gemm_backward_workspace(M, N, K, mode)
    ws = torch.empty(need, device=A.device, dtype=torch.uint8) if need else None
    rise_gemm_backward(dA, dB, dC, A, B, M, N, K, ldda=K, lddb=N, lddc=N, lda=K, ldb=N,
                       mode=mode, ws=ws)
    return dA, dB


@_on_stream
def stencil2d_backward(dOut, img, w, pad="clamp", *, need_din=True, need_dw=True):
    _require_dtype(dOut, torch.float32, "dOut")
    _require_dtype(img, torch.float32, "img")
    _require_cuda(dOut, img, w)
    dOut, img = dOut.contiguous(), img.contiguous()
    w = w.contiguous().to(device=img.device, dtype=torch.float32)
    H, W = img.shape
    kh, kw = w.shape
    dIn = torch.empty((H, W), device=img.device, dtype=torch.float32) if need_din else None
    dW = torch.empty((kh, kw), device=img.device, dtype=torch.float32) if need_dw else None
    ws = torch.empty(max(rise_stencil2d_backward_workspace(H, W, kh, kw), 256), device=img.device,
                     dtype=torch.uint8)
    rise_stencil2d_backward(dIn, dW, dOut, img, w, H, W, ld_din=W, ld_dout=W, ld_in=W, kh=kh,
                            kw=kw, pad=pad, ws=ws)
    return dIn, dW


@_on_stream
def conv2d(x, w, pad="zero"):
    """x: B x H x W x Cin bfloat16 (NHWC), w: Cout x Cin x 3 x 3 float32 -> bfloat16 NHWC."""
    _require_dtype(x, torch.bfloat16, "x")
    _require_cuda(x, w)
    x = x.contiguous()
    w = w.contiguous().to(device=x.device, dtype=torch.float32)
    B, H, W, Cin = x.shape
    Cout = w.shape[0]
    out = torch.empty((B, H, W, Cout), device=x.device, dtype=torch.bfloat16)
    ws = torch.empty(rise_conv2d_workspace(Cin, Cout), device=x.device, dtype=torch.uint8)
    rise_conv2d(out, x, w, B, Cin, Cout, H, W, kh=w.shape[2], kw=w.shape[3], pad=pad, ws=ws)
    return out


@_on_stream
def conv2d_backward(dOut, x, w, pad="zero", *, need_din=True, need_dw=True):
    _require_dtype(dOut, torch.bfloat16, "dOut")
    _require_dtype(x, torch.bfloat16, "x")
    _require_cuda(dOut, x, w)
    dOut, x = dOut.contiguous(), x.contiguous()
    w = w.contiguous().to(device=x.device, dtype=torch.float32)
    B, H, W, Cin = x.shape
    Cout = w.shape[0]
    dIn = torch.empty_like(x) if need_din else None
    dW = torch.empty_like(w) if need_dw else None
    ws = torch.empty(rise_conv2d_backward_workspace(B, Cin, Cout, H, W), device=x.device,
                     dtype=torch.uint8)
    rise_conv2d_backward(dIn, dW, dOut, x, w, B, Cin, Cout, H, W, kh=w.shape[2], kw=w.shape[3],
                         pad=pad, ws=ws)
    return dIn, dW


from .autograd import RiseConv2dFn, RiseGemmFn, RiseStencil2dFn  # noqa: E402,F401
