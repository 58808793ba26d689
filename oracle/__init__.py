"""The oracle: a plain CPU interpreter of the RISE pattern semantics (fp64).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports, links or
runs anything here, and this package never imports the GPU library.

Every function takes numpy arrays holding the stored input bits (float32,
bfloat16 bit patterns as uint16, float64) and returns float64 results computed
by rise_oracle.c, which cites the paper passage each definition follows.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "librise_oracle.so")
_lib = None

EL_F32, EL_F64, EL_BF16 = 0, 1, 2
PAD_CLAMP, PAD_ZERO = 0, 1
MODE_F32, MODE_BF16, MODE_BF16X3, MODE_BF16X6, MODE_FP8 = 0, 1, 2, 3, 4

# view-op codes of oracle_view_eval
V_IDX, V_SPLIT, V_JOIN, V_TRANSPOSE, V_SLIDE, V_PAD = 1, 2, 3, 4, 5, 6


class OracleError(RuntimeError):
    pass


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_INT = ctypes.c_int


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    sig = {
        "oracle_gemm": [_P, _I64, _P, _INT, _I64, _INT, _P, _INT, _I64, _INT, _I64, _I64, _I64],
        "oracle_gemm_sampled": [_P, _P, _P, _I64, _P, _INT, _I64, _INT, _P, _INT, _I64, _INT,
                                _I64, _I64, _I64],
        "oracle_gemm_tiled": [_P, _I64, _P, _INT, _I64, _INT, _P, _INT, _I64, _INT, _I64, _I64,
                              _I64, _I64, _I64, _I64],
        "oracle_stencil2d": [_P, _P, _INT, _I64, _I64, _I64, _P, _INT, _INT, _INT],
        "oracle_stencil2d_backward": [_P, _P, _P, _P, _INT, _I64, _I64, _I64, _P, _INT, _INT,
                                      _INT],
        "oracle_conv2d": [_P, _P, _INT, _P, _I64, _I64, _I64, _I64, _I64, _INT, _INT, _INT],
        "oracle_conv2d_backward": [_P, _P, _P, _P, _INT, _P, _I64, _I64, _I64, _I64, _I64, _INT,
                                   _INT, _INT],
        "oracle_view_eval": [_P, _I64, _P, _P, _P, _INT, _P, _P, _INT],
        "oracle_quant_bf16": [_P, _P, _I64],
        "oracle_split_bf16": [_P, _P, _P, _I64],
        "oracle_split3_bf16": [_P, _P, _P, _P, _I64],
        "oracle_quant_e4m3_blocks": [_P, _P, _P, _I64, _I64, _I64, _I64, _I64],
        "oracle_gemm_mode": [_P, _P, _P, _I64, _P, _I64, _P, _I64, _I64, _I64, _I64, _INT],
        "oracle_iterate_sum": [_P, _P, _I64, _I64, _I64, _INT],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = _INT
    for name in ("oracle_round_bf16", "oracle_round_e4m3"):
        fn = getattr(lib, name)
        fn.argtypes = [ctypes.c_double]
        fn.restype = ctypes.c_double
    lib.oracle_e4m3_decode.argtypes = [ctypes.c_uint8]
    lib.oracle_e4m3_decode.restype = ctypes.c_double
    lib.oracle_e4m3_block_exponent.argtypes = [ctypes.c_double]
    lib.oracle_e4m3_block_exponent.restype = _INT
    lib.oracle_num_threads.restype = _INT
    lib.oracle_last_threads.restype = _INT
    lib.oracle_set_threads.argtypes = [_INT]
    lib.oracle_set_threads.restype = _INT
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what}: oracle status {rc}")


def _elem(a):
    if a.dtype == np.float32:
        return EL_F32
    if a.dtype == np.float64:
        return EL_F64
    if a.dtype == np.uint16:
        return EL_BF16
    raise TypeError(f"oracle leaf arrays are float32, float64 or bf16 bits (uint16), got {a.dtype}")


def _c(a):
    return np.ascontiguousarray(a)


def num_threads():
    return _load().oracle_num_threads()


def last_threads():
    return _load().oracle_last_threads()


def set_threads(n):
    """OpenMP threads for the following calls; returns the previous setting."""
    return _load().oracle_set_threads(int(n))


# --------------------------------------------------------------------------
# GEMM
# --------------------------------------------------------------------------
def gemm(A, B, opA=0, opB=0):
    """C = A |> map(aRow => transpose(B) |> map(bCol => zip |> map(*) |> reduce(+,0))).

    opA/opB = 1 means the stored array is read through transpose (A stored K x M,
    B stored N x K)."""
    lib = _load()
    A, B = _c(A), _c(B)
    M, K = (A.shape if opA == 0 else A.shape[::-1])
    K2, N = (B.shape if opB == 0 else B.shape[::-1])
    if K != K2:
        raise OracleError("zip needs equal lengths: K of A and B differ")
    C = np.empty((M, N), dtype=np.float64)
    _check(lib.oracle_gemm(_ptr(C), N, _ptr(A), _elem(A), A.shape[1], opA, _ptr(B), _elem(B),
                           B.shape[1], opB, M, N, K), "gemm")
    return C


def gemm_sampled(A, B, rows, cols, opA=0, opB=0):
    lib = _load()
    A, B = _c(A), _c(B)
    M, K = (A.shape if opA == 0 else A.shape[::-1])
    K2, N = (B.shape if opB == 0 else B.shape[::-1])
    if K != K2:
        raise OracleError("zip needs equal lengths: K of A and B differ")
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.empty(rows.shape[0], dtype=np.float64)
    _check(lib.oracle_gemm_sampled(_ptr(out), _ptr(rows), _ptr(cols), rows.shape[0], _ptr(A),
                                   _elem(A), A.shape[1], opA, _ptr(B), _elem(B), B.shape[1], opB,
                                   M, N, K), "gemm_sampled")
    return out


def gemm_tiled(A, B, mt, nt, kt):
    lib = _load()
    A, B = _c(A), _c(B)
    M, K = A.shape
    _, N = B.shape
    C = np.empty((M, N), dtype=np.float64)
    _check(lib.oracle_gemm_tiled(_ptr(C), N, _ptr(A), _elem(A), K, 0, _ptr(B), _elem(B), N, 0,
                                 M, N, K, mt, nt, kt), "gemm_tiled")
    return C


def gemm_mode(A, B, mode, rows=None, cols=None):
    """The value a precision mode's arithmetic defines (see rise_oracle.c)."""
    lib = _load()
    A = _c(np.asarray(A, dtype=np.float32))
    B = _c(np.asarray(B, dtype=np.float32))
    M, K = A.shape
    _, N = B.shape
    if rows is None:
        C = np.empty((M, N), dtype=np.float64)
        _check(lib.oracle_gemm_mode(_ptr(C), None, None, 0, _ptr(A), K, _ptr(B), N, M, N, K,
                                    mode), "gemm_mode")
        return C
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.empty(rows.shape[0], dtype=np.float64)
    _check(lib.oracle_gemm_mode(_ptr(out), _ptr(rows), _ptr(cols), rows.shape[0], _ptr(A), K,
                                _ptr(B), N, M, N, K, mode), "gemm_mode")
    return out


# --------------------------------------------------------------------------
# stencil and stencil layer
# --------------------------------------------------------------------------
def stencil2d(img, w, pad=PAD_CLAMP):
    lib = _load()
    img = _c(img)
    w = _c(np.asarray(w, dtype=np.float32))
    H, W = img.shape
    kh, kw = w.shape
    out = np.empty((H, W), dtype=np.float64)
    _check(lib.oracle_stencil2d(_ptr(out), _ptr(img), _elem(img), W, H, W, _ptr(w), kh, kw, pad),
           "stencil2d")
    return out


def stencil2d_iterate(img, w, steps, pad=PAD_CLAMP):
    """iterate (Sec. VI) with the stencil as its size-preserving body: `steps`
    applications, each to the image the previous one produced, held in two
    float64 images that take turns (newDoubleBuffer); steps = 0 returns the
    input."""
    cur = np.asarray(img, dtype=np.float64)
    if steps == 0:
        return cur.copy()
    bufs = [None, None]
    for i in range(int(steps)):
        bufs[i & 1] = stencil2d(cur, w, pad)
        cur = bufs[i & 1]
    return cur


def stencil2d_backward(dout, img, w, pad=PAD_CLAMP, want_din=True, want_dw=True):
    lib = _load()
    img = _c(img)
    dout = _c(np.asarray(dout, dtype=np.float32))
    w = _c(np.asarray(w, dtype=np.float32))
    H, W = img.shape
    kh, kw = w.shape
    din = np.empty((H, W), dtype=np.float64) if want_din else None
    dw = np.empty((kh, kw), dtype=np.float64) if want_dw else None
    _check(lib.oracle_stencil2d_backward(_ptr(din), _ptr(dw), _ptr(dout), _ptr(img), _elem(img),
                                         W, H, W, _ptr(w), kh, kw, pad), "stencil2d_backward")
    return din, dw


def iterate_sum(x, n, m, k, binary32=False):
    """iterate(n, m, k, split(n) |> map(reduce(+, 0)), x) of Sec. VI: k rounds of
    summing groups of n neighbours, n^k * m values in, m out.  binary32 rounds
    every addition to float in the program's order; otherwise the sums are
    doubles."""
    lib = _load()
    x = _c(np.asarray(x, dtype=np.float32)).reshape(-1)
    if x.size != int(n) ** int(k) * int(m):
        raise OracleError(f"iterate_sum: {x.size} values, expected n^k*m = {n}^{k}*{m}")
    out = np.empty(int(m), dtype=np.float64)
    _check(lib.oracle_iterate_sum(_ptr(out), _ptr(x), int(n), int(m), int(k), int(binary32)),
           "iterate_sum")
    return out


def conv2d(x, w, pad=PAD_ZERO):
    """x: B x H x W x Cin (NHWC), w: Cout x Cin x kh x kw -> B x H x W x Cout."""
    lib = _load()
    x = _c(x)
    w = _c(np.asarray(w, dtype=np.float32))
    B, H, W, Cin = x.shape
    Cout, Cin2, kh, kw = w.shape
    if Cin != Cin2:
        raise OracleError("channel counts differ")
    out = np.empty((B, H, W, Cout), dtype=np.float64)
    _check(lib.oracle_conv2d(_ptr(out), _ptr(x), _elem(x), _ptr(w), B, Cin, Cout, H, W, kh, kw,
                             pad), "conv2d")
    return out


def conv2d_backward(dout, x, w, pad=PAD_ZERO, want_din=True, want_dw=True):
    lib = _load()
    x = _c(x)
    dout = _c(np.asarray(dout, dtype=np.float32))
    w = _c(np.asarray(w, dtype=np.float32))
    B, H, W, Cin = x.shape
    Cout, _, kh, kw = w.shape
    din = np.empty((B, H, W, Cin), dtype=np.float64) if want_din else None
    dw = np.empty((Cout, Cin, kh, kw), dtype=np.float64) if want_dw else None
    _check(lib.oracle_conv2d_backward(_ptr(din), _ptr(dw), _ptr(dout), _ptr(x), _elem(x),
                                      _ptr(w), B, Cin, Cout, H, W, kh, kw, pad),
           "conv2d_backward")
    return din, dw


# --------------------------------------------------------------------------
# views (pattern-law tests)
# --------------------------------------------------------------------------
def view_eval(data, ops):
    """Materialise a composition of view ops over a float64 array.

    ops: list of tuples (op, axis, p, q, mode) with op in V_IDX, V_SPLIT, V_JOIN,
    V_TRANSPOSE, V_SLIDE, V_PAD."""
    lib = _load()
    data = _c(np.asarray(data, dtype=np.float64))
    rank = data.ndim
    shape = np.array(data.shape, dtype=np.int64)
    enc = np.zeros((max(len(ops), 1), 5), dtype=np.int64)
    for k, o in enumerate(ops):
        o = tuple(o) + (0,) * (5 - len(o))
        enc[k] = o
    cap = 1
    # a generous bound: slide/pad can grow the element count
    cap = max(64, data.size * 64 + 4096)
    out = np.empty(cap, dtype=np.float64)
    out_rank = np.zeros(1, dtype=np.int64)
    out_shape = np.zeros(6, dtype=np.int64)
    _check(lib.oracle_view_eval(_ptr(out), cap, _ptr(out_rank), _ptr(out_shape), _ptr(data),
                                rank, _ptr(shape), _ptr(enc), len(ops)), "view_eval")
    r = int(out_rank[0])
    shp = tuple(int(s) for s in out_shape[:r])
    n = int(np.prod(shp)) if r else 1
    return out[:n].reshape(shp)


# --------------------------------------------------------------------------
# operand preparation
# --------------------------------------------------------------------------
def round_bf16(x):
    return _load().oracle_round_bf16(float(x))


def round_e4m3(x):
    return _load().oracle_round_e4m3(float(x))


def e4m3_decode(b):
    return _load().oracle_e4m3_decode(int(b))


def e4m3_block_exponent(amax):
    return _load().oracle_e4m3_block_exponent(float(amax))


def quant_bf16(x):
    """bf16 bit patterns (uint16) of round-to-nearest-even casts of float32 x."""
    lib = _load()
    x = _c(np.asarray(x, dtype=np.float32))
    out = np.empty(x.shape, dtype=np.uint16)
    lib.oracle_quant_bf16(_ptr(out), _ptr(x), x.size)
    return out


def split_bf16(x):
    lib = _load()
    x = _c(np.asarray(x, dtype=np.float32))
    hi = np.empty(x.shape, dtype=np.uint16)
    lo = np.empty(x.shape, dtype=np.uint16)
    lib.oracle_split_bf16(_ptr(hi), _ptr(lo), _ptr(x), x.size)
    return hi, lo


def split3_bf16(x):
    lib = _load()
    x = _c(np.asarray(x, dtype=np.float32))
    p = [np.empty(x.shape, dtype=np.uint16) for _ in range(3)]
    lib.oracle_split3_bf16(_ptr(p[0]), _ptr(p[1]), _ptr(p[2]), _ptr(x), x.size)
    return tuple(p)


def quant_e4m3_rows(x, blk=32):
    """Row vectors of a row-major M x K matrix, blocks along K.

    Returns (q uint8 M x K, scale uint8 M x ceil(K/blk))."""
    lib = _load()
    x = _c(np.asarray(x, dtype=np.float32))
    M, K = x.shape
    nb = (K + blk - 1) // blk
    q = np.empty((M, K), dtype=np.uint8)
    s = np.empty((M, nb), dtype=np.uint8)
    _check(lib.oracle_quant_e4m3_blocks(_ptr(q), _ptr(s), _ptr(x), M, K, K, 1, blk), "quant_e4m3")
    return q, s


def quant_e4m3_cols(x, blk=32):
    """Column vectors of a row-major K x N matrix, blocks along K.

    Returns (q uint8 N x K, scale uint8 N x ceil(K/blk))."""
    lib = _load()
    x = _c(np.asarray(x, dtype=np.float32))
    K, N = x.shape
    nb = (K + blk - 1) // blk
    q = np.empty((N, K), dtype=np.uint8)
    s = np.empty((N, nb), dtype=np.uint8)
    _check(lib.oracle_quant_e4m3_blocks(_ptr(q), _ptr(s), _ptr(x), N, K, 1, N, blk), "quant_e4m3")
    return q, s


def bf16_bits_to_f32(bits):
    """Widen bf16 bit patterns to float32 (exact)."""
    bits = np.asarray(bits, dtype=np.uint16)
    return (bits.astype(np.uint32) << 16).view(np.float32)
