"""The C ABI without a GPU: the library loads, exports every declared entry
point, and rejects invalid arguments before touching the device (every call
below returns from host-side validation; none launches a kernel)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rise.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rise_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2201_03611_amd import _lib

    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "rise_gemm" in names and "rise_stencil2d" in names
    for n in names:
        assert hasattr(lib, n), n


def test_binding_declares_every_header_function():
    from paper_2201_03611_amd import _lib

    assert set(declared_functions()) <= set(_lib.exported_names())


FAKE_A = 0x10000000
FAKE_B = 0x20000000
FAKE_C = 0x30000000
FAKE_W = 0x40000000


def gemm(lib, C=FAKE_C, ldc=64, A=FAKE_A, tA=0, lda=64, opA=0, B=FAKE_B, tB=0, ldb=64, opB=0,
         M=64, N=64, K=64, mode=0, tile=None, ws=None, ws_bytes=0):
    return lib.rise_gemm(C, ldc, A, tA, lda, opA, B, tB, ldb, opB, M, N, K, mode, tile, ws,
                         ws_bytes, None)


def test_gemm_rejections(lib):
    from paper_2201_03611_amd._lib import RiseTile

    assert gemm(lib, C=None) == 1                       # NULL
    assert gemm(lib, A=None) == 1
    assert gemm(lib, M=-1) == 2                         # SHAPE
    assert gemm(lib, M=1 << 31) == 2
    assert gemm(lib, ldc=63) == 2
    assert gemm(lib, lda=63) == 2
    assert gemm(lib, opA=1, lda=63) == 2                # stored K x M needs lda >= M
    assert gemm(lib, C=FAKE_A + 256) == 3               # ALIAS: C inside A
    assert gemm(lib, tA=1) == 4                         # DTYPE: F32 mode with bf16 A
    assert gemm(lib, tA=1, mode=2) == 4                 # split mode needs f32 operands
    assert gemm(lib, opA=2) == 5                        # UNSUPPORTED
    assert gemm(lib, mode=9) == 5
    assert gemm(lib, tile=ctypes.byref(RiseTile(96, 96, 32))) == 5
    assert gemm(lib, mode=1) == 6                       # WORKSPACE missing
    need = lib.rise_gemm_workspace(64, 64, 64, 1, None)
    assert need > 0
    assert gemm(lib, mode=1, ws=0x50000000, ws_bytes=need - 1) == 6
    assert gemm(lib, mode=1, ws=0x50000001, ws_bytes=need) == 6  # alignment
    assert gemm(lib, mode=1, ws=FAKE_A, ws_bytes=need) == 3      # workspace overlaps A
    assert lib.rise_last_error() != b""


def gemv(lib, y=FAKE_C, A=FAKE_A, lda=64, opA=0, x=FAKE_B, M=64, K=64, ws=None, ws_bytes=0):
    return lib.rise_gemv(y, A, lda, opA, x, M, K, ws, ws_bytes, None)


def test_gemv_rejections(lib):
    assert gemv(lib, y=None) == 1                       # NULL
    assert gemv(lib, x=None) == 1
    assert gemv(lib, M=-1) == 2                         # SHAPE
    assert gemv(lib, K=1 << 31) == 2
    assert gemv(lib, lda=63) == 2
    assert gemv(lib, opA=1, M=100, lda=99) == 2         # stored K x M needs lda >= M
    assert gemv(lib, y=FAKE_A + 128) == 3               # ALIAS: y inside A
    assert gemv(lib, opA=3) == 5                        # UNSUPPORTED
    need = lib.rise_gemv_workspace(64, 100000, 1)
    assert need > 0 and lib.rise_gemv_workspace(64, 100000, 0) == 0
    assert gemv(lib, opA=1, K=100000) == 6              # WORKSPACE missing
    assert gemv(lib, opA=1, K=100000, ws=0x50000000, ws_bytes=need - 1) == 6
    assert gemv(lib, opA=1, K=100000, ws=0x50000010, ws_bytes=need) == 6
    assert gemv(lib, opA=1, K=100000, ws=FAKE_A, ws_bytes=need) == 3
    assert gemv(lib, M=0, y=None) == 0                  # no-op


def test_gemv_noalloc_rejections(lib):
    # the same host-side checks as rise_gemv, minus the workspace (none is passed)
    def call(y=FAKE_C, A=FAKE_A, lda=64, opA=0, x=FAKE_B, M=64, K=64):
        return lib.rise_gemv_noalloc(y, A, lda, opA, x, M, K, None)

    assert call(y=None) == 1                            # NULL
    assert call(x=None) == 1
    assert call(M=-1) == 2                              # SHAPE
    assert call(K=1 << 31) == 2
    assert call(lda=63) == 2
    assert call(opA=1, M=100, lda=99) == 2
    assert call(y=FAKE_A + 128) == 3                    # ALIAS: y inside A
    assert call(opA=3) == 5                             # UNSUPPORTED
    assert call(M=0, y=None) == 0                       # no-op
    msg = lib.rise_last_error()
    assert msg in (None, b"")


def test_gemv_noalloc_scratch_covers_every_split(lib):
    # the library's largest split-K partial buffer fits the fixed scratch:
    # kchunks > 1 needs at most 1023 column blocks of 1024 outputs
    from paper_2201_03611_amd import RISE_GEMV_NOALLOC_SCRATCH_BYTES as cap

    worst = 0
    for M in [1, 1000, 1024, 1025, 4096, 16384, 100000, 1023 * 1024, 1023 * 1024 + 1, 1 << 20]:
        for K in [1, 64, 65, 4096, 1 << 20, (1 << 31) - 1]:
            worst = max(worst, lib.rise_gemv_workspace(M, K, 1))
    assert 0 < worst <= cap


def iterate(lib, out=FAKE_C, x=FAKE_A, n=2, m=1, k=26, ws=None, ws_bytes=0):
    return lib.rise_iterate_sum(out, x, n, m, k, ws, ws_bytes, None)


def test_iterate_rejections(lib):
    assert iterate(lib, out=None) == 1                   # NULL
    assert iterate(lib, x=None) == 1
    assert iterate(lib, n=0) == 2                        # SHAPE
    assert iterate(lib, k=-1) == 2
    assert iterate(lib, m=-3) == 2
    assert iterate(lib, n=2, k=40) == 2                  # 2^40 values: above the limit
    assert iterate(lib, n=8193, k=1) == 5                # UNSUPPORTED fan-in
    assert iterate(lib, out=FAKE_A + 4096) == 3          # ALIAS: out inside in
    # one pass (2^13 values fit one workgroup): no workspace; two passes: two halves
    assert lib.rise_iterate_sum_workspace(2, 1, 13) == 0
    need = lib.rise_iterate_sum_workspace(2, 1, 26)
    assert need == 2 * 8192 * 4
    assert iterate(lib) == 6                             # WORKSPACE missing
    assert iterate(lib, ws=0x50000000, ws_bytes=need - 1) == 6
    assert iterate(lib, ws=0x50000010, ws_bytes=need) == 6
    assert iterate(lib, ws=FAKE_A, ws_bytes=need) == 3   # workspace inside in
    assert iterate(lib, m=0, out=None, x=None) == 0      # no-op
    assert lib.rise_iterate_sum_workspace(1, 5, 10 ** 12) == 0


def sit(lib, out=FAKE_C, ldo=64, x=FAKE_A, ldi=64, H=64, W=64, w=FAKE_W, kh=5, kw=5, pad=0,
        steps=8, fuse=0, ws=None, ws_bytes=0):
    return lib.rise_stencil2d_iterate(out, ldo, x, ldi, H, W, w, kh, kw, pad, steps, fuse, ws,
                                      ws_bytes, None)


def test_stencil_iterate_rejections(lib):
    assert lib.rise_stencil2d_iterate_max_fuse() == 4
    img = ((64 * 64 * 4 + 255) // 256) * 256
    # default fuse 4 for 3x3: 8 steps are two launches, one workspace image;
    # default 1 for 5x5: eight launches through both images
    assert lib.rise_stencil2d_iterate_workspace(64, 64, 3, 3, 8, 0) == img
    assert lib.rise_stencil2d_iterate_workspace(64, 64, 5, 5, 8, 0) == 2 * img
    assert lib.rise_stencil2d_iterate_workspace(64, 64, 5, 5, 8, 4) == img
    assert lib.rise_stencil2d_iterate_workspace(64, 64, 5, 5, 4, 4) == 0
    assert lib.rise_stencil2d_iterate_workspace(64, 64, 7, 7, 2, 0) == img
    assert sit(lib, out=None) == 1                        # NULL
    assert sit(lib, w=None) == 1
    assert sit(lib, steps=-1) == 2                        # SHAPE
    assert sit(lib, ldi=63) == 2
    assert sit(lib, kh=4) == 5                            # UNSUPPORTED
    assert sit(lib, pad=7) == 5
    assert sit(lib, fuse=5) == 5                          # above the largest fuse
    assert sit(lib, fuse=-1) == 5
    assert sit(lib, kh=7, kw=7, fuse=2) == 5              # fused 7x7 not offered
    assert sit(lib, kh=3, kw=5, fuse=2) == 5
    assert sit(lib, out=FAKE_A + 256) == 3                # ALIAS
    assert sit(lib, fuse=4) == 6                          # WORKSPACE missing
    assert sit(lib, fuse=4, ws=0x50000000, ws_bytes=img - 1) == 6
    assert sit(lib, fuse=4, ws=0x50000010, ws_bytes=img) == 6
    assert sit(lib, fuse=4, ws=FAKE_A, ws_bytes=img) == 3
    assert sit(lib, H=0, out=None, x=None) == 0           # no-op


def test_gemm_degenerate_sizes_are_noops(lib):
    assert gemm(lib, M=0) == 0
    assert gemm(lib, N=0, C=None) == 0
    assert lib.rise_gemm_workspace(0, 0, 0, 0, None) == 0


def test_tiles_and_workspace_queries(lib):
    from paper_2201_03611_amd._lib import RiseTile

    for mode in range(5):
        n = lib.rise_gemm_tiles(mode, None, 0)
        assert n >= (1 if mode == 4 else 2)  # FP8: the 128 x 128 tile only
        arr = (RiseTile * n)()
        assert lib.rise_gemm_tiles(mode, arr, n) == n
        for t in arr:
            assert t.bm > 0 and t.bn > 0 and t.bk > 0
    assert lib.rise_gemm_workspace(4096, 4096, 4096, 0, None) == 0
    # bf16 hi/lo: two bf16 planes per operand
    ws3 = lib.rise_gemm_workspace(256, 256, 256, 2, None)
    assert ws3 >= 2 * 2 * 256 * 256 * 2
    assert lib.rise_prep_bytes(64, 64, 4) == 64 * 64 + 64 * 2
    assert lib.rise_prep_bytes(64, 64, 3) == 3 * 64 * 64 * 2


def test_strategy_queries():
    """The schedules the library picks when the caller leaves the choice to it
    (Sec. IV-B/C), reported by host-only queries."""
    import paper_2201_03611_amd as rise

    for mode in ("f32", "bf16", "bf16x3", "bf16x6", "fp8"):
        for mnk in ((4096, 4096, 4096), (64, 64, 64), (1000, 3000, 77), (0, 0, 0)):
            assert rise.rise_gemm_default_tile(*mnk, mode) in rise.rise_gemm_tiles(mode)
    assert rise.rise_gemm_default_tile(4096, 4096, 4096, "f32") == (256, 128, 16)
    with pytest.raises(rise.RiseError):
        rise.rise_gemm_default_tile(-1, 4, 4, "f32")

    scheds = rise.rise_stencil_schedules()
    assert rise.rise_stencil2d_default_schedule(4096, 4096, 5, 5) == ("lds", 8)
    assert rise.rise_stencil2d_default_schedule(4096, 4096, 7, 7) == ("lds", 16)
    for k in (1, 3, 5, 7):
        assert rise.rise_stencil2d_default_schedule(300, 517, k, k) in scheds
    assert rise.rise_stencil2d_default_schedule(64, 64, 9, 9) == ("direct", 0)
    assert rise.rise_stencil2d_default_schedule(64, 64, 3, 5) == ("direct", 0)
    with pytest.raises(rise.RiseError):
        rise.rise_stencil2d_default_schedule(64, 64, 4, 4)

    assert rise.rise_stencil2d_iterate_default_fuse(3, 3) == rise.rise_stencil2d_iterate_max_fuse()
    assert rise.rise_stencil2d_iterate_default_fuse(5, 5) == 1
    assert rise.rise_stencil2d_iterate_default_fuse(7, 7) == 1

    # every pass sums groups of n^rounds <= 8192 values inside one workgroup;
    # the passes together run all k rounds
    for n, m, k in ((2, 1, 26), (2, 4096, 14), (4, 3, 9), (3, 5, 7), (8192, 2, 2), (2, 7, 0)):
        rounds = rise.rise_iterate_sum_passes(n, m, k)
        assert sum(rounds) == k and all(n ** r <= 8192 for r in rounds), (n, m, k, rounds)
        assert (len(rounds) > 1) == (rise.rise_iterate_sum_workspace(n, m, k) > 0)
    assert rise.rise_iterate_sum_passes(2, 1, 26) == [13, 13]
    assert rise.rise_iterate_sum_passes(1, 4, 9) == [1]
    assert rise.rise_iterate_sum_passes(2, 0, 5) == []
    assert rise.rise_iterate_sum_passes(8193, 1, 1) == []

    for M, K in ((16384, 16384), (3000, 20000), (64, 64), (5, 0)):
        assert rise.rise_gemv_parts(M, K, rise.RISE_OP_N) == 1
        parts = rise.rise_gemv_parts(M, K, rise.RISE_OP_T)
        ws = rise.rise_gemv_workspace(M, K, rise.RISE_OP_T)
        assert parts >= 1 and (parts > 1) == (ws > 0)
        if parts > 1:
            assert ws == (parts * M * 4 + 255) // 256 * 256
    assert rise.rise_gemv_parts(-1, 4, rise.RISE_OP_T) == 0


def stencil(lib, out=FAKE_C, ld_out=100, inp=FAKE_A, ld_in=100, H=50, W=100, w=FAKE_W, kh=5,
            kw=5, pad=0, sched=None):
    return lib.rise_stencil2d(out, ld_out, inp, ld_in, H, W, w, kh, kw, pad, sched, None)


def test_stencil_rejections(lib):
    assert stencil(lib, out=None) == 1
    assert stencil(lib, w=None) == 1
    assert stencil(lib, kh=4) == 5
    assert stencil(lib, kw=17) == 5
    assert stencil(lib, kh=0) == 5
    assert stencil(lib, pad=7) == 5
    assert stencil(lib, ld_in=99) == 2
    assert stencil(lib, H=-3) == 2
    assert stencil(lib, out=FAKE_A + 400) == 3
    assert stencil(lib, w=FAKE_C + 4) == 3
    from paper_2201_03611_amd._lib import RiseStencilSchedule

    assert stencil(lib, sched=ctypes.byref(RiseStencilSchedule(1, 48))) == 5
    assert stencil(lib, sched=ctypes.byref(RiseStencilSchedule(7, 32))) == 5
    assert lib.rise_stencil_schedules(None, 0) >= 2
    assert stencil(lib, H=0) == 0
    assert stencil(lib, W=0, out=None) == 0


def test_prep_rejections(lib):
    P = lib.rise_prep_operand
    assert P(FAKE_C, 64, 64, FAKE_A, 64, 64, 64, 1, 0, None) == 5   # F32 has no preparation
    assert P(FAKE_C, 32, 64, FAKE_A, 64, 64, 64, 1, 1, None) == 2   # rows_out < rows
    assert P(FAKE_C, 64, 48, FAKE_A, 64, 40, 64, 1, 4, None) == 2   # FP8 needs k_out % 32 == 0
    assert P(None, 64, 64, FAKE_A, 64, 64, 64, 1, 1, None) == 1
    assert P(FAKE_A + 64, 64, 64, FAKE_A, 64, 64, 64, 1, 1, None) == 3


def test_status_strings(lib):
    for s in range(8):
        assert lib.rise_status_string(s)


def test_backward_rejections(lib):
    GB = lib.rise_gemm_backward
    # dA overlapping dC
    assert GB(FAKE_C, 64, None, 0, FAKE_C + 64, 64, FAKE_A, 64, FAKE_B, 64, 64, 64, 64, 0, None, 0,
              None) == 3
    assert GB(None, 0, None, 0, FAKE_C, 64, FAKE_A, 64, FAKE_B, 64, -1, 64, 64, 0, None, 0,
              None) == 2
    assert GB(None, 0, None, 0, FAKE_C, 64, FAKE_A, 64, FAKE_B, 64, 64, 64, 64, 0, None, 0,
              None) == 0  # nothing requested
    # dA overlapping A: dA is written before the dB product reads A
    assert GB(FAKE_A + 256, 64, 0x60000000, 64, FAKE_C, 64, FAKE_A, 64, FAKE_B, 64, 64, 64, 64,
              0, None, 0, None) == 3
    # dB overlapping B
    assert GB(0x60000000, 64, FAKE_B, 64, FAKE_C, 64, FAKE_A, 64, FAKE_B, 64, 64, 64, 64, 0,
              None, 0, None) == 3
    # workspace overlapping A (rewritten by the dA product's operand preparation)
    need = lib.rise_gemm_backward_workspace(64, 64, 64, 2)
    assert need > 0
    assert GB(0x60000000, 64, 0x68000000, 64, FAKE_C, 64, FAKE_A, 64, FAKE_B, 64, 64, 64, 64, 2,
              FAKE_A, need, None) == 3
    SB = lib.rise_stencil2d_backward
    need = lib.rise_stencil2d_backward_workspace(64, 64, 5, 5)
    assert need > 0
    args = dict(dIn=FAKE_C, ld_din=64, dW=0x60000000, dOut=FAKE_A, ld_dout=64, inp=FAKE_B,
                ld_in=64, H=64, W=64, w=FAKE_W, kh=5, kw=5, pad=0, ws=0x70000000, wsb=need)

    def call(**kw):
        a = dict(args, **kw)
        return SB(a["dIn"], a["ld_din"], a["dW"], a["dOut"], a["ld_dout"], a["inp"], a["ld_in"],
                  a["H"], a["W"], a["w"], a["kh"], a["kw"], a["pad"], a["ws"], a["wsb"], None)

    assert call(kh=4) == 5
    assert call(dOut=None) == 1
    assert call(wsb=need - 1) == 6
    assert call(ws=0x70000001) == 6
    assert call(dIn=FAKE_A) == 3
    assert call(dW=FAKE_C + 8) == 3
    assert call(ld_din=10) == 2
    assert call(dIn=None, dW=None) == 0


def test_batched_rejections(lib):
    from paper_2201_03611_amd._lib import RiseGemmProblem, RiseStencilProblem

    plan = ctypes.c_void_p()
    g = (RiseGemmProblem * 2)()
    g[0] = RiseGemmProblem(FAKE_C, FAKE_A, FAKE_B, 64, 64, 64, 64, 64, 64, 0, 0)
    g[1] = RiseGemmProblem(FAKE_C, FAKE_A + 4, FAKE_B, 64, 64, 64, 64, 64, 64, 0, 0)  # unaligned
    assert lib.rise_plan_create(ctypes.byref(plan), g, 2, None, 0, None, None) == 5
    g[1] = RiseGemmProblem(FAKE_C, FAKE_A, FAKE_B, 64, 64, 64, 60, 64, 64, 0, 0)  # lda < K
    assert lib.rise_plan_create(ctypes.byref(plan), g, 2, None, 0, None, None) == 2
    g[1] = RiseGemmProblem(FAKE_C, FAKE_A, FAKE_B, 64, 64, 60, 64, 64, 64, 1, 0)  # bf16 K % 8
    assert lib.rise_plan_create(ctypes.byref(plan), g, 2, None, 0, None, None) == 5
    g[1] = RiseGemmProblem(FAKE_A + 64, FAKE_A, FAKE_B, 64, 64, 64, 64, 64, 64, 0, 0)  # alias
    assert lib.rise_plan_create(ctypes.byref(plan), g, 2, None, 0, None, None) == 3
    s = (RiseStencilProblem * 1)()
    s[0] = RiseStencilProblem(FAKE_C, FAKE_A, FAKE_W, 64, 64, 64, 64, 9, 0)  # k = 9 not batched
    assert lib.rise_plan_create(ctypes.byref(plan), None, 0, s, 1, None, None) == 5
    s[0] = RiseStencilProblem(FAKE_C, FAKE_A, FAKE_W, 64, 64, 63, 64, 5, 0)  # ld < W
    assert lib.rise_plan_create(ctypes.byref(plan), None, 0, s, 1, None, None) == 2
    assert lib.rise_plan_create(None, None, 0, None, 0, None, None) == 1
    assert lib.rise_plan_launch(None, None) == 1
    assert lib.rise_plan_destroy(None) == 0


def test_autotune_rejections(lib, tmp_path):
    # validation happens before any device work (no GPU here)
    path = str(tmp_path / "tune.txt").encode()
    assert lib.rise_autotune_gemm(None, 64, 64, 64, 0, None) == 1
    assert lib.rise_autotune_gemm(path, 0, 64, 64, 0, None) == 2
    assert lib.rise_autotune_gemm(path, 64, 64, 1 << 31, 0, None) == 2
    assert lib.rise_autotune_gemm(path, 64, 64, 64, 9, None) == 5
    assert lib.rise_autotune_gemm(path, 1 << 20, 1 << 20, 1 << 20, 0, None) == 2  # > 16 GiB
    assert lib.rise_autotune_stencil(None, 64, 64, 5, None) == 1
    assert lib.rise_autotune_stencil(path, -1, 64, 5, None) == 2
    assert lib.rise_autotune_stencil(path, 64, 64, 9, None) == 5
    assert not os.path.exists(path)


def test_tune_cache_without_entries_keeps_the_defaults(lib, tmp_path):
    # an empty or unrelated cache leaves the built-in choices (which host-only
    # queries report without a device)
    from paper_2201_03611_amd._lib import RiseStencilSchedule, RiseTile

    p = tmp_path / "tune.txt"
    p.write_text("garbage line\nstencil gfx000 10 10 5 1 8 1.0\n")
    before = RiseTile()
    assert lib.rise_set_tune_cache(None) == 0
    assert lib.rise_gemm_default_tile(4096, 4096, 4096, 0, ctypes.byref(before)) == 0
    assert lib.rise_set_tune_cache(str(p).encode()) == 0
    t = RiseTile()
    assert lib.rise_gemm_default_tile(4096, 4096, 4096, 0, ctypes.byref(t)) == 0
    assert (t.bm, t.bn, t.bk) == (before.bm, before.bn, before.bk)
    sc = RiseStencilSchedule()
    assert lib.rise_stencil2d_default_schedule(4096, 4096, 5, 5, ctypes.byref(sc)) == 0
    assert lib.rise_set_tune_cache(None) == 0
