"""GPU parity of rise_gemm against the oracle.

Bar: FP32 mode within 1e-5 componentwise, |c_hat - c| <= 1e-5 (|A| |B|)_ij; the
reduced-precision modes within the same bound against the oracle's evaluation
of that mode's arithmetic (the value the mode defines); integer-valued inputs,
whose sums are exact in any order, bit for bit.
"""
import numpy as np
import pytest

import oracle
import rise_inputs as ri
from _helpers import componentwise, dev, gemm_scale, gemm_scale_sampled, host

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5


@pytest.fixture(scope="module")
def rise():
    import paper_2201_03611_amd as rise

    return rise


def run(rise, A, B, transA=False, transB=False, mode="f32", tile=None):
    print(f"gemm A{A.shape} B{B.shape} tA={transA} tB={transB} mode={mode} tile={tile}",
          flush=True)
    out = rise.gemm(dev(A), dev(B), transA=transA, transB=transB, mode=mode, tile=tile)
    return host(out)


def test_config_128_cubed_uniform(rise):
    A, B = ri.gemm_uniform(128, 128, 128, ri.SEED_GEMM_SMALL)
    C = run(rise, A, B)
    assert componentwise(C, oracle.gemm(A, B), gemm_scale(A, B)) <= TOL_F32


@pytest.mark.parametrize("tile", [(128, 128, 32), (128, 64, 32), (64, 128, 32), (64, 64, 32),
                                  (256, 128, 16)])
@pytest.mark.parametrize("ops", [(False, False), (False, True), (True, False), (True, True)])
def test_integer_exact_all_tiles_and_ops(rise, tile, ops):
    g = ri.rng(hash((tile, ops)) % 1000)
    M, N, K = 200, 136, 70  # ragged in all three dimensions for every tile
    A = ri.integer_matrix(g, M, K, bound=3)
    B = ri.integer_matrix(g, K, N, bound=3)
    As = np.ascontiguousarray(A.T) if ops[0] else A
    Bs = np.ascontiguousarray(B.T) if ops[1] else B
    C = run(rise, As, Bs, transA=ops[0], transB=ops[1], tile=tile)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)
    assert np.array_equal(C, exact)


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (1, 7, 3), (33, 65, 17), (64, 64, 64),
                                   (257, 129, 300), (31, 1000, 5)])
def test_ragged_uniform(rise, M, N, K):
    g = ri.rng(M * 7 + N * 3 + K)
    A = ri.uniform_matrix(g, M, K)
    B = ri.uniform_matrix(g, K, N)
    C = run(rise, A, B)
    assert componentwise(C, oracle.gemm(A, B), gemm_scale(A, B)) <= TOL_F32


def test_unaligned_leading_dimension_uses_scalar_loads(rise):
    import torch

    g = ri.rng(5)
    M, N, K = 70, 50, 45
    Abig = ri.uniform_matrix(g, M, K + 3)
    A = Abig[:, :K]
    B = ri.uniform_matrix(g, K, N)
    dA = dev(Abig)
    dB = dev(B)
    C = torch.empty((M, N), device="cuda", dtype=torch.float32)
    rise.rise_gemm(C, dA, dB, M, N, K, lda=K + 3, ldb=N, ldc=N)
    assert componentwise(host(C), oracle.gemm(np.ascontiguousarray(A), B), gemm_scale(
        np.ascontiguousarray(A), B)) <= TOL_F32


@pytest.mark.parametrize("ops", [(False, False), (False, True), (True, False), (True, True)])
@pytest.mark.parametrize("M,N,K", [(70, 50, 45), (130, 257, 131), (5, 3, 2)])
def test_padded_rows_ragged_edges_every_tile(rise, ops, M, N, K):
    # 16-byte rows (leading dimensions multiples of 4) with ragged M, N, K: the
    # vector loads reach into each row's padding, which holds NaN here, so any
    # element read past the operand and not zeroed would poison the result
    import torch

    g = ri.rng(M + N + K + 7 * ops[0] + 11 * ops[1])
    A = ri.uniform_matrix(g, M, K)
    B = ri.uniform_matrix(g, K, N)

    def padded(X):
        r, c = X.shape
        P = np.full((r, (c + 3) // 4 * 4 + 4), np.nan, np.float32)
        P[:, :c] = X
        return P

    As = padded(np.ascontiguousarray(A.T) if ops[0] else A)
    Bs = padded(np.ascontiguousarray(B.T) if ops[1] else B)
    dA, dB = dev(As), dev(Bs)
    ref = oracle.gemm(A, B)
    for tile in rise.rise_gemm_tiles("f32"):
        C = torch.empty((M, N), device="cuda", dtype=torch.float32)
        rise.rise_gemm(C, dA, dB, M, N, K, lda=As.shape[1], ldb=Bs.shape[1], ldc=N,
                       opA=int(ops[0]), opB=int(ops[1]), tile=tile)
        assert componentwise(host(C), ref, gemm_scale(A, B)) <= TOL_F32, tile


@pytest.mark.parametrize("ops", [(False, False), (False, True), (True, False), (True, True)])
@pytest.mark.parametrize("M,N,K", [(260, 132, 48), (300, 200, 16), (516, 388, 272),
                                   (4, 4, 16)])
def test_async_ring_ragged_mn_integer_exact(rise, ops, M, N, K):
    # K a multiple of 16 with 16-byte rows: the 256 x 128 x 16 tile runs the
    # asynchronous-ring schedule (rows and chunks past M and N are fetched from
    # the last valid ones and only feed outputs that are not stored); integer
    # inputs make every summation order exact, so the result is bit for bit
    g = ri.rng(M + 3 * N + 7 * K + 11 * ops[0] + 13 * ops[1])
    A = ri.integer_matrix(g, M, K, bound=3)
    B = ri.integer_matrix(g, K, N, bound=3)
    As = np.ascontiguousarray(A.T) if ops[0] else A
    Bs = np.ascontiguousarray(B.T) if ops[1] else B
    C = run(rise, As, Bs, transA=ops[0], transB=ops[1], tile=(256, 128, 16))
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)
    assert np.array_equal(C, exact)


@pytest.mark.parametrize("ops", [(False, False), (False, True), (True, False), (True, True)])
def test_async_ring_nan_padded_rows_oracle(rise, ops):
    # leading dimensions beyond the rows with NaN in the padding: a copy that
    # reached past a row (or a chunk past M or N not clamped) would poison C
    import torch

    M, N, K = 388, 260, 96
    g = ri.rng(17 + 2 * ops[0] + ops[1])
    A = ri.uniform_matrix(g, M, K)
    B = ri.uniform_matrix(g, K, N)

    def padded(X):
        r, c = X.shape
        P = np.full((r, c + 8), np.nan, np.float32)
        P[:, :c] = X
        return P

    As = padded(np.ascontiguousarray(A.T) if ops[0] else A)
    Bs = padded(np.ascontiguousarray(B.T) if ops[1] else B)
    C = torch.full((M, N), float("nan"), device="cuda", dtype=torch.float32)
    print(f"gemm async ring padded ops={ops}", flush=True)
    rise.rise_gemm(C, dev(As), dev(Bs), M, N, K, lda=As.shape[1], ldb=Bs.shape[1], ldc=N,
                   opA=int(ops[0]), opB=int(ops[1]), tile=(256, 128, 16))
    assert componentwise(host(C), oracle.gemm(A, B), gemm_scale(A, B)) <= TOL_F32


def test_k_zero_writes_zero(rise):
    import torch

    C = torch.full((5, 7), 3.0, device="cuda")
    A = torch.empty((5, 0), device="cuda")
    B = torch.empty((0, 7), device="cuda")
    rise.rise_gemm(C, A, B, 5, 7, 0, lda=1, ldb=7, ldc=7)
    assert np.array_equal(host(C), np.zeros((5, 7), np.float32))


def test_n_equals_one_is_mv(rise):
    # GEMM with N = 1 is the paper's matrix-vector program
    g = ri.rng(9)
    M = ri.uniform_matrix(g, 1000, 300)
    x = ri.uniform_matrix(g, 300, 1)
    y = run(rise, M, x)
    assert componentwise(y, oracle.gemm(M, x), gemm_scale(M, x)) <= TOL_F32


def test_config_4096_cubed_sampled(rise):
    # the timed FP32 workload, in the launch configuration the benchmark uses
    A, B = ri.gemm_uniform(4096, 4096, 4096, ri.SEED_GEMM_F32)
    C = run(rise, A, B)
    rows, cols = ri.sample_indices(ri.rng(77), 4096, 4096, 3000)
    ref = oracle.gemm_sampled(A, B, rows, cols)
    err = componentwise(C[rows, cols], ref, gemm_scale_sampled(A, B, rows, cols))
    print("4096^3 f32 componentwise max err", err)
    assert err <= TOL_F32
    assert np.all(np.isfinite(C))


# ---------------------------------------------------------------------------
# reduced-precision modes
# ---------------------------------------------------------------------------
MODES = {"bf16": oracle.MODE_BF16, "bf16x3": oracle.MODE_BF16X3, "bf16x6": oracle.MODE_BF16X6,
         "fp8": oracle.MODE_FP8}


@pytest.mark.parametrize("mode", list(MODES))
def test_modes_integer_exact(rise, mode):
    g = ri.rng(21)
    M, N, K = 300, 260, 200
    A = ri.integer_matrix(g, M, K, bound=2)
    B = ri.integer_matrix(g, K, N, bound=2)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)
    for tile in rise.rise_gemm_tiles(mode):
        C = run(rise, A, B, mode=mode, tile=tile)
        assert np.array_equal(C, exact), tile


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("K", [1, 16, 33, 96, 130])
def test_modes_short_k_every_tile(rise, mode, K):
    # fewer K slabs than the pipelines have stages, and ragged last slabs
    g = ri.rng(40 + K)
    M, N = 97, 260
    A = ri.integer_matrix(g, M, K, bound=2)
    B = ri.integer_matrix(g, K, N, bound=2)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)
    for tile in rise.rise_gemm_tiles(mode):
        C = run(rise, A, B, mode=mode, tile=tile)
        assert np.array_equal(C, exact), tile


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("ops", [(False, False), (True, True)])
def test_modes_match_mode_oracle(rise, mode, ops):
    M, N, K = 333, 290, 515
    A, B = ri.gemm_scaled_normal(M, N, K, ri.SEED_PRECISION)
    As = np.ascontiguousarray(A.T) if ops[0] else A
    Bs = np.ascontiguousarray(B.T) if ops[1] else B
    ref = oracle.gemm_mode(A, B, MODES[mode])
    for tile in rise.rise_gemm_tiles(mode):
        C = run(rise, As, Bs, transA=ops[0], transB=ops[1], mode=mode, tile=tile)
        err = componentwise(C, ref, gemm_scale(A, B))
        print(mode, tile, "err vs mode oracle", err, flush=True)
        assert err <= TOL_F32, tile


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("ops", [(False, False), (True, True)])
@pytest.mark.parametrize("pad", [4, 3])
def test_modes_padded_leading_dimensions_every_tile(rise, mode, ops, pad):
    # leading dimensions past the rows, NaN in the padding: pad 4 keeps 16-byte
    # rows (vector preparation), pad 3 forces the scalar one; both write the
    # row-major and the K-blocked operand layouts, which must agree bit for bit
    import torch

    M, N, K = 300, 270, 200
    g = ri.rng(101 + pad + 2 * ops[0])
    A = ri.integer_matrix(g, M, K, bound=2)
    B = ri.integer_matrix(g, K, N, bound=2)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)

    def padded(X):
        r, c = X.shape
        P = np.full((r, c + pad), np.nan, np.float32)
        P[:, :c] = X
        return P

    As = padded(np.ascontiguousarray(A.T) if ops[0] else A)
    Bs = padded(np.ascontiguousarray(B.T) if ops[1] else B)
    dA, dB = dev(As), dev(Bs)
    for tile in rise.rise_gemm_tiles(mode):
        C = torch.full((M, N), float("nan"), device="cuda", dtype=torch.float32)
        ws = torch.empty(rise.rise_gemm_workspace(M, N, K, mode, tile), device="cuda",
                         dtype=torch.uint8)
        print(f"gemm {mode} padded ld pad={pad} ops={ops} tile={tile}", flush=True)
        rise.rise_gemm(C, dA, dB, M, N, K, lda=As.shape[1], ldb=Bs.shape[1], ldc=N,
                       opA=int(ops[0]), opB=int(ops[1]), mode=mode, tile=tile, ws=ws)
        assert np.array_equal(host(C), exact), tile


def test_bf16_stored_operands(rise):
    import torch

    g = ri.rng(31)
    A = ri.uniform_matrix(g, 130, 96)
    B = ri.uniform_matrix(g, 96, 70)
    Ab = ri.bf16_bits_from_f32(A)
    Bb = ri.bf16_bits_from_f32(B)
    dA = dev(Ab).view(torch.bfloat16)
    dB = dev(Bb).view(torch.bfloat16)
    C = host(rise.gemm(dA, dB, mode="bf16"))
    ref = oracle.gemm(Ab, Bb)
    assert componentwise(C, ref, gemm_scale(oracle.bf16_bits_to_f32(Ab),
                                            oracle.bf16_bits_to_f32(Bb))) <= TOL_F32


def test_precision_config_sampled(rise):
    # 8192^3, N(0,1) 2^U(-4,4): every mode against its own definition on samples,
    # and the error of each mode against the exact product of the FP32 inputs
    A, B = ri.gemm_scaled_normal(8192, 8192, 8192, ri.SEED_PRECISION)
    rows, cols = ri.sample_indices(ri.rng(78), 8192, 8192, 600)
    exact = oracle.gemm_sampled(A, B, rows, cols)
    scale = gemm_scale_sampled(A, B, rows, cols)
    errs = {}
    for mode in ["f32"] + list(MODES):
        C = run(rise, A, B, mode=mode)[rows, cols]
        if mode != "f32":
            ref = oracle.gemm_mode(A, B, MODES[mode], rows, cols)
            assert componentwise(C, ref, scale) <= TOL_F32, mode
        errs[mode] = componentwise(C, exact, scale)
    print("componentwise error vs exact product:", errs, flush=True)
    assert errs["f32"] <= TOL_F32 and errs["bf16x3"] <= TOL_F32 and errs["bf16x6"] <= TOL_F32
    assert errs["bf16"] <= 2.0 ** -7 and errs["fp8"] <= 2.0 ** -3
