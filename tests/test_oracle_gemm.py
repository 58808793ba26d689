"""Pins of the oracle GEMM.

The oracle evaluates C = A |> map(aRow => transpose(B) |> map(bCol =>
zip(aRow, bCol) |> map(*) |> reduce(+, 0))), the paper's matrix-vector program
(Sec. IV, running example) mapped over the columns of B.  It is pinned here by
brute-force loops, closed forms, exact integer arithmetic, the MV index map of
the generated OpenCL kernel (Sec. V) and a torch float64 library cross-check.
"""
import numpy as np
import pytest
import torch

import oracle
import rise_inputs as ri


def brute_gemm(A, B):
    """Triple loop in Python floats (double), no library call."""
    M, K = A.shape
    _, N = B.shape
    C = np.zeros((M, N))
    for i in range(M):
        for j in range(N):
            s = 0.0
            for k in range(K):
                s += float(A[i, k]) * float(B[k, j])
            C[i, j] = s
    return C


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (3, 5, 7), (8, 4, 1), (5, 9, 16), (16, 3, 2)])
def test_matches_brute_force(M, N, K):
    g = ri.rng(7)
    A = ri.uniform_matrix(g, M, K)
    B = ri.uniform_matrix(g, K, N)
    C = oracle.gemm(A, B)
    np.testing.assert_allclose(C, brute_gemm(A, B), rtol=1e-13, atol=1e-13)


def test_identity_and_ones_closed_forms():
    g = ri.rng(3)
    B = ri.uniform_matrix(g, 6, 7)
    I = np.eye(6, dtype=np.float32)
    assert np.array_equal(oracle.gemm(I, B), B.astype(np.float64))
    ones_a = np.ones((4, 9), dtype=np.float32)
    ones_b = np.ones((9, 5), dtype=np.float32)
    assert np.array_equal(oracle.gemm(ones_a, ones_b), np.full((4, 5), 9.0))
    # A = 1 gives every row of C equal to the column sums of B
    Bc = ri.uniform_matrix(g, 9, 5)
    C = oracle.gemm(ones_a, Bc)
    colsum = np.array([sum(float(Bc[k, j]) for k in range(9)) for j in range(5)])
    for i in range(4):
        np.testing.assert_allclose(C[i], colsum, rtol=1e-14)


def test_integer_inputs_are_exact():
    g = ri.rng(11)
    A = ri.integer_matrix(g, 17, 33, bound=2)
    B = ri.integer_matrix(g, 33, 12, bound=2)
    exact = A.astype(np.int64) @ B.astype(np.int64)
    assert np.array_equal(oracle.gemm(A, B), exact.astype(np.float64))


def test_transposed_operands_read_the_transpose():
    g = ri.rng(5)
    A = ri.integer_matrix(g, 7, 4)
    B = ri.integer_matrix(g, 4, 6)
    ref = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    At = np.ascontiguousarray(A.T)
    Bt = np.ascontiguousarray(B.T)
    assert np.array_equal(oracle.gemm(At, B, opA=1), ref)
    assert np.array_equal(oracle.gemm(A, Bt, opB=1), ref)
    assert np.array_equal(oracle.gemm(At, Bt, opA=1, opB=1), ref)


def test_product_transpose_law():
    # (AB)^T = B^T A^T, bitwise on integer data
    g = ri.rng(13)
    A = ri.integer_matrix(g, 5, 8)
    B = ri.integer_matrix(g, 8, 3)
    lhs = oracle.gemm(A, B).T
    rhs = oracle.gemm(np.ascontiguousarray(B.T), np.ascontiguousarray(A.T))
    assert np.array_equal(lhs, rhs)


def test_n_equals_one_is_the_papers_mv_kernel():
    # The generated kernel (Sec. V, OpenCL listing) computes
    #   output[lId + s*wgId] = sum_i M[(i + lId*m) + m*s*wgId] * x[i]
    # over work-groups wgId < n/s and local ids lId < s (reading i += 1 for the
    # loop increment).  A GEMM with N = 1 must produce the same vector.
    n, m, s = 12, 7, 4
    g = ri.rng(17)
    M = ri.uniform_matrix(g, n, m)
    x = ri.uniform_matrix(g, m, 1)
    flatM = M.reshape(-1).astype(np.float64)
    xv = x.reshape(-1).astype(np.float64)
    output = np.zeros(n)
    for wgId in range(n // s):
        for lId in range(s):
            accum = 0.0
            for i in range(m):
                accum += flatM[(i + lId * m) + (m * s * wgId)] * xv[i]
            output[lId + s * wgId] = accum
    C = oracle.gemm(M, x)
    assert C.shape == (n, 1)
    np.testing.assert_allclose(C[:, 0], output, rtol=1e-14, atol=0)


@pytest.mark.parametrize("mt,nt,kt", [(1, 1, 1), (4, 2, 8), (8, 6, 4), (16, 12, 32)])
def test_tiled_form_equals_untiled(mt, nt, kt):
    g = ri.rng(19)
    A = ri.integer_matrix(g, 16, 32)
    B = ri.integer_matrix(g, 32, 12)
    assert np.array_equal(oracle.gemm_tiled(A, B, mt, nt, kt), oracle.gemm(A, B))
    Af = ri.uniform_matrix(g, 16, 32)
    Bf = ri.uniform_matrix(g, 32, 12)
    np.testing.assert_allclose(oracle.gemm_tiled(Af, Bf, mt, nt, kt), oracle.gemm(Af, Bf),
                               rtol=32 * 2.0 ** -52, atol=1e-14)


def test_tiled_form_rejects_non_divisible_split():
    A = np.ones((6, 8), dtype=np.float32)
    B = np.ones((8, 6), dtype=np.float32)
    with pytest.raises(oracle.OracleError):
        oracle.gemm_tiled(A, B, 4, 3, 4)


def test_k_zero_is_init():
    A = np.zeros((3, 0), dtype=np.float32)
    B = np.zeros((0, 4), dtype=np.float32)
    assert np.array_equal(oracle.gemm(A, B), np.zeros((3, 4)))


def test_library_cross_check_float64():
    A, B = ri.gemm_uniform(128, 128, 128, ri.SEED_GEMM_SMALL)
    ref = (torch.from_numpy(A).double() @ torch.from_numpy(B).double()).numpy()
    np.testing.assert_allclose(oracle.gemm(A, B), ref, rtol=1e-12, atol=1e-12)


def test_sampled_equals_full():
    g = ri.rng(23)
    A = ri.uniform_matrix(g, 33, 20)
    B = ri.uniform_matrix(g, 20, 17)
    full = oracle.gemm(A, B)
    rows, cols = ri.sample_indices(g, 33, 17, 40)
    assert np.array_equal(oracle.gemm_sampled(A, B, rows, cols), full[rows, cols])


def test_bf16_leaves_decode_exactly():
    g = ri.rng(29)
    A = ri.uniform_matrix(g, 9, 16)
    B = ri.uniform_matrix(g, 16, 5)
    Ab = ri.bf16_bits_from_f32(A)
    Bb = ri.bf16_bits_from_f32(B)
    Aw = oracle.bf16_bits_to_f32(Ab)
    Bw = oracle.bf16_bits_to_f32(Bb)
    np.testing.assert_array_equal(oracle.gemm(Ab, Bb), oracle.gemm(Aw, Bw))
