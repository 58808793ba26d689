"""GPU parity of the matrix-vector product (rise_gemv), the paper's running
example: y = A |> map(row => zip(row, x) |> map(*) |> reduce(+, 0)).  Bar: the
componentwise FP32 bound |y - y*| <= 1e-5 (|A| |x|) against the fp64 oracle (the
oracle's MV is its GEMM with N = 1, pinned to the index map of the paper's
generated matrix-vector kernel)."""
import numpy as np
import pytest

import oracle
import rise_inputs as ri
from _helpers import componentwise, dev, gemm_scale, host

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def rise():
    import paper_2201_03611_amd as rise

    return rise


def run(rise, A_stored, x, trans, lda=None, x_offset=0, M=None, K=None):
    import torch

    if M is None:
        M, K = (A_stored.shape[1], A_stored.shape[0]) if trans else A_stored.shape
    dA = dev(A_stored)
    xs = np.concatenate([np.zeros(x_offset, np.float32), x.reshape(-1)])
    dx = dev(xs)[x_offset:]
    y = torch.full((M,), float("nan"), device="cuda")
    op = rise.RISE_OP_T if trans else rise.RISE_OP_N
    n = rise.rise_gemv_workspace(M, K, op)
    ws = torch.empty(n, device="cuda", dtype=torch.uint8) if n else None
    print(f"gemv M={M} K={K} trans={trans} lda={lda} x_offset={x_offset}", flush=True)
    rise.rise_gemv(y, dA, dx, M, K, lda=lda or A_stored.shape[1], opA=op, ws=ws)
    return host(y)


@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("M,K", [(1, 1), (3, 5), (97, 300), (1000, 257), (4096, 1024),
                                 (257, 4097), (5, 20000)])
def test_gemv_vs_oracle(rise, trans, M, K):
    g = ri.rng(M * 31 + K + trans)
    A = ri.uniform_matrix(g, M, K)
    x = ri.uniform_matrix(g, K, 1)
    stored = np.ascontiguousarray(A.T) if trans else A
    y = run(rise, stored, x, trans)
    assert componentwise(y[:, None], oracle.gemm(A, x), gemm_scale(A, x)) <= TOL


@pytest.mark.parametrize("trans", [False, True])
def test_gemv_scalar_paths(rise, trans):
    # leading dimension not a multiple of 4 and a misaligned x: scalar loads
    g = ri.rng(77 + trans)
    M, K = 130, 203
    A = ri.uniform_matrix(g, M, K)
    x = ri.uniform_matrix(g, K, 1)
    stored = np.ascontiguousarray(A.T) if trans else A
    padded = np.zeros((stored.shape[0], stored.shape[1] + 3), np.float32)
    padded[:, :stored.shape[1]] = stored
    y = run(rise, padded, x, trans, lda=padded.shape[1], x_offset=1, M=M, K=K)
    assert componentwise(y[:, None], oracle.gemm(A, x), gemm_scale(A, x)) <= TOL


def test_gemv_integer_exact(rise):
    g = ri.rng(3)
    A = ri.integer_matrix(g, 500, 700, bound=3)
    x = ri.integer_matrix(g, 700, 1, bound=3)
    exact = (A.astype(np.int64) @ x.astype(np.int64)).astype(np.float32)[:, 0]
    assert np.array_equal(run(rise, A, x, False), exact)
    assert np.array_equal(run(rise, np.ascontiguousarray(A.T), x, True), exact)


def test_gemv_k_zero_writes_zero(rise):
    import torch

    y = torch.full((7,), 3.0, device="cuda")
    A = torch.empty((7, 0), device="cuda")
    x = torch.empty((0,), device="cuda")
    rise.rise_gemv(y, A, x, 7, 0, lda=1)
    assert np.array_equal(host(y), np.zeros(7, np.float32))


def test_gemv_equals_the_papers_mv_kernel(rise):
    # the index map of the paper's generated kernel: output[lId + s*wgId] =
    # sum_i M[(i + lId*m) + m*s*wgId] * x[i], evaluated in fp64 on the host
    n, m, s = 64, 33, 8
    g = ri.rng(17)
    M = ri.uniform_matrix(g, n, m)
    x = ri.uniform_matrix(g, m, 1)
    flatM, xv = M.reshape(-1).astype(np.float64), x.reshape(-1).astype(np.float64)
    ref = np.zeros(n)
    for wgId in range(n // s):
        for lId in range(s):
            ref[lId + s * wgId] = sum(flatM[(i + lId * m) + m * s * wgId] * xv[i] for i in range(m))
    y = run(rise, M, x, False)
    assert componentwise(y[:, None], ref[:, None], gemm_scale(M, x)) <= TOL


@pytest.mark.parametrize("trans", [False, True])
def test_gemv_16384_sampled(rise, trans):
    # the benchmark size and launch: 16384 x 16384 (1 GiB of A) drawn on the device
    # as the benchmark draws it; 200 sampled outputs plus the ends against the
    # oracle's MV (its GEMM with N = 1) on the same stored values
    import torch

    n = 16384
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1200 + trans)
    dA = torch.rand((n, n), device="cuda", generator=gen) * 2 - 1
    dx = torch.rand((n,), device="cuda", generator=gen) * 2 - 1
    y = torch.empty(n, device="cuda")
    op = rise.RISE_OP_T if trans else rise.RISE_OP_N
    nws = rise.rise_gemv_workspace(n, n, op)
    ws = torch.empty(nws, device="cuda", dtype=torch.uint8) if nws else None
    print(f"gemv {n} trans={trans} parts={rise.rise_gemv_parts(n, n, op)}", flush=True)
    rise.rise_gemv(y, dA, dx, n, n, lda=n, opA=op, ws=ws)
    rows = np.concatenate([ri.sample_indices(ri.rng(5), n, 1, 200)[0], [1, n - 2]])
    zeros = np.zeros_like(rows)
    Ah, xh, yh = host(dA), host(dx).reshape(n, 1), host(y)
    ref = oracle.gemm_sampled(Ah, xh, rows, zeros, opA=int(trans))
    scale = oracle.gemm_sampled(np.abs(Ah), np.abs(xh), rows, zeros, opA=int(trans))
    assert componentwise(yh[rows], ref, scale) <= TOL


@pytest.mark.parametrize("M,K", [(1000, 40000), (3000, 12001)])
def test_gemv_transposed_wide_split(rise, M, K):
    # grids of at least two workgroups per compute unit take the split-K kernel
    # with two rows of loads in flight per thread (the 16384^2 launch runs it too)
    parts = rise.rise_gemv_parts(M, K, rise.RISE_OP_T)
    mblocks = (M + 1023) // 1024
    assert mblocks * parts >= 2 * 256, (M, K, parts)
    g = ri.rng(M + K)
    A = ri.uniform_matrix(g, M, K)
    x = ri.uniform_matrix(g, K, 1)
    y = run(rise, np.ascontiguousarray(A.T), x, True)
    assert componentwise(y[:, None], oracle.gemm(A, x), gemm_scale(A, x)) <= TOL
