"""rise_gemv_noalloc, the matrix-vector entry point that allocates nothing,
against rise_gemv (the entry point with a caller workspace) through the C ABI.

Both run the same kernels in the same order, so the results must agree bit for
bit; each is also held to the componentwise FP32 bar (1e-5 of (|A| |x|)_i)
against the fp64 oracle.  Two calls in a row, the second smaller, check that
the second call does not depend on what the first left in the shared scratch.
"""
import numpy as np
import pytest

import oracle
import rise_inputs as ri
from _helpers import componentwise, dev, host

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def rise():
    import paper_2201_03611_amd as rise

    return rise


def both(rise, A_stored, x, trans):
    import torch

    M, K = (A_stored.shape[1], A_stored.shape[0]) if trans else A_stored.shape
    op = rise.RISE_OP_T if trans else rise.RISE_OP_N
    dA, dx = dev(A_stored), dev(x)
    y_ws = torch.full((M,), float("nan"), device="cuda")
    y_na = torch.full((M,), float("nan"), device="cuda")
    n = rise.rise_gemv_workspace(M, K, op)
    ws = torch.empty(n, device="cuda", dtype=torch.uint8) if n else None
    parts = rise.rise_gemv_parts(M, K, op)
    print(f"gemv_noalloc M={M} K={K} trans={trans} parts={parts} ws={n}", flush=True)
    rise.rise_gemv(y_ws, dA, dx, M, K, lda=A_stored.shape[1], opA=op, ws=ws)
    rise.rise_gemv_noalloc(y_na, dA, dx, M, K, lda=A_stored.shape[1], opA=op)
    torch.cuda.synchronize()
    A = A_stored.T if trans else A_stored
    ref = oracle.gemm(A, x.reshape(-1, 1)).reshape(-1)
    scale = oracle.gemm(np.abs(A), np.abs(x).reshape(-1, 1)).reshape(-1)
    return host(y_ws), host(y_na), ref, scale, parts


@pytest.mark.parametrize("trans", [True, False])
def test_noalloc_equals_workspace_call_twice_second_smaller(rise, trans):
    g = ri.rng(91)
    for (M, K) in [(3000, 5000), (700, 1300)]:
        A_stored = ri.uniform_matrix(g, K, M) if trans else ri.uniform_matrix(g, M, K)
        x = ri.uniform_matrix(g, 1, K).reshape(-1)
        y_ws, y_na, ref, scale, parts = both(rise, A_stored, x, trans)
        if trans:
            assert parts > 1  # the transposed product goes through the scratch
        assert np.array_equal(y_ws.view(np.uint32), y_na.view(np.uint32))
        assert componentwise(y_na, ref, scale) <= TOL
