"""The strategy queries report what the library runs: a call with the reported
tile or schedule passed explicitly gives the same bits as the call that leaves
the choice to the library (same kernel, same order of additions), and the
result of the default call is within the parity bar of the oracle.  Shapes are
chosen so that the default differs between them (several GEMM tiles, 5x5 and
7x7 stencil rows, one- and multi-pass tree reductions)."""
import numpy as np
import pytest

import oracle
import rise_inputs as ri
from _helpers import componentwise, dev, gemm_scale, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rise():
    import paper_2201_03611_amd as rise

    return rise


@pytest.mark.parametrize("mnk", [(1024, 1024, 300), (520, 260, 96), (100, 70, 33)])
@pytest.mark.parametrize("mode", ["f32", "bf16x3", "fp8"])
def test_gemm_default_tile_is_what_runs(rise, mnk, mode):
    M, N, K = mnk
    A, B = ri.gemm_uniform(M, N, K, 4100 + M)
    tile = rise.rise_gemm_default_tile(M, N, K, mode)
    print(f"strategy gemm {mnk} mode={mode} default tile {tile}", flush=True)
    want = host(rise.gemm(dev(A), dev(B), mode=mode))
    got = host(rise.gemm(dev(A), dev(B), mode=mode, tile=tile))
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    if mode == "f32":
        assert componentwise(want, oracle.gemm(A, B), gemm_scale(A, B)) <= 1e-5


@pytest.mark.parametrize("k", [3, 5, 7])
def test_stencil_default_schedule_is_what_runs(rise, k):
    H, W = 300, 517
    img = ri.image_uniform(H, W, 4200 + k)
    w = ri.gaussian_weights(k)
    sched = rise.rise_stencil2d_default_schedule(H, W, k, k)
    print(f"strategy stencil k={k} default schedule {sched}", flush=True)
    want = host(rise.stencil2d(dev(img), dev(w)))
    got = host(rise.stencil2d(dev(img), dev(w), schedule=sched))
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    # Gaussian weights and inputs in [0, 1): (|w| * |window|) is at most 1 per output
    assert np.max(np.abs(want - oracle.stencil2d(img, w))) <= 1e-5


@pytest.mark.parametrize("n,m,k", [(2, 3, 20), (4, 2, 5), (2, 1, 14)])
def test_iterate_sum_pass_plan(rise, n, m, k):
    # the workspace exists exactly when the plan has more than one pass, and the
    # result is the oracle's bit for bit whatever the plan
    import torch

    rounds = rise.rise_iterate_sum_passes(n, m, k)
    print(f"strategy iterate_sum n={n} m={m} k={k} rounds per pass {rounds}", flush=True)
    assert sum(rounds) == k
    assert (len(rounds) > 1) == (rise.rise_iterate_sum_workspace(n, m, k) > 0)
    x = ri.uniform_matrix(ri.rng(4300 + k), 1, m * n ** k).reshape(-1)
    got = host(rise.iterate_sum(torch.from_numpy(x).cuda(), n, k))
    want = oracle.iterate_sum(x, n, m, k, binary32=True).astype(np.float32)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
