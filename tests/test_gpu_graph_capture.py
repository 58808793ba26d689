"""Multi-launch entry points under HIP graph capture: rise_iterate_sum (two
kernel passes through the workspace double buffer), rise_stencil2d_iterate
(one launch per step, fused steps, and the zero-step copy) and the transposed
rise_gemv (split-K partials, then their reduction) are captured once on
a side stream with torch's graph API and replayed several times, with eager
work and synchronisations between the replays; every replay must reproduce the
eager result bit for bit (same kernels, same order of additions).  The inputs
are rewritten between replays, so a replay that read stale data would differ."""
import numpy as np
import pytest

import rise_inputs as ri
from _helpers import host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rise():
    import paper_2201_03611_amd as rise

    return rise


def capture(torch, fn):
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn(s)  # warm-up on the capture stream
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            fn(s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    return g


def test_iterate_sum_replays(rise):
    import torch

    n, m, k = 2, 3, 20  # two passes
    x = torch.empty(m * n ** k, device="cuda")
    out = torch.empty(m, device="cuda")
    ws = torch.empty(rise.rise_iterate_sum_workspace(n, m, k), device="cuda", dtype=torch.uint8)
    print(f"graph capture iterate_sum n={n} m={m} k={k}", flush=True)
    g = capture(torch, lambda s: rise.rise_iterate_sum(out, x, n, m, k, ws=ws, stream=s))
    for rep in range(3):
        vals = torch.from_numpy(ri.uniform_matrix(ri.rng(9500 + rep), 1, x.numel()).reshape(-1))
        x.copy_(vals.cuda())
        want = rise.iterate_sum(x, n, k)  # eager, on the current stream
        torch.cuda.synchronize()
        out.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(out).view(np.uint32), host(want).view(np.uint32)), rep


@pytest.mark.parametrize("k,steps,fuse", [(5, 3, 1), (3, 6, 4), (5, 5, 2), (5, 0, 0)])
def test_stencil_iterate_replays(rise, k, steps, fuse):
    import torch

    H, W = 300, 520
    img = torch.empty((H, W), device="cuda")
    w = torch.from_numpy(ri.gaussian_weights(k)).cuda()
    out = torch.empty((H, W), device="cuda")
    need = rise.rise_stencil2d_iterate_workspace(H, W, k, k, steps, fuse)
    ws = torch.empty(max(need, 1), device="cuda", dtype=torch.uint8)
    print(f"graph capture stencil_iterate k={k} steps={steps} fuse={fuse}", flush=True)
    g = capture(torch, lambda s: rise.rise_stencil2d_iterate(
        out, img, w, H, W, ld_out=W, ld_in=W, kh=k, kw=k, steps=steps, fuse=fuse, ws=ws,
        stream=s))
    for rep in range(3):
        img.copy_(torch.from_numpy(ri.image_uniform(H, W, 9600 + rep)).cuda())
        want = rise.stencil2d_iterate(img, w, steps, fuse=fuse)
        torch.cuda.synchronize()
        out.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(out).view(np.uint32), host(want).view(np.uint32)), rep


def test_gemv_transposed_replays(rise):
    # split-K partials in the workspace, then the fixed-order reduction kernel
    import torch

    M, K = 3000, 20000
    A = torch.empty((K, M), device="cuda")
    x = torch.empty(K, device="cuda")
    y = torch.empty(M, device="cuda")
    ws = torch.empty(max(rise.rise_gemv_workspace(M, K, rise.RISE_OP_T), 1), device="cuda",
                     dtype=torch.uint8)
    print(f"graph capture gemv transposed M={M} K={K}", flush=True)
    g = capture(torch, lambda s: rise.rise_gemv(y, A, x, M, K, lda=M, opA=rise.RISE_OP_T, ws=ws,
                                                stream=s))
    for rep in range(3):
        A.copy_(torch.from_numpy(ri.uniform_matrix(ri.rng(9700 + rep), K, M)).cuda())
        x.copy_(torch.from_numpy(ri.uniform_matrix(ri.rng(9800 + rep), 1, K).reshape(-1)).cuda())
        want = rise.gemv(A, x, transA=True)
        torch.cuda.synchronize()
        y.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(y).view(np.uint32), host(want).view(np.uint32)), rep
