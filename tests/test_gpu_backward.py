"""GPU parity of the adjoint kernels (rise_gemm_backward, rise_stencil2d_backward)
and the autograd wrappers, against the oracle gradients and finite differences.

Bar: componentwise 1e-5 against the oracle, with the scale the same adjoint
applied to absolute values; at full size sampled outputs plus a directional
finite-difference identity (the maps are bilinear, so it holds up to rounding).
"""
import numpy as np
import pytest

import oracle
import rise_inputs as ri
from _helpers import componentwise, dev, host

pytestmark = pytest.mark.gpu
TOL = 1e-5
PADS = {"clamp": oracle.PAD_CLAMP, "zero": oracle.PAD_ZERO}


@pytest.fixture(scope="module")
def rise():
    import paper_2201_03611_amd as rise

    return rise


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (33, 65, 17), (200, 136, 70), (128, 128, 128)])
@pytest.mark.parametrize("mode", ["f32", "bf16x3"])
def test_gemm_backward_vs_oracle(rise, M, N, K, mode):
    print(f"gemm_backward M={M} N={N} K={K} mode={mode}", flush=True)
    g = ri.rng(M + N + K)
    A = ri.uniform_matrix(g, M, K)
    B = ri.uniform_matrix(g, K, N)
    G = ri.uniform_matrix(g, M, N)
    dA, dB = rise.gemm_backward(dev(G), dev(A), dev(B), mode=mode)
    refA = oracle.gemm(G, np.ascontiguousarray(B), opB=1)
    refB = oracle.gemm(np.ascontiguousarray(A), G, opA=1)
    sA = oracle.gemm(np.abs(G), np.abs(B), opB=1)
    sB = oracle.gemm(np.abs(A), np.abs(G), opA=1)
    assert componentwise(host(dA), refA, sA) <= TOL
    assert componentwise(host(dB), refB, sB) <= TOL


def test_gemm_backward_integer_exact(rise):
    g = ri.rng(3)
    A = ri.integer_matrix(g, 97, 64)
    B = ri.integer_matrix(g, 64, 45)
    G = ri.integer_matrix(g, 97, 45)
    dA, dB = rise.gemm_backward(dev(G), dev(A), dev(B))
    iA, iB, iG = (x.astype(np.int64) for x in (A, B, G))
    assert np.array_equal(host(dA), (iG @ iB.T).astype(np.float32))
    assert np.array_equal(host(dB), (iA.T @ iG).astype(np.float32))


def test_gemm_backward_4096_sampled_and_directional(rise):
    import torch

    n = 4096
    g = ri.rng(ri.SEED_GEMM_BWD)
    A = ri.uniform_matrix(g, n, n)
    B = ri.uniform_matrix(g, n, n)
    G = ri.uniform_matrix(g, n, n)
    print("gemm_backward 4096^3", flush=True)
    dA, dB = rise.gemm_backward(dev(G), dev(A), dev(B))
    dA, dB = host(dA), host(dB)
    rows, cols = ri.sample_indices(ri.rng(5), n, n, 1000)
    refA = oracle.gemm_sampled(G, B, rows, cols, opB=1)
    sA = oracle.gemm_sampled(np.abs(G), np.abs(B), rows, cols, opB=1)
    refB = oracle.gemm_sampled(A, G, rows, cols, opA=1)
    sB = oracle.gemm_sampled(np.abs(A), np.abs(G), rows, cols, opA=1)
    assert componentwise(dA[rows, cols], refA, sA) <= TOL
    assert componentwise(dB[rows, cols], refB, sB) <= TOL
    # directional check: L(A) = <G, A B> is linear in A, so (L(A+hV) - L(A-hV)) / 2h = <G, V B>
    # must equal <dA, V>; V B runs on the GPU forward kernel
    V = ri.uniform_matrix(ri.rng(6), n, n)
    VB = host(rise.gemm(dev(V), dev(B))).astype(np.float64)
    fd = float(np.sum(G.astype(np.float64) * VB))
    lin = float(np.sum(dA.astype(np.float64) * V))
    scale = float(np.sum(np.abs(G.astype(np.float64)) * np.abs(VB))) + 1.0
    assert abs(fd - lin) <= 1e-6 * scale, (fd, lin)


def test_autograd_gemm(rise):
    import torch

    g = ri.rng(8)
    A = ri.uniform_matrix(g, 70, 50)
    B = ri.uniform_matrix(g, 50, 30)
    G = ri.uniform_matrix(g, 70, 30)
    tA = dev(A).requires_grad_(True)
    tB = dev(B).requires_grad_(True)
    C = rise.RiseGemmFn.apply(tA, tB)
    C.backward(dev(G))
    assert componentwise(host(C.detach()), oracle.gemm(A, B), oracle.gemm(np.abs(A), np.abs(B))) <= TOL
    assert componentwise(host(tA.grad), oracle.gemm(G, np.ascontiguousarray(B), opB=1),
                         oracle.gemm(np.abs(G), np.abs(B), opB=1)) <= TOL
    assert componentwise(host(tB.grad), oracle.gemm(np.ascontiguousarray(A), G, opA=1),
                         oracle.gemm(np.abs(A), np.abs(G), opA=1)) <= TOL


def stencil_bwd_case(rise, H, W, kh, kw, pad, seed):
    print(f"stencil_backward H={H} W={W} k={kh}x{kw} pad={pad}", flush=True)
    g = ri.rng(seed)
    img = ri.uniform_matrix(g, H, W, 0.0, 1.0)
    w = ri.uniform_matrix(g, kh, kw)
    G = ri.uniform_matrix(g, H, W)
    dIn, dW = rise.stencil2d_backward(dev(G), dev(img), dev(w), pad=pad)
    rin, rw = oracle.stencil2d_backward(G, img, w, PADS[pad])
    sin, sw = oracle.stencil2d_backward(np.abs(G), np.abs(img), np.abs(w), PADS[pad])
    assert componentwise(host(dIn), rin, sin) <= TOL
    assert componentwise(host(dW), rw, sw) <= TOL


@pytest.mark.parametrize("pad", list(PADS))
@pytest.mark.parametrize("H,W", [(1, 1), (2, 3), (5, 9), (33, 257), (70, 300), (100, 13)])
@pytest.mark.parametrize("k", [1, 3, 5, 7])
def test_stencil_backward_vs_oracle(rise, pad, H, W, k):
    stencil_bwd_case(rise, H, W, k, k, pad, H * 31 + W + k)


@pytest.mark.parametrize("kh,kw", [(9, 9), (3, 7), (15, 1)])
@pytest.mark.parametrize("pad", list(PADS))
def test_stencil_backward_other_windows(rise, kh, kw, pad):
    stencil_bwd_case(rise, 45, 77, kh, kw, pad, kh * 7 + kw)


def test_stencil_backward_4096(rise):
    H = W = 4096
    img = ri.image_uniform(H, W, ri.SEED_STENCIL)
    w = ri.gaussian_weights(5, 1.0)
    G = ri.uniform_matrix(ri.rng(12), H, W)
    print("stencil_backward 4096^2", flush=True)
    dIn, dW = rise.stencil2d_backward(dev(G), dev(img), dev(w), pad="clamp")
    rin, rw = oracle.stencil2d_backward(G, img, w, oracle.PAD_CLAMP)
    sin, sw = oracle.stencil2d_backward(np.abs(G), img, w, oracle.PAD_CLAMP)
    assert componentwise(host(dIn), rin, sin) <= TOL
    assert componentwise(host(dW), rw, sw) <= TOL


def test_autograd_stencil(rise):
    g = ri.rng(14)
    img = ri.uniform_matrix(g, 40, 70, 0.0, 1.0)
    w = ri.uniform_matrix(g, 5, 5)
    G = ri.uniform_matrix(g, 40, 70)
    ti = dev(img).requires_grad_(True)
    tw = dev(w).requires_grad_(True)
    out = rise.RiseStencil2dFn.apply(ti, tw, "zero")
    out.backward(dev(G))
    rin, rw = oracle.stencil2d_backward(G, img, w, oracle.PAD_ZERO)
    sin, sw = oracle.stencil2d_backward(np.abs(G), img, np.abs(w), oracle.PAD_ZERO)
    assert componentwise(host(ti.grad), rin, sin) <= TOL
    assert componentwise(host(tw.grad), rw, sw) <= TOL


def test_autograd_gemm_bf16_operands(rise):
    # mode "bf16" with bfloat16 operands: the backward products take the exactly
    # widened operands, round dC to bf16 as the mode does, and return gradients in
    # the operands' type (the oracle evaluates the same mode on the same values)
    import torch

    g = ri.rng(9)
    A = ri.uniform_matrix(g, 70, 48)
    B = ri.uniform_matrix(g, 48, 40)
    G = ri.uniform_matrix(g, 70, 40)
    Ab = oracle.bf16_bits_to_f32(ri.bf16_bits_from_f32(A)).reshape(A.shape)
    Bb = oracle.bf16_bits_to_f32(ri.bf16_bits_from_f32(B)).reshape(B.shape)
    tA = dev(Ab).to(torch.bfloat16).requires_grad_(True)
    tB = dev(Bb).to(torch.bfloat16).requires_grad_(True)
    C = rise.RiseGemmFn.apply(tA, tB, "bf16")
    C.backward(dev(G))
    assert tA.grad.dtype == torch.bfloat16 and tB.grad.dtype == torch.bfloat16
    refA = oracle.gemm_mode(G, np.ascontiguousarray(Bb.T), oracle.MODE_BF16)
    refB = oracle.gemm_mode(np.ascontiguousarray(Ab.T), G, oracle.MODE_BF16)
    # the gradient itself is rounded once to bf16 on return (relative 2^-8), on top of
    # the mode's FP32-accumulated product of bf16-rounded operands
    sA = oracle.gemm(np.abs(G), np.abs(Bb), opB=1)
    sB = oracle.gemm(np.abs(Ab), np.abs(G), opA=1)
    assert componentwise(host(tA.grad.float()), refA, sA) <= 2.0 ** -8 + TOL
    assert componentwise(host(tB.grad.float()), refB, sB) <= 2.0 ** -8 + TOL


def test_wrappers_on_a_side_stream(rise):
    # a wrapper called with stream= allocates its output and workspace on that
    # stream; the results equal the default-stream call bit for bit
    import torch

    g = ri.rng(10)
    A = dev(ri.uniform_matrix(g, 300, 200))
    B = dev(ri.uniform_matrix(g, 200, 260))
    img = dev(ri.uniform_matrix(g, 100, 300, 0.0, 1.0))
    w = dev(ri.gaussian_weights(5, 1.0))
    ref_c = rise.gemm(A, B, mode="bf16x3")
    ref_s = rise.stencil2d(img, w)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    for _ in range(3):
        c = rise.gemm(A, B, mode="bf16x3", stream=s)
        o = rise.stencil2d(img, w, stream=s)
    s.synchronize()
    assert torch.equal(c, ref_c) and torch.equal(o, ref_s)
