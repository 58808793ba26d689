"""Pins of the oracle gradients (adjoints of the bilinear GEMM, stencil and layer).

GEMM and the stencils are bilinear, so central finite differences of
L = <G, f(X)> are exact up to rounding for any step; the adjoint (dot-product)
identity <f(x), y> = <x, f^T(y)> is checked too, and torch float64 autograd is
the library cross-check.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
import rise_inputs as ri
from oracle import PAD_CLAMP, PAD_ZERO


def fd_grad(fun, X, h=0.5):
    """Central differences of a scalar function of a float64 array (exact for
    quadratic functions up to rounding)."""
    g = np.zeros_like(X)
    it = np.nditer(X, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        Xp = X.copy()
        Xm = X.copy()
        Xp[i] += h
        Xm[i] -= h
        g[i] = (fun(Xp) - fun(Xm)) / (2 * h)
    return g


def test_gemm_gradients_by_definition_and_fd():
    # dA = dC . B^T and dB = A^T . dC, written with the oracle's transposed views
    g = ri.rng(41)
    A = ri.uniform_matrix(g, 5, 4)
    B = ri.uniform_matrix(g, 4, 3)
    G = ri.uniform_matrix(g, 5, 3)
    dA = oracle.gemm(G, np.ascontiguousarray(B), opB=1)  # reads B^T through transpose
    dB = oracle.gemm(np.ascontiguousarray(A), G, opA=1)
    fA = lambda X: float((G.astype(np.float64) * oracle.gemm(X, B.astype(np.float64))).sum())
    fB = lambda X: float((G.astype(np.float64) * oracle.gemm(A.astype(np.float64), X)).sum())
    np.testing.assert_allclose(dA, fd_grad(fA, A.astype(np.float64)), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(dB, fd_grad(fB, B.astype(np.float64)), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("mode", [PAD_CLAMP, PAD_ZERO])
@pytest.mark.parametrize("k", [3, 5])
def test_stencil_gradients_fd(mode, k):
    g = ri.rng(43)
    H, W = 6, 7
    img = ri.uniform_matrix(g, H, W, 0.0, 1.0)
    w = ri.uniform_matrix(g, k, k)
    G = ri.uniform_matrix(g, H, W)
    din, dw = oracle.stencil2d_backward(G, img, w, mode)
    Gd = G.astype(np.float64)
    f_in = lambda X: float((Gd * oracle.stencil2d(X, w, mode)).sum())
    # the oracle reads f32 weights; f_w perturbs them through a float64 image instead
    np.testing.assert_allclose(din, fd_grad(f_in, img.astype(np.float64)), rtol=1e-11,
                               atol=1e-12)
    ref_dw = np.zeros((k, k))
    for dy in range(k):
        for dx in range(k):
            e = np.zeros((k, k), dtype=np.float32)
            e[dy, dx] = 1.0
            ref_dw[dy, dx] = float((Gd * oracle.stencil2d(img, e, mode)).sum())
    np.testing.assert_allclose(dw, ref_dw, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("mode", [PAD_CLAMP, PAD_ZERO])
def test_stencil_adjoint_identity_and_library(mode):
    g = ri.rng(47)
    H, W, k = 17, 13, 5
    x = ri.uniform_matrix(g, H, W)
    y = ri.uniform_matrix(g, H, W)
    w = ri.uniform_matrix(g, k, k)
    lhs = float((oracle.stencil2d(x, w, mode) * y.astype(np.float64)).sum())
    din, _ = oracle.stencil2d_backward(y, x, w, mode, want_dw=False)
    rhs = float((x.astype(np.float64) * din).sum())
    assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(lhs))
    # torch autograd cross-check
    xt = torch.from_numpy(x).double().requires_grad_(True)
    wt = torch.from_numpy(w).double().requires_grad_(True)
    r = (k - 1) // 2
    if mode == PAD_CLAMP:
        out = F.conv2d(F.pad(xt[None, None], (r, r, r, r), mode="replicate"), wt[None, None])
    else:
        out = F.conv2d(xt[None, None], wt[None, None], padding=r)
    (out[0, 0] * torch.from_numpy(y).double()).sum().backward()
    din2, dw2 = oracle.stencil2d_backward(y, x, w, mode)
    np.testing.assert_allclose(din2, xt.grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(dw2, wt.grad.numpy(), rtol=1e-12, atol=1e-11)


def test_conv_gradients_library_and_fd():
    g = ri.rng(53)
    x = g.standard_normal(size=(2, 4, 5, 3)).astype(np.float32)
    w = g.standard_normal(size=(2, 3, 3, 3)).astype(np.float32)
    G = g.standard_normal(size=(2, 4, 5, 2)).astype(np.float32)
    din, dw = oracle.conv2d_backward(G, x, w, PAD_ZERO)
    xt = torch.from_numpy(x).double().permute(0, 3, 1, 2).requires_grad_(True)
    wt = torch.from_numpy(w).double().requires_grad_(True)
    out = F.conv2d(xt, wt, padding=1).permute(0, 2, 3, 1)
    (out * torch.from_numpy(G).double()).sum().backward()
    np.testing.assert_allclose(din, xt.grad.permute(0, 2, 3, 1).numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(dw, wt.grad.numpy(), rtol=1e-12, atol=1e-12)
    Gd = G.astype(np.float64)
    f_in = lambda X: float((Gd * oracle.conv2d(X, w, PAD_ZERO)).sum())
    np.testing.assert_allclose(din, fd_grad(f_in, x.astype(np.float64)), rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("kh,kw", [(3, 3), (5, 3)])
def test_conv_gradients_clamp_padding(kh, kw):
    # clamp (replicate) padding of the layer: torch float64 autograd through
    # F.pad(mode="replicate") + F.conv2d, and central differences in both the
    # input and the weights; the adjoint sends every out-of-range tap to the
    # nearest edge pixel, so edge pixels collect several taps
    g = ri.rng(61 + kh)
    x = g.standard_normal(size=(2, 4, 6, 3)).astype(np.float32)
    w = g.standard_normal(size=(2, 3, kh, kw)).astype(np.float32)
    G = g.standard_normal(size=(2, 4, 6, 2)).astype(np.float32)
    din, dw = oracle.conv2d_backward(G, x, w, PAD_CLAMP)
    ry, rx = (kh - 1) // 2, (kw - 1) // 2
    xt = torch.from_numpy(x).double().permute(0, 3, 1, 2).requires_grad_(True)
    wt = torch.from_numpy(w).double().requires_grad_(True)
    out = F.conv2d(F.pad(xt, (rx, rx, ry, ry), mode="replicate"), wt).permute(0, 2, 3, 1)
    (out * torch.from_numpy(G).double()).sum().backward()
    np.testing.assert_allclose(din, xt.grad.permute(0, 2, 3, 1).numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(dw, wt.grad.numpy(), rtol=1e-12, atol=1e-12)
    Gd = G.astype(np.float64)
    f_in = lambda X: float((Gd * oracle.conv2d(X, w, PAD_CLAMP)).sum())
    np.testing.assert_allclose(din, fd_grad(f_in, x.astype(np.float64)), rtol=1e-11, atol=1e-11)
    # the layer is linear in w: <dW, V> = <G, conv(x, V)> for any V (the oracle takes
    # f32 weights, so the identity replaces differences of perturbed weights)
    V = g.standard_normal(size=w.shape).astype(np.float32)
    lhs = float(np.sum(dw * V.astype(np.float64)))
    rhs = float((Gd * oracle.conv2d(x, V, PAD_CLAMP)).sum())
    assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(rhs))
    # clamping maps taps only onto the first/last row and column: there the
    # gradient differs from zero padding's, everywhere else it is the same
    din0, _ = oracle.conv2d_backward(G, x, w, PAD_ZERO)
    assert not np.allclose(din[:, 0, 0], din0[:, 0, 0])
    np.testing.assert_allclose(din[:, 1:-1, 1:-1], din0[:, 1:-1, 1:-1], rtol=1e-12, atol=1e-12)
