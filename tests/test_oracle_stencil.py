"""Pins of the oracle 2D stencil and the multi-channel stencil layer.

The oracle evaluates in |> pad2D |> slide2D(k, 1) |> map(map(weighted reduce))
(pad/slide are paper-silent: clamp = replicate the nearest edge pixel, zero =
constant 0; cross-correlation order).  Pins: direct window sums written with
explicit clamp loops, closed forms on dyadic data (exact), and torch float64
library cross-checks (replicate pad + conv2d, which is a cross-correlation).
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
import rise_inputs as ri
from oracle import PAD_CLAMP, PAD_ZERO


def brute_stencil(img, w, mode):
    H, W = img.shape
    kh, kw = w.shape
    rh, rw = (kh - 1) // 2, (kw - 1) // 2
    out = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            s = 0.0
            for dy in range(kh):
                for dx in range(kw):
                    yy, xx = y + dy - rh, x + dx - rw
                    if mode == PAD_CLAMP:
                        yy = min(max(yy, 0), H - 1)
                        xx = min(max(xx, 0), W - 1)
                        v = float(img[yy, xx])
                    else:
                        v = float(img[yy, xx]) if (0 <= yy < H and 0 <= xx < W) else 0.0
                    s += v * float(w[dy, dx])
            out[y, x] = s
    return out


@pytest.mark.parametrize("mode", [PAD_CLAMP, PAD_ZERO])
@pytest.mark.parametrize("H,W,kh,kw", [(1, 1, 3, 3), (5, 7, 3, 3), (6, 4, 5, 5), (3, 9, 7, 3),
                                       (8, 8, 1, 1), (2, 3, 7, 7)])
def test_matches_brute_force(mode, H, W, kh, kw):
    g = ri.rng(101)
    img = ri.uniform_matrix(g, H, W, 0.0, 1.0)
    w = ri.uniform_matrix(g, kh, kw)  # asymmetric weights catch a flipped kernel
    np.testing.assert_allclose(oracle.stencil2d(img, w, mode), brute_stencil(img, w, mode),
                               rtol=1e-13, atol=1e-14)


def test_constant_image_binomial_kernel_is_exact():
    b = np.array([1, 4, 6, 4, 1], dtype=np.float64)
    w = (np.outer(b, b) / 256.0).astype(np.float32)  # dyadic, sums to exactly 1
    img = np.full((9, 11), 0.375, dtype=np.float32)
    assert np.array_equal(oracle.stencil2d(img, w, PAD_CLAMP), np.full((9, 11), 0.375))


def test_delta_kernel_is_identity_and_shifted_delta_is_clamped_shift():
    g = ri.rng(5)
    img = ri.uniform_matrix(g, 6, 7, 0.0, 1.0)
    d = np.zeros((5, 5), dtype=np.float32)
    d[2, 2] = 1.0
    assert np.array_equal(oracle.stencil2d(img, d, PAD_CLAMP), img.astype(np.float64))
    s = np.zeros((5, 5), dtype=np.float32)
    s[0, 4] = 1.0  # reads (y - 2, x + 2), clamped
    out = oracle.stencil2d(img, s, PAD_CLAMP)
    H, W = img.shape
    for y in range(H):
        for x in range(W):
            assert out[y, x] == img[max(y - 2, 0), min(x + 2, W - 1)]
    outz = oracle.stencil2d(img, s, PAD_ZERO)
    for y in range(H):
        for x in range(W):
            ref = img[y - 2, x + 2] if (y - 2 >= 0 and x + 2 < W) else 0.0
            assert outz[y, x] == ref


def test_symmetric_normalised_kernel_preserves_interior_ramp():
    w = ri.gaussian_weights(5, 1.0)
    H, W = 12, 14
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    img = (0.25 * yy + 0.5 * xx).astype(np.float32)
    out = oracle.stencil2d(img, w, PAD_CLAMP)
    s = float(w.astype(np.float64).sum())
    interior = out[2:-2, 2:-2]
    np.testing.assert_allclose(interior, s * img[2:-2, 2:-2].astype(np.float64), rtol=1e-12,
                               atol=1e-12)


def test_gaussian_weights_reading():
    w = ri.gaussian_weights(5, 1.0)
    assert w.shape == (5, 5) and w.dtype == np.float32
    assert abs(float(w.astype(np.float64).sum()) - 1.0) < 1e-6
    assert np.array_equal(w, w.T) and np.array_equal(w, w[::-1, ::-1])
    assert w[2, 2] == w.max()


@pytest.mark.parametrize("k", [3, 5, 7])
def test_library_cross_check_replicate_pad(k):
    g = ri.rng(17)
    img = ri.uniform_matrix(g, 23, 19, 0.0, 1.0)
    w = ri.uniform_matrix(g, k, k)
    r = (k - 1) // 2
    t = torch.from_numpy(img).double()[None, None]
    ref = F.conv2d(F.pad(t, (r, r, r, r), mode="replicate"),
                   torch.from_numpy(w).double()[None, None])[0, 0].numpy()
    np.testing.assert_allclose(oracle.stencil2d(img, w, PAD_CLAMP), ref, rtol=1e-12, atol=1e-13)
    refz = F.conv2d(t, torch.from_numpy(w).double()[None, None], padding=r)[0, 0].numpy()
    np.testing.assert_allclose(oracle.stencil2d(img, w, PAD_ZERO), refz, rtol=1e-12, atol=1e-13)


def test_rejects_even_kernel():
    with pytest.raises(oracle.OracleError):
        oracle.stencil2d(np.zeros((4, 4), np.float32), np.zeros((4, 4), np.float32))


def test_image_smaller_than_kernel_clamps():
    img = np.array([[2.0, 3.0]], dtype=np.float32)
    w = np.ones((5, 5), dtype=np.float32)
    out = oracle.stencil2d(img, w, PAD_CLAMP)
    # column x=0 window reads x-2..x+2 clamped -> [2,2,2,3,3], five rows identical
    assert np.array_equal(out, np.array([[5 * 12.0, 5 * 13.0]]))


def brute_conv(x, w, mode=PAD_ZERO):
    B, H, W, Cin = x.shape
    Cout = w.shape[0]
    out = np.zeros((B, H, W, Cout))
    for b in range(B):
        for co in range(Cout):
            for ci in range(Cin):
                out[b, :, :, co] += brute_stencil(x[b, :, :, ci], w[co, ci], mode)
    return out


def test_conv_matches_brute_force_and_library():
    g = ri.rng(31)
    x = g.standard_normal(size=(2, 5, 6, 3)).astype(np.float32)
    w = g.standard_normal(size=(4, 3, 3, 3)).astype(np.float32)
    got = oracle.conv2d(x, w, PAD_ZERO)
    np.testing.assert_allclose(got, brute_conv(x, w), rtol=1e-12, atol=1e-12)
    xt = torch.from_numpy(x).double().permute(0, 3, 1, 2)
    ref = F.conv2d(xt, torch.from_numpy(w).double(), padding=1).permute(0, 2, 3, 1).numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_conv_single_channel_equals_stencil():
    g = ri.rng(37)
    img = ri.uniform_matrix(g, 7, 9, 0.0, 1.0)
    w = ri.uniform_matrix(g, 5, 5)
    got = oracle.conv2d(img[None, :, :, None], w[None, None], PAD_CLAMP)[0, :, :, 0]
    assert np.array_equal(got, oracle.stencil2d(img, w, PAD_CLAMP))
