"""Pins of the oracle's iterated stencil (iterate of Sec. VI with the stencil as
its size-preserving body).  Fixed by closed forms, not by the oracle: the
binomial window spreads a point into products of binomial coefficients (exact
dyadic values), a one-hot window moves the image by r per step (with clamp
padding applied at every step, the edge row or column repeats), a constant
image stays constant under weights that sum to one, and zero steps leave the
input unchanged."""
from math import comb

import numpy as np
import pytest

import oracle


def test_zero_and_one_step():
    g = np.random.default_rng(5)
    img = g.random((9, 11), dtype=np.float32)
    w = g.random((3, 3), dtype=np.float32)
    assert np.array_equal(oracle.stencil2d_iterate(img, w, 0), img.astype(np.float64))
    for pad in (oracle.PAD_CLAMP, oracle.PAD_ZERO):
        assert np.array_equal(oracle.stencil2d_iterate(img, w, 1, pad), oracle.stencil2d(img, w, pad))


@pytest.mark.parametrize("steps", [1, 2, 5])
def test_binomial_spread_of_a_point(steps):
    # [1 2 1]/4 in each direction: after T steps the point at c becomes
    # C(2T, T+i) C(2T, T+j) / 4^(2T) at c + (i, j); zero padding far away
    n, c = 31, 15
    img = np.zeros((n, n), np.float32)
    img[c, c] = 1.0
    b = np.array([1, 2, 1], np.float32) / 4
    w = np.outer(b, b).astype(np.float32)
    got = oracle.stencil2d_iterate(img, w, steps, oracle.PAD_ZERO)
    T = steps
    want = np.zeros((n, n))
    for i in range(-T, T + 1):
        for j in range(-T, T + 1):
            want[c + i, c + j] = comb(2 * T, T + i) * comb(2 * T, T + j) / 4.0 ** (2 * T)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("pad", [oracle.PAD_ZERO, oracle.PAD_CLAMP])
@pytest.mark.parametrize("corner", ["first", "last"])
def test_one_hot_window_moves_the_image(pad, corner):
    # 5x5 window with a single 1: at (0, 0) output (y, x) reads input
    # (y - 2, x - 2), at (4, 4) input (y + 2, x + 2); T steps move by 2T, and
    # clamp padding, applied at each step, repeats the edge
    g = np.random.default_rng(6)
    H, W, T, R = 13, 17, 3, 2
    img = g.random((H, W), dtype=np.float32)
    w = np.zeros((5, 5), np.float32)
    s = -1 if corner == "first" else 1
    w[0 if corner == "first" else 4, 0 if corner == "first" else 4] = 1.0
    got = oracle.stencil2d_iterate(img, w, T, pad)
    want = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            sy, sx = y + s * R * T, x + s * R * T
            if pad == oracle.PAD_CLAMP:
                want[y, x] = img[min(max(sy, 0), H - 1), min(max(sx, 0), W - 1)]
            elif 0 <= sy < H and 0 <= sx < W:
                want[y, x] = img[sy, sx]
    assert np.array_equal(got, want)


def test_constant_image_is_a_fixed_point_with_clamp():
    b = np.array([1, 4, 6, 4, 1], np.float32) / 16  # dyadic, sums to 1
    w = np.outer(b, b).astype(np.float32)
    img = np.full((10, 23), 0.375, np.float32)
    got = oracle.stencil2d_iterate(img, w, 4, oracle.PAD_CLAMP)
    assert np.all(got == 0.375)
    # with zero padding the border loses mass, the centre does not yet
    got = oracle.stencil2d_iterate(img, w, 1, oracle.PAD_ZERO)
    assert got[5, 10] == 0.375 and got[0, 0] < 0.375
