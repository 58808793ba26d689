"""Pins of the oracle's view primitives against the pattern laws and direct slicing.

split/join follow the DPIA functional primitives (Sec. V-A) and the splitJoinMap
rewrite (Sec. IV-B); transpose, slide and pad are not defined in the paper and
take their standard readings (swap two dimensions; windows of sz elements every
sp; edge repeat or zeros).  Every expected value here comes from
numpy slicing or from the law itself, never from the oracle.
"""
import numpy as np
import pytest

import oracle
from oracle import V_IDX, V_JOIN, V_PAD, V_SLIDE, V_SPLIT, V_TRANSPOSE, PAD_CLAMP, PAD_ZERO


def arr(*shape, seed=0):
    return np.random.default_rng(seed).standard_normal(size=shape)


@pytest.mark.parametrize("n,m", [(1, 12), (3, 4), (4, 3), (12, 1)])
def test_split_then_join_is_identity(n, m):
    x = arr(n * m)
    y = oracle.view_eval(x, [(V_SPLIT, 0, n), (V_JOIN, 0)])
    assert y.shape == x.shape and np.array_equal(y, x)


def test_split_layout_matches_paper_mv_index():
    # split(s) puts element j*s + i at [j][i]: the generated MV kernel reads
    # row lId of work-group wgId at M[(i + lId*m) + m*s*wgId] (Sec. V, OpenCL listing)
    n, m, s = 6, 5, 3
    M = arr(n, m)
    flat = M.reshape(-1)
    t = oracle.view_eval(M, [(V_SPLIT, 0, s)])  # (n/s, s, m)
    assert t.shape == (n // s, s, m)
    for wg in range(n // s):
        for l in range(s):
            for i in range(m):
                assert t[wg, l, i] == flat[(i + l * m) + m * s * wg]


def test_join_then_split_is_identity():
    x = arr(4, 6)
    y = oracle.view_eval(x, [(V_JOIN, 0), (V_SPLIT, 0, 6)])
    assert np.array_equal(y, x)


def test_split_rejects_non_divisible_length():
    with pytest.raises(oracle.OracleError):
        oracle.view_eval(arr(10), [(V_SPLIT, 0, 3)])


def test_transpose_twice_is_identity_and_matches_numpy():
    x = arr(3, 5, 2)
    t = oracle.view_eval(x, [(V_TRANSPOSE, 0)])
    assert np.array_equal(t, x.transpose(1, 0, 2))
    tt = oracle.view_eval(x, [(V_TRANSPOSE, 0), (V_TRANSPOSE, 0)])
    assert np.array_equal(tt, x)
    t1 = oracle.view_eval(x, [(V_TRANSPOSE, 1)])
    assert np.array_equal(t1, x.transpose(0, 2, 1))


@pytest.mark.parametrize("N,sz,sp", [(10, 3, 1), (10, 4, 2), (7, 7, 1), (9, 1, 4), (13, 5, 4)])
def test_slide_window_count_and_contents(N, sz, sp):
    x = arr(N)
    w = oracle.view_eval(x, [(V_SLIDE, 0, sz, sp)])
    assert w.shape == ((N - sz) // sp + 1, sz)
    for i in range(w.shape[0]):
        assert np.array_equal(w[i], x[i * sp:i * sp + sz])


def test_slide_rejects_ragged_step_and_short_input():
    with pytest.raises(oracle.OracleError):
        oracle.view_eval(arr(10), [(V_SLIDE, 0, 4, 4)])
    with pytest.raises(oracle.OracleError):
        oracle.view_eval(arr(3), [(V_SLIDE, 0, 4, 1)])


@pytest.mark.parametrize("mode", [PAD_CLAMP, PAD_ZERO])
def test_pad_lengths_and_values(mode):
    x = arr(6)
    p = oracle.view_eval(x, [(V_PAD, 0, 2, 3, mode)])
    assert p.shape == (2 + 6 + 3,)
    np_mode = "edge" if mode == PAD_CLAMP else "constant"
    assert np.array_equal(p, np.pad(x, (2, 3), mode=np_mode))


@pytest.mark.parametrize("r", [0, 1, 2, 3])
def test_pad_then_slide_gives_one_window_per_element(r):
    N = 9
    x = arr(N)
    w = oracle.view_eval(x, [(V_PAD, 0, r, r, PAD_CLAMP), (V_SLIDE, 0, 2 * r + 1, 1)])
    assert w.shape == (N, 2 * r + 1)
    for i in range(N):
        idx = np.clip(np.arange(i - r, i + r + 1), 0, N - 1)
        assert np.array_equal(w[i], x[idx])


def test_slide2d_equals_direct_2d_indexing():
    # slide2D(k, 1) = map(slide(k, 1)) |> slide(k, 1) |> map(transpose)
    H, W, kh, kw = 6, 7, 3, 5
    x = arr(H, W)
    w = oracle.view_eval(x, [(V_SLIDE, 1, kw, 1), (V_SLIDE, 0, kh, 1), (V_TRANSPOSE, 1)])
    assert w.shape == (H - kh + 1, W - kw + 1, kh, kw)
    for y in range(H - kh + 1):
        for xx in range(W - kw + 1):
            assert np.array_equal(w[y, xx], x[y:y + kh, xx:xx + kw])


def test_idx_selects_along_axis():
    x = arr(3, 4, 5)
    assert np.array_equal(oracle.view_eval(x, [(V_IDX, 1, 2)]), x[:, 2, :])
    assert np.array_equal(oracle.view_eval(x, [(V_IDX, 0, 1)]), x[1])


def test_split_join_map_law_on_inner_axis():
    # map(f) = split(n) >> map(map(f)) >> join, here with f a view (transpose of rows)
    x = arr(6, 4, 3)
    direct = oracle.view_eval(x, [(V_TRANSPOSE, 1)])
    tiled = oracle.view_eval(x, [(V_SPLIT, 0, 2), (V_TRANSPOSE, 2), (V_JOIN, 0)])
    assert np.array_equal(direct, tiled)
