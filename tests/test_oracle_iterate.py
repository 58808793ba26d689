"""Pins of the oracle's iterate (Sec. VI) with the tree-reduction body
split(n) |> map(reduce(+, 0)).  Each check is fixed by arithmetic or by the
definition, not by the oracle itself: integer sums are exact, exact float
rounding of hand-worked cases separates a tree from a left fold and a fold from
index 0 from one from the end, one-hot inputs pin which segment a value lands
in, math.fsum gives the correctly rounded sum, and the float order's error
stays within the bound of recursive summation."""
import math

import numpy as np
import pytest

import oracle
import rise_inputs as ri


@pytest.mark.parametrize("n,m,k", [(2, 1, 5), (3, 4, 3), (4, 2, 4), (5, 3, 2), (7, 1, 1)])
@pytest.mark.parametrize("binary32", [False, True])
def test_integer_ramp_closed_form(n, m, k, binary32):
    # x_i = i: segment j sums i over [j*G, (j+1)*G), G = n^k, which is
    # G*(2*j*G + G - 1)/2; every partial sum is an integer below 2^24
    G = n ** k
    x = np.arange(G * m, dtype=np.float32)
    got = oracle.iterate_sum(x, n, m, k, binary32=binary32)
    want = [G * (2 * j * G + G - 1) / 2 for j in range(m)]
    assert got.tolist() == want


def test_tree_and_left_fold_round_differently():
    # binary32: 2^24 + 1 rounds back to 2^24 (ties to even), 1 + 1 is exact
    x = np.array([2.0 ** 24, 1, 1, 1], np.float32)
    # n = 2, k = 2: (2^24 + 1) + (1 + 1) = 2^24 + 2
    assert oracle.iterate_sum(x, 2, 1, 2, binary32=True).tolist() == [2.0 ** 24 + 2]
    # n = 4, k = 1: ((2^24 + 1) + 1) + 1, every step rounds back to 2^24
    assert oracle.iterate_sum(x, 4, 1, 1, binary32=True).tolist() == [2.0 ** 24]
    # in doubles both give the exact sum
    assert oracle.iterate_sum(x, 2, 1, 2).tolist() == [2.0 ** 24 + 3]
    assert oracle.iterate_sum(x, 4, 1, 1).tolist() == [2.0 ** 24 + 3]


def test_fold_runs_from_index_zero():
    # n = 3: ((0 + 2^24) + 1) + 1 = 2^24, but ((0 + 1) + 1) + 2^24 = 2^24 + 2
    big_first = np.array([2.0 ** 24, 1, 1], np.float32)
    big_last = np.array([1, 1, 2.0 ** 24], np.float32)
    assert oracle.iterate_sum(big_first, 3, 1, 1, binary32=True).tolist() == [2.0 ** 24]
    assert oracle.iterate_sum(big_last, 3, 1, 1, binary32=True).tolist() == [2.0 ** 24 + 2]


def test_rounds_pair_neighbours_not_strided_elements():
    # n = 2, k = 2 over [a, b, c, d] is (a + b) + (c + d).  With a = 2^24, b = 1,
    # c = -2^24, d = 1 that is 2^24 + (-2^24 + 1) = 1 in binary32 (2^24 + 1
    # rounds to 2^24); pairing a with c (a stride-2 tree) would give 0 + 2 = 2
    x = np.array([2.0 ** 24, 1, -2.0 ** 24, 1], np.float32)
    assert oracle.iterate_sum(x, 2, 1, 2, binary32=True).tolist() == [1.0]
    assert oracle.iterate_sum(x, 2, 1, 2).tolist() == [2.0]


@pytest.mark.parametrize("n,m,k", [(2, 3, 4), (3, 2, 3), (6, 5, 2)])
def test_one_hot_lands_in_its_segment(n, m, k):
    G = n ** k
    for p in [0, 1, G - 1, G, G * m - 1, (G * m) // 2]:
        x = np.zeros(G * m, np.float32)
        x[p] = 1.0
        got = oracle.iterate_sum(x, n, m, k)
        want = np.zeros(m)
        want[p // G] = 1.0
        assert got.tolist() == want.tolist(), p


@pytest.mark.parametrize("n,m,k,seed", [(2, 3, 10, 1), (3, 2, 6, 2), (16, 4, 2, 3)])
def test_doubles_match_correctly_rounded_sum(n, m, k, seed):
    G = n ** k
    x = ri.uniform_matrix(ri.rng(seed), m, G).reshape(-1)
    got = oracle.iterate_sum(x, n, m, k)
    for j in range(m):
        seg = [float(v) for v in x[j * G:(j + 1) * G]]
        exact = math.fsum(seg)
        # the double fold's error is far below float resolution
        assert abs(got[j] - exact) <= 1e-13 * math.fsum(abs(v) for v in seg)


@pytest.mark.parametrize("n,m,k,seed", [(2, 2, 12, 4), (3, 1, 7, 5), (8, 3, 4, 6)])
def test_float_order_within_recursive_summation_bound(n, m, k, seed):
    # each input passes through at most k*(n-1) float additions
    G = n ** k
    x = ri.uniform_matrix(ri.rng(seed), m, G).reshape(-1)
    f32 = oracle.iterate_sum(x, n, m, k, binary32=True)
    f64 = oracle.iterate_sum(x, n, m, k)
    u = 2.0 ** -24
    for j in range(m):
        l1 = float(np.abs(x[j * G:(j + 1) * G].astype(np.float64)).sum())
        assert abs(f32[j] - f64[j]) <= k * (n - 1) * u * l1 * 1.0001
        assert f32[j] == np.float32(f32[j])  # representable in binary32


def test_rounds_compose():
    # iterate k1 + k2 rounds = iterate k2 rounds over the result of k1 rounds
    n, m = 3, 2
    x = ri.uniform_matrix(ri.rng(7), m, n ** 5).reshape(-1)
    full = oracle.iterate_sum(x, n, m, 5, binary32=True)
    inner = oracle.iterate_sum(x, n, m * n ** 3, 2, binary32=True).astype(np.float32)
    outer = oracle.iterate_sum(inner, n, m, 3, binary32=True)
    assert full.tolist() == outer.tolist()


def test_degenerate_cases():
    x = np.array([1.5, -0.0, 2.0], np.float32)
    # k = 0: nothing is folded
    got = oracle.iterate_sum(x, 4, 3, 0, binary32=True)
    assert got.tolist() == [1.5, 0.0, 2.0] and math.copysign(1, got[1]) < 0
    # n = 1: each round adds 0, so -0 becomes +0 and nothing else changes
    for k in (1, 3):
        got = oracle.iterate_sum(x, 1, 3, k, binary32=True)
        assert got.tolist() == [1.5, 0.0, 2.0] and math.copysign(1, got[1]) > 0
    assert oracle.iterate_sum(np.zeros(0, np.float32), 2, 0, 3).size == 0
    with pytest.raises(oracle.OracleError):
        oracle.iterate_sum(np.zeros(7, np.float32), 2, 1, 3)
