"""GPU parity of iterate with the tree-reduction body (Sec. VI), rise_iterate_sum:
out = iterate(n, m, k, split(n) |> map(reduce(+, 0)), x).

The kernel adds in the order the definition gives, so the bar is bit-exact
equality with the oracle's binary32 evaluation of the same program; the fp64
oracle bounds the distance to the exact sums (k*(n-1) float additions per
input).  Cases cover one pass and several passes (the double buffer in the
workspace), fan-ins that fold in registers (2, 4) and in LDS (others), ragged
last workgroups, unaligned inputs, the largest fan-in, and the degenerate
k = 0, n = 1 and m = 0."""
import math

import numpy as np
import pytest

import oracle
import rise_inputs as ri
from _helpers import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rise():
    import paper_2201_03611_amd as rise

    return rise


def run(rise, x, n, m, k, offset=0):
    import torch

    xs = np.concatenate([np.zeros(offset, np.float32), x.reshape(-1)])
    dx = dev(xs)[offset:]
    out = torch.full((m + 64,), float("nan"), device="cuda")
    need = rise.rise_iterate_sum_workspace(n, m, k)
    ws = torch.empty(need, device="cuda", dtype=torch.uint8) if need else None
    print(f"iterate_sum n={n} m={m} k={k} offset={offset} ws={need}", flush=True)
    rise.rise_iterate_sum(out, dx, n, m, k, ws=ws)
    got = host(out)
    assert np.all(np.isnan(got[m:])), "wrote past out[m)"
    return got[:m]


def check(rise, x, n, m, k, offset=0):
    got = run(rise, x, n, m, k, offset)
    want = oracle.iterate_sum(x, n, m, k, binary32=True).astype(np.float32)
    bad = np.flatnonzero(got.view(np.uint32) != want.view(np.uint32))
    assert bad.size == 0, f"{bad.size} of {m} differ, first at {bad[0]}: {got[bad[0]]} vs {want[bad[0]]}"
    return got


CASES = [
    (2, 1, 13),      # one pass, one workgroup, rounds 1-2 in registers
    (2, 1, 14),      # two passes: 13 rounds, then 1
    (2, 3, 20),      # two passes, 3 segments
    (2, 1001, 10),   # 8 groups per workgroup, ragged last workgroup
    (2, 4097, 1),    # one round, last chunk of 2 values (tail fold)
    (4, 7, 7),       # fan-in 4: round 1 in registers
    (3, 5, 9),       # 3^8 values per group in the first pass, then 1 round
    (8, 3, 6),
    (16, 2, 5),
    (5, 1, 1),
    (7, 9, 4),
    (3, 4096, 2),    # 910 groups of 9 per workgroup (chunks not 16-byte aligned)
    (3, 8, 3),       # one aligned chunk of 8 groups of 27: 16-byte loads of 4 groups of 3
    (6, 500, 2),     # aligned chunks of 1362 first-round groups: 16-byte loads + 2-group tail
    (6, 4001, 1),    # one round per pass, ragged last workgroup
    (8, 1000, 3),    # 16 groups of 512 per workgroup, three rounds
    (8, 1027, 1),    # one round; the last workgroup holds 3 groups (tail only)
    (5, 3, 5),       # 5^5 per group, one group per workgroup
    (4, 1001, 2),    # fan-in 4 with 16-value groups, ragged last workgroup
    (4, 2051, 1),    # one round; the last workgroup holds 3 groups (tail only)
    (4097, 3, 1),    # one group per workgroup
    (8192, 2, 1),    # the largest fan-in
]


@pytest.mark.parametrize("n,m,k", CASES)
def test_bit_exact_against_binary32_program(rise, n, m, k):
    x = ri.uniform_matrix(ri.rng(9000 + n * 31 + k), m, n ** k).reshape(-1)
    check(rise, x, n, m, k)


@pytest.mark.parametrize("k", range(1, 14))
def test_binary_tree_every_round_count(rise, k):
    # n = 2 with k rounds in one pass: rounds in registers, across lanes and,
    # past 64 positions, across wavefronts; 37 groups leave a ragged last
    # workgroup whenever a workgroup holds several groups
    x = ri.uniform_matrix(ri.rng(9050 + k), 37, 2 ** k).reshape(-1)
    check(rise, x, 2, 37, k)


@pytest.mark.parametrize("n,m,k", [(2, 5, 12), (3, 4, 7), (4, 9, 5), (6, 3, 3)])
def test_unaligned_input(rise, n, m, k):
    # the input starts 4 bytes past a 16-byte boundary: plain loads, every
    # round in LDS
    x = ri.uniform_matrix(ri.rng(9100 + n), m, n ** k).reshape(-1)
    check(rise, x, n, m, k, offset=1)


def test_within_summation_bound_of_exact_sums(rise):
    n, m, k = 2, 4, 18
    G = n ** k
    x = ri.uniform_matrix(ri.rng(9200), m, G).reshape(-1)
    got = run(rise, x, n, m, k).astype(np.float64)
    exact = oracle.iterate_sum(x, n, m, k)
    l1 = np.abs(x.astype(np.float64)).reshape(m, G).sum(axis=1)
    assert np.all(np.abs(got - exact) <= k * (n - 1) * 2.0 ** -24 * l1)


def test_rounding_pattern_of_the_tree(rise):
    # (2^24 + 1) + (-2^24 + 1) = 1 in binary32, while the exact sum is 2
    x = np.array([2.0 ** 24, 1, -2.0 ** 24, 1] * 3, np.float32)
    assert run(rise, x, 2, 3, 2).tolist() == [1.0, 1.0, 1.0]
    # left fold of 4: ((2^24 + 1) + 1) + 1 stays 2^24
    y = np.array([2.0 ** 24, 1, 1, 1], np.float32)
    assert run(rise, y, 4, 1, 1).tolist() == [2.0 ** 24]


@pytest.mark.parametrize("n,m,k", [(2, 3, 12), (2, 5, 3), (4, 2, 6), (3, 2, 5)])
def test_signed_zeros_follow_the_fold_from_zero(rise, n, m, k):
    # every sum starts from +0, so (0 + -0) + -0 is +0; bit equality checks the
    # sign of each zero result
    g = ri.rng(9150 + n + k)
    x = np.where(g.random(m * n ** k) < 0.5, -0.0, 0.0).astype(np.float32)
    x[g.random(x.size) < 0.01] = 1.0
    check(rise, x, n, m, k)


def test_integer_ramp_is_exact(rise):
    n, m, k = 2, 3, 11
    G = n ** k
    x = np.arange(G * m, dtype=np.float32)
    got = run(rise, x, n, m, k)
    assert got.tolist() == [G * (2 * j * G + G - 1) / 2 for j in range(m)]


def test_degenerate_rounds(rise):
    x = np.array([1.5, -0.0, 2.0, -3.25, 0.0], np.float32)
    got = check(rise, x, 7, 5, 0)              # k = 0: a copy, -0 kept
    assert math.copysign(1, got[1]) < 0
    got = check(rise, x, 1, 5, 4)              # n = 1: 0 + x, so -0 becomes +0
    assert math.copysign(1, got[1]) > 0
    big = ri.uniform_matrix(ri.rng(9300), 1, 20011).reshape(-1)
    check(rise, big, 1, 20011, 2)              # n = 1 over several workgroups
    check(rise, big, 3, 20011, 0)              # k = 0 over several workgroups


def test_empty_is_a_noop(rise):
    import torch

    out = torch.full((4,), 7.0, device="cuda")
    rise.rise_iterate_sum(out, torch.empty(0, device="cuda"), 2, 0, 5)
    assert host(out).tolist() == [7.0] * 4


def test_full_size_tree_2_pow_26(rise):
    # the measured workload: 2^26 floats (256 MiB), binary tree, one output
    n, m, k = 2, 1, 26
    x = ri.uniform_matrix(ri.rng(9400), 1, n ** k).reshape(-1)
    check(rise, x, n, m, k)


def test_convenience_wrapper(rise):
    import torch

    x = torch.arange(3 * 4 ** 5, dtype=torch.float32, device="cuda")
    y = rise.iterate_sum(x, 4, 5)
    G = 4 ** 5
    assert host(y).tolist() == [G * (2 * j * G + G - 1) / 2 for j in range(3)]
