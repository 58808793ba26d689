"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws inputs.  It holds none of the GEMM, stencil or
quantisation arithmetic: both the oracle and the GPU library consume the exact
arrays produced here (float32, or bfloat16 bit patterns as uint16).

Seeds follow one convention: numpy.random.default_rng(1000 + i) for the i-th
workload (1: GEMM 128^3, 2: GEMM 4096^3, 3: stencil 4096^2, 4: precision GEMM
8192^3, 5: batched set, 6: stencil layer, 7: GEMM backward).
"""
import numpy as np

SEED_GEMM_SMALL = 1001
SEED_GEMM_F32 = 1002
SEED_STENCIL = 1003
SEED_PRECISION = 1004
SEED_BATCHED = 1005
SEED_CONV = 1006
SEED_GEMM_BWD = 1007


def rng(seed):
    return np.random.default_rng(seed)


def uniform_matrix(g, rows, cols, lo=-1.0, hi=1.0):
    """i.i.d. U(lo, hi) float32, row-major."""
    return g.uniform(lo, hi, size=(rows, cols)).astype(np.float32)


def gemm_uniform(M, N, K, seed):
    """A (M x K) and B (K x N), entries U(-1, 1), A drawn first."""
    g = rng(seed)
    A = uniform_matrix(g, M, K)
    B = uniform_matrix(g, K, N)
    return A, B


def gemm_scaled_normal(M, N, K, seed, spread=4.0):
    """A = N(0,1) * 2^u_i per row, B = N(0,1) * 2^v_j per column, u, v ~ U(-spread, spread).

    Entries are drawn first (A then B), then the row and column exponents; the
    products are rounded to float32 once and those stored values are the inputs."""
    g = rng(seed)
    A = g.standard_normal(size=(M, K))
    B = g.standard_normal(size=(K, N))
    u = g.uniform(-spread, spread, size=(M, 1))
    v = g.uniform(-spread, spread, size=(1, N))
    A = (A * np.exp2(u)).astype(np.float32)
    B = (B * np.exp2(v)).astype(np.float32)
    return A, B


def integer_matrix(g, rows, cols, bound=2):
    """Integer-valued float32 entries in [-bound, bound] (exact in f32, bf16 and fp8)."""
    return g.integers(-bound, bound + 1, size=(rows, cols)).astype(np.float32)


def image_uniform(H, W, seed):
    """H x W float32 image, entries U[0, 1)."""
    return rng(seed).random(size=(H, W), dtype=np.float64).astype(np.float32)


def gaussian_weights(k=5, sigma=1.0):
    """k x k Gaussian taps exp(-(dy^2 + dx^2) / (2 sigma^2)), dy, dx in [-(k-1)/2, (k-1)/2],
    normalised over the k^2 discrete taps in float64, then rounded to float32."""
    r = (k - 1) // 2
    d = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-(d[:, None] ** 2 + d[None, :] ** 2) / (2.0 * sigma * sigma))
    g = g / g.sum()
    return g.astype(np.float32)


def random_weights(g, k):
    """k x k weights u / sum(u) with u ~ U(0, 1) (taps that sum to 1)."""
    u = g.random(size=(k, k))
    return (u / u.sum()).astype(np.float32)


def batched_gemm_sizes(n=512, seed=SEED_BATCHED, lo=64, hi=1024, step=32):
    """n (M, N, K) triples, each i.i.d. uniform on the multiples of `step` in [lo, hi]."""
    g = rng(seed)
    choices = np.arange(lo, hi + 1, step)
    return g.choice(choices, size=(n, 3)).astype(np.int64)


def batched_stencil_specs(n=256, seed=SEED_BATCHED + 100, lo=256, hi=2048, ks=(3, 5, 7)):
    """n (side, k) pairs: side ~ U{lo..hi}, k ~ U(ks)."""
    g = rng(seed)
    sides = g.integers(lo, hi + 1, size=n)
    kk = g.choice(np.array(ks), size=n)
    return np.stack([sides, kk], axis=1).astype(np.int64)


def bf16_bits_from_f32(x):
    """bf16 bit patterns of float32 x via torch's round-to-nearest-even cast (used only to
    draw bf16-stored inputs)."""
    import torch

    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).numpy().view(np.uint16)


def conv_inputs(B, Cin, Cout, H, W, seed=SEED_CONV, k=3, w_std=0.02):
    """Stencil-layer inputs: x ~ N(0,1) stored as bf16 (NHWC, uint16 bits),
    weights N(0, w_std^2) float32 (Cout x Cin x k x k), dOut ~ N(0,1) stored as bf16."""
    g = rng(seed)
    x = g.standard_normal(size=(B, H, W, Cin), dtype=np.float32)
    w = (g.standard_normal(size=(Cout, Cin, k, k)) * w_std).astype(np.float32)
    dout = g.standard_normal(size=(B, H, W, Cout), dtype=np.float32)
    return bf16_bits_from_f32(x), w, bf16_bits_from_f32(dout)


def sample_indices(g, M, N, count):
    """`count` distinct-ish (row, col) samples plus the four corners."""
    rows = g.integers(0, M, size=count)
    cols = g.integers(0, N, size=count)
    rows = np.concatenate([rows, [0, 0, M - 1, M - 1]])
    cols = np.concatenate([cols, [0, N - 1, 0, N - 1]])
    return rows.astype(np.int64), cols.astype(np.int64)

