"""GPU parity of rise_stencil2d against the oracle.

Bar: |out_hat - out| <= 1e-5 * sum |w| |window| per output (the componentwise
FP32 tolerance); dyadic inputs whose sums are exact in FP32, bit for bit.
"""
import numpy as np
import pytest

import oracle
import rise_inputs as ri
from _helpers import componentwise, dev, host, stencil_scale

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5
PADS = {"clamp": oracle.PAD_CLAMP, "zero": oracle.PAD_ZERO}


@pytest.fixture(scope="module")
def rise():
    import paper_2201_03611_amd as rise

    return rise


def run(rise, img, w, pad, schedule=None):
    print(f"stencil img{img.shape} w{w.shape} pad={pad} schedule={schedule}", flush=True)
    return host(rise.stencil2d(dev(img), dev(w), pad=pad, schedule=schedule))


@pytest.mark.parametrize("pad", list(PADS))
@pytest.mark.parametrize("H,W", [(1, 1), (3, 5), (32, 256), (33, 257), (70, 300), (100, 13),
                                 (64, 1024)])
@pytest.mark.parametrize("k", [1, 3, 5, 7])
def test_tiled_kernel_vs_oracle(rise, pad, H, W, k):
    g = ri.rng(H * 1000 + W + k)
    img = ri.uniform_matrix(g, H, W, 0.0, 1.0)
    w = ri.uniform_matrix(g, k, k)  # asymmetric, signed: catches flips and sign errors
    ref = oracle.stencil2d(img, w, PADS[pad])
    scale = stencil_scale(img, w, PADS[pad])
    for sc in rise.rise_stencil_schedules():
        out = run(rise, img, w, pad, sc)
        assert componentwise(out, ref, scale) <= TOL_F32, sc


@pytest.mark.parametrize("pad", list(PADS))
@pytest.mark.parametrize("H,W", [(2050, 2100), (4099, 513)])
@pytest.mark.parametrize("k", [3, 5, 7])
def test_resident_grid_walks_several_tiles(rise, pad, H, W, k):
    # more tiles than resident workgroups, so each workgroup of the pipelined
    # schedule walks two or more tiles through both LDS buffers
    g = ri.rng(H + W * 7 + k)
    img = ri.uniform_matrix(g, H, W, 0.0, 1.0)
    w = ri.uniform_matrix(g, k, k)
    ref = oracle.stencil2d(img, w, PADS[pad])
    scale = stencil_scale(img, w, PADS[pad])
    for sc in [s for s in rise.rise_stencil_schedules() if s[0] != "stream"]:
        out = run(rise, img, w, pad, sc)
        assert componentwise(out, ref, scale) <= TOL_F32, sc


@pytest.mark.parametrize("kh,kw", [(9, 9), (3, 7), (15, 1), (11, 5)])
@pytest.mark.parametrize("pad", list(PADS))
def test_direct_kernel_vs_oracle(rise, kh, kw, pad):
    g = ri.rng(kh * 17 + kw)
    img = ri.uniform_matrix(g, 45, 77, 0.0, 1.0)
    w = ri.uniform_matrix(g, kh, kw)
    out = run(rise, img, w, pad)
    ref = oracle.stencil2d(img, w, PADS[pad])
    assert componentwise(out, ref, stencil_scale(img, w, PADS[pad])) <= TOL_F32


@pytest.mark.parametrize("k", [3, 5, 7])
def test_dyadic_inputs_bit_exact(rise, k):
    g = ri.rng(k)
    img = g.integers(0, 16, size=(97, 390)).astype(np.float32)
    w = (g.integers(-8, 9, size=(k, k)) / 64.0).astype(np.float32)
    for pad in PADS:
        ref = oracle.stencil2d(img, w, PADS[pad]).astype(np.float32)
        for sc in rise.rise_stencil_schedules():
            assert np.array_equal(run(rise, img, w, pad, sc), ref), (pad, sc)


def test_constant_image_binomial_closed_form(rise):
    b = np.array([1, 4, 6, 4, 1], dtype=np.float64)
    w = (np.outer(b, b) / 256.0).astype(np.float32)
    img = np.full((64, 300), 0.625, dtype=np.float32)
    for sc in rise.rise_stencil_schedules():
        assert np.array_equal(run(rise, img, w, "clamp", sc), img), sc


def test_unaligned_leading_dimension(rise):
    import torch

    g = ri.rng(11)
    H, W = 50, 121
    big = ri.uniform_matrix(g, H, W + 1, 0.0, 1.0)
    w = ri.gaussian_weights(5)
    img = np.ascontiguousarray(big[:, :W])
    ref = oracle.stencil2d(img, w, oracle.PAD_CLAMP)
    for sc in rise.rise_stencil_schedules():
        out = torch.empty((H, W + 3), device="cuda")
        rise.rise_stencil2d(out, dev(big), dev(w), H, W, ld_out=W + 3, ld_in=W + 1, kh=5, kw=5,
                            schedule=sc)
        assert componentwise(host(out)[:, :W], ref, stencil_scale(img, w, 0)) <= TOL_F32, sc


@pytest.mark.parametrize("pad", list(PADS))
@pytest.mark.parametrize("H,W,ld", [(50, 121, 124), (37, 258, 260), (300, 1022, 1024)])
def test_aligned_rows_with_ragged_width(rise, pad, H, W, ld):
    # 16-byte aligned rows (ld % 4 == 0) whose width is not a multiple of 4: the
    # last 16-byte chunk of a row straddles the image edge, so the kernels must
    # not take the whole-chunk fetch path
    import torch

    g = ri.rng(H + W + ld)
    big = ri.uniform_matrix(g, H, ld, 0.0, 1.0)
    img = np.ascontiguousarray(big[:, :W])
    w = ri.uniform_matrix(g, 5, 5)
    ref = oracle.stencil2d(img, w, PADS[pad])
    scale = stencil_scale(img, w, PADS[pad])
    for sc in rise.rise_stencil_schedules():
        out = torch.full((H, ld), float("nan"), device="cuda")
        print(f"stencil aligned ragged H={H} W={W} ld={ld} pad={pad} schedule={sc}", flush=True)
        rise.rise_stencil2d(out, dev(big), dev(w), H, W, ld_out=ld, ld_in=ld, kh=5, kw=5,
                            pad=pad, schedule=sc)
        o = host(out)
        assert np.all(np.isnan(o[:, W:])), sc
        assert componentwise(o[:, :W], ref, scale) <= TOL_F32, sc


def test_config_4096_gaussian_full(rise):
    # the timed stencil workload: 4096 x 4096 U[0,1), 5 x 5 Gaussian sigma = 1, clamp
    img = ri.image_uniform(4096, 4096, ri.SEED_STENCIL)
    w = ri.gaussian_weights(5, 1.0)
    ref = oracle.stencil2d(img, w, oracle.PAD_CLAMP)
    scale = stencil_scale(img, w, oracle.PAD_CLAMP)
    for sc in [None] + rise.rise_stencil_schedules():
        err = componentwise(run(rise, img, w, "clamp", sc), ref, scale)
        print("4096^2 stencil componentwise max err", sc, err)
        assert err <= TOL_F32, sc
