"""GPU parity of the iterated stencil (iterate of Sec. VI with the stencil as its
body), rise_stencil2d_iterate.

Bar against the fp64 oracle: each step is a chain of k*k FP32 fma from 0, so
|got - exact| <= steps * (k*k + 1) * 2^-24 * (|W|^steps |x|), the stencil of
|w| applied `steps` times to |img| (first-order propagation of the per-step
rounding through a linear map).  Between schedules the bar is bit equality:
fused steps (LDS double buffer) and one launch per step (HBM double buffer)
add the same products in the same order."""
import numpy as np
import pytest

import oracle
import rise_inputs as ri
from _helpers import dev, host

pytestmark = pytest.mark.gpu
U = 2.0 ** -24


@pytest.fixture(scope="module")
def rise():
    import paper_2201_03611_amd as rise

    return rise


def run(rise, img, w, steps, pad, fuse, ld_in=None, ld_out=None, offset=0):
    import torch

    H, W = img.shape
    ld_in = ld_in or W
    ld_out = ld_out or W
    buf = np.zeros(offset + H * ld_in, np.float32)
    buf[offset:].reshape(H, ld_in)[:, :W] = img
    dimg = dev(buf)[offset:]
    out = torch.full((H * ld_out + 64,), float("nan"), device="cuda")
    kh, kw = w.shape
    need = rise.rise_stencil2d_iterate_workspace(H, W, kh, kw, steps, fuse)
    ws = torch.empty(need, device="cuda", dtype=torch.uint8) if need else None
    print(f"stencil_iterate H={H} W={W} k={kh}x{kw} pad={pad} steps={steps} fuse={fuse} "
          f"ld_in={ld_in} ld_out={ld_out} offset={offset} ws={need}", flush=True)
    rise.rise_stencil2d_iterate(out, dimg, dev(w), H, W, ld_out=ld_out, ld_in=ld_in, kh=kh, kw=kw,
                                steps=steps, pad=pad, fuse=fuse, ws=ws)
    o = host(out)
    full = o[:H * ld_out].reshape(H, ld_out)
    if ld_out > W:
        assert np.all(np.isnan(full[:, W:])), "wrote into the row padding"
    assert np.all(np.isnan(o[H * ld_out:])), "wrote past the image"
    return full[:, :W]


def check_oracle(got, img, w, steps, pad):
    p = oracle.PAD_ZERO if pad == "zero" else oracle.PAD_CLAMP
    ref = oracle.stencil2d_iterate(img, w, steps, p)
    scale = oracle.stencil2d_iterate(np.abs(img), np.abs(w), steps, p)
    k2 = w.shape[0] * w.shape[1]
    tol = steps * (k2 + 1) * U * scale + 1e-30
    err = np.abs(got.astype(np.float64) - ref)
    assert np.all(err <= tol), f"max err/scale {np.max(err / np.maximum(scale, 1e-30)):.3e}"


def inputs(H, W, k, seed, kw=None):
    g = ri.rng(seed)
    img = ri.uniform_matrix(g, H, W, 0.0, 1.0)
    w = ri.random_weights(g, k) if kw is None else g.random((k, kw), dtype=np.float32)
    return img, np.ascontiguousarray(w, dtype=np.float32)


CASES = [
    # H, W, k, pad, steps, fuse
    (100, 300, 3, "clamp", 5, 0),    # default fuse 4: one fused launch, then one step
    (77, 250, 5, "zero", 8, 4),      # two fused launches through the workspace
    (64, 224, 5, "clamp", 3, 3),
    (33, 113, 5, "clamp", 6, 2),     # three launches: both workspace images
    (130, 517, 3, "zero", 7, 3),
    (5, 7, 5, "clamp", 4, 4),        # the halo region is larger than the image
    (5, 7, 3, "zero", 4, 4),
    (1, 1, 3, "zero", 3, 0),
    (1, 300, 3, "clamp", 4, 4),
    (300, 1, 5, "clamp", 4, 4),
    (97, 129, 5, "zero", 5, 1),      # one launch per step
    (50, 60, 7, "clamp", 2, 0),      # 7x7: default is one launch per step
]


@pytest.mark.parametrize("H,W,k,pad,steps,fuse", CASES)
def test_against_oracle(rise, H, W, k, pad, steps, fuse):
    img, w = inputs(H, W, k, 7000 + H + W + k + steps)
    got = run(rise, img, w, steps, pad, fuse)
    check_oracle(got, img, w, steps, pad)


def test_rectangular_window_one_launch_per_step(rise):
    img, w = inputs(40, 70, 3, 7101, kw=5)
    got = run(rise, img, w, 3, "clamp", 0)
    check_oracle(got, img, w, 3, "clamp")


def test_zero_steps_copies(rise):
    img, w = inputs(31, 45, 5, 7102)
    got = run(rise, img, w, 0, "clamp", 0, ld_in=48, ld_out=50)
    assert np.array_equal(got, img)


@pytest.mark.parametrize("k", [3, 5])
@pytest.mark.parametrize("pad", ["clamp", "zero"])
@pytest.mark.parametrize("fuse", [2, 3, 4])
def test_fused_equals_one_launch_per_step(rise, k, pad, fuse):
    img, w = inputs(130, 517, k, 7200 + k + fuse)
    steps = 2 * fuse + 1
    a = run(rise, img, w, steps, pad, fuse)
    b = run(rise, img, w, steps, pad, 1)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_strided_and_unaligned_images(rise):
    img, w = inputs(70, 90, 5, 7300)
    a = run(rise, img, w, 5, "clamp", 4, ld_in=97, ld_out=101, offset=1)
    check_oracle(a, img, w, 5, "clamp")
    b = run(rise, img, w, 5, "clamp", 1, ld_in=97, ld_out=101, offset=1)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_full_size_4096_sampled(rise):
    # 4096^2, 5x5 Gaussian, clamp, 8 steps fused by 4: sampled outputs against
    # the oracle on a crop.  An output after T steps depends on inputs within
    # r*T of it, and a crop edge inside the image disturbs only outputs within
    # r*T of that edge, so a crop reaching r*T past the sample (or to the real
    # image edge) gives the exact oracle value there.
    import torch

    H = W = 4096
    steps, R = 8, 2
    RT = R * steps
    img = ri.image_uniform(H, W, 1003)
    w = ri.gaussian_weights(5, 1.0)
    got = run(rise, img, w, steps, "clamp", 4)
    g = ri.rng(7400)
    ys = np.concatenate([[0, 1, H - 1, 17, H - 18], g.integers(0, H, 27)])
    xs = np.concatenate([[0, W - 1, 2, W - 3, 16], g.integers(0, W, 27)])
    for y, x in zip(ys, xs):
        y0, y1 = max(0, y - RT), min(H, y + RT + 1)
        x0, x1 = max(0, x - RT), min(W, x + RT + 1)
        crop = img[y0:y1, x0:x1]
        ref = oracle.stencil2d_iterate(crop, w, steps, oracle.PAD_CLAMP)[y - y0, x - x0]
        scale = oracle.stencil2d_iterate(np.abs(crop), w, steps, oracle.PAD_CLAMP)[y - y0, x - x0]
        assert abs(float(got[y, x]) - ref) <= steps * 26 * U * scale, (y, x)
    # and the fused launch equals one launch per step everywhere
    b = run(rise, img, w, steps, "clamp", 1)
    assert np.array_equal(got.view(np.uint32), b.view(np.uint32))
    del b
    torch.cuda.empty_cache()


def test_convenience_wrapper(rise):
    import torch

    img, w = inputs(64, 64, 3, 7500)
    y = rise.stencil2d_iterate(torch.from_numpy(img).cuda(), torch.from_numpy(w), 3)
    check_oracle(host(y), img, w, 3, "clamp")
