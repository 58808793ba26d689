"""GPU parity of the multi-channel stencil layer (rise_conv2d, rise_conv2d_backward).

The GPU rounds the FP32 weights to bfloat16 and its output to bfloat16; the
reference is the oracle layer evaluated on the same bf16 activations with the
weights rounded by the oracle's own bf16 rounding.  Bar per element:
|got - ref| <= 2^-8 (|ref| + 1e-5 s) + 1e-5 s,  s = sum |w| |window|
(one bf16 rounding of the FP32 result, nearest even: unit roundoff 2^-8 for 8
significant bits; 1e-5 s covers the FP32 accumulation),
and FP32 dW within 1e-5 componentwise.
"""
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


def bf16_dev(bits):
    import torch

    return dev(bits).view(torch.bfloat16)


def decode(t):
    import torch

    return oracle.bf16_bits_to_f32(host(t.contiguous().view(torch.int16)).view(np.uint16))


def wq(w):
    """weights as the matrix cores see them: bf16 (nearest even) widened back to f32"""
    return oracle.bf16_bits_to_f32(oracle.quant_bf16(w)).reshape(w.shape)


def check_out(got, ref, scale):
    err = np.abs(got.astype(np.float64) - ref)
    bound = 2.0 ** -8 * (np.abs(ref) + 1e-5 * scale) + 1e-5 * scale + 1e-30
    assert np.all(err <= bound), float(np.max(err / bound))


def case_inputs(B, H, W, Cin, Cout, seed):
    g = ri.rng(seed)
    x = ri.bf16_bits_from_f32(g.standard_normal((B, H, W, Cin)).astype(np.float32))
    w = (g.standard_normal((Cout, Cin, 3, 3)) * 0.05).astype(np.float32)
    dout = ri.bf16_bits_from_f32(g.standard_normal((B, H, W, Cout)).astype(np.float32))
    return x, w, dout


@pytest.mark.parametrize("Cin,Cout", [(16, 32), (32, 64), (64, 64), (64, 32), (16, 64), (32, 32)])
@pytest.mark.parametrize("pad", ["zero", "clamp"])
@pytest.mark.parametrize("H,W", [(5, 7), (9, 70), (4, 64)])
def test_forward_vs_oracle(rise, Cin, Cout, pad, H, W):
    print(f"conv fwd Cin={Cin} Cout={Cout} pad={pad} H={H} W={W}", flush=True)
    x, w, _ = case_inputs(2, H, W, Cin, Cout, Cin * 7 + Cout + H)
    out = decode(rise.conv2d(bf16_dev(x), dev(w), pad=pad))
    pm = oracle.PAD_ZERO if pad == "zero" else oracle.PAD_CLAMP
    ref = oracle.conv2d(x, wq(w), pm)
    scale = oracle.conv2d(np.abs(oracle.bf16_bits_to_f32(x)).reshape(x.shape), np.abs(wq(w)), pm)
    check_out(out, ref, scale)


def test_forward_small_integers_exact(rise):
    # |sum| <= 9 * 16 = 144 < 256: every sum and the bf16 output are exact
    g = ri.rng(4)
    x = g.integers(-1, 2, size=(2, 6, 67, 16)).astype(np.float32)
    w = g.integers(-1, 2, size=(32, 16, 3, 3)).astype(np.float32)
    out = decode(rise.conv2d(bf16_dev(ri.bf16_bits_from_f32(x)), dev(w)))
    assert np.array_equal(out, oracle.conv2d(x, w, oracle.PAD_ZERO).astype(np.float32))


@pytest.mark.parametrize("Cin,Cout", [(64, 64), (32, 64), (64, 32), (32, 32)])
@pytest.mark.parametrize("H,W", [(5, 7), (9, 70)])
def test_backward_vs_oracle(rise, Cin, Cout, H, W):
    print(f"conv bwd Cin={Cin} Cout={Cout} H={H} W={W}", flush=True)
    x, w, dout = case_inputs(2, H, W, Cin, Cout, Cin + Cout * 3 + W)
    dIn, dW = rise.conv2d_backward(bf16_dev(dout), bf16_dev(x), dev(w))
    xf = oracle.bf16_bits_to_f32(x).reshape(x.shape)
    gf = oracle.bf16_bits_to_f32(dout).reshape(dout.shape)
    rin, rw = oracle.conv2d_backward(gf, x, wq(w), oracle.PAD_ZERO)
    sin, sw = oracle.conv2d_backward(np.abs(gf), np.abs(xf), np.abs(wq(w)), oracle.PAD_ZERO)
    check_out(decode(dIn), rin, sin)
    err = np.abs(host(dW).astype(np.float64) - rw)
    assert np.all(err <= 1e-5 * sw + 1e-30), float(np.max(err / (sw + 1e-30)))


def test_config_layer_crops(rise):
    # the layer at its full size (batch 32, 64 -> 64 channels, 512 x 512): outputs of
    # two crops compared with the oracle on the same crops (halo included)
    import torch

    B, H, W, C = 32, 512, 512, 64
    x, w, dout = ri.conv_inputs(B, C, C, H, W)
    print("conv full-size forward", flush=True)
    dx = bf16_dev(x)
    out = rise.conv2d(dx, dev(w))
    torch.cuda.synchronize()
    for (b, y0, x0) in [(0, 0, 0), (17, 300, 200), (31, 496, 440)]:
        ys, xs = max(y0 - 1, 0), max(x0 - 1, 0)
        ye, xe = min(y0 + 17, H), min(x0 + 73, W)
        crop = np.ascontiguousarray(x[b:b + 1, ys:ye, xs:xe, :])
        ref = oracle.conv2d(crop, wq(w), oracle.PAD_ZERO)[0]
        scale = oracle.conv2d(np.abs(oracle.bf16_bits_to_f32(crop)).reshape(crop.shape),
                              np.abs(wq(w)), oracle.PAD_ZERO)[0]
        # keep the outputs whose window lies inside the crop (or on a true image edge)
        oy0, ox0 = y0 - ys, x0 - xs
        oy1 = min(16, (ye - ys) - oy0 - (1 if ye < H else 0))
        ox1 = min(72, (xe - xs) - ox0 - (1 if xe < W else 0))
        got = decode(out[b, y0:y0 + oy1, x0:x0 + ox1, :])
        check_out(got, ref[oy0:oy0 + oy1, ox0:ox0 + ox1], scale[oy0:oy0 + oy1, ox0:ox0 + ox1])


def test_config_layer_backward_directional(rise):
    # dW of the full layer: L(w) = <dOut, conv(x, w)> is linear in the (bf16-rounded)
    # weights, so <dW, V> = <dOut, conv(x, V)> for a bf16-exact direction V
    import torch

    B, H, W, C = 8, 512, 512, 64
    x, w, dout = ri.conv_inputs(B, C, C, H, W, seed=ri.SEED_CONV + 1)
    print("conv full-size backward", flush=True)
    dIn, dW = rise.conv2d_backward(bf16_dev(dout), bf16_dev(x), dev(w))
    V = wq((ri.rng(9).standard_normal((C, C, 3, 3)) * 0.05).astype(np.float32))
    LV = decode(rise.conv2d(bf16_dev(x), dev(V))).astype(np.float64)
    g = oracle.bf16_bits_to_f32(dout).reshape(dout.shape).astype(np.float64)
    fd = float(np.sum(g * LV))
    lin = float(np.sum(host(dW).astype(np.float64) * V))
    scale = float(np.sum(np.abs(g) * np.abs(LV)))
    assert abs(fd - lin) <= 2.0 ** -8 * scale, (fd, lin, scale)
    assert np.all(np.isfinite(decode(dIn)))


def test_autograd_layer(rise):
    import torch

    x, w, dout = case_inputs(2, 8, 66, 64, 64, 99)
    tx = bf16_dev(x).requires_grad_(True)
    tw = dev(w).requires_grad_(True)
    out = rise.RiseConv2dFn.apply(tx, tw)
    out.backward(bf16_dev(dout))
    gf = oracle.bf16_bits_to_f32(dout).reshape(dout.shape)
    rin, rw = oracle.conv2d_backward(gf, x, wq(w), oracle.PAD_ZERO)
    xf = oracle.bf16_bits_to_f32(x).reshape(x.shape)
    sin, sw = oracle.conv2d_backward(np.abs(gf), np.abs(xf), np.abs(wq(w)), oracle.PAD_ZERO)
    check_out(decode(tx.grad), rin, sin)
    err = np.abs(host(tw.grad).astype(np.float64) - rw)
    assert np.all(err <= 1e-5 * sw + 1e-30)
