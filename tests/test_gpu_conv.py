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


def _taps(img, pad):
    """The nine shifted views (dy, dx) of an NHWC batch under pad2D(1): element
    [b, y, x, c] of view (dy, dx) is img[b, y + dy - 1, x + dx - 1, c], outside the
    image 0 (zero) or the nearest edge pixel (clamp)."""
    B, H, W, C = img.shape
    p = np.pad(img, ((0, 0), (1, 1), (1, 1), (0, 0)), mode="edge" if pad == "clamp" else "constant")
    return [p[:, dy:dy + H, dx:dx + W, :] for dy in range(3) for dx in range(3)]


def dw_scale(g_abs, x_abs, pad):
    """sum over (b, y, x) of |dOut| * |window| per (co, ci, dy, dx): the componentwise
    scale of dW (a tolerance only; the expected values come from the oracle)."""
    Cout, Cin = g_abs.shape[-1], x_abs.shape[-1]
    G = g_abs.reshape(-1, Cout).astype(np.float64)
    out = np.empty((Cout, Cin, 9))
    for t, v in enumerate(_taps(x_abs, pad)):
        out[:, :, t] = G.T @ v.reshape(-1, Cin).astype(np.float64)
    return out.reshape(Cout, Cin, 3, 3)


def din_scale(g_abs, w_abs):
    """|dIn| scale under zero padding: sum over taps and co of |dOut| |w| at the
    pixels whose window holds this one (the adjoint applied to absolute values)."""
    B, H, W, Cout = g_abs.shape
    Cin = w_abs.shape[1]
    out = np.zeros((B, H, W, Cin))
    gp = np.pad(g_abs.astype(np.float64), ((0, 0), (1, 1), (1, 1), (0, 0)))
    for dy in range(3):
        for dx in range(3):
            # pixel (y, x) is tap (dy, dx) of output (y - dy + 1, x - dx + 1)
            src = gp[:, 2 - dy:2 - dy + H, 2 - dx:2 - dx + W, :]
            out += src @ w_abs[:, :, dy, dx].astype(np.float64)
    return out


def check_dw(got, ref, scale):
    err = np.abs(np.asarray(got, np.float64) - ref)
    assert np.all(err <= 1e-5 * scale + 1e-30), float(np.max(err / (scale + 1e-30)))


@pytest.mark.parametrize("pad", ["zero", "clamp"])
def test_layer_backward_multi_tile(rise, pad):
    # 8 x 200 x 129 (ragged in both dimensions) with 32 -> 32 channels: 2400 dW
    # tiles over 512 persistent workgroups, so every workgroup walks a run of
    # several tiles (with the next tile's loads in flight) before the fixed-order
    # reduction of the partials; all of dW and (zero padding) all of dIn against
    # the oracle.  dIn under clamp padding is refused by the library.
    B, H, W, C = 8, 200, 129, 32
    x, w, dout = ri.conv_inputs(B, C, C, H, W, seed=ri.SEED_CONV + 3, w_std=0.05)
    pm = oracle.PAD_ZERO if pad == "zero" else oracle.PAD_CLAMP
    print(f"conv bwd multi-tile pad={pad}", flush=True)
    dIn, dW = rise.conv2d_backward(bf16_dev(dout), bf16_dev(x), dev(w), pad=pad,
                                   need_din=pad == "zero")
    xf = oracle.bf16_bits_to_f32(x).reshape(x.shape)
    gf = oracle.bf16_bits_to_f32(dout).reshape(dout.shape)
    rin, rw = oracle.conv2d_backward(gf, x, wq(w), pm, want_din=pad == "zero")
    check_dw(host(dW), rw, dw_scale(np.abs(gf), np.abs(xf), pad))
    if pad == "zero":
        check_out(decode(dIn), rin, din_scale(np.abs(gf), np.abs(wq(w))))


def test_layer_backward_clamp_din_refused(rise):
    x, w, dout = case_inputs(1, 4, 8, 32, 32, 5)
    with pytest.raises(rise.RiseError, match="zero padding"):
        rise.conv2d_backward(bf16_dev(dout), bf16_dev(x), dev(w), pad="clamp")


def test_config_layer_backward(rise):
    # The layer's full size (batch 32, 64 -> 64 channels, 512 x 512), launched as
    # the benchmark launches it.
    #  * all of dW for image 0 (its own launch: 2048 tiles, four per persistent
    #    workgroup) against the oracle, element by element;
    #  * the batch's dW equals the sum of the 32 per-image dW (each a launch of
    #    its own), within the FP32 accumulation bound of the summed scales;
    #  * dIn of the batch launch on full-width bands of rows at the top, middle
    #    and bottom of three images against the oracle on the same bands (with
    #    their one-row halo of dOut).
    import torch

    B, H, W, C = 32, 512, 512, 64
    x, w, dout = ri.conv_inputs(B, C, C, H, W, seed=ri.SEED_CONV + 1)
    dx_, dg_ = bf16_dev(x), bf16_dev(dout)
    print("conv full-size backward", flush=True)
    dIn, dW = rise.conv2d_backward(dg_, dx_, dev(w))
    dW = host(dW).astype(np.float64)
    per = []
    for b in range(B):
        _, dWb = rise.conv2d_backward(dg_[b:b + 1], dx_[b:b + 1], dev(w), need_din=False)
        per.append(host(dWb).astype(np.float64))
    torch.cuda.synchronize()
    xf = oracle.bf16_bits_to_f32(x).reshape(x.shape)
    gf = oracle.bf16_bits_to_f32(dout).reshape(dout.shape)
    scales = [dw_scale(np.abs(gf[b:b + 1]), np.abs(xf[b:b + 1]), "zero") for b in range(B)]
    print("conv full-size backward: oracle dW of image 0", flush=True)
    _, rw0 = oracle.conv2d_backward(gf[:1], x[:1], wq(w), oracle.PAD_ZERO, want_din=False)
    check_dw(per[0], rw0, scales[0])
    check_dw(dW, np.sum(per, axis=0), 2 * np.sum(scales, axis=0))
    dIn_h = decode(dIn)
    for b, y0 in [(0, 0), (13, 200), (31, 448)]:
        ys, ye = max(y0 - 1, 0), min(y0 + 65, H)
        rin, _ = oracle.conv2d_backward(gf[b:b + 1, ys:ye], x[b:b + 1, ys:ye], wq(w),
                                        oracle.PAD_ZERO, want_dw=False)
        sin = din_scale(np.abs(gf[b:b + 1, ys:ye]), np.abs(wq(w)))
        # rows whose contributing dOut rows all lie in the band (or beyond an image edge)
        lo = y0 - ys
        hi = min(64, (ye - ys) - lo - (1 if ye < H else 0))
        check_out(dIn_h[b, y0:y0 + hi], rin[0, lo:lo + hi], sin[0, lo:lo + hi])


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
