"""Pins of the oracle's operand preparation for the reduced-precision GEMM modes.

bf16 rounding is round-to-nearest-even to 8 significant bits; torch's CPU cast is
the library cross-check and hand-built halfway cases pin tie-to-even.  The hi/lo
split obeys |a - hi - lo| <= 2^-16 |a|.  FP8 is OCP E4M3 (max 448, min normal
2^-6, subnormal quantum 2^-9), cross-checked against torch.float8_e4m3fn; block
exponents are pinned by their defining property (largest e with amax 2^e <= 448).
"""
import struct

import numpy as np
import pytest
import torch

import oracle
import rise_inputs as ri


def f32_from_bits(u):
    return struct.unpack("<f", struct.pack("<I", u))[0]


def test_bf16_round_matches_torch_cast():
    g = ri.rng(61)
    x = np.concatenate([
        g.standard_normal(100000).astype(np.float32),
        (g.standard_normal(1000) * 1e-30).astype(np.float32),
        (g.standard_normal(1000) * 1e30).astype(np.float32),
        np.array([0.0, -0.0, 1.0, -1.0, 3.0e38], dtype=np.float32),
    ])
    ours = oracle.quant_bf16(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


def test_bf16_ties_go_to_even():
    # 1 + 2^-8 is exactly halfway between 1 and 1 + 2^-7: ties to the even mantissa (1)
    assert oracle.round_bf16(1.0 + 2.0 ** -8) == 1.0
    # 1 + 3*2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6
    assert oracle.round_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    # just above halfway rounds up
    assert oracle.round_bf16(f32_from_bits(0x3F808001)) == 1.0 + 2.0 ** -7
    # truncation would give 1.0 here; nearest is 1 + 2^-7
    assert oracle.round_bf16(1.0 + 2.0 ** -7 - 2.0 ** -20) == 1.0 + 2.0 ** -7


def test_hi_lo_split_error_bound():
    g = ri.rng(67)
    x = (g.standard_normal(50000) * np.exp2(g.uniform(-4, 4, 50000))).astype(np.float32)
    hi, lo = oracle.split_bf16(x)
    h = oracle.bf16_bits_to_f32(hi).astype(np.float64)
    l = oracle.bf16_bits_to_f32(lo).astype(np.float64)
    xd = x.astype(np.float64)
    assert np.array_equal(hi, oracle.quant_bf16(x))
    assert np.all(np.abs(xd - h - l) <= 2.0 ** -16 * np.abs(xd))
    # lo is the bf16 rounding of the exact residual
    assert np.array_equal(lo, oracle.quant_bf16((xd - h).astype(np.float32)))
    p1, p2, p3 = oracle.split3_bf16(x)
    s = sum(oracle.bf16_bits_to_f32(p).astype(np.float64) for p in (p1, p2, p3))
    assert np.all(np.abs(xd - s) <= 2.0 ** -24 * np.abs(xd))


def test_e4m3_round_matches_torch_in_range():
    g = ri.rng(71)
    x = np.concatenate([
        g.uniform(-448, 448, 20000),
        g.standard_normal(20000) * 0.01,
        g.standard_normal(5000) * 1e-3,
        [0.0, 448.0, -448.0, 2.0 ** -9, 2.0 ** -10, 3 * 2.0 ** -11, 240.0, 464.0 - 1e-3],
    ]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    ours = np.array([oracle.round_e4m3(v) for v in x])
    ok = np.abs(x) <= 448
    assert np.array_equal(ours[ok], ref[ok])


def test_e4m3_saturates_and_decodes():
    assert oracle.round_e4m3(1000.0) == 448.0
    assert oracle.round_e4m3(-470.0) == -448.0
    assert oracle.e4m3_decode(0x7E) == 448.0
    assert oracle.e4m3_decode(0x01) == 2.0 ** -9
    assert oracle.e4m3_decode(0x08) == 2.0 ** -6
    assert oracle.e4m3_decode(0xB8) == -1.0
    assert np.isnan(oracle.e4m3_decode(0x7F))
    # every finite code decodes to a value that round-trips through the rounding
    for b in range(256):
        v = oracle.e4m3_decode(b)
        if not np.isnan(v):
            assert oracle.round_e4m3(v) == v


@pytest.mark.parametrize("amax", [448.0, 447.9, 448.1, 1.0, 0.875, 0.8751, 1e-3, 3.0e5, 2.0 ** -20])
def test_block_exponent_is_the_largest_that_fits(amax):
    a = float(np.float32(amax))
    e = oracle.e4m3_block_exponent(a)
    assert a * 2.0 ** e <= 448.0
    assert a * 2.0 ** (e + 1) > 448.0


def test_block_quantisation_layout_and_values():
    g = ri.rng(73)
    A = ri.gemm_scaled_normal(5, 3, 70, 1004)[0]
    q, s = oracle.quant_e4m3_rows(A, blk=32)
    assert q.shape == (5, 70) and s.shape == (5, 3)
    for i in range(5):
        for b in range(3):
            blk = A[i, 32 * b:min(32 * b + 32, 70)].astype(np.float64)
            e = 127 - int(s[i, b])
            assert np.max(np.abs(blk)) * 2.0 ** e <= 448.0
            deq = np.array([oracle.e4m3_decode(v) for v in q[i, 32 * b:32 * b + len(blk)]])
            ref = np.array([oracle.round_e4m3(v * 2.0 ** e) for v in blk])
            assert np.array_equal(deq, ref)
    # the column form of B equals the row form of B^T
    B = ri.gemm_scaled_normal(3, 6, 40, 1004)[1]
    qc, sc = oracle.quant_e4m3_cols(B, blk=32)
    qr, sr = oracle.quant_e4m3_rows(np.ascontiguousarray(B.T), blk=32)
    assert np.array_equal(qc, qr) and np.array_equal(sc, sr)


def test_gemm_modes_on_exact_integers():
    # integers with |v| <= 16 are exact in bf16 and E4M3: every mode gives the exact product
    g = ri.rng(79)
    A = ri.integer_matrix(g, 9, 64, bound=2)
    B = ri.integer_matrix(g, 64, 7, bound=2)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    for mode in (oracle.MODE_F32, oracle.MODE_BF16, oracle.MODE_BF16X3, oracle.MODE_BF16X6,
                 oracle.MODE_FP8):
        assert np.array_equal(oracle.gemm_mode(A, B, mode), exact), mode


def test_gemm_mode_definitions():
    g = ri.rng(83)
    A, B = ri.gemm_scaled_normal(6, 5, 48, 1004)
    Ad, Bd = A.astype(np.float64), B.astype(np.float64)
    np.testing.assert_allclose(oracle.gemm_mode(A, B, oracle.MODE_F32), Ad @ Bd, rtol=1e-13)
    bf = lambda X: oracle.bf16_bits_to_f32(oracle.quant_bf16(X)).astype(np.float64)
    np.testing.assert_allclose(oracle.gemm_mode(A, B, oracle.MODE_BF16), bf(A) @ bf(B),
                               rtol=1e-13, atol=1e-13)
    Ah, Al = [oracle.bf16_bits_to_f32(p).astype(np.float64) for p in oracle.split_bf16(A)]
    Bh, Bl = [oracle.bf16_bits_to_f32(p).astype(np.float64) for p in oracle.split_bf16(B)]
    np.testing.assert_allclose(oracle.gemm_mode(A, B, oracle.MODE_BF16X3),
                               Ah @ Bh + Ah @ Bl + Al @ Bh, rtol=1e-13, atol=1e-13)
    # BF16X6: exactly the six products A_i B_j with i + j <= 4 of the three-way
    # splits -- neither fewer nor more (A2 B3, A3 B2 and A3 B3 are left out)
    A1, A2, A3 = [oracle.bf16_bits_to_f32(p).astype(np.float64).reshape(A.shape)
                  for p in oracle.split3_bf16(A)]
    B1, B2, B3 = [oracle.bf16_bits_to_f32(p).astype(np.float64).reshape(B.shape)
                  for p in oracle.split3_bf16(B)]
    six = A1 @ B1 + A1 @ B2 + A2 @ B1 + A1 @ B3 + A2 @ B2 + A3 @ B1
    x6 = oracle.gemm_mode(A, B, oracle.MODE_BF16X6)
    sc = np.abs(Ad) @ np.abs(Bd)
    # each left-out product reaches well above 1e-14 of the scale somewhere, so a
    # seventh product would show; the comparisons allow only fp64 reordering
    for P in (A2 @ B3, A3 @ B2, A3 @ B3):
        assert np.max(np.abs(P) / sc) > 1e-12
    dropped = A2 @ B3 + A3 @ B2 + A3 @ B3
    assert np.max(np.abs(x6 - six) / sc) < 1e-14
    full = (A1 + A2 + A3) @ (B1 + B2 + B3)
    assert np.max(np.abs(x6 + dropped - full) / sc) < 1e-14
    qa, sa = oracle.quant_e4m3_rows(A)
    qb, sb = oracle.quant_e4m3_cols(B)
    dec = np.vectorize(oracle.e4m3_decode)
    Aq = dec(qa) * np.exp2(np.repeat(sa.astype(np.float64) - 127, 32, axis=1)[:, :48])
    Bq = (dec(qb) * np.exp2(np.repeat(sb.astype(np.float64) - 127, 32, axis=1)[:, :48])).T
    np.testing.assert_allclose(oracle.gemm_mode(A, B, oracle.MODE_FP8), Aq @ Bq, rtol=1e-13,
                               atol=1e-13)
    # the compensated forms get closer to the f32 product than plain bf16
    ref = Ad @ Bd
    scale = np.abs(Ad) @ np.abs(Bd)
    e1 = np.max(np.abs(oracle.gemm_mode(A, B, oracle.MODE_BF16) - ref) / scale)
    e3 = np.max(np.abs(oracle.gemm_mode(A, B, oracle.MODE_BF16X3) - ref) / scale)
    e6 = np.max(np.abs(oracle.gemm_mode(A, B, oracle.MODE_BF16X6) - ref) / scale)
    assert e3 < 2.0 ** -14 < e1 and e6 < 2.0 ** -20
