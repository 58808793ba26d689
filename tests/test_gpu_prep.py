"""GPU parity of the operand preparation (bf16 rounding, hi/lo and three-way
splits, FP8 E4M3 with block scales): byte work, compared bit for bit with the
oracle's encodings, including the zero padding."""
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


def prep(rise, src, mode, rows, K, ld_r, ld_k, rows_out, k_out):
    print(f"prep {mode} rows={rows} K={K} ld=({ld_r},{ld_k}) out=({rows_out},{k_out})",
          flush=True)
    return host(rise.prep_operand(dev(src), mode, rows=rows, K=K, ld_r=ld_r, ld_k=ld_k,
                                  rows_out=rows_out, k_out=k_out))


def planes16(buf, parts, rows_out, k_out):
    return buf.view(np.uint16).reshape(parts, rows_out, k_out)


CASES = [(64, 64, 64, 64), (100, 70, 128, 96), (5, 3, 64, 64), (130, 200, 256, 256)]


@pytest.mark.parametrize("rows,K,rows_out,k_out", CASES)
@pytest.mark.parametrize("layout", ["rowmajor", "colmajor", "strided"])
def test_bf16_splits_bit_exact(rise, rows, K, rows_out, k_out, layout):
    g = ri.rng(rows + K)
    X = (g.standard_normal((rows, K)) * np.exp2(g.uniform(-4, 4, (rows, 1)))).astype(np.float32)
    if layout == "rowmajor":
        src, ld_r, ld_k = X, K, 1
    elif layout == "colmajor":
        src, ld_r, ld_k = np.ascontiguousarray(X.T), 1, rows
    else:  # padded rows, odd leading dimension: scalar loads
        src = np.zeros((rows, K + 3), np.float32)
        src[:, :K] = X
        ld_r, ld_k = K + 3, 1
    refs = {"bf16": (oracle.quant_bf16(X),), "bf16x3": oracle.split_bf16(X),
            "bf16x6": oracle.split3_bf16(X)}
    for mode, parts in refs.items():
        got = planes16(prep(rise, src, mode, rows, K, ld_r, ld_k, rows_out, k_out), len(parts),
                       rows_out, k_out)
        for p, ref in enumerate(parts):
            assert np.array_equal(got[p, :rows, :K], ref), (mode, p)
            assert not got[p, rows:, :].any() and not got[p, :, K:].any()


@pytest.mark.parametrize("rows,K,rows_out,k_out", [(64, 64, 64, 64), (100, 70, 128, 96),
                                                   (33, 200, 64, 224)])
@pytest.mark.parametrize("layout", ["rowmajor", "colmajor"])
def test_fp8_blocks_bit_exact(rise, rows, K, rows_out, k_out, layout):
    g = ri.rng(3 * rows + K)
    X = (g.standard_normal((rows, K)) * np.exp2(g.uniform(-4, 4, (rows, 1)))).astype(np.float32)
    X[0, :min(K, 32)] = 0.0           # an all-zero block: scale exponent 0
    X[min(1, rows - 1), 0] = 448.0    # a block whose amax is exactly the format maximum
    if rows > 2:
        X[2, :] *= 1e-6               # subnormal E4M3 codes
    if layout == "rowmajor":
        src, ld_r, ld_k = X, K, 1
    else:
        src, ld_r, ld_k = np.ascontiguousarray(X.T), 1, rows
    buf = prep(rise, src, "fp8", rows, K, ld_r, ld_k, rows_out, k_out)
    q = buf[:rows_out * k_out].reshape(rows_out, k_out)
    s = buf[rows_out * k_out:].reshape(rows_out, k_out // 32)
    qref, sref = oracle.quant_e4m3_rows(X, blk=32)
    nb = (K + 31) // 32
    assert np.array_equal(q[:rows, :K], qref)
    assert np.array_equal(s[:rows, :nb], sref)
    assert not q[rows:, :].any() and not q[:, K:].any()


def test_bf16_rounding_edge_values(rise):
    vals = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 3.0e38, -3.4e38,
                     1e-40, -1e-40, 0.0, -0.0, np.float32(np.inf), 65504.0, 1.00390625],
                    dtype=np.float32)
    X = np.tile(vals, (1, 1))
    got = prep(rise, X, "bf16", 1, vals.size, vals.size, 1, 1, vals.size)
    assert np.array_equal(got.view(np.uint16).reshape(1, -1)[0], oracle.quant_bf16(vals))
