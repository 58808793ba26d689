"""GPU parity of the batched persistent launch (rise_plan_*): every problem of a
batch against the oracle, graph replays against each other, and the chosen
tiles.  Each problem is checked with the same bar as its one-problem entry point
(componentwise 1e-5 for FP32; bf16-stored GEMMs against the oracle on the same
bf16 operands)."""
import ctypes
import os
import tempfile

import numpy as np
import pytest

import oracle
import rise_inputs as ri
from _helpers import componentwise, dev, gemm_scale_sampled, host, stencil_scale

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def rise():
    import paper_2201_03611_amd as rise

    return rise


def make_batch(g, n_f32, n_bf16, n_st, lo, hi, slo, shi, sizes=None):
    """Host inputs of a mixed batch: FP32 GEMMs, bf16 GEMMs, stencils."""
    gemms = []
    for i in range(n_f32 + n_bf16):
        if sizes is not None:
            M, N, K = (int(v) for v in sizes[i % len(sizes)])
        else:
            M, N, K = (int(v) for v in g.choice(np.arange(lo, hi + 1, 32), size=3))
        opB = int(g.integers(0, 2))
        A = ri.uniform_matrix(g, M, K)
        B = ri.uniform_matrix(g, K, N)
        bf16 = i >= n_f32
        gemms.append(dict(M=M, N=N, K=K, opB=opB, A=A, B=B, bf16=bf16))
    stencils = []
    for i in range(n_st):
        side = int(g.integers(slo, shi + 1))
        k = int(g.choice([3, 5, 7]))
        img = ri.uniform_matrix(g, side, side, 0.0, 1.0)
        w = ri.random_weights(g, k)
        stencils.append(dict(H=side, W=side, k=k, img=img, w=w, pad=int(g.integers(0, 2))))
    return gemms, stencils


def to_device(rise, gemms, stencils):
    import torch

    from paper_2201_03611_amd._lib import RISE_BF16, RISE_F32

    keep = []
    gp = (rise.RiseGemmProblem * max(len(gemms), 1))()
    for i, p in enumerate(gemms):
        if p["bf16"]:
            A = dev(ri.bf16_bits_from_f32(p["A"])).view(torch.bfloat16)
            Bh = p["B"] if p["opB"] == 0 else np.ascontiguousarray(p["B"].T)
            B = dev(ri.bf16_bits_from_f32(Bh)).view(torch.bfloat16)
        else:
            A = dev(p["A"])
            B = dev(p["B"] if p["opB"] == 0 else np.ascontiguousarray(p["B"].T))
        C = torch.full((p["M"], p["N"]), float("nan"), device="cuda")
        keep += [A, B, C]
        p["dC"] = C
        gp[i] = rise.RiseGemmProblem(C.data_ptr(), A.data_ptr(), B.data_ptr(), p["M"], p["N"],
                                     p["K"], p["K"], B.shape[1], p["N"],
                                     RISE_BF16 if p["bf16"] else RISE_F32, p["opB"])
    sp = (rise.RiseStencilProblem * max(len(stencils), 1))()
    for i, p in enumerate(stencils):
        img = dev(p["img"])
        w = dev(p["w"])
        out = torch.full((p["H"], p["W"]), float("nan"), device="cuda")
        keep += [img, w, out]
        p["dOut"] = out
        sp[i] = rise.RiseStencilProblem(out.data_ptr(), img.data_ptr(), w.data_ptr(), p["H"],
                                        p["W"], p["W"], p["W"], p["k"], p["pad"])
    return gp, sp, keep


def check_gemm(p, C, samples=None):
    A, B = p["A"], p["B"]
    if p["bf16"]:
        A = oracle.bf16_bits_to_f32(ri.bf16_bits_from_f32(A)).reshape(A.shape)
        B = oracle.bf16_bits_to_f32(ri.bf16_bits_from_f32(B)).reshape(B.shape)
    if samples is None:
        ref = oracle.gemm(A, B)
        assert componentwise(C, ref, oracle.gemm(np.abs(A), np.abs(B))) <= TOL
    else:
        rows, cols = ri.sample_indices(ri.rng(samples), p["M"], p["N"], 16)
        ref = oracle.gemm_sampled(A, B, rows, cols)
        assert componentwise(C[rows, cols], ref, gemm_scale_sampled(A, B, rows, cols)) <= TOL


def check_stencil(p, out, rows=None):
    pad = oracle.PAD_ZERO if p["pad"] == 1 else oracle.PAD_CLAMP
    if rows is None:
        ref = oracle.stencil2d(p["img"], p["w"], pad)
        assert componentwise(out, ref, stencil_scale(p["img"], p["w"], pad)) <= TOL
        return
    r = (p["k"] - 1) // 2
    for y in rows:
        y0, y1 = max(0, y - r), min(p["H"], y + r + 1)
        crop = np.ascontiguousarray(p["img"][y0:y1])
        # rows of the crop at true image edges are padded like the image; interior crop
        # edges are never read by row y's window
        ref = oracle.stencil2d(crop, p["w"], pad)[y - y0]
        sc = stencil_scale(crop, p["w"], pad)[y - y0]
        assert componentwise(out[y], ref, sc) <= TOL


def test_small_mixed_batch_and_graph_replays(rise):
    import torch

    g = ri.rng(2024)
    gemms, stencils = make_batch(g, 24, 12, 14, 32, 320, 20, 600)
    gp, sp, keep = to_device(rise, gemms, stencils)
    print(f"batch: {len(gemms)} gemms, {len(stencils)} stencils", flush=True)
    plan = rise.Plan(gp, len(gemms), sp, len(stencils))
    assert plan.items() > 0
    for rep in range(3):
        for p in gemms:
            p["dC"].fill_(float("nan"))
        for p in stencils:
            p["dOut"].fill_(float("nan"))
        torch.cuda.synchronize()
        if rep == 0:
            plan.launch()
        elif rep == 1:  # back to back: the plan's two graph instances in turn
            plan.launch()
            plan.launch()
        else:
            plan.launch_direct()
        torch.cuda.synchronize()
        for p in gemms:
            check_gemm(p, host(p["dC"]))
        for p in stencils:
            check_stencil(p, host(p["dOut"]))
    for i, p in enumerate(gemms):
        bm, bn, bk = plan.tile(i)
        # the persistent kernel's FP32 tiles are 16 deep in K, its bf16 tiles 64
        assert bm in (64, 128) and bn in (64, 128) and bk == (64 if p["bf16"] else 16)
    with pytest.raises(rise.RiseError, match="not a GEMM problem"):
        plan.tile(len(gemms))  # the first stencil
    with pytest.raises(rise.RiseError, match="outside the plan"):
        plan.tile(len(gemms) + len(stencils))
    plan.destroy()


def test_f32_tiles_both_schedules(rise):
    # K a multiple of 16 takes the asynchronous-ring tile, any other K the
    # register-staged one (zero-filled k past K); both in one plan, both opB
    import torch

    g = ri.rng(31)
    sizes = [(96, 160, 64), (200, 72, 44), (128, 128, 100), (64, 96, 20), (136, 264, 48)]
    gemms = []
    for i, (M, N, K) in enumerate(sizes * 2):
        gemms.append(dict(M=M, N=N, K=K, opB=i % 2, A=ri.uniform_matrix(g, M, K),
                          B=ri.uniform_matrix(g, K, N), bf16=False))
    gp, sp, keep = to_device(rise, gemms, [])
    print(f"batch: {len(gemms)} f32 gemms, K in {sorted(set(s[2] for s in sizes))}", flush=True)
    plan = rise.Plan(gp, len(gemms), sp, 0)
    plan.launch()
    torch.cuda.synchronize()
    for p in gemms:
        check_gemm(p, host(p["dC"]))
    plan.destroy()


def test_bf16_items_ragged(rise):
    # bf16 GEMMs with M and N ragged against the 64 and 128 tiles and K a
    # multiple of 8 that is not a whole number of 64-k slabs (zero-filled chunks)
    import torch

    g = ri.rng(4242)
    sizes = [(70, 136, 96), (200, 72, 64), (130, 264, 288), (64, 64, 32),
             (50, 72, 40), (130, 200, 200), (257, 136, 72), (33, 8, 264)]
    gemms = []
    for opB in (0, 1):
        for M, N, K in sizes:
            gemms.append(dict(M=M, N=N, K=K, opB=opB, A=ri.uniform_matrix(g, M, K),
                              B=ri.uniform_matrix(g, K, N), bf16=True))
    gp, sp, keep = to_device(rise, gemms, [])
    print(f"batch: {len(gemms)} bf16 gemms", flush=True)
    plan = rise.Plan(gp, len(gemms), sp, 0)
    for rep in range(2):
        for p in gemms:
            p["dC"].fill_(float("nan"))
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for p in gemms:
            check_gemm(p, host(p["dC"]))
    for i in range(len(gemms)):
        assert plan.tile(i)[2] == 64
    plan.destroy()


def test_batched_equals_single_calls(rise):
    import torch

    g = ri.rng(7)
    gemms, stencils = make_batch(g, 6, 0, 4, 64, 256, 100, 300)
    gp, sp, keep = to_device(rise, gemms, stencils)
    rise.rise_gemm_batched(gp, len(gemms))
    rise.rise_stencil2d_batched(sp, len(stencils))
    torch.cuda.synchronize()
    for p in gemms:
        single = rise.gemm(dev(p["A"]), dev(p["B"]))
        assert componentwise(host(p["dC"]), host(single).astype(np.float64),
                             oracle.gemm(np.abs(p["A"]), np.abs(p["B"]))) <= 2 * TOL
    for p in stencils:
        single = rise.stencil2d(dev(p["img"]), dev(p["w"]), pad="zero" if p["pad"] else "clamp")
        assert np.array_equal(host(p["dOut"]), host(single))  # same tile code, same order


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_config_batch_sampled(rise, dtype):
    # the batched workload: 512 GEMMs with M, N, K uniform on {64, 96, ..., 1024},
    # plus 256 stencils with side U{256..2048}, k in {3, 5, 7}, weights summing to 1
    import torch

    sizes = ri.batched_gemm_sizes()
    specs = ri.batched_stencil_specs()
    g = ri.rng(ri.SEED_BATCHED + 1)
    gemms = []
    for i in range(512):
        M, N, K = (int(v) for v in sizes[i])
        gemms.append(dict(M=M, N=N, K=K, opB=0, A=ri.uniform_matrix(g, M, K),
                          B=ri.uniform_matrix(g, K, N), bf16=dtype == "bf16"))
    stencils = []
    for i in range(256):
        side, k = (int(v) for v in specs[i])
        stencils.append(dict(H=side, W=side, k=k, img=ri.uniform_matrix(g, side, side, 0.0, 1.0),
                             w=ri.random_weights(g, k), pad=0))
    gp, sp, keep = to_device(rise, gemms, stencils)
    print(f"config batch {dtype}", flush=True)
    plan = rise.Plan(gp, 512, sp, 256)
    plan.launch()
    torch.cuda.synchronize()
    for i, p in enumerate(gemms):
        check_gemm(p, host(p["dC"]), samples=i)
    for i, p in enumerate(stencils):
        H = p["H"]
        check_stencil(p, host(p["dOut"]), rows=[0, 1, H // 2, H - 1])
    plan.destroy()


def test_autotune_table(rise):
    path = os.path.join(tempfile.mkdtemp(), "tune.txt")
    print("autotune", flush=True)
    rise.rise_autotune_batched(path)
    rows = [l.split() for l in open(path) if l.strip()]
    names = {r[0] for r in rows}
    assert len(rows) == 20 and "f32_128x128_N" in names and "stencil_5_scalar" in names
    for r in rows:
        a, b = float(r[1]), float(r[2])
        assert a + b * 1024 > 0
    # a plan built from the measured table works
    g = ri.rng(1)
    gemms, stencils = make_batch(g, 3, 1, 2, 64, 192, 50, 120)
    gp, sp, keep = to_device(rise, gemms, stencils)
    plan = rise.Plan(gp, len(gemms), sp, len(stencils), tune_table=path)
    plan.launch()
    import torch

    torch.cuda.synchronize()
    for p in gemms:
        check_gemm(p, host(p["dC"]))
    plan.destroy()


def test_stencils_with_aligned_rows_and_ragged_width(rise):
    # row pitch a multiple of 4 floats, width not: the last 16-byte chunk of a
    # row straddles the edge, which the whole-chunk fetch must not be used for
    import torch

    g = ri.rng(31)
    specs = [(50, 121, 124, 5, 0), (37, 258, 260, 3, 1), (70, 1021, 1024, 7, 0), (33, 6, 8, 5, 1)]
    sp = (rise.RiseStencilProblem * len(specs))()
    keep, refs = [], []
    for i, (H, W, ld, k, pad) in enumerate(specs):
        big = ri.uniform_matrix(g, H, ld, 0.0, 1.0)
        img = np.ascontiguousarray(big[:, :W])
        w = ri.random_weights(g, k)
        din, dw = dev(big), dev(w)
        out = torch.full((H, ld), float("nan"), device="cuda")
        keep += [din, dw, out]
        sp[i] = rise.RiseStencilProblem(out.data_ptr(), din.data_ptr(), dw.data_ptr(), H, W, ld, ld,
                                        k, pad)
        refs.append((img, w, pad, out, W))
    print(f"batched stencils, aligned rows with ragged widths: {specs}", flush=True)
    rise.rise_stencil2d_batched(sp, len(specs))
    torch.cuda.synchronize()
    for img, w, pad, out, W in refs:
        p = oracle.PAD_ZERO if pad == 1 else oracle.PAD_CLAMP
        o = host(out)
        assert np.all(np.isnan(o[:, W:]))
        assert componentwise(o[:, :W], oracle.stencil2d(img, w, p), stencil_scale(img, w, p)) <= TOL
