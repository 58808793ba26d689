"""Benchmark of the dense RISE patterns on one MI355X.

A step is one pass of the timed workload: the FP32 GEMM C = A B with
M = N = K = 4096 (A, B ~ U(-1,1)) followed by the 4096 x 4096 FP32 stencil with
the 5 x 5 normalised Gaussian (sigma 1), clamp padding.  Inputs are resident
in HBM before timing starts; the stencil rotates over several input/output
buffer sets (more than the 256 MB last-level cache) so each launch reads HBM.

One JSON line is printed.  Besides the contract fields it carries
  roofline          GEMM kernel (dominant): algorithmic flops / event time
  roofline_stencil  stencil kernel: algorithmic bytes (8 B per pixel) / event time
  precision         8192^3 GEMM, N(0,1) 2^U(-4,4): time and componentwise error vs
                    the exact product per mode, and the FP32 / BF16X3 speedup
  cpu_baseline      the oracle on a bounded sample of the same workload
  strategy          beside each result, the schedule the library chose for it
                    (tile, stencil schedule, passes, K split, steps per launch)
Kernel times come from HIP events recorded on the stream the kernels run on.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA = 157.3   # TFLOP/s, MI355X dense FP32 matrix
PEAK_BF16 = 2516.6       # TFLOP/s dense
PEAK_FP8 = 5033.0
PEAK_HBM = 8000.0        # GB/s
PEAK_F32_VEC = 157.3     # TFLOP/s, MI355X FP32 vector (counts packed dual-issue FP32)

M = N = K = 4096
H = W = 4096
KS = 5


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--no-precision", action="store_true", help="skip the 8192^3 precision leg")
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline leg")
    p.add_argument("--no-extra", action="store_true",
                   help="skip the batched, stencil-layer, GEMV and iterate legs")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 1 GiB device copy (HBM counter calibration)")
    p.add_argument("--only", default=None,
                   choices=["gemm_f32", "gemm_bf16", "gemm_bf16x3", "gemm_fp8", "stencil",
                            "conv_fwd", "conv_bwd", "batched", "gemv", "gemv_t", "iterate_sum",
                            "iterate_sum_fanin3", "iterate_sum_fanin8", "stencil_iterate",
                            "stencil_iterate_1"],
                   help="run one kernel of the path --reps times (for profilers) and exit")
    p.add_argument("--reps", type=int, default=5)
    return p.parse_args()


def src_hash(*rel):
    h = hashlib.sha256()
    for r in rel:
        with open(os.path.join(ROOT, r), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(kernel, source_files, launches_per_unit=1):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        tab = json.load(f)
    row = tab.get(kernel)
    if not row or row.get("source_hash") != src_hash(*source_files):
        return None
    return row.get("bytes_per_launch")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build has no multi-GPU path); "
              f"got --gpus {args.gpus}", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2201_03611_amd as rise
    import rise_inputs as ri

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    if args.only:
        run_only(args.only, args.reps, rise, ri, torch, dev, stream)
        return

    if args.copy_calibration:
        a = torch.empty(1 << 28, device=dev, dtype=torch.float32)  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": a.numel() * 4}))
        return

    # ---- inputs --------------------------------------------------------------
    A, B = ri.gemm_uniform(M, N, K, ri.SEED_GEMM_F32)
    img = ri.image_uniform(H, W, ri.SEED_STENCIL)
    wts = ri.gaussian_weights(KS, 1.0)
    dA, dB = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
    dC = torch.empty((M, N), device=dev, dtype=torch.float32)
    nsets = 6  # 6 x 128 MiB > 256 MB last-level cache
    imgs = [torch.from_numpy(img).to(dev) for _ in range(nsets)]
    outs = [torch.empty((H, W), device=dev, dtype=torch.float32) for _ in range(nsets)]
    dw = torch.from_numpy(wts).to(dev)
    torch.cuda.synchronize()

    def step(i, ev=None):
        if ev is not None:
            ev[0].record(stream)
        rise.rise_gemm(dC, dA, dB, M, N, K, lda=K, ldb=N, ldc=N, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        s = i % nsets
        rise.rise_stencil2d(outs[s], imgs[s], dw, H, W, ld_out=W, ld_in=W, kh=KS, kw=KS,
                            pad="clamp", stream=stream)
        if ev is not None:
            ev[2].record(stream)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i, evs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    t_gemm = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps  # ms
    t_sten = sum(e[1].elapsed_time(e[2]) for e in evs) / args.steps

    flops_gemm = 2.0 * M * N * K
    flops_sten = 2.0 * KS * KS * H * W
    bytes_sten = 8.0 * H * W
    gemm_tf = flops_gemm / (t_gemm * 1e-3) / 1e12
    sten_gbs = bytes_sten / (t_sten * 1e-3) / 1e9
    value = (flops_gemm + flops_sten) / (ms_step * 1e-3) / 1e12

    # the 256 x 128 x 16 tile runs the asynchronous-ring kernel for these operands
    # (contiguous, 16-byte aligned rows, K a multiple of 16); other tiles run the
    # register-staged one
    gt = rise.rise_gemm_default_tile(M, N, K, "f32")
    gemm_kernel = "gemm_f32_async_kernel" if tuple(gt) == (256, 128, 16) else "gemm_f32_kernel"
    gemm_traffic = traffic_for(gemm_kernel, ["paper_2201_03611_amd/csrc/gemm_f32.hip",
                                             "paper_2201_03611_amd/csrc/async_copy.h",
                                             "paper_2201_03611_amd/csrc/tiles.h",
                                             "paper_2201_03611_amd/csrc/common.h"])
    sten_traffic = traffic_for("stencil2d_tiled", ["paper_2201_03611_amd/csrc/stencil.hip",
                                                   "paper_2201_03611_amd/csrc/tiles.h",
                                                   "paper_2201_03611_amd/csrc/common.h"])
    # the schedules the library chose for the two calls (tile=None, sched=None)
    sv, srows = rise.rise_stencil2d_default_schedule(H, W, KS, KS)
    result = {
        "metric": "GEMM TFLOP/s + stencil GB/s vs roofline; BF16-comp vs FP32 speedup at equal error",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "FP32 GEMM 4096^3 U(-1,1) + FP32 stencil 4096x4096 5x5 Gaussian "
                               "sigma=1 clamp", "gemm_mnk": [M, N, K], "stencil_hw": [H, W],
                   "stencil_k": KS, "parallelism": "single-gpu"},
        "gemm_tflops": round(gemm_tf, 2),
        "stencil_gbps": round(sten_gbs, 1),
        "roofline": {"bound": "mfma", "achieved": round(gemm_tf, 2), "peak": PEAK_FP32_MFMA,
                     "unit": "TFLOP/s", "frac": round(gemm_tf / PEAK_FP32_MFMA, 4),
                     "traffic": gemm_traffic,
                     "kernel": f"{gemm_kernel}<{gt[0]},{gt[1]},{gt[2]}>",
                     "ms": round(t_gemm, 4)},
        "roofline_stencil": {"bound": "hbm", "achieved": round(sten_gbs, 1), "peak": PEAK_HBM,
                             "unit": "GB/s", "frac": round(sten_gbs / PEAK_HBM, 4),
                             "traffic": sten_traffic,
                             "kernel": f"stencil2d_tiled<{KS},{srows} rows>",
                             "ms": round(t_sten, 5)},
    }

    result["strategy"] = {"gemm": f"f32 tile {gt[0]}x{gt[1]}x{gt[2]}" + (
                              ", slabs through a 3-slab asynchronous LDS ring"
                              if gemm_kernel == "gemm_f32_async_kernel" else ""),
                          "stencil": f"{sv} halo tile, {srows} output rows x 256 columns"}

    # measured ceilings of this GPU beside the spec peaks
    ceil = ceilings_leg(rise, torch, dev, stream)
    result["ceilings"] = ceil
    result["roofline"]["frac_measured_ceiling"] = round(gemm_tf / ceil["mfma_f32_tflops"], 4)
    result["roofline_stencil"]["frac_measured_ceiling"] = round(sten_gbs / ceil["hbm_copy_gbps"], 4)

    # the stencil's events above start when the GEMM ends, so they include the
    # dispatch gap after it; the same launches back to back (rotating buffers)
    # give the kernel's own rate beside it
    ms_b2b = event_ms(torch, stream, lambda: [rise.rise_stencil2d(
        outs[j], imgs[j], dw, H, W, ld_out=W, ld_in=W, kh=KS, kw=KS, pad="clamp", stream=stream)
        for j in range(nsets)], 5) / nsets
    result["roofline_stencil"]["ms_back_to_back"] = round(ms_b2b, 5)
    result["roofline_stencil"]["achieved_back_to_back"] = round(bytes_sten / (ms_b2b * 1e-3) / 1e9, 1)
    result["roofline_stencil"]["frac_back_to_back"] = round(
        bytes_sten / (ms_b2b * 1e-3) / 1e9 / PEAK_HBM, 4)

    result["gemm_backward"] = gemm_backward_leg(rise, ri, torch, dev, stream, result["ceilings"])
    if not args.no_precision:
        result["precision"] = precision_leg(rise, ri, np, torch, dev, stream)
    if not args.no_extra:
        result["batched"] = batched_leg(rise, ri, torch, dev, stream)
        result["layer"] = layer_leg(rise, torch, dev, stream)
        result["gemv"] = gemv_leg(rise, torch, dev, stream)
        result["iterate_sum"] = iterate_leg(rise, torch, dev, stream)
        result["stencil_iterate"] = stencil_iterate_leg(rise, ri, torch, dev, stream)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_leg(ri, np, A, B, img, wts, value, ms_step)
    print(json.dumps(result), flush=True)


def run_only(what, reps, rise, ri, torch, dev, stream):
    """One kernel of the path, `reps` launches, on seeded synthetic data of the
    benchmark sizes (for rocprofv3 runs)."""
    g = torch.Generator(device=dev)
    g.manual_seed(1000)
    if what.startswith("gemm"):
        n = 4096 if what == "gemm_f32" else 8192
        mode = what[5:]
        A = torch.randn((n, n), device=dev, generator=g)
        B = torch.randn((n, n), device=dev, generator=g)
        C = torch.empty((n, n), device=dev)
        ws = torch.empty(max(rise.rise_gemm_workspace(n, n, n, mode), 1), device=dev,
                         dtype=torch.uint8)
        call = lambda i: rise.rise_gemm(C, A, B, n, n, n, lda=n, ldb=n, ldc=n, mode=mode, ws=ws,
                                        stream=stream)
    elif what == "stencil":
        imgs = [torch.rand((H, W), device=dev, generator=g) for _ in range(6)]
        outs = [torch.empty((H, W), device=dev) for _ in range(6)]
        w = torch.from_numpy(ri.gaussian_weights(KS, 1.0)).to(dev)
        call = lambda i: rise.rise_stencil2d(outs[i % 6], imgs[i % 6], w, H, W, ld_out=W,
                                             ld_in=W, kh=KS, kw=KS, stream=stream)
    elif what.startswith("conv"):
        Bn, C, Hc, Wc = 32, 64, 512, 512
        x = torch.randn((Bn, Hc, Wc, C), device=dev, generator=g).to(torch.bfloat16)
        dout = torch.randn((Bn, Hc, Wc, C), device=dev, generator=g).to(torch.bfloat16)
        w = torch.randn((C, C, 3, 3), device=dev, generator=g) * 0.02
        if what == "conv_fwd":
            out = torch.empty_like(x)
            ws = torch.empty(rise.rise_conv2d_workspace(C, C), device=dev, dtype=torch.uint8)
            call = lambda i: rise.rise_conv2d(out, x, w, Bn, C, C, Hc, Wc, ws=ws, stream=stream)
        else:
            dIn = torch.empty_like(x)
            dW = torch.empty_like(w)
            ws = torch.empty(rise.rise_conv2d_backward_workspace(Bn, C, C, Hc, Wc), device=dev,
                             dtype=torch.uint8)
            call = lambda i: rise.rise_conv2d_backward(dIn, dW, dout, x, w, Bn, C, C, Hc, Wc,
                                                       ws=ws, stream=stream)
    elif what in ("gemv", "gemv_t"):
        n = 16384
        A = torch.rand((n, n), device=dev, generator=g) * 2 - 1
        x = torch.rand((n,), device=dev, generator=g) * 2 - 1
        y = torch.empty(n, device=dev)
        op = rise.RISE_OP_T if what == "gemv_t" else rise.RISE_OP_N
        ws = torch.empty(max(rise.rise_gemv_workspace(n, n, op), 1), device=dev,
                         dtype=torch.uint8)
        call = lambda i: rise.rise_gemv(y, A, x, n, n, lda=n, opA=op, ws=ws, stream=stream)
    elif what in ("stencil_iterate", "stencil_iterate_1"):
        img = torch.rand((H, W), device=dev, generator=g)
        out = torch.empty_like(img)
        w = torch.from_numpy(ri.gaussian_weights(KS, 1.0)).to(dev)
        fuse = 1 if what.endswith("_1") else 4
        ws = torch.empty(max(rise.rise_stencil2d_iterate_workspace(H, W, KS, KS, 16, fuse), 1),
                         device=dev, dtype=torch.uint8)
        call = lambda i: rise.rise_stencil2d_iterate(out, img, w, H, W, ld_out=W, ld_in=W, kh=KS,
                                                     kw=KS, steps=16, fuse=fuse, ws=ws,
                                                     stream=stream)
    elif what == "iterate_sum":
        x = torch.rand((1 << 26,), device=dev, generator=g) * 2 - 1
        out = torch.empty(1, device=dev)
        ws = torch.empty(max(rise.rise_iterate_sum_workspace(2, 1, 26), 1), device=dev,
                         dtype=torch.uint8)
        call = lambda i: rise.rise_iterate_sum(out, x, 2, 1, 26, ws=ws, stream=stream)
    elif what in ("iterate_sum_fanin3", "iterate_sum_fanin8"):
        n, m, k = (3, 2, 16) if what.endswith("3") else (8, 4, 8)
        x = torch.rand((m * n ** k,), device=dev, generator=g) * 2 - 1
        out = torch.empty(m, device=dev)
        ws = torch.empty(max(rise.rise_iterate_sum_workspace(n, m, k), 1), device=dev,
                         dtype=torch.uint8)
        call = lambda i: rise.rise_iterate_sum(out, x, n, m, k, ws=ws, stream=stream)
    else:  # batched
        plan, keep = batched_plan(rise, ri, torch, dev, "f32")
        call = lambda i: plan.launch(stream)
    for i in range(reps):
        call(i)
    torch.cuda.synchronize()
    print(json.dumps({"only": what, "reps": reps}), flush=True)


def batched_plan(rise, ri, torch, dev, dtype):
    """The batched workload: 512 GEMMs with M, N, K uniform on {64, 96, ..., 1024}
    (FP32 or bf16 operands) and 256 FP32 stencils, side U{256..2048}, k in {3, 5, 7},
    weights summing to 1, clamp padding; device data from a seeded generator."""
    import numpy as np

    from paper_2201_03611_amd._lib import RISE_BF16, RISE_F32

    sizes = ri.batched_gemm_sizes()
    specs = ri.batched_stencil_specs()
    g = torch.Generator(device=dev)
    g.manual_seed(ri.SEED_BATCHED)
    keep = []
    gp = (rise.RiseGemmProblem * 512)()
    flops = 0.0
    for i in range(512):
        M, N, K = (int(v) for v in sizes[i])
        A = torch.rand((M, K), device=dev, generator=g) * 2 - 1
        B = torch.rand((K, N), device=dev, generator=g) * 2 - 1
        if dtype == "bf16":
            A, B = A.to(torch.bfloat16), B.to(torch.bfloat16)
        C = torch.empty((M, N), device=dev)
        keep += [A, B, C]
        gp[i] = rise.RiseGemmProblem(C.data_ptr(), A.data_ptr(), B.data_ptr(), M, N, K, K, N, N,
                                     RISE_BF16 if dtype == "bf16" else RISE_F32, 0)
        flops += 2.0 * M * N * K
    sp = (rise.RiseStencilProblem * 256)()
    rng = ri.rng(ri.SEED_BATCHED + 200)
    bytes_ = 0.0
    for i in range(256):
        side, k = (int(v) for v in specs[i])
        img = torch.rand((side, side), device=dev, generator=g)
        w = torch.from_numpy(ri.random_weights(rng, k)).to(dev)
        out = torch.empty_like(img)
        keep += [img, w, out]
        sp[i] = rise.RiseStencilProblem(out.data_ptr(), img.data_ptr(), w.data_ptr(), side, side,
                                        side, side, k, 0)
        bytes_ += 8.0 * side * side
    plan = rise.Plan(gp, 512, sp, 256)
    keep.append((flops, bytes_, gp, sp))
    return plan, keep


def event_ms(torch, stream, fn, reps, warm=3):
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def ceilings_leg(rise, torch, dev, stream):
    """What this GPU reaches outside the patterns: a 2 GiB streaming device copy
    (read + write bytes / time) and back-to-back matrix instructions on every
    SIMD for FP32, BF16 and FP8 (rise_ceiling_*)."""
    n = 1 << 29  # floats: 2 GiB per buffer
    src = torch.empty(n, device=dev, dtype=torch.float32).fill_(1.0)
    dst = torch.empty_like(src)
    ms = event_ms(torch, stream, lambda: rise.rise_ceiling_copy(dst, src, stream=stream), 5)
    out = {"hbm_copy_gbps": round(2.0 * 4 * n / (ms * 1e-3) / 1e9, 1),
           "hbm_copy_bytes": 2 * 4 * n}
    del src, dst
    torch.cuda.empty_cache()
    sink = torch.empty(rise.rise_ceiling_mfma_sink_floats(), device=dev, dtype=torch.float32)
    for mode, iters in (("f32", 4096), ("bf16", 4096), ("fp8", 4096)):
        fl = rise.rise_ceiling_mfma(mode, iters, sink, stream=stream)
        ms = event_ms(torch, stream, lambda: rise.rise_ceiling_mfma(mode, iters, sink,
                                                                    stream=stream), 5)
        out[f"mfma_{mode}_tflops"] = round(fl / (ms * 1e-3) / 1e12, 1)
    out["spec"] = {"hbm_gbps": PEAK_HBM, "mfma_f32_tflops": PEAK_FP32_MFMA,
                   "mfma_bf16_tflops": PEAK_BF16, "mfma_fp8_tflops": PEAK_FP8}
    return out


def gemm_backward_leg(rise, ri, torch, dev, stream, ceil):
    """GEMM 4096^3 backward (dA = dC B^T, dB = A^T dC; A, B, dC ~ U(-1,1)): each
    product timed on its own (the transposed-operand instantiations of the FP32
    kernel), algorithmic 2 M N K flops each."""
    n = 4096
    A, B = ri.gemm_uniform(n, n, n, ri.SEED_GEMM_BWD)
    G = ri.uniform_matrix(ri.rng(ri.SEED_GEMM_BWD + 1), n, n)
    dA_, dB_, dG = (torch.from_numpy(x).to(dev) for x in (A, B, G))
    gA = torch.empty_like(dA_)
    gB = torch.empty_like(dB_)
    fl = 2.0 * n ** 3
    res = {}
    for name, call in (
            ("dA", lambda: rise.rise_gemm_backward(gA, None, dG, dA_, dB_, n, n, n, ldda=n,
                                                   lddb=n, lddc=n, lda=n, ldb=n, stream=stream)),
            ("dB", lambda: rise.rise_gemm_backward(None, gB, dG, dA_, dB_, n, n, n, ldda=n,
                                                   lddb=n, lddc=n, lda=n, ldb=n, stream=stream))):
        ms = event_ms(torch, stream, call, 10)
        tf = fl / (ms * 1e-3) / 1e12
        res[name] = {"ms": round(ms, 4), "tflops": round(tf, 2),
                     "frac_mfma_peak": round(tf / PEAK_FP32_MFMA, 4),
                     "frac_measured_ceiling": round(tf / ceil["mfma_f32_tflops"], 4)}
    t = rise.rise_gemm_default_tile(n, n, n, "f32")
    res["dA"]["strategy"] = f"f32 tile {t[0]}x{t[1]}x{t[2]}, B read through transpose"
    res["dB"]["strategy"] = f"f32 tile {t[0]}x{t[1]}x{t[2]}, A read through transpose"
    tot = res["dA"]["ms"] + res["dB"]["ms"]
    res["both"] = {"ms": round(tot, 4), "tflops": round(2 * fl / (tot * 1e-3) / 1e12, 2)}
    del dA_, dB_, dG, gA, gB
    torch.cuda.empty_cache()
    return res


def batched_leg(rise, ri, torch, dev, stream):
    """512 GEMMs + 256 stencils: one graph launch of the persistent kernel, the same
    kernel without the graph, and 768 separate one-problem launches; lower bounds
    from the spec peaks (additive: compute + memory; overlapped: their max)."""
    out = {}
    for dtype in ("f32", "bf16"):
        plan, keep = batched_plan(rise, ri, torch, dev, dtype)
        flops, sbytes, gp, sp = keep[-1]
        gbytes = 0.0
        for i in range(512):
            p = gp[i]
            e = 4 if dtype == "f32" else 2
            gbytes += e * (p.M * p.K + p.K * p.N) + 4 * p.M * p.N
        # the first mode timed after the set-up ran 0.12-0.15 ms slower per launch
        # with a single warm-up launch, whichever it was: warm up for 10
        ms_graph = event_ms(torch, stream, lambda: plan.launch(stream), 10, warm=10)
        ms_direct = event_ms(torch, stream, lambda: plan.launch_direct(stream), 10, warm=10)

        def separate():
            for i in range(512):
                A, B, C = keep[3 * i:3 * i + 3]
                q = gp[i]
                rise.rise_gemm(C, A, B, q.M, q.N, q.K, lda=q.lda, ldb=q.ldb, ldc=q.ldc,
                               stream=stream)
            for i in range(256):
                img, w, o = keep[1536 + 3 * i:1536 + 3 * i + 3]
                q = sp[i]
                rise.rise_stencil2d(o, img, w, q.H, q.W, ld_out=q.ld_out, ld_in=q.ld_in,
                                    kh=q.k, kw=q.k, pad=q.pad, stream=stream)

        ms_sep = event_ms(torch, stream, separate, 3) if dtype == "f32" else None
        peak = PEAK_FP32_MFMA if dtype == "f32" else PEAK_BF16
        t_flop = flops / (peak * 1e12) * 1e3
        t_mem = (sbytes + gbytes) / (PEAK_HBM * 1e9) * 1e3
        out[dtype] = {"ms_graph": round(ms_graph, 3), "ms_direct": round(ms_direct, 3),
                      "ms_separate_launches": round(ms_sep, 3) if ms_sep else None,
                      "items": plan.items(), "gemm_gflop": round(flops / 1e9, 1),
                      "stencil_gb": round(sbytes / 1e9, 2),
                      "bound_ms_additive": round(t_flop + t_mem, 3),
                      "bound_ms_overlapped": round(max(t_flop, t_mem), 3),
                      "frac_of_additive_bound": round((t_flop + t_mem) / ms_graph, 3),
                      "frac_of_overlapped_bound": round(max(t_flop, t_mem) / ms_graph, 3)}
        if ms_sep:
            out[dtype]["speedup_vs_separate"] = round(ms_sep / ms_graph, 2)
        kinds = {}
        for i in range(512):
            t = plan.tile(i)
            key = f"{t[0]}x{t[1]}x{t[2]}"
            kinds[key] = kinds.get(key, 0) + 1
        out[dtype]["strategy"] = {"gemm_tiles": dict(sorted(kinds.items())),
                                  "stencil": "one kernel per window side and load width, one workgroup per LDS halo tile"}
        plan.destroy()
        del keep
        torch.cuda.empty_cache()
    out["note"] = ("separate launches: 512 rise_gemm + 256 rise_stencil2d calls with the "
                   "library's default tiles (FP32 set only; the bf16 set needs its operand "
                   "preparation per call)")
    return out


def gemv_leg(rise, torch, dev, stream):
    """The paper's matrix-vector program at 16384 x 16384 FP32 (1 GiB of A, read
    once per call): HBM GB/s against the 8 TB/s peak, both storage orders."""
    n = 16384
    g = torch.Generator(device=dev)
    g.manual_seed(1200)
    A = torch.rand((n, n), device=dev, generator=g) * 2 - 1
    x = torch.rand((n,), device=dev, generator=g) * 2 - 1
    y = torch.empty(n, device=dev)
    res = {}
    for name, op in (("row_major", rise.RISE_OP_N), ("transposed", rise.RISE_OP_T)):
        nws = rise.rise_gemv_workspace(n, n, op)
        ws = torch.empty(max(nws, 1), device=dev, dtype=torch.uint8)
        ms = event_ms(torch, stream, lambda: rise.rise_gemv(y, A, x, n, n, lda=n, opA=op, ws=ws,
                                                            stream=stream), 20)
        gbs = 4.0 * n * n / (ms * 1e-3) / 1e9
        parts = rise.rise_gemv_parts(n, n, op)
        res[name] = {"us": round(ms * 1e3, 1), "gbps": round(gbs, 1),
                     "frac_hbm_peak": round(gbs / PEAK_HBM, 3),
                     "strategy": (f"K split in {parts} slices + ordered reduction" if parts > 1
                                  else "one pass, rows per wavefront")}
    del A
    torch.cuda.empty_cache()
    return res


def stencil_iterate_leg(rise, ri, torch, dev, stream):
    """16 steps of the 4096^2 5x5 Gaussian clamp stencil (iterate, Sec. VI): one
    launch per step through the double buffer of two images, and 4 steps per
    launch in the LDS double buffer.  Pixel-steps per second; the fused schedule
    against the FP32 vector peak (k*k FMAs per pixel-step).  The per-step
    schedule's working set (input, two 64 MiB intermediates, output) fits the
    256 MB last-level cache, which serves most of its reads: its bytes per
    second are an equivalent rate, not an HBM fraction."""
    steps = 16
    img = torch.from_numpy(ri.image_uniform(H, W, 1003)).to(dev)
    w = torch.from_numpy(ri.gaussian_weights(KS, 1.0)).to(dev)
    out = torch.empty_like(img)
    res = {}
    for name, fuse in (("per_step", 1), ("fused4", 4)):
        need = rise.rise_stencil2d_iterate_workspace(H, W, KS, KS, steps, fuse)
        ws = torch.empty(max(need, 1), device=dev, dtype=torch.uint8)
        ms = event_ms(torch, stream, lambda: rise.rise_stencil2d_iterate(
            out, img, w, H, W, ld_out=W, ld_in=W, kh=KS, kw=KS, steps=steps, fuse=fuse, ws=ws,
            stream=stream), 5)
        pxs = H * W * steps / (ms * 1e-3)
        res[name] = {"ms": round(ms, 3), "us_per_step": round(ms * 1e3 / steps, 1),
                     "gpix_steps_per_s": round(pxs / 1e9, 1),
                     "tflops": round(pxs * 2 * KS * KS / 1e12, 1),
                     "hbm_gbps_equiv": round(pxs * 8 / 1e9, 1),
                     "strategy": f"{fuse} step(s) per launch, {-(-steps // fuse)} launches"}
    res["default_fuse"] = rise.rise_stencil2d_iterate_default_fuse(KS, KS)
    res["fused4"]["frac_fp32_vector_peak"] = round(res["fused4"]["tflops"] / PEAK_F32_VEC, 3)
    res["per_step"]["note"] = "reads served largely by the last-level cache; not an HBM figure"
    res["speedup_fused"] = round(res["per_step"]["ms"] / res["fused4"]["ms"], 2)
    return res


def iterate_leg(rise, torch, dev, stream):
    """iterate with the tree-reduction body (binary tree, n = 2) over 2^26 FP32
    values (256 MiB, read once) to one sum, and over 4096 rows of 2^14 values
    to 4096 sums; fan-ins 3 (2 x 3^16 values) and 8 (4 x 8^8 values): HBM GB/s
    of the input read against the 8 TB/s peak.  The launches rotate over three
    inputs (above the 256 MB last-level cache), so every launch reads its input
    from HBM."""
    res = {}
    for name, n, m, k in (("tree_2pow26_to_1", 2, 1, 26), ("rows_4096x2pow14", 2, 4096, 14),
                          ("fanin3_2x3pow16", 3, 2, 16), ("fanin8_4x8pow8", 8, 4, 8)):
        total = m * n ** k
        g = torch.Generator(device=dev)
        g.manual_seed(1300)
        xs = [torch.rand((total,), device=dev, generator=g) * 2 - 1 for _ in range(3)]
        out = torch.empty(m, device=dev)
        need = rise.rise_iterate_sum_workspace(n, m, k)
        ws = torch.empty(max(need, 1), device=dev, dtype=torch.uint8)
        ms = event_ms(torch, stream, lambda: [rise.rise_iterate_sum(out, x, n, m, k, ws=ws,
                                                                    stream=stream)
                                              for x in xs], 7) / len(xs)
        gbs = 4.0 * (total + m) / (ms * 1e-3) / 1e9
        rounds = rise.rise_iterate_sum_passes(n, m, k)
        res[name] = {"us": round(ms * 1e3, 1), "gbps": round(gbs, 1),
                     "frac_hbm_peak": round(gbs / PEAK_HBM, 3),
                     "strategy": f"{len(rounds)} pass(es), rounds per pass {rounds}"}
        del xs
    torch.cuda.empty_cache()
    return res


def layer_leg(rise, torch, dev, stream):
    """Stencil layer, batch 32, 64 -> 64 channels, 512 x 512, 3 x 3, bf16 NHWC:
    forward, dIn and dW (each 618.5 GFLOP), seeded device data."""
    Bn, C, Hc, Wc = 32, 64, 512, 512
    g = torch.Generator(device=dev)
    g.manual_seed(1006)
    x = torch.randn((Bn, Hc, Wc, C), device=dev, generator=g).to(torch.bfloat16)
    dout = torch.randn((Bn, Hc, Wc, C), device=dev, generator=g).to(torch.bfloat16)
    w = torch.randn((C, C, 3, 3), device=dev, generator=g) * 0.02
    out = torch.empty_like(x)
    dIn = torch.empty_like(x)
    dW = torch.empty_like(w)
    wsf = torch.empty(rise.rise_conv2d_workspace(C, C), device=dev, dtype=torch.uint8)
    wsb = torch.empty(rise.rise_conv2d_backward_workspace(Bn, C, C, Hc, Wc), device=dev,
                      dtype=torch.uint8)
    fl = 2.0 * Bn * Hc * Wc * C * C * 9
    act = 2.0 * Bn * Hc * Wc * C
    ms_f = event_ms(torch, stream, lambda: rise.rise_conv2d(out, x, w, Bn, C, C, Hc, Wc, ws=wsf,
                                                            stream=stream), 10)
    ms_di = event_ms(torch, stream, lambda: rise.rise_conv2d_backward(
        dIn, None, dout, x, w, Bn, C, C, Hc, Wc, ws=wsb, stream=stream), 10)
    ms_dw = event_ms(torch, stream, lambda: rise.rise_conv2d_backward(
        None, dW, dout, x, w, Bn, C, C, Hc, Wc, ws=wsb, stream=stream), 10)
    res = {}
    for name, ms, by in (("forward", ms_f, 2 * act), ("dIn", ms_di, 2 * act), ("dW", ms_dw, 2 * act)):
        tf = fl / (ms * 1e-3) / 1e12
        gbs = by / (ms * 1e-3) / 1e9
        res[name] = {"ms": round(ms, 3), "tflops": round(tf, 1),
                     "frac_bf16_peak": round(tf / PEAK_BF16, 3), "gbps": round(gbs, 1),
                     "frac_hbm_peak": round(gbs / PEAK_HBM, 3)}
    res["bound_ms_forward"] = round(max(fl / (PEAK_BF16 * 1e9), 2 * act / (PEAK_HBM * 1e6)), 3)
    res["strategy"] = {"forward": "bf16 MFMA, weights in registers, halo tiles of two rows per wave",
                       "dIn": "the forward kernel with rotated, channel-transposed weights",
                       "dW": "per-workgroup partial sums over pixel tiles + ordered reduction"}
    return res


def precision_leg(rise, ri, np, torch, dev, stream):
    """8192^3, N(0,1) 2^U(-4,4): every mode timed with events (operand preparation
    included) and its componentwise error vs the exact product on sampled outputs."""
    import oracle

    n = 8192
    A, B = ri.gemm_scaled_normal(n, n, n, ri.SEED_PRECISION)
    rows, cols = ri.sample_indices(ri.rng(78), n, n, 600)
    exact = oracle.gemm_sampled(A, B, rows, cols)
    scale = oracle.gemm_sampled(np.abs(A), np.abs(B), rows, cols)
    dA, dB = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
    dC = torch.empty((n, n), device=dev, dtype=torch.float32)
    out = {}
    peaks = {"f32": PEAK_FP32_MFMA, "bf16": PEAK_BF16, "bf16x3": PEAK_BF16, "bf16x6": PEAK_BF16,
             "fp8": PEAK_FP8}
    for mode in ["f32", "bf16", "bf16x3", "bf16x6", "fp8"]:
        need = rise.rise_gemm_workspace(n, n, n, mode)
        ws = torch.empty(max(need, 1), device=dev, dtype=torch.uint8)
        call = lambda: rise.rise_gemm(dC, dA, dB, n, n, n, lda=n, ldb=n, ldc=n, mode=mode, ws=ws,
                                      stream=stream)
        call()
        torch.cuda.synchronize()
        reps = 5
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            call()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        C = dC.cpu().numpy()[rows, cols]
        diff = np.abs(C.astype(np.float64) - exact)
        err = float(np.max(diff / scale))
        # normwise max|c_hat - c| / max|c| and elementwise |c_hat - c| / |c| over
        # outputs with |c| >= 1e-3 max|c| (both over the same samples)
        big = np.abs(exact) >= 1e-3 * np.max(np.abs(exact))
        tf = 2.0 * n ** 3 / (ms * 1e-3) / 1e12
        tl = rise.rise_gemm_default_tile(n, n, n, mode)
        ms_prep = None
        if mode != "f32":
            # the operand preparation alone (A as rows of K, B read as columns), so
            # the contraction's own rate can be read beside the end-to-end one
            pa = torch.empty(rise.rise_prep_bytes(n, n, mode), device=dev, dtype=torch.uint8)
            pb = torch.empty_like(pa)
            ms_prep = event_ms(torch, stream, lambda: (
                rise.rise_prep_operand(pa, n, n, dA, n, n, n, 1, mode, stream=stream),
                rise.rise_prep_operand(pb, n, n, dB, n, n, 1, n, mode, stream=stream)), 5)
            del pa, pb
        out[mode] = {"ms": round(ms, 3), "tflops_useful": round(tf, 1),
                     "strategy": f"{mode} tile {tl[0]}x{tl[1]}x{tl[2]}",
                     "frac_of_own_peak": round(tf / peaks[mode], 4),
                     "err_componentwise_max": err,
                     "err_normwise": float(np.max(diff) / np.max(np.abs(exact))),
                     "err_elementwise_floored_max": float(np.max(diff[big] / np.abs(exact[big])))}
        if ms_prep is not None:
            out[mode]["ms_prep"] = round(ms_prep, 3)
            out[mode]["tflops_contraction"] = round(2.0 * n ** 3 / ((ms - ms_prep) * 1e-3) / 1e12, 1)
        del ws
    for mode in ["bf16", "bf16x3", "bf16x6", "fp8"]:
        out[mode]["err_ratio_to_f32"] = round(out[mode]["err_componentwise_max"] /
                                              out["f32"]["err_componentwise_max"], 2)
    out["speedup_bf16x3_vs_f32"] = round(out["f32"]["ms"] / out["bf16x3"]["ms"], 3)
    out["speedup_bf16x6_vs_f32"] = round(out["f32"]["ms"] / out["bf16x6"]["ms"], 3)
    out["equal_error_bound"] = 1e-5
    out["note"] = ("times include operand preparation; errors over 604 sampled outputs against "
                   "the exact product of the FP32 inputs: componentwise max |c_hat - c| / "
                   "(|A||B|)_ij (the bar), normwise, and elementwise over |c| >= 1e-3 max|c|; "
                   "ms_prep is the row-major preparation of rise_prep_operand, while the "
                   "256x256 tiles prepare their operands K-blocked inside rise_gemm (same "
                   "bytes, a different write order)")
    return out


def cpu_leg(ri, np, A, B, img, wts, gpu_value, ms_step):
    """The oracle (fp64 view interpreter, OpenMP) on a bounded sample of the
    step: 65536 sampled outputs of the 4096^3 GEMM and the full 4096^2 stencil,
    rated in the metric's unit (flops of the sample / wall time)."""
    import oracle

    g = ri.rng(99)
    rows, cols = ri.sample_indices(g, M, N, 65532)
    t0 = time.perf_counter()
    oracle.gemm_sampled(A, B, rows, cols)
    t1 = time.perf_counter()
    threads = oracle.last_threads()
    oracle.stencil2d(img, wts)
    t2 = time.perf_counter()
    flops = 2.0 * K * rows.size + 2.0 * KS * KS * img.size
    tflops = flops / (t2 - t0) / 1e12
    # the same oracle on one core, on a smaller sample of the same workload
    prev = oracle.set_threads(1)
    r1, c1 = rows[:4096], cols[:4096]
    crop = np.ascontiguousarray(img[:512])
    t3 = time.perf_counter()
    oracle.gemm_sampled(A, B, r1, c1)
    t4 = time.perf_counter()
    oracle.stencil2d(crop, wts)
    t5 = time.perf_counter()
    oracle.set_threads(prev)
    flops1 = 2.0 * K * r1.size + 2.0 * KS * KS * crop.size
    return {"value": tflops, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{rows.size} of the 4096^2 GEMM outputs ({t1 - t0:.2f} s, "
                      f"{2.0 * K * rows.size / (t1 - t0) / 1e9:.3f} GFLOP/s) + the full "
                      f"4096^2 5x5 stencil ({t2 - t1:.2f} s, {8.0 * img.size / (t2 - t1) / 1e9:.3f} "
                      f"GB/s)",
            "one_core": {"value": flops1 / (t5 - t3) / 1e12, "unit": "TFLOP/s",
                         "sample": f"{r1.size} GEMM outputs ({t4 - t3:.2f} s) + 512 x 4096 "
                                   f"rows of the stencil ({t5 - t4:.2f} s)"},
            "gpu_over_cpu": round(gpu_value / tflops, 1)}


if __name__ == "__main__":
    main()
