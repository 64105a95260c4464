"""Throughput of the Mosaic Flow predictor on one MI355X.

One step = one full pass of the hot path over one synthetic domain: the
predictor loop of Alg. 2 (200 four-colour sweeps, CROSS targets) followed by
the overlap-averaged assembly, on a 16 x 16 unit domain (513 x 513 grid,
961 placements) with a width-256 SDNet (Xavier weights, seed 0) and GP
boundary data (length scale 2, seed 1). The value is SDNet point
evaluations per second over the whole step (sweeps + assembly), float32.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Prints one JSON line. The "roofline" object reports the colour-phase kernel
(the dominant kernel): algorithmic flops per launch over its average launch
duration, timed with HIP events on the launch stream during the timed
region. The "cpu_baseline" object times the float64 oracle on the host
cores on a bounded sample of the same workload.

Beside the headline the line carries: the assembly timed on its own; the
2 x 2-unit workload in microseconds per sweep; one GPU's share of the
64 x 64-unit domain split eight ways; the standalone gather and scatter in
GB/s on a field larger than the last-level cache; the GEMM rates torch.mm
reaches (achievable peaks); FP32 against BF16 on the 64 x 64-unit domain;
the training step; optionally the 48-domain batch and its adjoint (--c5).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SDNet point-evals/s in MF sweep (BF16 vs FP32 @ stated L2 err); train steps/s"
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2516.6
PEAK_HBM_BYTES_PER_S = 8.0e12
CROSS_T = 61
INTERIOR_T = 961

# HBM traffic of the colour-phase kernel per launch on this workload, by tile
# shape, from two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE; KiB per
# dispatch) scaled by what the same counters read for a plain 512 MiB device
# copy (FETCH_SIZE reads half the copied bytes on this part: factor 2.0;
# WRITE_SIZE: 1.0). It is reported only while the kernel sources hash to the
# value the counters were taken with; otherwise "traffic" is null. Summary:
# profiles/*_traffic.md.
MEASURED_TRAFFIC = {
    "sources_sha256": "943990a6e26f9dddd7633f39e00bb5db39c67fc87b01d2af7ff5b4ab8bf6939a",
    "bytes_per_launch": {"64": (5148.3 * 2.0 + 261.9) * 1024,
                         "64|stream": (5100.3 * 2.0 + 261.9) * 1024,
                         "32": (6014.4 * 2.0 + 268.6) * 1024},
}
KERNEL_SOURCES = ("paper_2308_14258_amd/csrc/sweep_kernels.hip",
                  "paper_2308_14258_amd/csrc/mf_device.h")


def kernel_sources_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def flops_per_point(width: int, T: int) -> float:
    """Algorithmic flops of one SDNet evaluation in a phase with T targets per
    placement: three d x d hidden layers (6 d^2), the coordinate term of the
    first layer (4 d), the output layer (2 d), and the boundary projection
    2 * 128 * d amortised over the placement's T points."""
    d = width
    return 6.0 * d * d + 6.0 * d + 2.0 * 128 * d / T


def sweep_points(ux: int, uy: int, T: int) -> int:
    return (2 * ux - 1) * (2 * uy - 1) * T


def host_info():
    """CPU model, logical CPU count and the BLAS torch's CPU operations use."""
    import torch
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = ""
    for line in torch.__config__.show().splitlines():
        if "BLAS_INFO" in line:
            blas = line.split("BLAS_INFO=")[1].split(",")[0]
    return {"cpu_model": model, "nproc": os.cpu_count(), "blas": blas}


def cpu_baseline(field, params, width, ux, uy, sample_sweeps):
    import torch
    from oracle import sweep as sw
    torch.set_num_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    solver = sw.sdnet_solver(torch.from_numpy(params.astype(np.float64)), width)
    u = torch.from_numpy(field.astype(np.float64))
    t0 = time.perf_counter()
    for _ in range(sample_sweeps):
        u = sw.sweep(u, ux, uy, solver)
    sw.assemble(u, ux, uy, solver)
    dt = time.perf_counter() - t0
    evals = sample_sweeps * sweep_points(ux, uy, CROSS_T) + sweep_points(ux, uy, INTERIOR_T)
    return {"value": evals / dt, "unit": "point-evals/s", "cores": torch.get_num_threads(),
            "kind": "oracle", "host": host_info(),
            "sample": f"{sample_sweeps} CROSS sweeps + 1 assembly of the same 16x16-unit, "
                      f"width-{width} workload, float64, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sweeps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-sweeps", type=int, default=20)
    ap.add_argument("--mode", choices=["solve", "copy"], default="solve",
                    help="copy: one plain device copy of --copy-mb MiB, the reference "
                         "kernel for scaling HBM counters")
    ap.add_argument("--copy-mb", type=int, default=512)
    ap.add_argument("--no-bf16", action="store_true",
                    help="skip the 64x64-unit BF16-vs-FP32 comparison")
    ap.add_argument("--bf16-sweeps", type=int, default=500)
    ap.add_argument("--only-bf16", action="store_true",
                    help="run only the 64x64-unit comparison (for counter collection)")
    ap.add_argument("--no-train", action="store_true", help="skip the training-step measurement")
    ap.add_argument("--train-steps", type=int, default=20)
    ap.add_argument("--c5", action="store_true",
                    help="also time the 48-domain batch (BF16 sweeps + FP32 adjoint); its GP "
                         "inputs take about a minute to generate on the host")
    ap.add_argument("--only-c5", action="store_true")
    ap.add_argument("--only-train", action="store_true", help="only the training-step measurement")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip C1, the per-GPU share, gather/scatter bandwidth and the GEMM peaks")
    ap.add_argument("--only-io", action="store_true", help="only the gather/scatter bandwidth")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "runs on one GPU only: the sweep holds the whole domain on "
                                   "a single device; splitting a domain's placement rows over "
                                   "GPUs with a halo exchange per colour phase is not built",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import mf_inputs as mi
    from paper_2308_14258_amd import Context, MF_CROSS, MF_FP32, mf_autotune, mf_solve

    if args.mode == "copy":
        n = args.copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read": 4 * n, "bytes_written": 4 * n}), flush=True)
        return

    if args.only_bf16 or args.only_c5 or args.only_train or args.only_io:
        ctx = Context(0)
        if args.only_io:
            out = {"gather_scatter": io_measurement(ctx)}
        elif args.only_bf16:
            out = {"bf16_vs_fp32": bf16_comparison(ctx, args.bf16_sweeps)}
        elif args.only_c5:
            out = {"batched": batched_measurement(ctx)}
        else:
            out = {"train": train_measurement(ctx, args.train_steps)}
        print(json.dumps(out), flush=True)
        ctx.close()
        return

    w = mi.WORKLOADS["C2"]
    ux, uy = w["units"]
    width = w["width"]
    K = args.sweeps
    field = mi.workload_field("C2")
    params_np = mi.xavier_params(width, 0)

    dev = torch.device("cuda:0")
    ctx = Context(0)
    params = torch.from_numpy(params_np).to(dev)
    u0 = torch.from_numpy(field).to(dev)
    u = u0.clone()
    u_out = torch.empty_like(u)

    # tile height chosen by the autotuner on a scratch copy (outside the timed region)
    tile_rows = mf_autotune(ctx, params, u0.clone(), (ux, uy), MF_CROSS, MF_FP32, trials=3)

    def step():
        u.copy_(u0)
        mf_solve(ctx, params, u, (ux, uy), K, targets=MF_CROSS, prec=MF_FP32, u_out=u_out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.timing_read()                      # drop anything recorded so far
    ctx.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.timing(False)
    launches, phase_ms, phase_rows = ctx.timing_read()

    evals_per_step = K * sweep_points(ux, uy, CROSS_T) + sweep_points(ux, uy, INTERIOR_T)
    value = evals_per_step * args.steps / dt
    fpp = flops_per_point(width, CROSS_T)
    achieved = phase_rows * fpp / (phase_ms * 1e-3) / 1e12
    avg_us = phase_ms * 1e3 / max(launches, 1)

    # parity of the last step against stored oracle values (16x16, 200 sweeps)
    parity = None
    gpath = os.path.join(ROOT, "tests", "golden", "c2_fp32.npz")
    if K == 200 and os.path.exists(gpath):
        from oracle.sweep import skeleton_mask
        g = np.load(gpath)
        uh = u.cpu().numpy().astype(np.float64)
        m = skeleton_mask(*field.shape).numpy()
        e_s = np.linalg.norm(uh[m] - g["skel200"]) / np.linalg.norm(g["skel200"])
        uo = u_out.cpu().numpy().astype(np.float64)[g["sample_j"], g["sample_i"]]
        e_o = np.linalg.norm(uo - g["u_out_sample"]) / np.linalg.norm(g["u_out_sample"])
        parity = {"rel_l2_skeleton_vs_oracle": float(e_s), "rel_l2_u_out_vs_oracle": float(e_o)}

    traffic = (MEASURED_TRAFFIC["bytes_per_launch"].get(tile_shape_name(tile_rows))
               if MEASURED_TRAFFIC["sources_sha256"] == kernel_sources_sha() else None)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "point-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "C2: plain Mosaic Flow, 16x16 units (513x513 grid, 961 "
                               "placements), SDNet width 256, GP ring data (l=2, seed 1), "
                               f"{K} CROSS sweeps + assembly",
                   "units": [ux, uy], "width": width, "sweeps": K, "targets": "cross",
                   "evals_per_step": evals_per_step, "tile_shape": tile_shape_name(tile_rows)},
        "sweep_phase": {"launches": launches, "avg_launch_us": avg_us,
                        "point_evals_per_s": phase_rows / (phase_ms * 1e-3)},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_MFMA_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA_TFLOPS,
                     "traffic": traffic,
                     "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE/WRITE_SIZE)",
                     "hbm_gbps": traffic / (avg_us * 1e3) if traffic else None,
                     "hbm_frac": traffic / (avg_us * 1e-6) / PEAK_HBM_BYTES_PER_S if traffic else None,
                     "kernel": "tile_kernel<256,R,CROSS,FP32> (colour phase)",
                     "flops_per_point_eval": fpp},
        "parity": parity,
    }
    out["assembly"] = assembly_measurement(ctx, params, u0, (ux, uy))
    if not args.no_extras:
        out["c1"] = c1_measurement(ctx)
        out["per_gpu_share"] = per_gpu_share_measurement(ctx)
        out["gather_scatter"] = io_measurement(ctx)
        out["achievable_peaks"] = achievable_peaks()
        out["roofline"]["frac_of_achievable"] = achieved / out["achievable_peaks"]["fp32_tflops"]
    if not args.no_bf16:
        out["bf16_vs_fp32"] = bf16_comparison(ctx, args.bf16_sweeps)
    if not args.no_train:
        out["train"] = train_measurement(ctx, args.train_steps)
    if args.c5:
        out["batched"] = batched_measurement(ctx)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(field, params_np, width, ux, uy, args.cpu_sample_sweeps)
    print(json.dumps(out), flush=True)
    ctx.close()


def train_measurement(ctx, steps):
    """Physics-informed training step (Alg. 1 + Adam): 1024 GP boundary
    conditions x (128 boundary + 256 collocation points), width 128, fp32.
    Algorithmic flops per step count the forward Taylor streams (4 streams of
    3 hidden d x d GEMMs per collocation point, 1 for a data point) and twice
    that for the reverse pass (input adjoints + weight gradients)."""
    import torch
    import mf_inputs as mi
    from paper_2308_14258_amd import sdnet_train_step
    w = mi.WORKLOADS["C3"]
    d = w["width"]
    G = torch.from_numpy(mi.gp_perimeter_batch(w["n_bc"], w["length"], w["bc_seed"])).cuda()
    Xc = torch.from_numpy(mi.collocation_points(w["n_bc"], w["n_colloc"], w["colloc_seed"])).cuda()
    Xb = torch.from_numpy(mi.unit_perimeter_nodes().astype(np.float32)).cuda()
    p = torch.from_numpy(mi.xavier_params(d, 0)).cuda()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    for k in range(2):
        sdnet_train_step(ctx, p, m, v, k + 1, G, Xb, Xc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        loss = sdnet_train_step(ctx, p, m, v, k + 3, G, Xb, Xc)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rows = w["n_bc"] * (4 * w["n_colloc"] + 128)
    flops = 3 * (3 * 2.0 * d * d * rows)
    return {"workload": "C3: 1024 conditions x (128 + 256) points, width 128, Adam",
            "steps_per_s": steps / dt, "ms_per_step": dt * 1e3 / steps,
            "gemm_tflops": flops * steps / dt / 1e12,
            "frac_of_fp32_mfma_peak": flops * steps / dt / 1e12 / PEAK_FP32_MFMA_TFLOPS,
            "last_loss": [float(x) for x in loss.cpu()]}


def _event_ms(fn, reps):
    """Average milliseconds of fn() over reps calls, timed with events on the
    current stream (the stream every library call is given)."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def achievable_peaks():
    """Dense GEMM rates the platform library reaches on this GPU (torch.mm,
    8192^3, fp32 and bf16): the achievable denominators beside the published
    peaks."""
    import torch
    out = {}
    n = 8192
    for name, dt in (("fp32", torch.float32), ("bf16", torch.bfloat16)):
        a = torch.randn(n, n, device="cuda").to(dt)
        b = torch.randn(n, n, device="cuda").to(dt)
        ms = _event_ms(lambda: torch.mm(a, b), 10)
        out[name + "_tflops"] = 2.0 * n ** 3 / (ms * 1e-3) / 1e12
        del a, b
    out["method"] = "torch.mm 8192x8192x8192, mean of 10 after one warm-up"
    return out


def assembly_measurement(ctx, params, field, units):
    """The overlap-averaged assembly on its own (INTERIOR targets, every
    placement, four colour launches plus the ring copy): mf_solve with zero
    sweeps and u_out."""
    import torch
    from paper_2308_14258_amd import mf_solve
    ux, uy = units
    u = field.clone()
    u_out = torch.empty_like(u)
    ms = _event_ms(lambda: mf_solve(ctx, params, u, units, 0, u_out=u_out), 10)
    evals = sweep_points(ux, uy, INTERIOR_T)
    return {"ms": ms, "point_evals": evals, "point_evals_per_s": evals / (ms * 1e-3),
            "tflops": evals * flops_per_point(params_width(params), INTERIOR_T) / (ms * 1e-3) / 1e12}


def params_width(params):
    from paper_2308_14258_amd.api import width_of
    return width_of(params)


def c1_measurement(ctx):
    """2 x 2 units, width 128, 50 sweeps (graph replay): launch-bound, so
    microseconds per sweep."""
    import torch
    import mf_inputs as mi
    from paper_2308_14258_amd import mf_solve
    w = mi.WORKLOADS["C1"]
    units = w["units"]
    f = torch.from_numpy(mi.workload_field("C1")).cuda()
    params = torch.from_numpy(mi.xavier_params(w["width"], 0)).cuda()
    u = f.clone()
    ms = _event_ms(lambda: mf_solve(ctx, params, u, units, w["sweeps"]), 20)
    return {"workload": "C1: 2x2 units, width 128, 50 CROSS sweeps", "us_per_sweep": ms * 1e3 / w["sweeps"]}


def per_gpu_share_measurement(ctx):
    """One GPU's block of the 64 x 64-unit domain under a 2 x 4 processor
    grid: a 32 x 16-unit domain (1,953 placements, against 16,129 / 8 = 2,016
    for an even split), width 256, 20 sweeps, FP32 and BF16."""
    import torch
    import mf_inputs as mi
    from paper_2308_14258_amd import MF_BF16, MF_FP32, mf_autotune, mf_solve
    ux, uy = 32, 16
    f = torch.from_numpy(mi.expsin_field(ux, uy)).cuda()
    params = torch.from_numpy(mi.xavier_params(256, 0)).cuda()
    K = 20
    out = {"workload": "32x16 units (one GPU's share of 64x64 on 8 GPUs), width 256, 20 CROSS sweeps"}
    for name, prec in (("fp32", MF_FP32), ("bf16", MF_BF16)):
        mf_autotune(ctx, params, f.clone(), (ux, uy), 0, prec, trials=2)
        u = f.clone()
        ms = _event_ms(lambda: mf_solve(ctx, params, u, (ux, uy), K, prec=prec), 3)
        evals = K * sweep_points(ux, uy, CROSS_T)
        out[name] = {"ms_per_sweep": ms / K, "point_evals_per_s": evals / (ms * 1e-3)}
    return out


def io_measurement(ctx):
    """Standalone boundary gather and target scatter of each colour on a
    256 x 256-unit field (8193^2 floats, 268 MB: larger than the last-level
    cache). Algorithmic bytes: gather 512 B read + 512 B written per
    placement; scatter 4 B read + 4 B written per target."""
    import torch
    import mf_inputs as mi
    from paper_2308_14258_amd import MF_CROSS, MF_INTERIOR, mf_colour_placements, mf_gather, mf_scatter
    ux = uy = 256
    u = torch.from_numpy(mi.random_interior_field(ux, uy, 15).astype(np.float32)).cuda()
    res = {"field": "256x256 units, 8193x8193 float32 (268 MB)"}
    tot = {"gather": [0.0, 0.0], "scatter_cross": [0.0, 0.0], "scatter_interior": [0.0, 0.0]}
    for c in range(4):
        n = mf_colour_placements((ux, uy), c)
        G = torch.empty(n, 128, device="cuda")
        ms = _event_ms(lambda: mf_gather(ctx, u, (ux, uy), c, G), 20)
        tot["gather"][0] += ms
        tot["gather"][1] += n * 1024.0
        for key, targets, T in (("scatter_cross", MF_CROSS, 61), ("scatter_interior", MF_INTERIOR, 961)):
            pred = torch.randn(n, T, device="cuda")
            ms = _event_ms(lambda: mf_scatter(ctx, pred, u, (ux, uy), c, targets), 20)
            tot[key][0] += ms
            tot[key][1] += n * T * 8.0
            del pred
    for key, (ms, nbytes) in tot.items():
        gbps = nbytes / (ms * 1e-3) / 1e9
        res[key] = {"us_per_launch": ms * 1e3 / 4, "algorithmic_bytes_per_sweep": nbytes,
                    "GB_per_s": gbps, "frac_of_hbm_peak": gbps * 1e9 / PEAK_HBM_BYTES_PER_S}
    return res


def batched_measurement(ctx):
    """48 independent domains (4..48 units per side, seed 7), width 256: 20
    BF16 sweeps + assembly in one persistent launch per colour, and the FP32
    adjoint of J = sum u_out^2 through 20 sweeps with checkpoints every 5."""
    import torch
    import mf_inputs as mi
    from paper_2308_14258_amd import MF_BF16, MF_CROSS, Batch, mf_solve, mf_solve_adjoint
    w = mi.WORKLOADS["C5"]
    t0 = time.perf_counter()
    sizes, fields = mi.batched_domains(w["n_domains"], 4, 48, w["length"], w["seed"])
    gen_s = time.perf_counter() - t0
    params = torch.from_numpy(mi.xavier_params(w["width"], 0)).cuda()
    batch = Batch(fields)
    base = batch.buf.clone()
    out = torch.empty_like(batch.buf)
    K = w["sweeps"]
    mf_solve(ctx, params, batch, None, 2, prec=MF_BF16)
    batch.buf.copy_(base)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mf_solve(ctx, params, batch, None, K, prec=MF_BF16, u_out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    placements = int(sum((2 * ux - 1) * (2 * uy - 1) for ux, uy in sizes))
    evals = K * placements * CROSS_T + placements * INTERIOR_T
    t0 = time.perf_counter()
    ub, J = mf_solve_adjoint(ctx, params, Batch(fields), None, K, w["ckpt"])
    torch.cuda.synchronize()
    dta = time.perf_counter() - t0
    return {"workload": f"C5: 48 domains, {placements} placements, width 256, {K} sweeps",
            "input_generation_s": gen_s,
            "bf16_solve": {"s": dt, "point_evals_per_s": evals / dt},
            "fp32_adjoint": {"s": dta, "J": float(J.item()),
                             "grad_norm": float(ub.double().norm().item())}}


def tile_shape_name(code):
    """Readable tile shape: height plus the MF_TILE_WIDE / MF_TILE_STREAM flags."""
    name = str(code & 0xFFFF)
    if code & (1 << 16):
        name += "|wide"
    if code & (1 << 17):
        name += "|stream"
    if code & (1 << 18):
        name += "|rowsplit"
    return name


def bf16_comparison(ctx, sweeps):
    """64 x 64 units (2049^2 grid, 16,129 placements), width 256, e^x sin y
    ring data: the same solve in FP32 and with BF16 hidden GEMMs, one timed
    run each after a short warm-up; error of BF16 against the FP32 run."""
    import torch
    import mf_inputs as mi
    from paper_2308_14258_amd import MF_BF16, MF_CROSS, MF_FP32, mf_solve
    w = mi.WORKLOADS["C4"]
    ux, uy = w["units"]
    width = w["width"]
    field = torch.from_numpy(mi.workload_field("C4")).cuda()
    params = torch.from_numpy(mi.xavier_params(width, 0)).cuda()
    res = {"workload": f"C4: 64x64 units, width {width}, e^x sin y scaled, {sweeps} CROSS sweeps "
                       "+ assembly"}
    outs = {}
    gpath = os.path.join(ROOT, "tests", "golden", "c4_fp64.npz")   # oracle values, 500 sweeps
    evals = sweeps * sweep_points(ux, uy, CROSS_T) + sweep_points(ux, uy, INTERIOR_T)
    from paper_2308_14258_amd import mf_autotune
    for name, prec in (("fp32", MF_FP32), ("bf16", MF_BF16)):
        shape = mf_autotune(ctx, params, field.clone(), (ux, uy), MF_CROSS, prec, trials=2)
        u = field.clone()
        u_out = torch.empty_like(u)
        mf_solve(ctx, params, u, (ux, uy), 2, targets=MF_CROSS, prec=prec)   # warm-up + capture
        u.copy_(field)
        ctx.timing_read()
        ctx.timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mf_solve(ctx, params, u, (ux, uy), sweeps, targets=MF_CROSS, prec=prec, u_out=u_out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.timing(False)
        launches, ms, rows = ctx.timing_read()
        fpp = flops_per_point(width, CROSS_T)
        peak = PEAK_FP32_MFMA_TFLOPS if prec == MF_FP32 else PEAK_BF16_MFMA_TFLOPS
        ach = rows * fpp / (ms * 1e-3) / 1e12
        res[name] = {"point_evals_per_s": evals / dt, "s_per_solve": dt, "tile_shape": tile_shape_name(shape),
                     "phase_avg_us": ms * 1e3 / max(launches, 1),
                     "phase_tflops": ach, "phase_frac_of_mfma_peak": ach / peak}
        if sweeps == w["sweeps"] and os.path.exists(gpath):
            g = np.load(gpath)
            sk = u.cpu().numpy().astype(np.float64)[g["skel_j"], g["skel_i"]]
            uo = u_out.cpu().numpy().astype(np.float64)[g["sample_j"], g["sample_i"]]
            res[name]["rel_l2_skeleton_vs_oracle"] = float(np.linalg.norm(sk - g["skel500"]) /
                                                           np.linalg.norm(g["skel500"]))
            res[name]["rel_l2_u_out_vs_oracle"] = float(np.linalg.norm(uo - g["u_out_sample"]) /
                                                        np.linalg.norm(g["u_out_sample"]))
        outs[name] = u_out.double()
    d = outs["bf16"][1:-1, 1:-1] - outs["fp32"][1:-1, 1:-1]
    res["rel_l2_bf16_vs_fp32_u_out"] = float(d.norm() / outs["fp32"][1:-1, 1:-1].norm())
    res["speedup_bf16_over_fp32"] = res["bf16"]["point_evals_per_s"] / res["fp32"]["point_evals_per_s"]
    return res


if __name__ == "__main__":
    main()
