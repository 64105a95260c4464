"""Throughput of the Mosaic Flow predictor on one MI355X.

One step = one full pass of the hot path over one synthetic domain: the
predictor loop of Alg. 2 (500 four-colour sweeps, CROSS targets) followed by
the overlap-averaged assembly, on a 64 x 64-unit domain (2049 x 2049 grid,
16,129 placements) with a width-256 SDNet (Xavier weights, seed 0) and
e^x sin y ring data scaled to [0, 1]. The headline value is SDNet point
evaluations per second over the whole step (sweeps + assembly) in float32;
the same steps with 16-bit GEMM operands are reported beside it ("bf16",
"fp16"), each with its error against the float64 oracle, and FP16 sweeps
held to the float32 iteration by a periodically refreshed correction
("fp16_mixed").

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Prints one JSON line. The "roofline" object reports the colour-phase kernel
(the dominant kernel): algorithmic flops per launch over its average launch
duration, timed with HIP events on the launch stream during the timed
region. The "cpu_baseline" object times the float64 oracle on the host
cores on a bounded sample of the same workload.

Beside the headline the line carries: errors along the trajectory against
stored oracle values; the 16 x 16-unit workload; the 48-domain batch (BF16
sweeps, parity at its 20 sweeps) and its adjoint; the training step; the
paper's convolutional-embedding GELU network on the 64 x 64-unit domain; a
trained network's accuracy against the global 5-point solve; the
assembly timed on its own; the 2 x 2-unit workload in microseconds per
sweep; one GPU's share of the 64 x 64-unit domain split eight ways; the
standalone gather and scatter in GB/s on a field larger than the last-level
cache; the GEMM rates torch.mm reaches (achievable peaks).
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
GOLDEN = os.path.join(ROOT, "tests", "golden")

# HBM traffic of the colour-phase kernel per launch on the 64 x 64-unit
# workload, by precision and tile shape, from two rocprofv3 --pmc passes
# (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) scaled by what the same counters
# read for a plain 512 MiB device copy (FETCH_SIZE reads half the copied bytes
# on this part: factor 2.0; WRITE_SIZE: 1.0). It is reported only while the
# kernel sources hash to the value the counters were taken with; otherwise
# "traffic" is null. Summary: profiles/tile_kernel_c4_traffic.md.
MEASURED_TRAFFIC = {
    "sources_sha256": "e3ca4b81af6293e60782b6b9091a014c1dc7af10e691b00029a32eacddb8ccee",
    "bytes_per_launch": {"C4:fp32:64|stream": (27791.9 * 2.0 + 4396.5) * 1024,
                         "C4:bf16:256|rowsplit": (14265.9 * 2.0 + 4312.4) * 1024,
                         "C4:fp16:256|rowsplit": (14268.5 * 2.0 + 4312.4) * 1024},
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
    """The float64 oracle's sweep rate on the host cores: `sample_sweeps`
    CROSS sweeps of the headline domain from its initial field, in
    point-evals/s. The step's assembly (one INTERIOR pass, 16x the points of
    a sweep) is not in the sample; its rate per point is the sweep's within
    the projection's share (T = 961 instead of 61)."""
    import torch
    from oracle import sweep as sw
    torch.set_num_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    solver = sw.sdnet_solver(torch.from_numpy(params.astype(np.float64)), width)
    u = torch.from_numpy(field.astype(np.float64))
    t0 = time.perf_counter()
    for _ in range(sample_sweeps):
        u = sw.sweep(u, ux, uy, solver)
    dt = time.perf_counter() - t0
    evals = sample_sweeps * sweep_points(ux, uy, CROSS_T)
    return {"value": evals / dt, "unit": "point-evals/s", "cores": torch.get_num_threads(),
            "kind": "oracle", "host": host_info(),
            "sample": f"{sample_sweeps} CROSS sweeps of the same 64x64-unit, width-{width} workload "
                      f"from its initial field, float64, {dt:.1f} s; the rate stands for the "
                      f"500-sweep step by extrapolation (the assembly is not in the sample)"}


def _rel(a, b) -> float:
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def _timed_steps(ctx, step, steps, warmup):
    """Warm-up, then `steps` timed calls of step() bracketed by device
    synchronisation; returns (total seconds, per-step seconds, colour-phase
    launches, their summed ms, their rows) with library timing on."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.timing_read()                      # drop anything recorded so far
    ctx.timing(True)
    per = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        t1 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        per.append(time.perf_counter() - t1)
    dt = time.perf_counter() - t0
    ctx.timing(False)
    launches, phase_ms, phase_rows = ctx.timing_read()
    return dt, per, launches, phase_ms, phase_rows


def _roofline(prec, width, launches, phase_ms, phase_rows, shape, workload=""):
    fpp = flops_per_point(width, CROSS_T)
    achieved = phase_rows * fpp / (phase_ms * 1e-3) / 1e12
    avg_us = phase_ms * 1e3 / max(launches, 1)
    # bf16 and fp16 share the dense MFMA peak (2.5 PFLOP/s)
    peak = PEAK_FP32_MFMA_TFLOPS if prec == "fp32" else PEAK_BF16_MFMA_TFLOPS
    key = f"{workload}:{prec}:{shape}"
    traffic = (MEASURED_TRAFFIC["bytes_per_launch"].get(key)
               if MEASURED_TRAFFIC["sources_sha256"] == kernel_sources_sha() else None)
    return {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": traffic,
            "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE/WRITE_SIZE)",
            "hbm_gbps": traffic / (avg_us * 1e3) if traffic else None,
            "hbm_frac": traffic / (avg_us * 1e-6) / PEAK_HBM_BYTES_PER_S if traffic else None,
            "kernel": f"tile_kernel (colour phase, {prec}, tile {shape})",
            "avg_launch_us": avg_us, "launches": launches,
            "flops_per_point_eval": fpp,
            "units_per_launch": phase_rows / max(launches, 1)}


def trajectory_parity(ctx, params, field, units, prec, gold_skel, ks, skel_j, skel_i, spread=None):
    """Error of the skeleton samples against oracle values after each sweep
    count in ks (mf_solve in segments; resuming is exact), and its maximum."""
    import torch
    from paper_2308_14258_amd import mf_solve
    u = field.clone()
    done = 0
    errs = {}
    for i, k in enumerate(ks):
        mf_solve(ctx, params, u, units, int(k) - done, prec=prec)
        done = int(k)
        torch.cuda.synchronize()
        got = u.cpu().numpy().astype(np.float64)[skel_j, skel_i]
        errs[int(k)] = _rel(got, gold_skel[i])
    out = {"rel_l2_skeleton_by_sweep": errs, "max": max(errs.values()),
           "argmax_sweep": max(errs, key=errs.get)}
    if spread is not None:
        out["float32_oracle_spread_by_sweep"] = spread
    return out


def c4_section(ctx, args, prec_name):
    """The 64 x 64-unit step in one precision: autotuned tile shape, warm-up,
    `steps` timed steps, the phase roofline, errors at 500 sweeps and along
    the trajectory."""
    import torch
    import mf_inputs as mi
    from paper_2308_14258_amd import MF_BF16, MF_CROSS, MF_FP16, MF_FP32, mf_autotune, mf_solve
    w = mi.WORKLOADS["C4"]
    ux, uy = w["units"]
    width = w["width"]
    K = args.sweeps
    prec = {"fp32": MF_FP32, "bf16": MF_BF16, "fp16": MF_FP16}[prec_name]
    field = torch.from_numpy(mi.workload_field("C4")).cuda()
    params = torch.from_numpy(mi.xavier_params(width, 0)).cuda()
    # tile shape chosen by the autotuner on a scratch copy (outside the timed region)
    shape = mf_autotune(ctx, params, field.clone(), (ux, uy), MF_CROSS, prec, trials=2)
    u = field.clone()
    u_out = torch.empty_like(u)

    def step():
        u.copy_(field)
        mf_solve(ctx, params, u, (ux, uy), K, targets=MF_CROSS, prec=prec, u_out=u_out)

    steps = args.steps if prec_name == "fp32" else max(args.steps, 5)
    dt, per, launches, phase_ms, phase_rows = _timed_steps(ctx, step, steps, args.warmup)
    evals = K * sweep_points(ux, uy, CROSS_T) + sweep_points(ux, uy, INTERIOR_T)
    res = {"value": evals * steps / dt, "steps": steps, "ms_per_step": dt * 1e3 / steps,
           "step_ms": {"median": float(np.median(per)) * 1e3, "min": min(per) * 1e3,
                       "max": max(per) * 1e3},
           "evals_per_step": evals, "tile_shape": tile_shape_name(shape),
           "roofline": _roofline(prec_name, width, launches, phase_ms, phase_rows, tile_shape_name(shape), "C4")}
    gpath = os.path.join(GOLDEN, "c4_fp64.npz")
    if K == w["sweeps"] and os.path.exists(gpath):
        g = np.load(gpath)
        sk = u.cpu().numpy().astype(np.float64)[g["skel_j"], g["skel_i"]]
        uo = u_out.cpu().numpy().astype(np.float64)[g["sample_j"], g["sample_i"]]
        res["parity"] = {"rel_l2_skeleton_vs_oracle": _rel(sk, g["skel500"]),
                         "rel_l2_u_out_vs_oracle": _rel(uo, g["u_out_sample"])}
        tpath = os.path.join(GOLDEN, "c4_traj.npz")
        if os.path.exists(tpath):
            t = np.load(tpath)
            spread = None
            cpath = os.path.join(GOLDEN, "c4_cond.npz")
            if os.path.exists(cpath):
                c = np.load(cpath)
                ref = {int(k): t["fp64"][list(t["K"]).index(k)] for k in c["K_fp32"] if k in t["K"]}
                spread = {int(k): _rel(c["fp32"][i], ref[int(k)]) for i, k in enumerate(c["K_fp32"])
                          if int(k) in ref}
            res["parity"]["trajectory"] = trajectory_parity(ctx, params, field, (ux, uy), prec, t["fp64"],
                                                            t["K"], g["skel_j"], g["skel_i"], spread)
    return res, u_out


def c4_mixed_section(ctx, args, refresh=50, assembly_fp16=False):
    """The 64 x 64-unit step with FP16 sweeps held to the float32 iteration
    by a correction refreshed every `refresh` sweeps (mf_solve_mixed; the
    refresh sweeps run each phase in float32 and in FP16, the assembly runs
    in float32, or in FP16 with assembly_fp16): throughput in the step's
    point evaluations (each refresh evaluates its points twice; that is
    overhead, not counted) and the error against the oracle at the step's
    sweep count."""
    import torch
    import mf_inputs as mi
    from paper_2308_14258_amd import MF_FP16, MF_FP32, mf_solve_mixed
    w = mi.WORKLOADS["C4"]
    asm = MF_FP16 if assembly_fp16 else MF_FP32
    ux, uy = w["units"]
    K = args.sweeps
    field = torch.from_numpy(mi.workload_field("C4")).cuda()
    params = torch.from_numpy(mi.xavier_params(w["width"], 0)).cuda()
    u = field.clone()
    u_out = torch.empty_like(u)

    def step():
        u.copy_(field)
        mf_solve_mixed(ctx, params, u, (ux, uy), K, refresh_every=refresh, prec=MF_FP16, u_out=u_out,
                       assembly_prec=asm)

    steps = max(args.steps, 5)
    dt, per, _, _, _ = _timed_steps(ctx, step, steps, 1)
    evals = K * sweep_points(ux, uy, CROSS_T) + sweep_points(ux, uy, INTERIOR_T)
    res = {"value": evals * steps / dt, "ms_per_step": dt * 1e3 / steps, "refresh_every": refresh,
           "assembly": "fp16" if assembly_fp16 else "fp32",
           "step_ms": {"median": float(np.median(per)) * 1e3, "min": min(per) * 1e3, "max": max(per) * 1e3}}
    gpath = os.path.join(GOLDEN, "c4_fp64.npz")
    if K == w["sweeps"] and os.path.exists(gpath):
        g = np.load(gpath)
        sk = u.cpu().numpy().astype(np.float64)[g["skel_j"], g["skel_i"]]
        uo = u_out.cpu().numpy().astype(np.float64)[g["sample_j"], g["sample_i"]]
        res["parity"] = {"rel_l2_skeleton_vs_oracle": _rel(sk, g["skel500"]),
                         "rel_l2_u_out_vs_oracle": _rel(uo, g["u_out_sample"])}
    return res


def c2_section(ctx, args):
    """16 x 16 units (961 placements), width 256, GP ring data, 200 sweeps +
    assembly, FP32: throughput and error against the oracle, with the
    trajectory."""
    import torch
    import mf_inputs as mi
    from paper_2308_14258_amd import MF_CROSS, MF_FP32, mf_autotune, mf_solve
    w = mi.WORKLOADS["C2"]
    ux, uy = w["units"]
    K = w["sweeps"]
    f = mi.workload_field("C2")
    field = torch.from_numpy(f).cuda()
    params = torch.from_numpy(mi.xavier_params(w["width"], 0)).cuda()
    shape = mf_autotune(ctx, params, field.clone(), (ux, uy), MF_CROSS, MF_FP32, trials=2)
    u = field.clone()
    u_out = torch.empty_like(u)

    def step():
        u.copy_(field)
        mf_solve(ctx, params, u, (ux, uy), K, u_out=u_out)

    dt, per, launches, phase_ms, phase_rows = _timed_steps(ctx, step, 5, 1)
    evals = K * sweep_points(ux, uy, CROSS_T) + sweep_points(ux, uy, INTERIOR_T)
    res = {"workload": "C2: 16x16 units (513x513 grid, 961 placements), width 256, GP ring data "
                       "(l=2, seed 1), 200 CROSS sweeps + assembly, FP32",
           "point_evals_per_s": evals * 5 / dt, "ms_per_step": dt * 1e3 / 5,
           "tile_shape": tile_shape_name(shape),
           "roofline": _roofline("fp32", w["width"], launches, phase_ms, phase_rows, tile_shape_name(shape), "C2")}
    gpath = os.path.join(GOLDEN, "c2_fp32.npz")
    if os.path.exists(gpath):
        from oracle.sweep import skeleton_mask
        g = np.load(gpath)
        uh = u.cpu().numpy().astype(np.float64)
        m = skeleton_mask(*f.shape).numpy()
        uo = u_out.cpu().numpy().astype(np.float64)[g["sample_j"], g["sample_i"]]
        res["parity"] = {"rel_l2_skeleton_vs_oracle": _rel(uh[m], g["skel200"]),
                         "rel_l2_u_out_vs_oracle": _rel(uo, g["u_out_sample"])}
    tpath = os.path.join(GOLDEN, "c2_traj.npz")
    if os.path.exists(tpath):
        t = np.load(tpath)
        spread = {int(k): _rel(t["fp32"][i], t["fp64"][i]) for i, k in enumerate(t["K"])}
        res.setdefault("parity", {})["trajectory"] = trajectory_parity(
            ctx, params, field, (ux, uy), MF_FP32, t["fp64"], t["K"], t["skel_j"], t["skel_i"], spread)
    return res


def gelu_section(ctx):
    """The paper's SDNet architecture (Sec. 3.1): circular convolutional
    boundary embedding (4 channels) + GELU layers, width 256, Xavier weights
    (seed 0), on the 64 x 64-unit workload: 20 CROSS sweeps + assembly,
    float32, three timed steps. Each colour phase is the per-placement
    embedding and projection, then the row kernels (first layer, three
    MFMA GEMMs with the GELU epilogue, output layer and scatter)."""
    import torch
    import mf_inputs as mi
    from paper_2308_14258_amd import mf_solve
    w = mi.WORKLOADS["C4"]
    ux, uy = w["units"]
    d, C, K = 256, 4, 20
    field = torch.from_numpy(mi.workload_field("C4")).cuda()
    params = torch.from_numpy(mi.xavier_conv_params(d, C, 0)).cuda()
    u = field.clone()
    u_out = torch.empty_like(u)

    def step():
        u.copy_(field)
        mf_solve(ctx, params, u, (ux, uy), K, u_out=u_out)

    dt, per, launches, phase_ms, phase_rows = _timed_steps(ctx, step, 3, 1)
    evals = K * sweep_points(ux, uy, CROSS_T) + sweep_points(ux, uy, INTERIOR_T)
    E = 128 * C
    fpp = 6.0 * d * d + 6.0 * d + (2.0 * E * d + 10.0 * 128 * C * (1 + C)) / CROSS_T
    ach = phase_rows * fpp / (phase_ms * 1e-3) / 1e12
    return {"workload": f"64x64 units, conv-embedding GELU SDNet (C={C}, width {d}), {K} CROSS sweeps + assembly, "
                        "float32",
            "point_evals_per_s": evals * 3 / dt, "ms_per_step": dt * 1e3 / 3,
            "colour_phase": {"avg_us": phase_ms * 1e3 / max(launches, 1), "tflops": ach,
                             "frac_of_fp32_mfma_peak": ach / PEAK_FP32_MFMA_TFLOPS,
                             "flops_per_point_eval": fpp,
                             "kernels": "embed_project + fwd_layer1<GELU> + 3 x taylor_gemm<GELU> + rows_output"}}


def trained_section(ctx):
    """A trained SDNet (weights/sdnet_laplace_d256.npz) and the predictor's
    accuracy against the global 5-point solve (oracle values stored in
    tests/golden/mfp_global.npz): the 4 x 4-unit problem after 100 sweeps,
    and on the 64 x 64-unit problem the float32 sweep count and time to MAE
    0.05 (checked every 100 sweeps) and the MAE after 2000 sweeps."""
    import torch
    import mf_inputs as mi
    from paper_2308_14258_amd import MF_BF16, MF_FP16, MF_FP32, mf_solve, mf_solve_mixed
    from paper_2308_14258_amd.sdnet_training import WEIGHTS_DIR, load_trained
    params, width, cfg, hist = load_trained(os.path.join(WEIGHTS_DIR, "sdnet_laplace_d256.npz"))
    p = torch.from_numpy(params).cuda()
    gpath = os.path.join(GOLDEN, "mfp_global.npz")
    if not os.path.exists(gpath):
        return None
    g = np.load(gpath)
    res = {"network": f"width {width}, tanh, {cfg['epochs']} epochs on {cfg['n_bc']} GP conditions, "
                      f"validation MSE {hist['val_mse'][-1]:.2e}"}
    f4 = mi.gp_field(4, 4, 1.0, seed=31)
    for name, prec in (("fp32", MF_FP32), ("bf16", MF_BF16), ("fp16", MF_FP16)):
        u = torch.from_numpy(f4).cuda()
        uo = torch.empty_like(u)
        mf_solve(ctx, p, u, (4, 4), 100, prec=prec, u_out=uo)
        torch.cuda.synchronize()
        res.setdefault("fig1_4x4_units_100_sweeps_mae", {})[name] = float(
            np.abs(uo.cpu().numpy().astype(np.float64) - g["u4"])[1:-1, 1:-1].mean())
    f64 = mi.gp_field(64, 64, 2.0, seed=41)

    def mae(uo):
        return float(np.mean(np.abs(uo.cpu().numpy()[g["sample_j"], g["sample_i"]] - g["u64_sample"])))

    t4 = {}
    # plain sweeps in each precision, and 16-bit sweeps with a float32
    # correction refreshed every `refresh` sweeps (mf_solve_mixed)
    # (the assembly in float32, or in the sweeps' precision: asm16)
    runs = (("fp32", MF_FP32, 0, MF_FP32), ("bf16", MF_BF16, 0, MF_FP32), ("fp16", MF_FP16, 0, MF_FP32),
            ("fp16_mixed_refresh50", MF_FP16, 50, MF_FP32), ("fp16_mixed_refresh50_asm16", MF_FP16, 50, MF_FP16),
            ("bf16_mixed_refresh5", MF_BF16, 5, MF_FP32))
    for name, prec, refresh, asm in runs:
        def solve(u, n, uo=None):
            if refresh:
                mf_solve_mixed(ctx, p, u, (64, 64), n, refresh_every=refresh, prec=prec, u_out=uo,
                               assembly_prec=asm)
            else:
                mf_solve(ctx, p, u, (64, 64), n, prec=prec, u_out=uo)
        u = torch.from_numpy(f64).cuda()
        uo = torch.empty_like(u)
        hit = None
        curve = {}
        for k in range(100, 2001, 100):
            solve(u, 100, uo)
            torch.cuda.synchronize()
            curve[k] = mae(uo)
            if hit is None and curve[k] < 0.05:
                hit = k
        r = {"mae_by_sweeps": curve, "sweeps_to_mae_0.05": hit}
        if hit is not None:
            u = torch.from_numpy(f64).cuda()
            solve(u, 10)
            u.copy_(torch.from_numpy(f64).cuda())
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            solve(u, hit, uo)
            torch.cuda.synchronize()
            r["seconds_to_mae_0.05"] = time.perf_counter() - t0
        t4[name] = r
    res["table4_64x64_units"] = t4
    # the paper's network (convolutional embedding, GELU), trained the same way
    gw = os.path.join(WEIGHTS_DIR, "sdnet_laplace_gelu_c4_d256.npz")
    if os.path.exists(gw):
        gparams, gwidth, gcfg, ghist = load_trained(gw)
        gp = torch.from_numpy(gparams).cuda()
        u = torch.from_numpy(f4).cuda()
        uo = torch.empty_like(u)
        mf_solve(ctx, gp, u, (4, 4), 100, u_out=uo)
        torch.cuda.synchronize()
        r = {"network": f"width {gwidth}, conv embedding C={gcfg['channels']} + GELU, {gcfg['epochs']} epochs, "
                        f"validation MSE {ghist['val_mse'][-1]:.2e}",
             "fig1_4x4_units_100_sweeps_mae_fp32": float(
                 np.abs(uo.cpu().numpy().astype(np.float64) - g["u4"])[1:-1, 1:-1].mean())}
        u = torch.from_numpy(f64).cuda()
        uo = torch.empty_like(u)
        curve = {}
        for k in range(100, 2001, 100):
            mf_solve(ctx, gp, u, (64, 64), 100, u_out=uo)
            torch.cuda.synchronize()
            curve[k] = mae(uo)
        r["table4_64x64_mae_by_sweeps_fp32"] = curve
        res["papers_network"] = r
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sweeps", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-sweeps", type=int, default=3)
    ap.add_argument("--mode", choices=["solve", "copy"], default="solve",
                    help="copy: one plain device copy of --copy-mb MiB, the reference "
                         "kernel for scaling HBM counters")
    ap.add_argument("--copy-mb", type=int, default=512)
    ap.add_argument("--headline-only", action="store_true",
                    help="only the 64x64-unit FP32 and BF16 steps (for profiling and counters)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip C1, the per-GPU share, gather/scatter bandwidth and the GEMM peaks")
    ap.add_argument("--no-c5", action="store_true", help="skip the 48-domain batch and its adjoint")
    ap.add_argument("--no-train", action="store_true", help="skip the training-step measurement")
    ap.add_argument("--train-steps", type=int, default=20)
    ap.add_argument("--only-c5", action="store_true")
    ap.add_argument("--only-train", action="store_true", help="only the training-step measurement")
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
    from paper_2308_14258_amd import Context

    if args.mode == "copy":
        n = args.copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read": 4 * n, "bytes_written": 4 * n}), flush=True)
        return

    if args.only_c5 or args.only_train or args.only_io:
        ctx = Context(0)
        if args.only_io:
            out = {"gather_scatter": io_measurement(ctx)}
        elif args.only_c5:
            out = {"c5": batched_measurement(ctx)}
        else:
            out = {"train": train_measurement(ctx, args.train_steps)}
        print(json.dumps(out), flush=True)
        ctx.close()
        return

    w = mi.WORKLOADS["C4"]
    ux, uy = w["units"]
    width = w["width"]
    ctx = Context(0)
    fp32, uo32 = c4_section(ctx, args, "fp32")
    print(f"# fp32 64x64: {fp32['value']:.4g} point-evals/s", file=sys.stderr, flush=True)
    half = {}
    for name in ("bf16", "fp16"):
        r, uo = c4_section(ctx, args, name)
        print(f"# {name} 64x64: {r['value']:.4g} point-evals/s", file=sys.stderr, flush=True)
        d = uo.double()[1:-1, 1:-1] - uo32.double()[1:-1, 1:-1]
        r["rel_l2_vs_fp32_u_out"] = float(d.norm() / uo32.double()[1:-1, 1:-1].norm())
        r["speedup_over_fp32"] = r["value"] / fp32["value"]
        half[name] = r
        del uo
    del uo32
    out = {
        "metric": METRIC,
        "value": fp32["value"],
        "unit": "point-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "C4: plain Mosaic Flow, 64x64 units (2049x2049 grid, 16,129 placements), "
                               "SDNet width 256 (Xavier-normal, seed 0), e^x sin y ring data scaled to "
                               f"[0, 1], {args.sweeps} CROSS sweeps + overlap-averaged assembly",
                   "units": [ux, uy], "width": width, "sweeps": args.sweeps, "targets": "cross",
                   "evals_per_step": fp32["evals_per_step"], "tile_shape": fp32["tile_shape"]},
        "step_ms": fp32["step_ms"],
        "roofline": fp32["roofline"],
        "parity": fp32.get("parity"),
        "bf16": half["bf16"],
        "fp16": half["fp16"],
    }
    mixed = c4_mixed_section(ctx, args)
    mixed["speedup_over_fp32"] = mixed["value"] / fp32["value"]
    out["fp16_mixed"] = mixed
    mixed16 = c4_mixed_section(ctx, args, assembly_fp16=True)
    mixed16["speedup_over_fp32"] = mixed16["value"] / fp32["value"]
    out["fp16_mixed_asm16"] = mixed16
    print(f"# fp16 mixed 64x64: {mixed['value']:.4g} point-evals/s, with the FP16 assembly "
          f"{mixed16['value']:.4g}", file=sys.stderr, flush=True)
    if not args.headline_only:
        out["c2"] = c2_section(ctx, args)
        print("# c2 done", file=sys.stderr, flush=True)
        if not args.no_c5:
            out["c5"] = batched_measurement(ctx)
            print("# c5 done", file=sys.stderr, flush=True)
        if not args.no_train:
            out["train"] = train_measurement(ctx, args.train_steps)
        out["gelu_conv_sdnet"] = gelu_section(ctx)
        print("# gelu done", file=sys.stderr, flush=True)
        out["trained"] = trained_section(ctx)
        print("# trained done", file=sys.stderr, flush=True)
        params = torch.from_numpy(mi.xavier_params(width, 0)).cuda()
        out["assembly"] = assembly_measurement(ctx, params, torch.from_numpy(mi.workload_field("C4")).cuda(),
                                               (ux, uy))
        if not args.no_extras:
            out["c1"] = c1_measurement(ctx)
            out["per_gpu_share"] = per_gpu_share_measurement(ctx)
            out["gather_scatter"] = io_measurement(ctx)
            out["achievable_peaks"] = achievable_peaks()
            out["roofline"]["frac_of_achievable"] = (out["roofline"]["achieved"] /
                                                     out["achievable_peaks"]["fp32_tflops"])
            for name in ("bf16", "fp16"):
                out[name]["roofline"]["frac_of_achievable"] = (out[name]["roofline"]["achieved"] /
                                                               out["achievable_peaks"][name + "_tflops"])
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(mi.workload_field("C4"), mi.xavier_params(width, 0), width,
                                               ux, uy, args.cpu_sample_sweeps)
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
    res = {"workload": "C3: 1024 conditions x (128 + 256) points, width 128, Adam",
           "steps_per_s": steps / dt, "ms_per_step": dt * 1e3 / steps,
           "gemm_tflops": flops * steps / dt / 1e12,
           "frac_of_fp32_mfma_peak": flops * steps / dt / 1e12 / PEAK_FP32_MFMA_TFLOPS,
           "last_loss": [float(x) for x in loss.cpu()]}
    res["lamb"] = train_lamb_measurement(ctx, steps, G, Xb, Xc, d)
    res["gelu_conv_sdnet"] = train_gelu_measurement(ctx, steps, G, Xb, Xc, d)
    return res


def train_gelu_measurement(ctx, steps, G, Xb, Xc, d, C=4):
    """The same training step (Alg. 1 + Adam, same conditions and points) for
    the paper's network: the convolutional embedding (C channels) and GELU
    layers at the same width."""
    import torch
    import mf_inputs as mi
    from paper_2308_14258_amd import sdnet_train_step
    p = torch.from_numpy(mi.xavier_conv_params(d, C, 0, bias_scale=0.1)).cuda()
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
    return {"network": f"conv embedding (C={C}) + GELU, width {d}", "steps_per_s": steps / dt,
            "ms_per_step": dt * 1e3 / steps, "last_loss": [float(x) for x in loss.cpu()]}


def train_lamb_measurement(ctx, steps, G, Xb, Xc, d):
    """The same step with the paper's optimiser (Sec. 5.2): the loss and
    gradient (sdnet_loss_grad), then LAMB (sdnet_lamb_step) at the
    schedule's learning rate (peak 1e-3, 0.1% warm-up, linear decay over
    500 x steps iterations), gradient clipped to norm 1; and the LAMB
    kernel alone."""
    import torch
    import mf_inputs as mi
    from paper_2308_14258_amd import lr_at, lr_schedule, sdnet_lamb_step, sdnet_loss_grad
    p = torch.from_numpy(mi.xavier_params(d, 0)).cuda()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    sched = lr_schedule(1e-3, 500 * steps)
    hp = dict(weight_decay=0.0, max_grad_norm=1.0, trust_without_decay=True)
    loss, grad = sdnet_loss_grad(ctx, p, G, Xb, Xc)
    for k in range(2):
        sdnet_loss_grad(ctx, p, G, Xb, Xc, loss=loss, grad_out=grad)
        sdnet_lamb_step(ctx, p, m, v, grad, k + 1, lr=lr_at(sched, k + 1), **hp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        sdnet_loss_grad(ctx, p, G, Xb, Xc, loss=loss, grad_out=grad)
        sdnet_lamb_step(ctx, p, m, v, grad, k + 3, lr=lr_at(sched, k + 3), **hp)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lamb_ms = _event_ms(lambda: sdnet_lamb_step(ctx, p, m, v, grad, 100, lr=1e-4, **hp), 20)
    n = p.numel()
    return {"optimizer": "LAMB (trust ratio per tensor, clip 1.0), warm-up + linear decay",
            "steps_per_s": steps / dt, "ms_per_step": dt * 1e3 / steps,
            "lamb_kernel_us": lamb_ms * 1e3,
            # algorithmic bytes: p, m, v, g read once, p, m, v written once
            "lamb_kernel_gbps": 7 * 4 * n / (lamb_ms * 1e-3) / 1e9,
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
    for name, dt in (("fp32", torch.float32), ("bf16", torch.bfloat16), ("fp16", torch.float16)):
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
    # the skeleton side layout: vertical edges and centre lines from the
    # transposed skeleton columns, the field's rows padded to a multiple of
    # 32 floats (128 bytes) so that even-offset edges start on a cache line
    from paper_2308_14258_amd import SkeletonCols, mf_gather_skel, mf_scatter_skel, mf_skeleton_pack, mf_skeleton_unpack
    ny, nx = u.shape
    padded = torch.empty(ny, (nx + 31) // 32 * 32, device="cuda")[:, :nx]
    padded.copy_(u)
    del u
    u = padded
    res["side_layout_row_pitch_floats"] = int(u.stride(0))
    cols = SkeletonCols(u, (ux, uy))
    pack_ms = _event_ms(lambda: mf_skeleton_pack(ctx, u, cols), 5)
    unpack_ms = _event_ms(lambda: mf_skeleton_unpack(ctx, cols, u), 5)
    tot["gather_side_layout"] = [0.0, 0.0]
    tot["scatter_cross_side_layout"] = [0.0, 0.0]
    for c in range(4):
        n = mf_colour_placements((ux, uy), c)
        G = torch.empty(n, 128, device="cuda")
        ms = _event_ms(lambda: mf_gather_skel(ctx, u, cols, c, G), 20)
        tot["gather_side_layout"][0] += ms
        tot["gather_side_layout"][1] += n * 1024.0
        pred = torch.randn(n, 61, device="cuda")
        ms = _event_ms(lambda: mf_scatter_skel(ctx, pred, u, cols, c), 20)
        tot["scatter_cross_side_layout"][0] += ms
        tot["scatter_cross_side_layout"][1] += n * 61 * 8.0
        del pred, G
    for key, (ms, nbytes) in tot.items():
        gbps = nbytes / (ms * 1e-3) / 1e9
        res[key] = {"us_per_launch": ms * 1e3 / 4, "algorithmic_bytes_per_sweep": nbytes,
                    "GB_per_s": gbps, "frac_of_hbm_peak": gbps * 1e9 / PEAK_HBM_BYTES_PER_S}
    res["side_layout_pack_us"] = pack_ms * 1e3
    res["side_layout_unpack_us"] = unpack_ms * 1e3
    return res


def batched_measurement(ctx):
    """48 independent domains (4..48 units per side, seed 7), width 256, GP
    ring data: 20 sweeps + assembly in one launch per colour for the whole
    batch, BF16 (the workload's precision), FP16 and FP32, each timed over three
    steps and checked at its smallest, median and largest domain against
    oracle values along the 20 sweeps; then the FP32 adjoint of
    J = sum u_out^2 through the 20 sweeps with checkpoints every 5, checked
    on the smallest domain against the oracle's gradient."""
    import torch
    import mf_inputs as mi
    from paper_2308_14258_amd import MF_BF16, MF_CROSS, MF_FP16, MF_FP32, Batch, mf_autotune, mf_solve, mf_solve_adjoint
    w = mi.WORKLOADS["C5"]
    t0 = time.perf_counter()
    sizes, fields = mi.batched_domains(w["n_domains"], 4, 48, w["length"], w["seed"])
    gen_s = time.perf_counter() - t0
    params = torch.from_numpy(mi.xavier_params(w["width"], 0)).cuda()
    batch = Batch(fields)
    base = batch.buf.clone()
    out = torch.empty_like(batch.buf)
    K = w["sweeps"]
    placements = int(sum((2 * ux - 1) * (2 * uy - 1) for ux, uy in sizes))
    evals = K * placements * CROSS_T + placements * INTERIOR_T
    res = {"workload": f"C5: 48 domains (4..48 units per side, seed 7), {placements} placements, width 256, "
                       f"GP ring data (l=1), {K} CROSS sweeps + assembly",
           "input_generation_s": gen_s}
    gpath = os.path.join(GOLDEN, "c5_k20.npz")
    g = np.load(gpath) if os.path.exists(gpath) else None
    for name, prec in (("bf16", MF_BF16), ("fp16", MF_FP16), ("fp32", MF_FP32)):
        # tile shape for the whole domain list from the autotuner (outside the timed region)
        shape = mf_autotune(ctx, params, batch, None, MF_CROSS, prec, trials=1)

        def step():
            batch.buf.copy_(base)
            mf_solve(ctx, params, batch, None, K, prec=prec, u_out=out)

        dt, per, launches, phase_ms, phase_rows = _timed_steps(ctx, step, 3, 1)
        r = {"point_evals_per_s": evals * 3 / dt, "ms_per_step": dt * 1e3 / 3, "tile_shape": tile_shape_name(shape),
             "roofline": _roofline(name, w["width"], launches, phase_ms, phase_rows, tile_shape_name(shape))}
        if g is not None:
            # errors at the stored sweep counts (solve in segments; resuming is exact)
            batch.buf.copy_(base)
            done = 0
            traj = {}
            for i, k in enumerate(g["K"]):
                k = int(k)
                mf_solve(ctx, params, batch, None, k - done, prec=prec, u_out=out if k == K else None)
                done = k
                torch.cuda.synchronize()
                for n, d in enumerate(g["picks"]):
                    u = batch.field(int(d)).cpu().numpy().astype(np.float64)
                    e = _rel(u[g[f"skel_j{n}"], g[f"skel_i{n}"]], g[f"skel_fp64_{n}"][i])
                    traj.setdefault(int(d), {})[k] = e
            par = {}
            for n, d in enumerate(g["picks"]):
                d = int(d)
                uo = batch.field(d, out).cpu().numpy().astype(np.float64)
                par[d] = {"units": [int(v) for v in sizes[d]],
                          "rel_l2_skeleton_vs_oracle_by_sweep": traj[d],
                          "trajectory_max": max(traj[d].values()),
                          "rel_l2_u_out_vs_oracle": _rel(uo[g[f"sample_j{n}"], g[f"sample_i{n}"]],
                                                         g[f"u_out_fp64_{n}"]),
                          "float32_oracle_spread_at_K": _rel(g[f"skel_fp32_{n}"][-1], g[f"skel_fp64_{n}"][-1])}
            r["parity"] = par
        res[name] = r
    batch.buf.copy_(base)
    ub, J = mf_solve_adjoint(ctx, params, batch, None, K, w["ckpt"])   # sizes the workspace
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ub, J = mf_solve_adjoint(ctx, params, batch, None, K, w["ckpt"], u0_bar=ub, J=J)
    torch.cuda.synchronize()
    dta = time.perf_counter() - t0
    adj = {"s": dta, "ratio_to_fp32_forward": dta * 1e3 / res["fp32"]["ms_per_step"],
           "J": float(J.item()), "grad_norm": float(ub.double().norm().item())}
    apath = os.path.join(GOLDEN, "c5_adjoint.npz")
    if os.path.exists(apath):
        a = np.load(apath)
        got = batch.field(int(a["domain"]), ub).cpu().numpy().astype(np.float64)
        adj["rel_l2_u0_bar_vs_oracle_smallest_domain"] = _rel(got, a["u0_bar"])
    res["fp32_adjoint"] = adj
    return res


def tile_shape_name(code):
    """Readable tile shape: height plus the MF_TILE_WIDE / STREAM / ROWSPLIT / PERSIST flags."""
    name = str(code & 0xFFFF)
    if code & (1 << 16):
        name += "|wide"
    if code & (1 << 17):
        name += "|stream"
    if code & (1 << 18):
        name += "|rowsplit"
    if code & (1 << 19):
        name += "|persist"
    return name


if __name__ == "__main__":
    main()
