"""Write the stored expected values used by the GPU parity tests.

Every value here comes from the float64 oracle (``oracle/``) run on the
seeded inputs of ``mf_inputs``; nothing is read from the HIP path.

    python tests/golden/make_golden.py [name ...]

c3_train.npz -- the training workload: full-batch gradient at the initial
    parameters and the loss curve of 100 Adam steps.
c4_fp64.npz -- 64 x 64 units, 500 sweeps: sampled skeleton values and
    sampled assembly points.
c4_one_sweep.npz -- the same 64 x 64-unit problem after ONE sweep from the
    initial field: the skeleton at the c4 sample points and the assembly of
    that state at the c4 assembly points (a full-size check of the sweep map
    that does not pass through the early transient, where an untrained
    network amplifies float32 rounding differences by orders of magnitude).
c5_one_sweep.npz -- the 48-domain batch (sizes 4..48 units, GP data length
    1.0, seed 7), width 256: for its smallest, median and largest domain (by
    placement count) one sweep from the initial field, as 4096 sampled
    skeleton values, and the assembly of that state at 256 sampled points.
c2_fp32.npz -- 16 x 16 units, width 256, GP ring data (length 2, seed 1),
    Xavier weights seed 0, 200 CROSS sweeps then the assembly. Holds the
    skeleton after 20 and 200 sweeps and u_out at 8192 sampled interior
    points (seed 123).
c2_traj.npz -- the 16 x 16-unit workload's skeleton at 8192 sampled points
    (seed 124) after each sweep count in TRAJ_K (up to 200) for three runs
    of the oracle: float64 on the
    stored parameters ("fp64"), float64 on parameters moved by a relative
    amount of float32 rounding size ("fp64_perturbed"), and the same
    algorithm evaluated in float32 ("fp32"). The last two measure how far
    rounding at float32 level alone moves the trajectory (its conditioning).
c4_traj.npz -- 64 x 64 units: the c4 sampled skeleton values after each sweep
    count in TRAJ_K (float64, up to 500 sweeps).
c4_cond.npz -- 64 x 64 units, the "fp64_perturbed" run of the same samples
    up to 50 sweeps (K) and the "fp32" run up to 500 (K_fp32).
c5_k20.npz -- the 48-domain batch's smallest, median and largest domain at
    its stated 20 sweeps: sampled skeleton after 1, 5, 10, 15 and 20 sweeps
    and the assembly after 20 at sampled points, for the three runs above.
mfp_global.npz -- ground truth for the trained network's accuracy: the global
    5-point Dirichlet solution (the oracle's sparse direct solve) of a
    4 x 4-unit domain with GP ring data (length 1, seed 31), whole, and of a
    64 x 64-unit domain with GP ring data (length 2, seed 41) at 65536
    sampled interior points (seed 557).
c5_adjoint.npz -- the smallest domain of that batch: u0_bar after 20 sweeps
    and the assembly for J = sum of squared interior values, and for a
    random seed u_out_bar (default_rng(77) normals), both full fields.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import mf_inputs as mi  # noqa: E402
from oracle import sweep as sw  # noqa: E402


def _sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]


def c2():
    w = mi.WORKLOADS["C2"]
    ux, uy = w["units"]
    field = mi.workload_field("C2")
    params = mi.xavier_params(w["width"], seed=0)
    solver = sw.sdnet_solver(torch.from_numpy(params.astype(np.float64)), w["width"])
    u = torch.from_numpy(field.astype(np.float64))
    t0 = time.time()
    skel20 = None
    for k in range(1, w["sweeps"] + 1):
        u = sw.sweep(u, ux, uy, solver)
        if k == 20:
            skel20 = sw.skeleton_values(u).numpy()
        if k % 20 == 0:
            print(f"c2: sweep {k} ({time.time() - t0:.0f} s)", flush=True)
    skel = sw.skeleton_values(u).numpy()
    u_out = sw.assemble(u, ux, uy, solver).numpy()
    rng = np.random.default_rng(123)
    ny, nx = u_out.shape
    jj = rng.integers(1, ny - 1, 8192)
    ii = rng.integers(1, nx - 1, 8192)
    np.savez_compressed(os.path.join(HERE, "c2_fp32.npz"), skel20=skel20, skel200=skel,
                        sample_j=jj.astype(np.int32), sample_i=ii.astype(np.int32),
                        u_out_sample=u_out[jj, ii], field_sha=_sha(field), params_sha=_sha(params))
    print(f"c2: done in {time.time() - t0:.0f} s", flush=True)


def c3():
    """1024 GP boundary conditions (l = 0.5, seed 2) x 256 collocation points
    (seed 3), width 128, Xavier seed 0: the full-batch gradient at the initial
    parameters and the (L_data, L_pde) curve of 100 Adam steps (lr 1e-3)."""
    from oracle import train
    w = mi.WORKLOADS["C3"]
    G32 = mi.gp_perimeter_batch(w["n_bc"], w["length"], w["bc_seed"])
    Xc32 = mi.collocation_points(w["n_bc"], w["n_colloc"], w["colloc_seed"])
    Xb = torch.from_numpy(mi.unit_perimeter_nodes())
    G = torch.from_numpy(G32.astype(np.float64))
    Xc = torch.from_numpy(Xc32.astype(np.float64))
    th0 = mi.xavier_params(w["width"], 0)
    th = torch.from_numpy(th0.astype(np.float64))
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    t0 = time.time()
    ld, lp, gd, gp = train.gradient(th, w["width"], G, Xb, Xc)
    grad0 = (gd + gp).numpy()
    curve = []
    for step in range(1, w["steps"] + 1):
        th, m, v, ld, lp = train.train_step(th, m, v, step, w["width"], G, Xb, Xc)
        curve.append((ld, lp))
        if step % 5 == 0:
            print(f"c3: step {step} L_data {ld:.6e} L_pde {lp:.6e} ({time.time() - t0:.0f} s)",
                  flush=True)
    np.savez_compressed(os.path.join(HERE, "c3_train.npz"), grad0=grad0, curve=np.array(curve),
                        G_sha=_sha(G32), Xc_sha=_sha(Xc32), params_sha=_sha(th0))
    print(f"c3: done in {time.time() - t0:.0f} s", flush=True)


def c4():
    """64 x 64 units (2049^2 grid), width 256, e^x sin y ring data, Xavier
    seed 0, 500 CROSS sweeps: 32768 sampled skeleton values after 20 and 500
    sweeps and the assembly at 2048 sampled interior points (seed 321)."""
    w = mi.WORKLOADS["C4"]
    ux, uy = w["units"]
    field = mi.workload_field("C4")
    params = mi.xavier_params(w["width"], seed=0)
    solver = sw.sdnet_solver(torch.from_numpy(params.astype(np.float64)), w["width"])
    u = torch.from_numpy(field.astype(np.float64))
    mask = sw.skeleton_mask(*field.shape).numpy()
    sj, si = np.nonzero(mask)
    rng = np.random.default_rng(321)
    pick = rng.choice(sj.size, 32768, replace=False)
    sj, si = sj[pick], si[pick]
    t0 = time.time()
    skel20 = None
    for k in range(1, w["sweeps"] + 1):
        u = sw.sweep(u, ux, uy, solver)
        if k == 20:
            skel20 = u.numpy()[sj, si].copy()
        if k % 10 == 0:
            print(f"c4: sweep {k} ({time.time() - t0:.0f} s)", flush=True)
    skel500 = u.numpy()[sj, si].copy()
    ny, nx = field.shape
    aj = rng.integers(1, ny - 1, 2048)
    ai = rng.integers(1, nx - 1, 2048)
    u_out = sw.assemble_at(u, ux, uy, solver, list(zip(aj.tolist(), ai.tolist()))).numpy()
    np.savez_compressed(os.path.join(HERE, "c4_fp64.npz"), skel_j=sj.astype(np.int32),
                        skel_i=si.astype(np.int32), skel20=skel20, skel500=skel500,
                        sample_j=aj.astype(np.int32), sample_i=ai.astype(np.int32),
                        u_out_sample=u_out, field_sha=_sha(field), params_sha=_sha(params))
    print(f"c4: done in {time.time() - t0:.0f} s", flush=True)


def c4_one():
    """One sweep of the 64 x 64-unit workload from its initial field, sampled
    at the c4 points (which it reads from c4_fp64.npz, itself oracle output)."""
    g = np.load(os.path.join(HERE, "c4_fp64.npz"))
    w = mi.WORKLOADS["C4"]
    ux, uy = w["units"]
    field = mi.workload_field("C4")
    params = mi.xavier_params(w["width"], seed=0)
    solver = sw.sdnet_solver(torch.from_numpy(params.astype(np.float64)), w["width"])
    t0 = time.time()
    u1 = sw.sweep(torch.from_numpy(field.astype(np.float64)), ux, uy, solver)
    skel1 = u1.numpy()[g["skel_j"], g["skel_i"]].copy()
    pts = list(zip(g["sample_j"].tolist(), g["sample_i"].tolist()))
    out1 = sw.assemble_at(u1, ux, uy, solver, pts).numpy()
    np.savez_compressed(os.path.join(HERE, "c4_one_sweep.npz"), skel1=skel1, u_out_sample=out1,
                        field_sha=_sha(field), params_sha=_sha(params))
    print(f"c4_one: done in {time.time() - t0:.0f} s", flush=True)


def c5_one():
    """One sweep of three sampled domains of the batched workload (their
    fields come from the same seeded generator as the whole batch)."""
    w = mi.WORKLOADS["C5"]
    t0 = time.time()
    sizes, fields = mi.batched_domains(w["n_domains"], 4, 48, w["length"], w["seed"])
    print(f"c5_one: inputs in {time.time() - t0:.0f} s", flush=True)
    params = mi.xavier_params(w["width"], seed=0)
    solver = sw.sdnet_solver(torch.from_numpy(params.astype(np.float64)), w["width"])
    places = [(2 * int(ux) - 1) * (2 * int(uy) - 1) for ux, uy in sizes]
    order = np.argsort(places, kind="stable")
    picks = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    out = {"picks": np.array(picks, dtype=np.int32), "sizes": sizes.astype(np.int32),
           "params_sha": _sha(params)}
    rng = np.random.default_rng(555)
    for n, d in enumerate(picks):
        ux, uy = (int(v) for v in sizes[d])
        f = fields[d]
        u1 = sw.sweep(torch.from_numpy(f.astype(np.float64)), ux, uy, solver)
        mask = sw.skeleton_mask(*f.shape).numpy()
        sj, si = np.nonzero(mask)
        pick = rng.choice(sj.size, min(4096, sj.size), replace=False)
        aj = rng.integers(1, f.shape[0] - 1, 256)
        ai = rng.integers(1, f.shape[1] - 1, 256)
        out[f"skel_j{n}"] = sj[pick].astype(np.int32)
        out[f"skel_i{n}"] = si[pick].astype(np.int32)
        out[f"skel1_{n}"] = u1.numpy()[sj[pick], si[pick]].copy()
        out[f"sample_j{n}"] = aj.astype(np.int32)
        out[f"sample_i{n}"] = ai.astype(np.int32)
        out[f"u_out{n}"] = sw.assemble_at(u1, ux, uy, solver, list(zip(aj.tolist(), ai.tolist()))).numpy()
        out[f"field_sha{n}"] = _sha(f)
        print(f"c5_one: domain {d} ({ux}x{uy}) done at {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, "c5_one_sweep.npz"), **out)


TRAJ_K = (1, 5, 10, 15, 20, 30, 50, 100, 150, 200, 300, 400, 500)


def _perturbed(params: np.ndarray, seed: int) -> np.ndarray:
    """float64 copy of the float32 parameters, each entry scaled by
    1 + r 2^-24 with r uniform in [-1, 1]: a change of float32 rounding size."""
    r = np.random.default_rng(seed).uniform(-1.0, 1.0, params.shape)
    return params.astype(np.float64) * (1.0 + r * 2.0 ** -24)


def _runs(params: np.ndarray, width: int):
    """(name, solver, dtype) of the three oracle runs of a conditioning study."""
    out = []
    for name, th, dt in (("fp64", params.astype(np.float64), torch.float64),
                         ("fp64_perturbed", _perturbed(params, 901), torch.float64),
                         ("fp32", params, torch.float32)):
        out.append((name, sw.sdnet_solver(torch.from_numpy(th).to(dt), width), dt))
    return out


def c2_traj():
    w = mi.WORKLOADS["C2"]
    ux, uy = w["units"]
    field = mi.workload_field("C2")
    params = mi.xavier_params(w["width"], seed=0)
    sj, si = np.nonzero(sw.skeleton_mask(*field.shape).numpy())
    pick = np.sort(np.random.default_rng(124).choice(sj.size, 8192, replace=False))
    sj, si = torch.from_numpy(sj[pick]), torch.from_numpy(si[pick])
    ks = [k for k in TRAJ_K if k <= w["sweeps"]]
    out = {"K": np.array(ks, dtype=np.int32), "skel_j": sj.numpy().astype(np.int32),
           "skel_i": si.numpy().astype(np.int32), "field_sha": _sha(field), "params_sha": _sha(params)}
    t0 = time.time()
    for name, solver, dt in _runs(params, w["width"]):
        u = torch.from_numpy(field).to(dt)
        rows = []
        for k in range(1, w["sweeps"] + 1):
            u = sw.sweep(u, ux, uy, solver)
            if k in ks:
                rows.append(u[sj, si].to(torch.float64).numpy())
        out[name] = np.stack(rows)
        print(f"c2_traj: {name} done ({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "c2_traj.npz"), **out)


def _c4_samples():
    g = np.load(os.path.join(HERE, "c4_fp64.npz"))
    return g["skel_j"], g["skel_i"]


def c4_traj():
    w = mi.WORKLOADS["C4"]
    ux, uy = w["units"]
    field = mi.workload_field("C4")
    params = mi.xavier_params(w["width"], seed=0)
    sj, si = _c4_samples()
    solver = sw.sdnet_solver(torch.from_numpy(params.astype(np.float64)), w["width"])
    u = torch.from_numpy(field.astype(np.float64))
    rows = []
    t0 = time.time()
    for k in range(1, w["sweeps"] + 1):
        u = sw.sweep(u, ux, uy, solver)
        if k in TRAJ_K:
            rows.append(u.numpy()[sj, si].copy())
            print(f"c4_traj: sweep {k} ({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "c4_traj.npz"), K=np.array(TRAJ_K, dtype=np.int32),
                        fp64=np.stack(rows), field_sha=_sha(field), params_sha=_sha(params))


def c4_cond():
    """The "fp64_perturbed" run up to 50 sweeps and the "fp32" run up to the
    workload's 500, at the c4 sample points."""
    w = mi.WORKLOADS["C4"]
    ux, uy = w["units"]
    field = mi.workload_field("C4")
    params = mi.xavier_params(w["width"], seed=0)
    sj, si = _c4_samples()
    out = {"field_sha": _sha(field), "params_sha": _sha(params)}
    t0 = time.time()
    for name, solver, dt in _runs(params, w["width"])[1:]:
        ks = [k for k in TRAJ_K if k <= (50 if name == "fp64_perturbed" else w["sweeps"])]
        out["K" if name == "fp64_perturbed" else "K_fp32"] = np.array(ks, dtype=np.int32)
        u = torch.from_numpy(field).to(dt)
        rows = []
        for k in range(1, ks[-1] + 1):
            u = sw.sweep(u, ux, uy, solver)
            if k in ks:
                rows.append(u.to(torch.float64).numpy()[sj, si].copy())
                print(f"c4_cond: {name} sweep {k} ({time.time() - t0:.0f} s)", flush=True)
        out[name] = np.stack(rows)
    np.savez_compressed(os.path.join(HERE, "c4_cond.npz"), **out)


def _c5_picks(sizes):
    places = [(2 * int(ux) - 1) * (2 * int(uy) - 1) for ux, uy in sizes]
    order = np.argsort(places, kind="stable")
    return [int(order[0]), int(order[len(order) // 2]), int(order[-1])]


def c5_k20():
    w = mi.WORKLOADS["C5"]
    t0 = time.time()
    sizes, fields = mi.batched_domains(w["n_domains"], 4, 48, w["length"], w["seed"])
    print(f"c5_k20: inputs in {time.time() - t0:.0f} s", flush=True)
    params = mi.xavier_params(w["width"], seed=0)
    picks = _c5_picks(sizes)
    ks = [k for k in TRAJ_K if k <= w["sweeps"]]
    out = {"picks": np.array(picks, dtype=np.int32), "sizes": sizes.astype(np.int32),
           "K": np.array(ks, dtype=np.int32), "params_sha": _sha(params)}
    rng = np.random.default_rng(556)
    runs = _runs(params, w["width"])
    for n, d in enumerate(picks):
        ux, uy = (int(v) for v in sizes[d])
        f = fields[d]
        mask = sw.skeleton_mask(*f.shape).numpy()
        sj, si = np.nonzero(mask)
        pick = rng.choice(sj.size, min(4096, sj.size), replace=False)
        sj, si = sj[pick], si[pick]
        aj = rng.integers(1, f.shape[0] - 1, 256)
        ai = rng.integers(1, f.shape[1] - 1, 256)
        out[f"skel_j{n}"], out[f"skel_i{n}"] = sj.astype(np.int32), si.astype(np.int32)
        out[f"sample_j{n}"], out[f"sample_i{n}"] = aj.astype(np.int32), ai.astype(np.int32)
        out[f"field_sha{n}"] = _sha(f)
        for name, solver, dt in runs:
            u = torch.from_numpy(f).to(dt)
            rows = []
            for k in range(1, w["sweeps"] + 1):
                u = sw.sweep(u, ux, uy, solver)
                if k in ks:
                    rows.append(u.to(torch.float64).numpy()[sj, si].copy())
            out[f"skel_{name}_{n}"] = np.stack(rows)
            pts = list(zip(aj.tolist(), ai.tolist()))
            out[f"u_out_{name}_{n}"] = sw.assemble_at(u, ux, uy, solver, pts).to(
                torch.float64).numpy()
            print(f"c5_k20: domain {d} ({ux}x{uy}) {name} done at {time.time() - t0:.0f} s",
                  flush=True)
    np.savez_compressed(os.path.join(HERE, "c5_k20.npz"), **out)


def c5_adjoint():
    from oracle import adjoint
    w = mi.WORKLOADS["C5"]
    sizes, fields = mi.batched_domains(w["n_domains"], 4, 48, w["length"], w["seed"])
    d = _c5_picks(sizes)[0]
    ux, uy = (int(v) for v in sizes[d])
    f = fields[d]
    params = mi.xavier_params(w["width"], seed=0)
    solver = sw.sdnet_solver(torch.from_numpy(params.astype(np.float64)), w["width"])
    u0 = torch.from_numpy(f.astype(np.float64))
    t0 = time.time()
    J, g = adjoint.solve_adjoint(u0, ux, uy, solver, w["sweeps"])
    seed = np.random.default_rng(77).standard_normal(f.shape).astype(np.float32)
    Js, gs = adjoint.solve_adjoint(u0, ux, uy, solver, w["sweeps"],
                                   uout_bar=torch.from_numpy(seed.astype(np.float64)))
    np.savez_compressed(os.path.join(HERE, "c5_adjoint.npz"), domain=np.int32(d),
                        units=np.array([ux, uy], dtype=np.int32), J=J, u0_bar=g.numpy(),
                        seed=seed, J_seed=Js, u0_bar_seed=gs.numpy(), field_sha=_sha(f),
                        params_sha=_sha(params))
    print(f"c5_adjoint: domain {d} ({ux}x{uy}) done in {time.time() - t0:.0f} s", flush=True)


def mfp_global():
    from oracle import fd
    t0 = time.time()
    f4 = mi.gp_field(4, 4, 1.0, seed=31)
    u4 = fd.global_solve(f4)
    f64 = mi.gp_field(64, 64, 2.0, seed=41)
    u64 = fd.global_solve(f64)
    rng = np.random.default_rng(557)
    jj = rng.integers(1, f64.shape[0] - 1, 65536)
    ii = rng.integers(1, f64.shape[1] - 1, 65536)
    np.savez_compressed(os.path.join(HERE, "mfp_global.npz"), u4=u4, field4_sha=_sha(f4),
                        sample_j=jj.astype(np.int32), sample_i=ii.astype(np.int32), u64_sample=u64[jj, ii],
                        field64_sha=_sha(f64))
    print(f"mfp_global: done in {time.time() - t0:.0f} s", flush=True)


JOBS = {"mfp_global": mfp_global, "c2": c2, "c3": c3, "c4": c4, "c4_one": c4_one, "c5_one": c5_one, "c2_traj": c2_traj,
        "c4_traj": c4_traj, "c4_cond": c4_cond, "c5_k20": c5_k20, "c5_adjoint": c5_adjoint}

if __name__ == "__main__":
    torch.set_num_threads(int(os.environ.get("GOLDEN_THREADS", os.cpu_count() or 1)))
    for name in (sys.argv[1:] or list(JOBS)):
        JOBS[name]()
