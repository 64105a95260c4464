"""GPU parity of the HIP sweep against the float64 oracle, through the C ABI.

Tolerance: float32 results match the oracle to relative L2 <= 1e-5 over the
points the run writes (interior skeleton points for CROSS sweeps, every
interior point for INTERIOR sweeps and for the assembly). BF16 results
(bf16 projection and hidden GEMMs, float32 everywhere else) are held to
<= 2e-2. FP16 results (the same GEMMs on IEEE half operands, whose unit
roundoff 2^-11 = 4.9e-4 is 8x finer) are held to <= 5e-3, ten unit
roundoffs (measured 5.7e-4 to 1.0e-3).
"""
import os

import numpy as np
import pytest
import torch

import mf_inputs as mi
from oracle import fd, sweep as sw
from paper_2308_14258_amd import MF_BF16, MF_CROSS, MF_FP16, MF_FP32, MF_INTERIOR, MF_TILE_STREAM, Context
from paper_2308_14258_amd import mf_solve, mf_sweep, mf_sweep_operator

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host64(t):
    return t.detach().cpu().double()


def rel_l2(got, want, mask=None):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    if mask is not None:
        got, want = got[mask], want[mask]
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


def skel_interior_mask(ny, nx):
    m = sw.skeleton_mask(ny, nx).numpy()
    m[0, :] = m[-1, :] = False
    m[:, 0] = m[:, -1] = False
    return m


def interior_mask(ny, nx):
    m = np.zeros((ny, nx), dtype=bool)
    m[1:-1, 1:-1] = True
    return m


def oracle_solver(params32, width):
    return sw.sdnet_solver(torch.from_numpy(params32.astype(np.float64)), width)


# ---------------------------------------------------------------------------
# check mode: exact 5-point subdomain solver
# ---------------------------------------------------------------------------

def test_operator_sweep_reproduces_x2_minus_y2(ctx):
    print("case: operator sweep, 2x2 units, x^2-y^2, 50 sweeps", flush=True)
    f = mi.x2_minus_y2_field(2, 2)
    exact = mi.full_analytic(2, 2, lambda x, y: x * x - y * y)
    Hc = dev(fd.subdomain_operator("cross").numpy())
    Hi = dev(fd.subdomain_operator("interior").numpy())
    u = dev(f)
    for _ in range(50):
        mf_sweep_operator(ctx, Hc, u, (2, 2), -1, MF_CROSS)
    u_out = torch.empty_like(u)
    mf_sweep_operator(ctx, Hi, u, (2, 2), 4, MF_INTERIOR, u_out=u_out)
    torch.cuda.synchronize()
    m = skel_interior_mask(65, 65)
    # float32 fixed point: a few ulps of |u| <= 4 per 128-term dot product
    assert np.abs(u.cpu().numpy() - exact)[m].max() <= 2e-5
    assert rel_l2(u.cpu().numpy(), exact, m) <= 2e-6
    assert rel_l2(u_out.cpu().numpy(), exact, interior_mask(65, 65)) <= 2e-6


def test_operator_sweep_matches_oracle_trajectory(ctx):
    print("case: operator sweep vs oracle, 3x2 units, GP data", flush=True)
    f = mi.gp_field(3, 2, 0.7, seed=4)
    Hc = dev(fd.subdomain_operator("cross").numpy())
    u = dev(f)
    uo = torch.from_numpy(f.astype(np.float64))
    solver = fd.operator_solver()
    m = skel_interior_mask(*f.shape)
    for k in range(5):
        mf_sweep_operator(ctx, Hc, u, (3, 2), -1, MF_CROSS)
        uo = sw.sweep(uo, 3, 2, solver)
        assert rel_l2(u.cpu().numpy(), uo.numpy(), m) <= 1e-6, k


# ---------------------------------------------------------------------------
# SDNet sweeps, float32
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("units", [(2, 2), (3, 2), (1, 1), (1, 3), (5, 4)])
@pytest.mark.parametrize("width", [128, 256])
@pytest.mark.parametrize("targets", [MF_CROSS, MF_INTERIOR])
def test_one_sweep_matches_oracle(ctx, units, width, targets):
    print(f"case: one sweep units={units} width={width} targets={targets}", flush=True)
    ux, uy = units
    params = mi.random_params(width, seed=3)
    f = mi.random_interior_field(ux, uy, seed=5)
    u = dev(f)
    mf_sweep(ctx, dev(params), u, units, -1, targets, MF_FP32)
    kind = "cross" if targets == MF_CROSS else "interior"
    want = sw.sweep(torch.from_numpy(f.astype(np.float64)), ux, uy, oracle_solver(params, width), kind)
    got = u.cpu().numpy()
    ny, nx = f.shape
    m = skel_interior_mask(ny, nx) if targets == MF_CROSS else interior_mask(ny, nx)
    assert rel_l2(got, want.numpy(), m) <= 1e-5
    # points outside the targets are never written (ring included)
    np.testing.assert_array_equal(got[~m], f[~m])


@pytest.mark.parametrize("colour", [0, 1, 2, 3])
def test_single_colour_phase(ctx, colour):
    print(f"case: colour phase {colour}, 3x3 units", flush=True)
    params = mi.random_params(128, seed=7)
    f = mi.random_interior_field(3, 3, seed=colour)
    u = dev(f)
    mf_sweep(ctx, dev(params), u, (3, 3), colour, MF_CROSS, MF_FP32)
    want = sw.colour_phase(torch.from_numpy(f.astype(np.float64)), 3, 3, colour,
                           oracle_solver(params, 128))
    got = u.cpu().numpy()
    changed = want.numpy() != f.astype(np.float64)
    assert changed.sum() > 0
    assert rel_l2(got, want.numpy(), changed) <= 1e-5
    np.testing.assert_array_equal(got[~changed], f[~changed])


def test_solve_c1_full(ctx):
    """2x2 units, width 128, x^2 - y^2 ring, Xavier seed 0, 50 sweeps + assembly."""
    print("case: mf_solve C1 (2x2, d=128, 50 sweeps)", flush=True)
    w = mi.WORKLOADS["C1"]
    params = mi.xavier_params(w["width"], 0)
    f = mi.workload_field("C1")
    u = dev(f)
    u_out = torch.empty_like(u)
    done, last = mf_solve(ctx, dev(params), u, (2, 2), w["sweeps"], u_out=u_out, report=True)
    assert done == 50 and np.isnan(last)
    uK, uo, _, _ = sw.solve(torch.from_numpy(f.astype(np.float64)), 2, 2,
                            oracle_solver(params, w["width"]), w["sweeps"])
    assert rel_l2(u.cpu().numpy(), uK.numpy(), skel_interior_mask(65, 65)) <= 1e-5
    assert rel_l2(u_out.cpu().numpy(), uo.numpy(), interior_mask(65, 65)) <= 1e-5
    ring = ~interior_mask(65, 65)
    np.testing.assert_array_equal(u_out.cpu().numpy()[ring], f[ring])


def test_solve_c2_full_golden(ctx):
    """16x16 units, width 256, GP data, 200 sweeps: against stored oracle values."""
    print("case: mf_solve C2 (16x16, d=256, 200 sweeps) vs golden", flush=True)
    g = np.load(os.path.join(HERE, "golden", "c2_fp32.npz"))
    w = mi.WORKLOADS["C2"]
    params = mi.xavier_params(w["width"], 0)
    f = mi.workload_field("C2")
    u = dev(f)
    mf_solve(ctx, dev(params), u, (16, 16), 20)
    torch.cuda.synchronize()
    mask = sw.skeleton_mask(*f.shape).numpy()
    err20 = rel_l2(u.cpu().numpy()[mask], g["skel20"])
    u_out = torch.empty_like(u)
    mf_solve(ctx, dev(params), u, (16, 16), w["sweeps"] - 20, u_out=u_out)
    torch.cuda.synchronize()
    err200 = rel_l2(u.cpu().numpy()[mask], g["skel200"])
    uo = u_out.cpu().numpy()[g["sample_j"], g["sample_i"]]
    err_out = rel_l2(uo, g["u_out_sample"])
    print(f"C2 fp32 rel L2 vs oracle: skeleton@20 {err20:.3e} skeleton@200 {err200:.3e} "
          f"u_out {err_out:.3e}", flush=True)
    assert err200 <= 1e-5 and err_out <= 1e-5
    assert err20 <= 1e-4   # transient amplification of a random network (reported)


def test_solve_delta_stops(ctx):
    print("case: mf_solve delta early stop", flush=True)
    params = mi.xavier_params(128, 0)
    f = mi.workload_field("C1")
    u = dev(f)
    done, last = mf_solve(ctx, dev(params), u, (2, 2), 40, eps=0.01, check_every=2, report=True)
    traj = []
    sw.solve(torch.from_numpy(f.astype(np.float64)), 2, 2, oracle_solver(params, 128), 40,
             trajectory=traj, assemble_out=False)
    skel = [sw.skeleton_values(t) for t in traj]
    want_k = None
    for k in range(2, 41, 2):
        d = sw.delta(skel[k - 1], skel[k - 2])
        if d < 0.01:
            want_k, want_d = k, d
            break
    assert want_k is not None
    assert done == want_k
    # delta is a difference of float32 fields of norm ~1: absolute error ~1e-6
    assert abs(last - want_d) <= 2e-5


def test_resume_and_determinism(ctx):
    print("case: resume and determinism", flush=True)
    params = dev(mi.random_params(256, seed=2))
    f = mi.gp_field(4, 3, 1.0, seed=3)
    a = dev(f)
    mf_solve(ctx, params, a, (4, 3), 9)
    b = dev(f)
    mf_solve(ctx, params, b, (4, 3), 4)
    mf_solve(ctx, params, b, (4, 3), 5)
    c = dev(f)
    mf_solve(ctx, params, c, (4, 3), 9)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(a, c)


def test_padded_pitch(ctx):
    print("case: padded row pitch", flush=True)
    params = mi.random_params(128, seed=4)
    f = mi.random_interior_field(2, 3, seed=8)
    big = torch.full((f.shape[0], f.shape[1] + 37), 7.0, dtype=torch.float32, device="cuda")
    u = big[:, : f.shape[1]]
    u.copy_(dev(f))
    mf_sweep(ctx, dev(params), u, (2, 3), -1, MF_CROSS, MF_FP32)
    want = sw.sweep(torch.from_numpy(f.astype(np.float64)), 2, 3, oracle_solver(params, 128))
    assert rel_l2(u.cpu().numpy(), want.numpy(), skel_interior_mask(*f.shape)) <= 1e-5
    assert torch.all(big[:, f.shape[1]:] == 7.0)


def test_zero_sweeps_is_assembly_only(ctx):
    print("case: zero sweeps", flush=True)
    params = mi.random_params(128, seed=6)
    f = mi.random_interior_field(2, 2, seed=9)
    u = dev(f)
    u_out = torch.empty_like(u)
    mf_solve(ctx, dev(params), u, (2, 2), 0, u_out=u_out)
    want = sw.assemble(torch.from_numpy(f.astype(np.float64)), 2, 2, oracle_solver(params, 128))
    np.testing.assert_array_equal(u.cpu().numpy(), f)
    assert rel_l2(u_out.cpu().numpy(), want.numpy(), interior_mask(65, 65)) <= 1e-5


# ---------------------------------------------------------------------------
# BF16 hidden GEMMs
# ---------------------------------------------------------------------------

def test_bf16_solve_c1_error(ctx):
    print("case: mf_solve C1 bf16", flush=True)
    w = mi.WORKLOADS["C1"]
    params = mi.xavier_params(w["width"], 0)
    f = mi.workload_field("C1")
    u = dev(f)
    u_out = torch.empty_like(u)
    mf_solve(ctx, dev(params), u, (2, 2), w["sweeps"], prec=MF_BF16, u_out=u_out)
    uK, uo, _, _ = sw.solve(torch.from_numpy(f.astype(np.float64)), 2, 2,
                            oracle_solver(params, w["width"]), w["sweeps"])
    e_skel = rel_l2(u.cpu().numpy(), uK.numpy(), skel_interior_mask(65, 65))
    e_out = rel_l2(u_out.cpu().numpy(), uo.numpy(), interior_mask(65, 65))
    print(f"C1 bf16 rel L2 vs oracle: skeleton {e_skel:.3e} u_out {e_out:.3e}", flush=True)
    assert e_skel <= 2e-2 and e_out <= 2e-2


def test_bf16_solve_c2_error(ctx):
    print("case: mf_solve C2 bf16 vs golden", flush=True)
    g = np.load(os.path.join(HERE, "golden", "c2_fp32.npz"))
    w = mi.WORKLOADS["C2"]
    params = mi.xavier_params(w["width"], 0)
    f = mi.workload_field("C2")
    u = dev(f)
    u_out = torch.empty_like(u)
    mf_solve(ctx, dev(params), u, (16, 16), w["sweeps"], prec=MF_BF16, u_out=u_out)
    torch.cuda.synchronize()
    mask = sw.skeleton_mask(*f.shape).numpy()
    e_skel = rel_l2(u.cpu().numpy()[mask], g["skel200"])
    e_out = rel_l2(u_out.cpu().numpy()[g["sample_j"], g["sample_i"]], g["u_out_sample"])
    print(f"C2 bf16 rel L2 vs oracle: skeleton {e_skel:.3e} u_out {e_out:.3e}", flush=True)
    assert e_skel <= 2e-2 and e_out <= 2e-2


@pytest.mark.parametrize("prec,tol", [(MF_FP32, 1e-5), (MF_BF16, 2e-2), (MF_FP16, 5e-3)])
def test_solve_c4_full_size_golden(ctx, prec, tol):
    """64 x 64 units (2049^2 grid, 16,129 placements), width 256: the
    benchmark's BF16-vs-FP32 workload at full size, in the launch
    configuration the benchmark uses (autotuned tile shape, graphs), against
    oracle values at 32768 sampled skeleton points and 2048 assembly points:
    after one sweep (the sweep map itself) and after 500 sweeps (the end
    state). After 20 sweeps the untrained network's iteration is in a
    transient that amplifies rounding at every phase: the same algorithm
    evaluated in float32 on the CPU is 6.8e-3 away from float64 there (0.6
    at 30 sweeps, c4_cond.npz). Float32 is held to 10x that spread; BF16 is
    reported."""
    print(f"case: mf_solve C4 (64x64, d=256) prec {prec} vs golden", flush=True)
    from paper_2308_14258_amd import mf_autotune
    g = np.load(os.path.join(HERE, "golden", "c4_fp64.npz"))
    g1 = np.load(os.path.join(HERE, "golden", "c4_one_sweep.npz"))
    w = mi.WORKLOADS["C4"]
    params = mi.xavier_params(w["width"], 0)
    f = mi.workload_field("C4")
    p = dev(params)
    sj, si = g["skel_j"], g["skel_i"]
    aj, ai = g["sample_j"], g["sample_i"]
    mf_autotune(ctx, p, dev(f), (64, 64), MF_CROSS, prec, trials=1)
    u = dev(f)
    u_out = torch.empty_like(u)
    mf_solve(ctx, p, u, (64, 64), 1, prec=prec, u_out=u_out)
    torch.cuda.synchronize()
    err1 = rel_l2(u.cpu().numpy()[sj, si], g1["skel1"])
    err1_out = rel_l2(u_out.cpu().numpy()[aj, ai], g1["u_out_sample"])
    mf_solve(ctx, p, u, (64, 64), 19, prec=prec)
    torch.cuda.synchronize()
    err20 = rel_l2(u.cpu().numpy()[sj, si], g["skel20"])
    mf_solve(ctx, p, u, (64, 64), w["sweeps"] - 20, prec=prec, u_out=u_out)
    torch.cuda.synchronize()
    err500 = rel_l2(u.cpu().numpy()[sj, si], g["skel500"])
    err_out = rel_l2(u_out.cpu().numpy()[aj, ai], g["u_out_sample"])
    print(f"C4 prec {prec} rel L2 vs oracle: sweep 1 skeleton {err1:.3e} u_out {err1_out:.3e}; "
          f"skeleton@20 {err20:.3e} (reported); skeleton@500 {err500:.3e} u_out {err_out:.3e}",
          flush=True)
    assert err1 <= tol and err1_out <= tol
    assert err500 <= tol and err_out <= tol
    if prec == MF_FP32:
        c = np.load(os.path.join(HERE, "golden", "c4_cond.npz"))
        e32 = rel_l2(c["fp32"][list(c["K_fp32"]).index(20)], g["skel20"])
        print(f"C4 sweep 20: float32 oracle spread {e32:.3e}, bound {max(1e-5, 10 * e32):.3e}", flush=True)
        assert err20 <= max(1e-5, 10.0 * e32)


@pytest.mark.parametrize("prec", [MF_FP32, MF_BF16, MF_FP16])
def test_solve_c4_trajectory(ctx, prec):
    """64 x 64 units, width 256, 500 sweeps: the skeleton at 32768 sampled
    points after each stored sweep count against the float64 oracle. Float32
    is held to max(1e-5, 10 x the float32 oracle's spread at that count);
    BF16 to 2e-2 and FP16 to 5e-3 where that spread is <= 1e-6 (outside
    the transient) and reported elsewhere; the trajectory maxima are printed."""
    print(f"case: C4 trajectory vs golden prec {prec}", flush=True)
    t = np.load(os.path.join(HERE, "golden", "c4_traj.npz"))
    c = np.load(os.path.join(HERE, "golden", "c4_cond.npz"))
    g = np.load(os.path.join(HERE, "golden", "c4_fp64.npz"))
    w = mi.WORKLOADS["C4"]
    assert str(t["field_sha"]) == str(c["field_sha"])
    p = dev(mi.xavier_params(w["width"], 0))
    u = dev(mi.workload_field("C4"))
    sj, si = g["skel_j"], g["skel_i"]
    kf = list(c["K_fp32"])
    done = 0
    worst = 0.0
    for i, k in enumerate(t["K"]):
        mf_solve(ctx, p, u, (64, 64), int(k) - done, prec=prec)
        done = int(k)
        torch.cuda.synchronize()
        e = rel_l2(u.cpu().numpy()[sj, si], t["fp64"][i])
        e32 = rel_l2(c["fp32"][kf.index(k)], t["fp64"][i])
        worst = max(worst, e)
        print(f"C4 prec {prec} K={int(k)}: rel L2 skeleton {e:.3e} (float32 oracle spread {e32:.3e})", flush=True)
        if prec == MF_FP32:
            assert e <= max(1e-5, 10.0 * e32), (int(k), e, e32)
        elif e32 <= 1e-6:
            assert e <= (2e-2 if prec == MF_BF16 else 5e-3), (int(k), e, e32)
    print(f"C4 prec {prec} trajectory max {worst:.3e}", flush=True)


def test_solve_c2_trajectory(ctx):
    """16 x 16 units, width 256, 200 sweeps: the skeleton at 8192 sampled
    points after each stored sweep count against the float64 oracle, held to
    max(1e-5, 10 x the float32 oracle's spread at that count); reports the
    trajectory maximum."""
    print("case: C2 trajectory vs golden", flush=True)
    t = np.load(os.path.join(HERE, "golden", "c2_traj.npz"))
    w = mi.WORKLOADS["C2"]
    p = dev(mi.xavier_params(w["width"], 0))
    u = dev(mi.workload_field("C2"))
    done = 0
    worst = 0.0
    for i, k in enumerate(t["K"]):
        mf_solve(ctx, p, u, (16, 16), int(k) - done)
        done = int(k)
        torch.cuda.synchronize()
        e = rel_l2(u.cpu().numpy()[t["skel_j"], t["skel_i"]], t["fp64"][i])
        e32 = rel_l2(t["fp32"][i], t["fp64"][i])
        worst = max(worst, e)
        print(f"C2 K={int(k)}: rel L2 skeleton {e:.3e} (float32 oracle spread {e32:.3e})", flush=True)
        assert e <= max(1e-5, 10.0 * e32), (int(k), e, e32)
    print(f"C2 trajectory max {worst:.3e}", flush=True)


def test_graph_replay_equals_direct_launches(ctx):
    print("case: graph replay vs direct launches", flush=True)
    params = dev(mi.random_params(256, seed=12))
    f = mi.gp_field(3, 4, 1.0, seed=6)
    a = dev(f)
    b = dev(f)
    ctx.graphs(False)
    mf_solve(ctx, params, a, (3, 4), 37)
    ctx.graphs(True)
    mf_solve(ctx, params, b, (3, 4), 37)
    mf_solve(ctx, params, b, (3, 4), 0)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("prec", [MF_FP32, MF_BF16])
def test_graph_replay_sees_new_parameter_values(ctx, prec):
    """A cached graph holds buffer addresses, not values: overwriting the
    parameters in place between two solves on the same buffers must give
    the result of the new parameters (the network is prepared outside the
    graph on every call)."""
    print(f"case: graph replay after an in-place parameter update prec={prec}", flush=True)
    pa, pb = mi.random_params(256, seed=41), mi.random_params(256, seed=42)
    f = mi.gp_field(4, 3, 1.0, seed=8)
    params = dev(pa)
    u = dev(f)
    ctx.graphs(True)
    mf_solve(ctx, params, u, (4, 3), 32, prec=prec)       # captures and replays with pa
    params.copy_(dev(pb))
    u.copy_(dev(f))
    mf_solve(ctx, params, u, (4, 3), 32, prec=prec)       # same addresses, new values
    ctx.graphs(False)
    v = dev(f)
    mf_solve(ctx, dev(pb), v, (4, 3), 32, prec=prec)
    ctx.graphs(True)
    torch.cuda.synchronize()
    assert torch.equal(u, v)


@pytest.mark.parametrize("prec,rows", [(MF_FP32, 32), (MF_FP32, 64), (MF_FP32, 64 | (1 << 17)), (MF_BF16, 64),
                                       (MF_BF16, 128), (MF_BF16, 256), (MF_BF16, 128 | (1 << 16)),
                                       (MF_BF16, 256 | (1 << 16)), (MF_BF16, 256 | (1 << 18)),
                                       (MF_BF16, 128 | (1 << 18)), (MF_FP16, 64), (MF_FP16, 128), (MF_FP16, 256),
                                       (MF_FP16, 256 | (1 << 18)), (MF_FP16, 128 | (1 << 18))])
@pytest.mark.parametrize("targets", [MF_CROSS, MF_INTERIOR])
def test_every_tile_height(ctx, prec, rows, targets):
    print(f"case: tile rows {rows} prec {prec} targets {targets}", flush=True)
    params = mi.random_params(256, seed=31)
    f = mi.random_interior_field(6, 5, seed=4)
    u = dev(f)
    ctx.tile_rows(prec, rows)
    try:
        mf_sweep(ctx, dev(params), u, (6, 5), -1, targets, prec)
        torch.cuda.synchronize()
    finally:
        ctx.tile_rows(prec, 0)
    kind = "cross" if targets == MF_CROSS else "interior"
    want = sw.sweep(torch.from_numpy(f.astype(np.float64)), 6, 5, oracle_solver(params, 256), kind)
    ny, nx = f.shape
    m = skel_interior_mask(ny, nx) if targets == MF_CROSS else interior_mask(ny, nx)
    err = rel_l2(u.cpu().numpy(), want.numpy(), m)
    print(f"tile rows {rows} prec {prec} targets {targets}: rel L2 {err:.3e}", flush=True)
    assert err <= {MF_FP32: 1e-5, MF_BF16: 2e-2, MF_FP16: 5e-3}[prec]
    np.testing.assert_array_equal(u.cpu().numpy()[~m], f[~m])


def test_autotune_picks_a_candidate_and_is_used(ctx):
    print("case: autotune", flush=True)
    from paper_2308_14258_amd import mf_autotune
    params = dev(mi.xavier_params(256, 0))
    f = mi.gp_field(8, 8, 1.0, seed=2)
    scratch = dev(f)
    best = mf_autotune(ctx, params, scratch, (8, 8), MF_CROSS, MF_BF16, trials=2)
    assert best in (64, 128, 256, 128 | (1 << 16), 256 | (1 << 16), 256 | (1 << 18), 128 | (1 << 18))
    a = dev(f)
    mf_solve(ctx, params, a, (8, 8), 5, prec=MF_BF16)
    ctx.tile_rows(MF_BF16, best)
    b = dev(f)
    mf_solve(ctx, params, b, (8, 8), 5, prec=MF_BF16)
    ctx.tile_rows(MF_BF16, 0)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("units,width,targets", [((2, 2), 128, MF_CROSS), ((3, 2), 256, MF_CROSS),
                                                 ((2, 3), 128, MF_INTERIOR), ((1, 1), 256, MF_INTERIOR)])
def test_additive_sweep_matches_oracle(ctx, units, width, targets):
    print(f"case: additive sweep units={units} width={width} targets={targets}", flush=True)
    from paper_2308_14258_amd import MF_ADDITIVE
    ux, uy = units
    params = mi.random_params(width, seed=17)
    f = mi.random_interior_field(ux, uy, seed=3)
    u = dev(f)
    mf_sweep(ctx, dev(params), u, units, -1, targets, MF_FP32, mode=MF_ADDITIVE)
    kind = "cross" if targets == MF_CROSS else "interior"
    want = sw.sweep_additive(torch.from_numpy(f.astype(np.float64)), ux, uy,
                             oracle_solver(params, width), kind)
    ny, nx = f.shape
    m = skel_interior_mask(ny, nx) if targets == MF_CROSS else interior_mask(ny, nx)
    assert rel_l2(u.cpu().numpy(), want.numpy(), m) <= 1e-5
    np.testing.assert_array_equal(u.cpu().numpy()[~m], f[~m])


def test_additive_solve_c1(ctx):
    print("case: additive solve C1", flush=True)
    from paper_2308_14258_amd import MF_ADDITIVE
    params = mi.xavier_params(128, 0)
    f = mi.workload_field("C1")
    u = dev(f)
    u_out = torch.empty_like(u)
    mf_solve(ctx, dev(params), u, (2, 2), 20, u_out=u_out, mode=MF_ADDITIVE)
    uK, uo, _, _ = sw.solve(torch.from_numpy(f.astype(np.float64)), 2, 2, oracle_solver(params, 128), 20,
                            mode="additive")
    assert rel_l2(u.cpu().numpy(), uK.numpy(), skel_interior_mask(65, 65)) <= 1e-5
    assert rel_l2(u_out.cpu().numpy(), uo.numpy(), interior_mask(65, 65)) <= 1e-5


@pytest.mark.parametrize("prec,tol", [(MF_BF16, 2e-2), (MF_FP16, 5e-3)])
@pytest.mark.parametrize("width", [128, 256])
def test_rowsplit_tile_solve_and_assembly(ctx, width, prec, tol):
    """The row-split 16-bit tile (each wave owns 32 rows, weights streamed
    through LDS; 8 waves or 4) in a full solve: sweeps and the overlap-averaged
    assembly against the oracle, and bit for bit against the column-split tile
    of the same precision."""
    print(f"case: row-split tile prec {prec}, width {width}, 5x4 units, 3 sweeps + assembly", flush=True)
    ux, uy = 5, 4
    params = mi.xavier_params(width, 2)
    f = mi.gp_field(ux, uy, 1.0, seed=6)
    outs = {}
    for name, rows in (("rowsplit", 256 | (1 << 18)), ("rowsplit128", 128 | (1 << 18)), ("default", 0)):
        u = dev(f)
        u_out = torch.empty_like(u)
        ctx.tile_rows(prec, rows)
        try:
            mf_solve(ctx, dev(params), u, (ux, uy), 3, prec=prec, u_out=u_out)
            torch.cuda.synchronize()
        finally:
            ctx.tile_rows(prec, 0)
        outs[name] = (u.cpu().numpy(), u_out.cpu().numpy())
    _, want, _, _ = sw.solve(torch.from_numpy(f.astype(np.float64)), ux, uy, oracle_solver(params, width), 3)
    ny, nx = f.shape
    e_or = rel_l2(outs["rowsplit"][1], want.numpy(), interior_mask(ny, nx))
    e_cs = rel_l2(outs["rowsplit"][1], outs["default"][1], interior_mask(ny, nx))
    print(f"row-split prec {prec} width {width}: u_out rel L2 vs oracle {e_or:.3e}, vs column-split {e_cs:.3e}",
          flush=True)
    assert e_or <= tol
    # same k order in every MFMA, same tanh and output sums: identical results
    for name in ("rowsplit128", "default"):
        np.testing.assert_array_equal(outs["rowsplit"][0], outs[name][0])
        np.testing.assert_array_equal(outs["rowsplit"][1], outs[name][1])


@pytest.mark.parametrize("width", [128, 256])
def test_fp32_tile_forms_agree_bit_for_bit(ctx, width):
    """The fp32 tiles with register-resident weights (64 rows; each weight
    register is reloaded with the next layer's operand right after its last
    MFMA) and with weights streamed from L2 (32 and 64 rows) run the same
    arithmetic per row: same k order in every MFMA, same tanh and output sums.
    Sweeps and assembly must agree bit for bit, and with the oracle to 1e-5."""
    print(f"case: fp32 tile forms, width {width}, 5x4 units, 3 sweeps + assembly", flush=True)
    ux, uy = 5, 4
    params = mi.xavier_params(width, 4)
    f = mi.gp_field(ux, uy, 1.0, seed=8)
    outs = {}
    for name, rows in (("registers", 64), ("stream64", 64 | MF_TILE_STREAM), ("stream32", 32)):
        u = dev(f)
        u_out = torch.empty_like(u)
        ctx.tile_rows(MF_FP32, rows)
        try:
            mf_solve(ctx, dev(params), u, (ux, uy), 3, u_out=u_out)
            torch.cuda.synchronize()
        finally:
            ctx.tile_rows(MF_FP32, 0)
        outs[name] = (u.cpu().numpy(), u_out.cpu().numpy())
    _, want, _, _ = sw.solve(torch.from_numpy(f.astype(np.float64)), ux, uy, oracle_solver(params, width), 3)
    ny, nx = f.shape
    err = rel_l2(outs["registers"][1], want.numpy(), interior_mask(ny, nx))
    print(f"fp32 register-weight tile width {width}: u_out rel L2 vs oracle {err:.3e}", flush=True)
    assert err <= 1e-5
    for name in ("stream64", "stream32"):
        np.testing.assert_array_equal(outs["registers"][0], outs[name][0], err_msg=name)
        np.testing.assert_array_equal(outs["registers"][1], outs[name][1], err_msg=name)
