"""Batched independent domains (one persistent launch per colour) through
the C ABI: the batch must equal the same domains solved one by one, and the
float64 oracle."""
import numpy as np
import pytest
import torch

import mf_inputs as mi
from oracle import sweep as sw
from paper_2308_14258_amd import MF_BF16, MF_CROSS, MF_FP16, MF_FP32, MF_INTERIOR, Batch, Context
from paper_2308_14258_amd import mf_solve, mf_sweep

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


def _fields(seed=7, n=7, lo=1, hi=6):
    sizes, fields = mi.batched_domains(n, lo, hi, 1.0, seed)
    return sizes, fields


@pytest.mark.parametrize("prec", [MF_FP32, MF_BF16, MF_FP16])
@pytest.mark.parametrize("targets", [MF_CROSS, MF_INTERIOR])
def test_batch_equals_one_by_one(ctx, prec, targets):
    print(f"case: batch vs single prec={prec} targets={targets}", flush=True)
    sizes, fields = _fields()
    params = torch.from_numpy(mi.random_params(256, seed=5)).cuda()
    batch = Batch(fields)
    out = torch.empty_like(batch.buf)
    mf_solve(ctx, params, batch, None, 6, targets=targets, prec=prec, u_out=out)
    for i, f in enumerate(fields):
        ux, uy = sizes[i]
        u = torch.from_numpy(f).cuda()
        uo = torch.empty_like(u)
        # the single domain may get another tile height than the batch; results
        # do not depend on it
        mf_solve(ctx, params, u, (int(ux), int(uy)), 6, targets=targets, prec=prec, u_out=uo)
        got = batch.field(i)
        torch.cuda.synchronize()
        assert torch.equal(got, u), i
        assert torch.equal(batch.field(i, out), uo), i


def test_batch_matches_oracle(ctx):
    print("case: batch vs oracle", flush=True)
    sizes, fields = _fields(seed=3, n=5, lo=1, hi=4)
    params_np = mi.random_params(128, seed=9)
    batch = Batch(fields)
    out = torch.empty_like(batch.buf)
    mf_solve(ctx, torch.from_numpy(params_np).cuda(), batch, None, 3, u_out=out)
    solver = sw.sdnet_solver(torch.from_numpy(params_np.astype(np.float64)), 128)
    for i, f in enumerate(fields):
        ux, uy = (int(v) for v in sizes[i])
        uK, uo, _, _ = sw.solve(torch.from_numpy(f.astype(np.float64)), ux, uy, solver, 3)
        got = batch.field(i, out).cpu().numpy().astype(np.float64)[1:-1, 1:-1]
        want = uo.numpy()[1:-1, 1:-1]
        assert np.linalg.norm(got - want) / np.linalg.norm(want) <= 1e-5, i


def test_batch_delta_and_sweep(ctx):
    print("case: batch delta + single sweep", flush=True)
    sizes, fields = _fields(seed=11, n=4, lo=2, hi=3)
    params = torch.from_numpy(mi.xavier_params(128, 0)).cuda()
    a = Batch(fields)
    done, last = mf_solve(ctx, params, a, None, 30, eps=1e-3, check_every=1, report=True)
    assert 1 <= done <= 30 and (last < 1e-3 or done == 30)
    b = Batch(fields)
    for _ in range(done):
        mf_sweep(ctx, params, b)
    torch.cuda.synchronize()
    assert torch.equal(a.buf, b.buf)


def test_batch_additive_equals_one_by_one(ctx):
    print("case: batch additive vs single", flush=True)
    from paper_2308_14258_amd import MF_ADDITIVE
    sizes, fields = _fields(seed=5, n=4, lo=1, hi=4)
    params = torch.from_numpy(mi.random_params(128, seed=8)).cuda()
    batch = Batch(fields)
    mf_solve(ctx, params, batch, None, 5, mode=MF_ADDITIVE)
    for i, f in enumerate(fields):
        ux, uy = (int(v) for v in sizes[i])
        u = torch.from_numpy(f).cuda()
        mf_solve(ctx, params, u, (ux, uy), 5, mode=MF_ADDITIVE)
        torch.cuda.synchronize()
        assert torch.equal(batch.field(i), u), i


@pytest.mark.parametrize("prec,tol", [(MF_FP32, 1e-5), (MF_BF16, 2e-2), (MF_FP16, 5e-3)])
def test_full_batch_one_sweep_sampled_domains(ctx, prec, tol):
    """The 48-domain batch (4..48 units per side, 138,286 placements), width
    256, in the launch configuration the benchmark uses (one persistent
    launch per colour for all domains): one sweep and the assembly, checked
    on its smallest, median and largest domain against float64 oracle values
    at sampled skeleton and assembly points."""
    import os
    print(f"case: 48-domain batch one sweep prec={prec}", flush=True)
    g = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_one_sweep.npz"))
    w = mi.WORKLOADS["C5"]
    sizes, fields = mi.batched_domains(w["n_domains"], 4, 48, w["length"], w["seed"])
    np.testing.assert_array_equal(sizes, g["sizes"])
    params = torch.from_numpy(mi.xavier_params(w["width"], 0)).cuda()
    batch = Batch(fields)
    out = torch.empty_like(batch.buf)
    mf_solve(ctx, params, batch, None, 1, prec=prec, u_out=out)
    torch.cuda.synchronize()
    for n, d in enumerate(g["picks"]):
        u = batch.field(int(d)).cpu().numpy().astype(np.float64)
        uo = batch.field(int(d), out).cpu().numpy().astype(np.float64)
        s_want = g[f"skel1_{n}"]
        s_got = u[g[f"skel_j{n}"], g[f"skel_i{n}"]]
        o_want = g[f"u_out{n}"]
        o_got = uo[g[f"sample_j{n}"], g[f"sample_i{n}"]]
        e_s = np.linalg.norm(s_got - s_want) / np.linalg.norm(s_want)
        e_o = np.linalg.norm(o_got - o_want) / np.linalg.norm(o_want)
        print(f"domain {int(d)} {tuple(int(v) for v in sizes[d])}: rel L2 skeleton {e_s:.3e} u_out {e_o:.3e}", flush=True)
        assert e_s <= tol and e_o <= tol, (int(d), e_s, e_o)


# Float32 results after many sweeps are held to the spread that float32
# rounding alone causes along the same trajectory: the oracle's algorithm
# evaluated in float32 on the CPU (the "fp32" run stored with the float64
# values) differs from float64 by e32(K); the GPU float32 error must stay
# within max(1e-5, COND_FACTOR * e32(K)). BF16 is held to 2e-2 and FP16 to
# 5e-3 where the trajectory is well conditioned (e32 <= 1e-6) and their
# errors are reported elsewhere.
COND_FACTOR = 10.0


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("prec", [MF_FP32, MF_BF16, MF_FP16])
def test_full_batch_k20_sampled_domains(ctx, prec):
    """The 48-domain batch at its stated 20 sweeps, in the benchmark's
    launch configuration: sampled skeleton of the smallest, median and
    largest domain after 1, 5, 10, 15 and 20 sweeps and the assembly after
    20, against the float64 oracle, with the trajectory maximum reported."""
    import os
    print(f"case: 48-domain batch K=20 prec={prec}", flush=True)
    g = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_k20.npz"))
    w = mi.WORKLOADS["C5"]
    sizes, fields = mi.batched_domains(w["n_domains"], 4, 48, w["length"], w["seed"])
    np.testing.assert_array_equal(sizes, g["sizes"])
    params = torch.from_numpy(mi.xavier_params(w["width"], 0)).cuda()
    batch = Batch(fields)
    out = torch.empty_like(batch.buf)
    ks = [int(k) for k in g["K"]]
    assert ks[-1] == w["sweeps"]
    done = 0
    worst = {}
    for i, k in enumerate(ks):
        mf_solve(ctx, params, batch, None, k - done, prec=prec, u_out=out if k == ks[-1] else None)
        done = k
        torch.cuda.synchronize()
        for n, d in enumerate(g["picks"]):
            u = batch.field(int(d)).cpu().numpy().astype(np.float64)
            got = u[g[f"skel_j{n}"], g[f"skel_i{n}"]]
            want = g[f"skel_fp64_{n}"][i]
            e = _rel(got, want)
            e32 = _rel(g[f"skel_fp32_{n}"][i], want)
            worst[n] = max(worst.get(n, 0.0), e)
            print(f"K={k} domain {int(d)} {tuple(int(v) for v in sizes[d])}: rel L2 skeleton {e:.3e} "
                  f"(float32 oracle spread {e32:.3e})", flush=True)
            if prec == MF_FP32:
                assert e <= max(1e-5, COND_FACTOR * e32), (k, int(d), e, e32)
            elif e32 <= 1e-6:
                assert e <= (2e-2 if prec == MF_BF16 else 5e-3), (k, int(d), e, e32)
    for n, d in enumerate(g["picks"]):
        uo = batch.field(int(d), out).cpu().numpy().astype(np.float64)
        got = uo[g[f"sample_j{n}"], g[f"sample_i{n}"]]
        want = g[f"u_out_fp64_{n}"]
        e = _rel(got, want)
        e32 = _rel(g[f"u_out_fp32_{n}"], want)
        print(f"K=20 domain {int(d)}: rel L2 u_out {e:.3e} (float32 oracle spread {e32:.3e}); "
              f"trajectory max skeleton {worst[n]:.3e}", flush=True)
        if prec == MF_FP32:
            assert e <= max(1e-5, COND_FACTOR * e32), (int(d), e, e32)
        elif e32 <= 1e-6:
            assert e <= (2e-2 if prec == MF_BF16 else 5e-3), (int(d), e, e32)


def test_autotune_on_a_batch_and_the_persistent_row_split_form(ctx):
    """mf_autotune takes a batch (candidates include the persistent
    row-split launch); its choice is used by later solves of the same
    domain list, and every bf16 batched form gives the same fields as the
    one-tile-per-workgroup row-split form, bit for bit."""
    print("case: batch autotune + persistent row-split", flush=True)
    from paper_2308_14258_amd import MF_TILE_PERSIST, MF_TILE_ROWSPLIT, mf_autotune
    sizes, fields = _fields(seed=13, n=6, lo=2, hi=9)
    params = torch.from_numpy(mi.xavier_params(256, 0)).cuda()
    rs = 256 | MF_TILE_ROWSPLIT
    scratch = Batch(fields)
    best = mf_autotune(ctx, params, scratch, None, MF_CROSS, MF_BF16, trials=2)
    rs128 = 128 | MF_TILE_ROWSPLIT
    assert best in (64, 128, 256, 128 | (1 << 16), 256 | (1 << 16), rs, rs128, rs | MF_TILE_PERSIST), best
    print(f"batch autotune chose {best:#x}", flush=True)
    outs = {}
    for code in (rs, rs | MF_TILE_PERSIST, rs128, rs128 | MF_TILE_PERSIST, 0):   # 0: the tuned choice
        ctx.tile_rows(MF_BF16, code)
        b = Batch(fields)
        o = torch.empty_like(b.buf)
        mf_solve(ctx, params, b, None, 4, prec=MF_BF16, u_out=o)
        torch.cuda.synchronize()
        outs[code] = (b.buf.clone(), o)
    ctx.tile_rows(MF_BF16, 0)
    for code in (rs | MF_TILE_PERSIST, rs128, rs128 | MF_TILE_PERSIST):
        assert torch.equal(outs[rs][0], outs[code][0]), hex(code)
        assert torch.equal(outs[rs][1], outs[code][1]), hex(code)
    if best in (rs, rs | MF_TILE_PERSIST, rs128):
        assert torch.equal(outs[0][0], outs[rs][0])
