"""Batched independent domains (one persistent launch per colour) through
the C ABI: the batch must equal the same domains solved one by one, and the
float64 oracle."""
import numpy as np
import pytest
import torch

import mf_inputs as mi
from oracle import sweep as sw
from paper_2308_14258_amd import MF_BF16, MF_CROSS, MF_FP32, MF_INTERIOR, Batch, Context
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


@pytest.mark.parametrize("prec", [MF_FP32, MF_BF16])
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
