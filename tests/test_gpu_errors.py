"""Error paths of mf_solve on the GPU, through the C ABI: a NaN in the
Dirichlet data makes the delta test (Alg. 2's convergence check) report
MF_ENONFINITE; an eps that is never reached reports MF_ENOTCONVERGED when
the caller asks for it; MF_FAULT_INJECT makes a solve fail between two
colour phases with the field left as the earlier phases made it."""
import os

import numpy as np
import pytest
import torch

import mf_inputs as mi
from paper_2308_14258_amd import Context, MosaicError, mf_solve, mf_sweep
from paper_2308_14258_amd._lib import MF_EDEVICE, MF_ENONFINITE, MF_ENOTCONVERGED

pytestmark = pytest.mark.gpu

FAIL_IF_NOT_CONVERGED = 1


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


def test_nan_in_the_data_is_reported(ctx):
    print("case: NaN on the ring, eps > 0 -> MF_ENONFINITE", flush=True)
    f = mi.gp_field(3, 2, 0.8, seed=4)
    f[0, 40] = np.nan                     # a ring point: never overwritten, gathered every sweep
    u = torch.from_numpy(f).cuda()
    params = torch.from_numpy(mi.xavier_params(128, 0)).cuda()
    with pytest.raises(MosaicError) as e:
        mf_solve(ctx, params, u, (3, 2), 10, eps=1e-4, check_every=1)
    assert e.value.status == MF_ENONFINITE
    assert "not finite" in str(e.value)
    # without the delta test the same solve runs to the end (no check, no error)
    u = torch.from_numpy(f).cuda()
    mf_solve(ctx, params, u, (3, 2), 3)
    torch.cuda.synchronize()


def test_not_converged_is_reported_only_on_request(ctx):
    print("case: eps never reached -> MF_ENOTCONVERGED with the flag", flush=True)
    f = mi.gp_field(2, 2, 0.8, seed=5)
    params = torch.from_numpy(mi.xavier_params(128, 0)).cuda()
    u = torch.from_numpy(f).cuda()
    done, last = mf_solve(ctx, params, u, (2, 2), 4, eps=1e-30, check_every=1, report=True)
    assert done == 4 and last >= 1e-30
    u = torch.from_numpy(f).cuda()
    with pytest.raises(MosaicError) as e:
        mf_solve(ctx, params, u, (2, 2), 4, eps=1e-30, check_every=1, flags=FAIL_IF_NOT_CONVERGED)
    assert e.value.status == MF_ENOTCONVERGED
    # the sweeps still ran: the field equals four plain sweeps
    v = torch.from_numpy(f).cuda()
    for _ in range(4):
        mf_sweep(ctx, params, v, (2, 2))
    torch.cuda.synchronize()
    assert torch.equal(u, v)


def test_injected_fault_leaves_the_earlier_phases(monkeypatch):
    print("case: MF_FAULT_INJECT=3:2", flush=True)
    monkeypatch.setenv("MF_FAULT_INJECT", "3:2")
    ctx = Context(0)                      # the spec is read when the context is created
    try:
        f = mi.gp_field(3, 3, 0.8, seed=6)
        params = torch.from_numpy(mi.xavier_params(128, 0)).cuda()
        u = torch.from_numpy(f).cuda()
        with pytest.raises(MosaicError) as e:
            mf_solve(ctx, params, u, (3, 3), 6, u_out=torch.empty_like(u))
        assert e.value.status == MF_EDEVICE and "injected" in str(e.value)
    finally:
        ctx.close()
    monkeypatch.delenv("MF_FAULT_INJECT")
    ref = Context(0)
    try:
        v = torch.from_numpy(f).cuda()
        for _ in range(2):
            mf_sweep(ref, params, v, (3, 3))
        for c in range(2):
            mf_sweep(ref, params, v, (3, 3), colour=c)
        torch.cuda.synchronize()
        assert torch.equal(u, v)
        # recovery: the remaining phases and sweeps give the uninterrupted solve
        for c in range(2, 4):
            mf_sweep(ref, params, u, (3, 3), colour=c)
        for _ in range(3):
            mf_sweep(ref, params, u, (3, 3))
        w = torch.from_numpy(f).cuda()
        mf_solve(ref, params, w, (3, 3), 6)
        torch.cuda.synchronize()
        assert torch.equal(u, w)
    finally:
        ref.close()
    assert os.environ.get("MF_FAULT_INJECT") is None
