"""The workspace-free sweep (mf_sweep_noalloc, for callers that cannot
allocate device memory) against mf_sweep, through the C ABI.

Both run the same kernels, the no-alloc form reading the prepared network
and the batch table from the library's static device scratch instead of a
caller's workspace, so the fields must agree bit for bit. Two calls in a
row, the second with a smaller input (fewer domains, a narrower network,
another precision), show that nothing stale from the first call's scratch
contents leaks into the second.
"""
import numpy as np
import pytest
import torch

import mf_inputs as mi
from paper_2308_14258_amd import (MF_BF16, MF_CROSS, MF_FP32, MF_INTERIOR, Batch, Context, MosaicError,
                                  mf_sweep, mf_sweep_noalloc)
from paper_2308_14258_amd._lib import MF_ENOMEM

pytestmark = pytest.mark.gpu


def _fields(sizes, seed):
    return [mi.random_interior_field(ux, uy, seed + i, 0.5) for i, (ux, uy) in enumerate(sizes)]


def test_noalloc_equals_mf_sweep_twice_second_smaller():
    ctx = Context(0)
    try:
        # call 1: a batch of three domains, width 256, bf16, full sweep
        print("case: noalloc call 1: batch of 3 domains (5x4, 3x6, 2x2 units), width 256, bf16", flush=True)
        fields = _fields([(5, 4), (3, 6), (2, 2)], 40)
        p256 = torch.from_numpy(mi.random_params(256, 3)).cuda()
        ref = Batch(fields)
        got = Batch(fields)
        mf_sweep(ctx, p256, ref, None, -1, MF_CROSS, MF_BF16)
        mf_sweep_noalloc(ctx, p256, got, None, -1, MF_CROSS, MF_BF16)
        torch.cuda.synchronize()
        assert not torch.equal(ref.buf, Batch(fields).buf)        # the sweep did change the field
        assert torch.equal(ref.buf, got.buf)
        # call 2: one smaller domain, width 128, fp32, one INTERIOR colour phase
        print("case: noalloc call 2: one 3x2-unit domain, width 128, fp32, INTERIOR colour 2", flush=True)
        f = torch.from_numpy(mi.random_interior_field(3, 2, 77, 0.5)).cuda()
        p128 = torch.from_numpy(mi.random_params(128, 5)).cuda()
        u_ref = f.clone()
        u_got = f.clone()
        mf_sweep(ctx, p128, u_ref, (3, 2), 2, MF_INTERIOR, MF_FP32)
        mf_sweep_noalloc(ctx, p128, u_got, (3, 2), 2, MF_INTERIOR, MF_FP32)
        torch.cuda.synchronize()
        assert not torch.equal(u_ref, f)
        assert torch.equal(u_ref, u_got)
        # a request past the static scratch is refused before any device work
        with pytest.raises(MosaicError) as ei:
            mf_sweep_noalloc(ctx, p256, Batch([np.zeros((33, 33), np.float32)] * 2300), None)
        assert ei.value.status == MF_ENOMEM
    finally:
        ctx.close()
