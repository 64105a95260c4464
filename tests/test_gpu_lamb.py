"""GPU parity of sdnet_lamb_step (the LAMB step of the SDNet training,
Sec. 5.2) against the float64 oracle, through the C ABI.

Inputs are seeded; the oracle runs on the same float32 values in float64.
Bars: the moments to relative 1e-5 of their largest entry (fp32 roundings,
and the clipping factor from a float32 norm of 231,169 squares); the
parameter change over the steps to relative 1e-5 of its largest entry (the
update divides by sqrt(v_hat) and multiplies by a ratio of two float32
norms, each a sum of up to 65,536 squares) plus the rounding of the stored
float32 parameters, half an ulp per step (doubled in the bound). Tensors whose trust
ratio is 1 (zero norm) and tensors with zero gradient and no decay are
checked exactly.
"""
import numpy as np
import pytest
import torch

import mf_inputs as mi
from oracle import optim
from paper_2308_14258_amd import (Context, MF_GELU, lr_at, lr_schedule, param_segments, sdnet_lamb_step,
                                  sdnet_loss_grad)
from paper_2308_14258_amd.api import sdnet_desc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


def _d(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _t64(a):
    return torch.from_numpy(np.asarray(a, dtype=np.float64))


def _run(ctx, params, grads, seg, steps, **hp):
    p, m, v = _d(params), torch.zeros(params.size, device="cuda"), torch.zeros(params.size, device="cuda")
    for t in range(1, steps + 1):
        sdnet_lamb_step(ctx, p, m, v, _d(grads[t - 1]), t, segments=seg, **hp)
    torch.cuda.synchronize()
    x, mo, vo = _t64(params), torch.zeros(params.size, dtype=torch.float64), torch.zeros(params.size,
                                                                                          dtype=torch.float64)
    for t in range(1, steps + 1):
        x, mo, vo = optim.lamb_update(x, mo, vo, _t64(grads[t - 1]), t, seg, **hp)
    return (p.cpu().numpy().astype(np.float64), m.cpu().numpy().astype(np.float64),
            v.cpu().numpy().astype(np.float64)), (x.numpy(), mo.numpy(), vo.numpy())


def _check(params, got, want, tag, steps):
    """Parameter change: within 1e-5 of its largest entry plus the float32
    storage of the parameters (half an ulp per step, 2^-24 |p|, doubled);
    moments within 1e-5 of their largest entry."""
    p0 = params.astype(np.float64)
    dp_g, dp_w = got[0] - p0, want[0] - p0
    tol = 1e-5 * np.abs(dp_w).max() + steps * 2.0 ** -23 * np.abs(p0)
    r_p = (np.abs(dp_g - dp_w) / tol).max()
    e_m = np.abs(got[1] - want[1]).max() / np.abs(want[1]).max()
    e_v = np.abs(got[2] - want[2]).max() / np.abs(want[2]).max()
    print(f"{tag}: parameter change error / bound {r_p:.2f} (largest change "
          f"{np.abs(dp_w).max():.2e}), m rel {e_m:.2e}, v rel {e_v:.2e}", flush=True)
    assert r_p <= 1.0 and e_m <= 1e-5 and e_v <= 1e-5


HP = {
    "published": dict(lr=1e-3, weight_decay=0.0, max_grad_norm=0.0, trust_without_decay=True),
    "decay_clip": dict(lr=2e-3, weight_decay=0.01, max_grad_norm=1.0, trust_without_decay=True),
    "paper_apex_default": dict(lr=1e-3, weight_decay=0.0, max_grad_norm=1.0, trust_without_decay=False),
    "decay_no_trust_flag": dict(lr=1e-3, weight_decay=0.05, max_grad_norm=0.0, trust_without_decay=False),
}


@pytest.mark.parametrize("name", list(HP))
def test_lamb_steps_match_the_oracle(ctx, name):
    """Five steps on the width-256 tanh layout; the second step's gradient
    is large, so clipping acts there."""
    print(f"case: LAMB {name}, width 256, 5 steps", flush=True)
    params = mi.xavier_params(256, 3)
    seg = param_segments(_d(params))
    assert seg == optim.tanh_segments(256)
    rng = np.random.default_rng(7)
    grads = [(rng.standard_normal(params.size) * (0.5 if t == 1 else 1e-3)).astype(np.float32) for t in range(5)]
    got, want = _run(ctx, params, grads, seg, 5, **HP[name])
    _check(params, got, want, name, 5)


def test_lamb_on_the_gelu_layout(ctx):
    print("case: LAMB on the convolutional-embedding network's 14 tensors", flush=True)
    desc = sdnet_desc(128, MF_GELU, 4)
    seg = param_segments(desc)
    assert seg == optim.conv_segments(128, 4) and len(seg) == 15
    rng = np.random.default_rng(8)
    params = (rng.standard_normal(seg[-1]) * 0.05).astype(np.float32)
    grads = [(rng.standard_normal(seg[-1]) * 1e-2).astype(np.float32) for _ in range(3)]
    got, want = _run(ctx, params, grads, seg, 3, lr=1e-3, weight_decay=0.01, max_grad_norm=0.5)
    _check(params, got, want, "gelu layout", 3)


def test_degenerate_tensors(ctx):
    """A tensor of zeros takes the plain step (ratio 1); a tensor with zero
    gradient and no decay does not move; a one-element tensor and an empty
    tensor are handled."""
    print("case: LAMB degenerate tensors", flush=True)
    seg = [0, 300, 300, 301, 2000, 2500]
    rng = np.random.default_rng(9)
    params = (rng.standard_normal(2500) * 0.1).astype(np.float32)
    params[301:2000] = 0.0
    grads = [(rng.standard_normal(2500) * 1e-2).astype(np.float32) for _ in range(2)]
    for g in grads:
        g[2000:] = 0.0
    got, want = _run(ctx, params, grads, seg, 2, lr=1e-2, weight_decay=0.0)
    _check(params, got, want, "degenerate", 2)
    assert np.array_equal(got[0][2000:], params[2000:].astype(np.float64))
    assert np.all(got[0][301:2000] != 0.0)


def test_single_tensor_and_repeatability(ctx):
    """One tensor of one element; and the same call twice gives the same
    bits (fixed reduction order)."""
    print("case: LAMB one element; repeatability", flush=True)
    got, want = _run(ctx, np.array([0.5], np.float32), [np.array([0.25], np.float32)], [0, 1], 1, lr=1e-2)
    assert got[0][0] == pytest.approx(want[0][0], rel=1e-6)
    params = mi.xavier_params(128, 4)
    g = (np.random.default_rng(10).standard_normal(params.size) * 1e-2).astype(np.float32)
    outs = []
    for _ in range(2):
        p, m, v = _d(params), torch.zeros(params.size, device="cuda"), torch.zeros(params.size, device="cuda")
        sdnet_lamb_step(ctx, p, m, v, _d(g), 1, lr=1e-3, weight_decay=0.01, max_grad_norm=0.1)
        torch.cuda.synchronize()
        outs.append(p.cpu())
    assert torch.equal(outs[0], outs[1])


def test_training_with_lamb_and_the_schedule_tracks_the_oracle(ctx):
    """Alg. 1 on the device (sdnet_loss_grad: both passes, gradients summed)
    followed by sdnet_lamb_step, with the warm-up + linear-decay learning
    rate, for 20 steps on 8 conditions x 32 collocation points (width 128,
    boundary-match data term) against the oracle's gradient and LAMB in
    float64: the loss curves agree to relative 1e-3."""
    print("case: LAMB training, width 128, 8 x 32, 20 steps", flush=True)
    width, B, nc, steps = 128, 8, 32, 20
    G = mi.gp_perimeter_batch(B, 0.5, 12)
    Xc = mi.collocation_points(B, nc, 13)
    Xb = mi.unit_perimeter_nodes().astype(np.float32)
    params = mi.xavier_params(width, 5)
    sched = lr_schedule(1e-3, steps, warmup_frac=0.2)
    hp = dict(weight_decay=0.0, max_grad_norm=1.0, trust_without_decay=True)
    p = _d(params)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    Gd, Xbd, Xcd = _d(G), _d(Xb), _d(Xc)
    curve = []
    for t in range(1, steps + 1):
        loss, grad = sdnet_loss_grad(ctx, p, Gd, Xbd, Xcd)
        sdnet_lamb_step(ctx, p, m, v, grad, t, lr=lr_at(sched, t), **hp)
        curve.append(loss[:2].clone())
    got = torch.stack(curve).cpu().numpy().astype(np.float64)
    th = _t64(params)
    mo, vo = torch.zeros_like(th), torch.zeros_like(th)
    want = []
    for t in range(1, steps + 1):
        lr = optim.lr_at(t, steps, 1e-3, 0.2)
        th, mo, vo, ld, lp = optim.lamb_train_step(th, mo, vo, t, width, _t64(G), _t64(Xb), _t64(Xc), lr=lr, **hp)
        want.append((ld, lp))
    want = np.array(want)
    rel = np.abs(got - want) / np.abs(want)
    print(f"LAMB training curve: max rel diff {rel.max():.3e}; L_data {got[0, 0]:.4e} -> {got[-1, 0]:.4e}",
          flush=True)
    assert rel.max() <= 1e-3
    assert got[-1].sum() < got[0].sum()
