"""Pins for the oracle's LAMB step and learning-rate schedule (Sec. 5.2,
"Hyperparameters"), against torch's optimisers and schedulers and against
properties that follow from LAMB's definition (You et al., ICLR 2020)."""
import math

import numpy as np
import pytest
import torch

from oracle import optim, sdnet, sdnet_conv


def _rand(n, seed, scale=1.0):
    return torch.from_numpy(np.random.default_rng(seed).standard_normal(n) * scale)


def test_segments_are_the_layout_tensors():
    d = 16
    seg = optim.tanh_segments(d)
    th = torch.arange(seg[-1], dtype=torch.float64)
    tensors = [t for layer in sdnet.unpack(th, d) for t in layer]
    assert len(tensors) == len(seg) - 1
    for t, a, b in zip(tensors, seg[:-1], seg[1:]):
        assert t.numel() == b - a and t.reshape(-1)[0].item() == a
    seg = optim.conv_segments(d, 3)
    th = torch.arange(seg[-1], dtype=torch.float64)
    convs, layers = sdnet_conv.unpack(th, d, 3)
    tensors = [t for pair in convs + layers for t in pair]
    assert len(tensors) == len(seg) - 1
    for t, a, b in zip(tensors, seg[:-1], seg[1:]):
        assert t.numel() == b - a and t.reshape(-1)[0].item() == a


def test_without_trust_ratio_lamb_is_adam():
    seg = [0, 30, 31, 80]
    th = _rand(80, 1)
    p = torch.nn.Parameter(th.clone())
    opt = torch.optim.Adam([p], lr=2e-3, betas=(0.8, 0.99), eps=1e-6)
    x, m, v = th.clone(), torch.zeros(80, dtype=torch.float64), torch.zeros(80, dtype=torch.float64)
    for t in range(1, 6):
        g = _rand(80, 10 + t)
        p.grad = g.clone()
        opt.step()
        x, m, v = optim.lamb_update(x, m, v, g, t, seg, lr=2e-3, beta1=0.8, beta2=0.99, eps=1e-6,
                                    trust_without_decay=False)
    assert torch.allclose(x, p.detach(), rtol=1e-12, atol=1e-15)


def test_clipping_is_adam_on_the_clipped_gradient():
    seg = [0, 50, 64]
    th = _rand(64, 2)
    p = torch.nn.Parameter(th.clone())
    opt = torch.optim.Adam([p], lr=1e-3, eps=1e-6)
    x, m, v = th.clone(), torch.zeros(64, dtype=torch.float64), torch.zeros(64, dtype=torch.float64)
    for t, scale in enumerate((10.0, 0.05, 3.0), start=1):   # clipped, not clipped, clipped
        g = _rand(64, 20 + t, scale)
        p.grad = g.clone()
        torch.nn.utils.clip_grad_norm_([p], 1.0)
        opt.step()
        x, m, v = optim.lamb_update(x, m, v, g, t, seg, lr=1e-3, max_grad_norm=1.0, trust_without_decay=False)
    # torch divides by (norm + 1e-6): agreement to that relative size
    assert torch.allclose(x, p.detach(), rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("wd", [0.0, 0.01])
def test_trust_ratio_fixes_each_tensors_step_length(wd):
    seg = [0, 100, 110, 300, 301]
    th = _rand(301, 3)
    th[100:110] = 0.0                                   # a tensor with zero norm: ratio 1
    m, v = _rand(301, 4, 0.01), _rand(301, 5, 0.01).abs()
    g = _rand(301, 6)
    new, m1, v1 = optim.lamb_update(th, m, v, g, 7, seg, lr=3e-3, weight_decay=wd)
    u = (m1 / (1 - 0.9 ** 7)) / (torch.sqrt(v1 / (1 - 0.999 ** 7)) + 1e-6) + wd * th
    for a, b in zip(seg[:-1], seg[1:]):
        step = torch.linalg.vector_norm(new[a:b] - th[a:b]).item()
        wn = torch.linalg.vector_norm(th[a:b]).item()
        if wn > 0:
            assert step == pytest.approx(3e-3 * wn, rel=1e-12)
        else:
            assert torch.allclose(new[a:b], -3e-3 * u[a:b], rtol=1e-12, atol=0)


def test_step_is_invariant_to_gradient_scale_without_eps():
    seg = [0, 40, 41, 90]
    th = _rand(90, 7)
    a = (th.clone(), torch.zeros(90, dtype=torch.float64), torch.zeros(90, dtype=torch.float64))
    b = (th.clone(), torch.zeros(90, dtype=torch.float64), torch.zeros(90, dtype=torch.float64))
    for t in range(1, 4):
        g = _rand(90, 30 + t)
        a = optim.lamb_update(*a, g, t, seg, lr=1e-2, eps=0.0, weight_decay=0.0)
        b = optim.lamb_update(*b, 7.0 * g, t, seg, lr=1e-2, eps=0.0, weight_decay=0.0)
    assert torch.allclose(a[0], b[0], rtol=1e-12, atol=1e-15)


def test_tensors_do_not_interact():
    """Swapping two tensors' data swaps their results (the ratio is per
    tensor, the moments per element)."""
    n1, n2 = 30, 45
    th, g = _rand(n1 + n2, 8), _rand(n1 + n2, 9)
    z = torch.zeros(n1 + n2, dtype=torch.float64)
    x, _, _ = optim.lamb_update(th, z, z, g, 1, [0, n1, n1 + n2], lr=1e-2, weight_decay=0.1)
    sw = lambda t: torch.cat([t[n1:], t[:n1]])
    y, _, _ = optim.lamb_update(sw(th), z, z, sw(g), 1, [0, n2, n1 + n2], lr=1e-2, weight_decay=0.1)
    assert torch.allclose(sw(x), y, rtol=1e-14, atol=0)


def test_schedule_is_torch_linear_warmup_then_polynomial_decay():
    T, frac, lr0, power = 400, 0.05, 1e-3, 1.0
    W = optim.warmup_steps(T, frac)
    assert W == 20
    p = torch.nn.Parameter(torch.zeros(1))
    opt = torch.optim.SGD([p], lr=lr0)
    warm = torch.optim.lr_scheduler.LinearLR(opt, start_factor=1.0 / W, end_factor=1.0, total_iters=W - 1)
    for step in range(1, W + 1):                   # torch's epoch step - 1
        assert optim.lr_at(step, T, lr0, frac, power) == pytest.approx(opt.param_groups[0]["lr"], rel=1e-12)
        opt.step()
        warm.step()
    for power in (1.0, 2.0):
        opt = torch.optim.SGD([p], lr=lr0)
        dec = torch.optim.lr_scheduler.PolynomialLR(opt, total_iters=T - W, power=power)
        for step in range(W, T + 1):               # torch's epoch step - W
            want = opt.param_groups[0]["lr"]
            assert optim.lr_at(step, T, lr0, frac, power) == pytest.approx(want, rel=1e-9, abs=1e-18)
            opt.step()
            dec.step()
    assert optim.lr_at(W, T, lr0, frac) == lr0
    assert optim.lr_at(T, T, lr0, frac) == 0.0 and optim.lr_at(T + 5, T, lr0, frac) == 0.0
    assert optim.lr_at(W + (T - W) // 2, T, lr0, frac) == pytest.approx(lr0 / 2, rel=1e-12)


def test_the_papers_settings():
    """0.1% warm-up of 50,000 iterations is 50; peak 1e-3 (Sec. 5.2)."""
    assert optim.warmup_steps(50000, 0.001) == 50
    assert optim.lr_at(50, 50000, 1e-3, 0.001) == 1e-3
    lr, frac = optim.scaled_schedule(1e-3, 0.001, 4.0)
    assert lr == pytest.approx(2e-3) and frac == pytest.approx(0.004)
    assert optim.scaled_schedule(1e-3, 0.5, 8.0)[1] == 1.0
    assert math.isclose(optim.scaled_schedule(1e-3, 0.001, 1.0)[0], 1e-3)


def test_step_direction_is_adamw_with_decoupled_decay():
    """With weight decay the LAMB step of each tensor points along
    torch.optim.AdamW's step (decoupled decay), rescaled to lr ||w_s||."""
    seg = [0, 64, 72, 200]
    th, g = _rand(200, 11), _rand(200, 12)
    p = torch.nn.Parameter(th.clone())
    opt = torch.optim.AdamW([p], lr=1.0, weight_decay=0.3, eps=1e-6)
    p.grad = g.clone()
    opt.step()
    d_adamw = p.detach() - th
    z = torch.zeros(200, dtype=torch.float64)
    new, _, _ = optim.lamb_update(th, z, z, g, 1, seg, lr=5e-3, weight_decay=0.3)
    for a, b in zip(seg[:-1], seg[1:]):
        want = 5e-3 * torch.linalg.vector_norm(th[a:b]) / torch.linalg.vector_norm(d_adamw[a:b]) * d_adamw[a:b]
        assert torch.allclose(new[a:b] - th[a:b], want, rtol=1e-10, atol=1e-16)
