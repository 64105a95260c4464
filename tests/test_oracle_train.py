"""Pins for the oracle's training loss, gradient and Adam (Alg. 1, Eq. 3).

The gradient is checked against float64 central finite differences on a
4 x 8 sub-batch (first 4 conditions, their first 8 collocation points, and
8 boundary nodes k = 0, 16, ..., 112), in random directions and on random
single coordinates; Adam against torch.optim.Adam.
"""
import numpy as np
import pytest
import torch

import mf_inputs as mi
from oracle import train


D = 32


@pytest.fixture(scope="module")
def batch():
    G = torch.from_numpy(mi.gp_perimeter_batch(4, 0.5, seed=2).astype(np.float64))
    Xb = torch.from_numpy(mi.unit_perimeter_nodes()[::16].copy())
    Xc = torch.from_numpy(mi.collocation_points(4, 8, seed=3).astype(np.float64))
    Gb = G[:, ::16].contiguous()
    th = torch.from_numpy(mi.random_params(D, 21).astype(np.float64))
    return th, G, Gb, Xb, Xc


def _loss(th, G, Gb, Xb, Xc):
    # boundary match on the 8 sampled nodes only: targets are the matching
    # entries of the boundary vector
    from oracle import sdnet
    layers = sdnet.unpack(th, D)
    u_b = sdnet.forward(layers, G, Xb)
    l_data = torch.mean((u_b - Gb) ** 2)
    _, _, _, lap = sdnet.derivatives(layers, G, Xc, create_graph=True)
    return l_data + torch.mean(lap ** 2)


def test_gradient_matches_finite_differences(batch):
    th, G, Gb, Xb, Xc = batch
    t = th.clone().requires_grad_(True)
    (grad,) = torch.autograd.grad(_loss(t, G, Gb, Xb, Xc), t)
    rng = np.random.default_rng(0)
    h = 1e-5
    for _ in range(16):
        v = torch.from_numpy(rng.standard_normal(th.numel()))
        v /= torch.linalg.vector_norm(v)
        fd = (_loss(th + h * v, G, Gb, Xb, Xc) - _loss(th - h * v, G, Gb, Xb, Xc)) / (2 * h)
        an = torch.dot(grad, v)
        assert abs(fd.item() - an.item()) <= 1e-4 * max(abs(an.item()), 1e-3 * grad.norm().item())
    idx = rng.choice(th.numel(), 256, replace=False)
    h = 1e-4
    scale = grad.abs().max().item()
    for i in idx:
        e = torch.zeros_like(th); e[i] = h
        fd = (_loss(th + e, G, Gb, Xb, Xc) - _loss(th - e, G, Gb, Xb, Xc)) / (2 * h)
        assert abs(fd.item() - grad[i].item()) <= 1e-4 * max(abs(grad[i].item()), 1e-3 * scale)


def test_full_loss_gradient_is_sum_of_parts(batch):
    """Alg. 1: the collocation gradient is accumulated onto the data one."""
    th, G, _, _, Xc = batch
    Xb = torch.from_numpy(mi.unit_perimeter_nodes())
    ld, lp, gd, gp = train.gradient(th, D, G, Xb, Xc)
    t = th.clone().requires_grad_(True)
    a, b = train.losses(t, D, G, Xb, Xc)
    (g,) = torch.autograd.grad(a + b, t)
    assert torch.allclose(g, gd + gp, rtol=1e-12, atol=1e-15)
    assert ld == pytest.approx(a.item()) and lp == pytest.approx(b.item())


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(4)
    th = torch.from_numpy(rng.standard_normal(50))
    p = torch.nn.Parameter(th.clone())
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = torch.zeros(50, dtype=torch.float64)
    v = torch.zeros(50, dtype=torch.float64)
    x = th.clone()
    for step in range(1, 8):
        g = torch.from_numpy(rng.standard_normal(50))
        p.grad = g.clone()
        opt.step()
        x, m, v = train.adam_update(x, m, v, g, step)
    assert torch.allclose(x, p.detach(), rtol=0, atol=1e-15)


def test_training_decreases_loss():
    G = torch.from_numpy(mi.gp_perimeter_batch(8, 0.5, seed=2).astype(np.float64))
    Xb = torch.from_numpy(mi.unit_perimeter_nodes())
    Xc = torch.from_numpy(mi.collocation_points(8, 16, seed=3).astype(np.float64))
    th = torch.from_numpy(mi.xavier_params(D).astype(np.float64))
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    first = None
    for step in range(1, 31):
        th, m, v, ld, lp = train.train_step(th, m, v, step, D, G, Xb, Xc, lr=3e-3)
        first = first if first is not None else ld + lp
    assert ld + lp < 0.7 * first
