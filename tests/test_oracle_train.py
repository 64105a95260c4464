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


def _zero_params(d):
    return torch.zeros(mi.param_count(d), dtype=torch.float64)


def test_losses_hand_computed_constant_network():
    """Only b5 non-zero: every hidden activation is tanh(0) = 0, so u = b5
    everywhere and the Laplacian vanishes. With boundary data constant per
    condition (1 and 3) and b5 = 0.5 the data loss is, by hand,
    ((0.5 - 1)^2 + (0.5 - 3)^2) / 2 = (0.25 + 6.25) / 2 = 3.25: the mean
    over conditions and nodes (a sum over the 256 entries would give 832, a
    half-squared error 1.625)."""
    d = 32
    th = _zero_params(d)
    th[-1] = 0.5
    G = torch.cat([torch.full((1, 128), 1.0), torch.full((1, 128), 3.0)]).double()
    Xb = torch.from_numpy(mi.unit_perimeter_nodes())
    Xc = torch.from_numpy(mi.collocation_points(2, 5, seed=4).astype(np.float64))
    l_data, l_pde = train.losses(th, d, G, Xb, Xc)
    assert l_data.item() == pytest.approx(3.25, rel=1e-15)
    assert l_pde.item() == 0.0


def test_losses_hand_computed_laplacian():
    """A single-unit chain: W1x row 0 = (a, b), W2..W4 entry (0, 0) = beta,
    w5 entry 0 = gamma, everything else zero. Then u = gamma T4(s) with
    s = a x + b y, T1 = tanh s, T_{l+1} = tanh(beta T_l), and
    Laplacian u = (a^2 + b^2) gamma T4''(s). The derivatives follow from
    tanh' = 1 - tanh^2 by the chain rule:
        T1' = 1 - T1^2,  T1'' = -2 T1 (1 - T1^2),
        T' = beta (1 - T^2) T_prev',
        T'' = beta (1 - T^2) T_prev'' - 2 beta^2 T (1 - T^2) T_prev'^2.
    All collocation points sit at one (x0, y0), so the mean of the squared
    residual is that one value squared: any sum/mean or factor slip in the
    PDE term changes it by a factor of 12 (the point count) or 2."""
    d = 32
    a, b, beta, gamma = 1.3, -0.7, 1.1, 0.9
    th = _zero_params(d)
    off_w1, off_b1 = 0, d * 130
    th[off_w1 + 128] = a
    th[off_w1 + 129] = b
    lstride = d * d + d
    off_w2 = off_b1 + d
    for layer in range(3):
        th[off_w2 + layer * lstride] = beta
    off_w5 = off_w2 + 3 * lstride
    th[off_w5] = gamma
    x0, y0 = 0.37, 0.81
    s = a * x0 + b * y0
    T = np.tanh(s)
    dT = 1.0 - T * T
    ddT = -2.0 * T * (1.0 - T * T)
    for _ in range(3):
        Tn = np.tanh(beta * T)
        dTn = beta * (1.0 - Tn * Tn) * dT
        ddTn = beta * (1.0 - Tn * Tn) * ddT - 2.0 * beta * beta * Tn * (1.0 - Tn * Tn) * dT * dT
        T, dT, ddT = Tn, dTn, ddTn
    lap = (a * a + b * b) * gamma * ddT
    G = torch.from_numpy(mi.gp_perimeter_batch(3, 0.5, seed=5).astype(np.float64))
    Xb = torch.from_numpy(mi.unit_perimeter_nodes())
    Xc = torch.tensor([x0, y0], dtype=torch.float64).expand(3, 4, 2).contiguous()
    _, l_pde = train.losses(th, d, G, Xb, Xc)
    assert l_pde.item() == pytest.approx(lap * lap, rel=1e-12)
    assert abs(lap) > 0.05                       # the case is not degenerate


def test_losses_hand_computed_per_condition_data_targets():
    """The data term against per-condition targets at per-condition points
    (the supervised form with solution values): with only b5 = 2 non-zero,
    u = 2 everywhere, so for targets y = [[1, 2, 4], [0, 2, 3]] the loss is,
    by hand, ((1 + 0 + 4) + (4 + 0 + 1)) / 6 = 10 / 6."""
    d = 32
    th = _zero_params(d)
    th[-1] = 2.0
    G = torch.from_numpy(mi.gp_perimeter_batch(2, 0.5, seed=6).astype(np.float64))
    Xd = torch.from_numpy(mi.collocation_points(2, 3, seed=7).astype(np.float64))
    Yd = torch.tensor([[1.0, 2.0, 4.0], [0.0, 2.0, 3.0]], dtype=torch.float64)
    Xc = torch.from_numpy(mi.collocation_points(2, 5, seed=8).astype(np.float64))
    l_data, l_pde = train.losses(th, d, G, Xd, Xc, Yd)
    assert l_data.item() == pytest.approx(10.0 / 6.0, rel=1e-15)
    assert l_pde.item() == 0.0


def test_boundary_match_is_the_data_term_with_targets_g():
    """Yd = None is the data term with the boundary vector as targets."""
    G = torch.from_numpy(mi.gp_perimeter_batch(3, 0.5, seed=9).astype(np.float64))
    Xb = torch.from_numpy(mi.unit_perimeter_nodes())
    Xc = torch.from_numpy(mi.collocation_points(3, 4, seed=10).astype(np.float64))
    th = torch.from_numpy(mi.random_params(D, 23).astype(np.float64))
    a = train.losses(th, D, G, Xb, Xc)
    b = train.losses(th, D, G, Xb.expand(3, 128, 2), Xc, G)
    assert a[0].item() == b[0].item() and a[1].item() == b[1].item()


def test_conv_network_losses_hand_computed_constant_network():
    """The paper's network (convolutional embedding, GELU) with only b5
    non-zero: GELU(0) = 0 in every layer, so u = b5 everywhere and the
    Laplacian vanishes; with boundary data 1 and 3 and b5 = 0.5 the data
    loss is, by hand, ((0.5 - 1)^2 + (0.5 - 3)^2) / 2 = 3.25."""
    from oracle import sdnet_conv
    d, C = 16, 2
    th = torch.zeros(sdnet_conv.param_count(d, C), dtype=torch.float64)
    th[-1] = 0.5
    G = torch.cat([torch.full((1, 128), 1.0), torch.full((1, 128), 3.0)]).double()
    Xb = torch.from_numpy(mi.unit_perimeter_nodes())
    Xc = torch.from_numpy(mi.collocation_points(2, 5, seed=4).astype(np.float64))
    l_data, l_pde = train.losses_conv(th, d, C, G, Xb, Xc)
    assert l_data.item() == pytest.approx(3.25, rel=1e-15)
    assert l_pde.item() == 0.0


def test_conv_network_gradient_matches_finite_differences():
    """gradient_conv (autograd through the embedding, the GELU layers and
    the Laplacian) against float64 central differences of losses_conv in
    random directions, width 16, 2 channels, 3 conditions x 6 points."""
    from oracle import sdnet_conv
    d, C = 16, 2
    rng = np.random.default_rng(5)
    th = torch.from_numpy(rng.standard_normal(sdnet_conv.param_count(d, C)) * 0.3)
    G = torch.from_numpy(mi.gp_perimeter_batch(3, 0.5, seed=8).astype(np.float64))
    Xb = torch.from_numpy(mi.unit_perimeter_nodes()[::16].copy())
    Gb = G[:, ::16].contiguous()
    Xc = torch.from_numpy(mi.collocation_points(3, 6, seed=9).astype(np.float64))
    ld, lp, gd, gp = train.gradient_conv(th, d, C, G, Xb, Xc, Yd=Gb)
    grad = gd + gp

    def L(t):
        a, b = train.losses_conv(t, d, C, G, Xb, Xc, Yd=Gb)
        return (a + b).item()
    h = 1e-5
    for _ in range(12):
        v = torch.from_numpy(rng.standard_normal(th.numel()))
        v /= torch.linalg.vector_norm(v)
        fd = (L(th + h * v) - L(th - h * v)) / (2 * h)
        an = torch.dot(grad, v).item()
        assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-3 * grad.norm().item())
