"""Pins for the oracle's convolutional-embedding GELU SDNet (Sec. 3.1,
Fig. 3; Sec. 3.2, Eq. 8): GELU against its definition with the scalar
error function, the circular convolutions against brute-force loops, the
input split against the input concat, a one-unit chain whose Laplacian is
worked out by hand with the GELU derivatives Phi + a phi and phi (2 - a^2),
and autograd derivatives against central differences."""
import math

import numpy as np
import pytest
import torch

import mf_inputs as mi
from oracle import sdnet_conv as sc
from oracle import sweep as sw

D, C = 16, 3


def _params(seed=1, bias=0.1):
    th = torch.from_numpy(mi.xavier_conv_params(D, C, seed, bias_scale=bias).astype(np.float64))
    return th, sc.unpack(th, D, C)


def test_param_count_and_layout():
    assert sc.param_count(D, C) == mi.conv_param_count(D, C)
    assert sc.param_count(256, 4) == 4 * 5 + 4 + 4 * 4 * 5 + 4 + 256 * 514 + 256 + 3 * (256 * 256 + 256) + 257


def test_gelu_is_a_phi():
    a = np.linspace(-6.0, 6.0, 241)
    want = np.array([x * 0.5 * (1.0 + math.erf(x / math.sqrt(2.0))) for x in a])
    got = sc.gelu(torch.from_numpy(a)).numpy()
    assert np.max(np.abs(got - want)) <= 1e-15
    assert np.max(np.abs(torch.nn.functional.gelu(torch.from_numpy(a)).numpy() - want)) <= 1e-15


def test_circular_convolution_brute_force():
    rng = np.random.default_rng(2)
    h = rng.standard_normal((2, 3, 128))
    w = rng.standard_normal((4, 3, 5))
    b = rng.standard_normal(4)
    got = sc.conv_circular(torch.from_numpy(h), torch.from_numpy(w), torch.from_numpy(b)).numpy()
    want = np.zeros((2, 4, 128))
    for n in range(2):
        for o in range(4):
            for k in range(128):
                acc = b[o]
                for i in range(3):
                    for t in range(5):
                        acc += w[o, i, t] * h[n, i, (k + t - 2) % 128]
                want[n, o, k] = acc
    assert np.max(np.abs(got - want)) <= 1e-12


def test_input_split_equals_concat():
    _, params = _params()
    G = torch.from_numpy(mi.gp_perimeter_batch(3, 0.5, seed=4).astype(np.float64))
    X = torch.from_numpy(mi.collocation_points(3, 7, seed=5).astype(np.float64))
    a = sc.forward(params, G, X)
    b = sc.forward_concat(params, G, X)
    assert torch.max(torch.abs(a - b)).item() <= 1e-13
    Xs = X[0]
    assert torch.max(torch.abs(sc.forward(params, G, Xs) - sc.forward_concat(params, G, Xs))).item() <= 1e-13


def _phi(a):
    return math.exp(-0.5 * a * a) / math.sqrt(2.0 * math.pi)


def _Phi(a):
    return 0.5 * (1.0 + math.erf(a / math.sqrt(2.0)))


def test_laplacian_hand_computed_gelu_chain():
    """Zero embedding (all convolution parameters zero: GELU(0) = 0), W1x
    row 0 = (a, b), W2..W4 entry (0, 0) = beta, w5 entry 0 = gamma. Then
    u = gamma T4(s), s = a x + b y, T1 = GELU(s), T_{l+1} = GELU(beta T_l),
    and with GELU' = Phi + a phi, GELU'' = phi (2 - a^2):
        T' = g1(beta T_prev) beta T_prev',
        T'' = g1(beta T_prev) beta T_prev'' + g2(beta T_prev) beta^2 T_prev'^2,
    Laplacian u = (a^2 + b^2) gamma T4''(s)."""
    d, ch = 8, 2
    a, b, beta, gamma = 1.3, -0.7, 1.6, 0.9
    th = torch.zeros(sc.param_count(d, ch), dtype=torch.float64)
    E = ch * 128
    off_w1 = ch * 5 + ch + ch * ch * 5 + ch
    th[off_w1 + E] = a
    th[off_w1 + E + 1] = b
    off_w2 = off_w1 + d * (E + 2) + d
    for layer in range(3):
        th[off_w2 + layer * (d * d + d)] = beta
    th[off_w2 + 3 * (d * d + d)] = gamma
    x0, y0 = 0.37, 0.81
    s = a * x0 + b * y0
    g1 = lambda z: _Phi(z) + z * _phi(z)
    g2 = lambda z: _phi(z) * (2.0 - z * z)
    T, dT, ddT = s * _Phi(s), g1(s), g2(s)
    for _ in range(3):
        z = beta * T
        T, dT, ddT = z * _Phi(z), g1(z) * beta * dT, g1(z) * beta * ddT + g2(z) * beta * beta * dT * dT
    lap_want = (a * a + b * b) * gamma * ddT
    params = sc.unpack(th, d, ch)
    G = torch.from_numpy(mi.gp_perimeter_batch(2, 0.5, seed=6).astype(np.float64))
    X = torch.tensor([x0, y0], dtype=torch.float64).expand(2, 3, 2).contiguous()
    u, ux, uy, lap = sc.derivatives(params, G, X)
    assert torch.allclose(u, torch.full_like(u, gamma * T), rtol=1e-14, atol=0)
    assert torch.allclose(lap, torch.full_like(lap, lap_want), rtol=1e-12, atol=0)
    assert torch.allclose(ux, torch.full_like(ux, gamma * dT * a), rtol=1e-13, atol=0)
    assert abs(lap_want) > 0.01


def test_derivatives_against_central_differences():
    _, params = _params(seed=3)
    G = torch.from_numpy(mi.gp_perimeter_batch(2, 0.5, seed=7).astype(np.float64))
    X = torch.from_numpy(mi.collocation_points(2, 5, seed=8).astype(np.float64))
    u, ux, uy, lap = sc.derivatives(params, G, X)
    h = 1e-4
    ex = torch.tensor([h, 0.0], dtype=torch.float64)
    ey = torch.tensor([0.0, h], dtype=torch.float64)
    f = lambda P: sc.forward(params, G, P)
    fdx = (f(X + ex) - f(X - ex)) / (2 * h)
    fdy = (f(X + ey) - f(X - ey)) / (2 * h)
    fdl = (f(X + ex) + f(X - ex) + f(X + ey) + f(X - ey) - 4 * f(X)) / (h * h)
    assert torch.allclose(ux, fdx, atol=1e-8) and torch.allclose(uy, fdy, atol=1e-8)
    assert torch.allclose(lap, fdl, atol=1e-5)


def test_sweep_with_the_conv_network_batched_equals_sequential():
    th, _ = _params(seed=9)
    solve = sc.solver(th, D, C)
    u0 = torch.from_numpy(mi.gp_field(3, 2, 0.8, seed=10).astype(np.float64))
    a = sw.sweep(u0, 3, 2, solve)
    b = sw.sweep(u0, 3, 2, solve, sequential=True)
    assert torch.max(torch.abs(a - b)).item() <= 1e-14 * torch.max(torch.abs(a)).item()
