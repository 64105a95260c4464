"""Pins for the oracle's SDNet (Sec. 3.1-3.2, Eqs. 5-8) and its derivatives."""
import numpy as np
import torch

import mf_inputs as mi
from oracle import sdnet



def _theta(width, seed=5):
    return torch.from_numpy(mi.random_params(width, seed).astype(np.float64))


def test_split_equals_concat():
    """Eq. 8 (input-split) is an exact rewrite of Eq. 6 (input-concat)."""
    layers = sdnet.unpack(_theta(64), 64)
    rng = np.random.default_rng(0)
    G = torch.from_numpy(rng.standard_normal((5, 128)))
    X = torch.from_numpy(rng.uniform(size=(5, 7, 2)))
    a = sdnet.forward(layers, G, X)
    b = sdnet.forward_concat(layers, G, X)
    assert torch.max(torch.abs(a - b)) <= 1e-14 * torch.max(torch.abs(b))
    Xs = X[0]
    assert torch.allclose(sdnet.forward(layers, G, Xs), sdnet.forward_concat(layers, G, Xs),
                          rtol=0, atol=1e-14)


def test_matches_independent_sequential():
    """A torch.nn.Sequential built from the same flat vector by hand."""
    d = 32
    th = _theta(d)
    seq = torch.nn.Sequential(
        torch.nn.Linear(130, d), torch.nn.Tanh(),
        torch.nn.Linear(d, d), torch.nn.Tanh(),
        torch.nn.Linear(d, d), torch.nn.Tanh(),
        torch.nn.Linear(d, d), torch.nn.Tanh(),
        torch.nn.Linear(d, 1)).double()
    off = 0
    with torch.no_grad():
        for m in seq:
            if isinstance(m, torch.nn.Linear):
                n = m.weight.numel()
                m.weight.copy_(th[off:off + n].reshape(m.weight.shape)); off += n
                n = m.bias.numel()
                m.bias.copy_(th[off:off + n]); off += n
    assert off == th.numel()
    rng = np.random.default_rng(1)
    G = torch.from_numpy(rng.standard_normal((3, 128)))
    X = torch.from_numpy(rng.uniform(size=(3, 4, 2)))
    inp = torch.cat([G[:, None, :].expand(3, 4, 128), X], -1)
    want = seq(inp)[..., 0]
    got = sdnet.forward(sdnet.unpack(th, d), G, X)
    assert torch.max(torch.abs(got - want)) <= 1e-13


def test_one_layer_closed_form_derivatives():
    """u = w . tanh(W1 [g; x] + b1) + b5 has
    u_x = sum_k w_k (1 - t_k^2) W1x[k, 0] and
    Lap u = sum_k w_k (-2 t_k (1 - t_k^2)) (W1x[k,0]^2 + W1x[k,1]^2)."""
    rng = np.random.default_rng(2)
    d = 16
    W1 = torch.from_numpy(rng.standard_normal((d, 130)))
    b1 = torch.from_numpy(rng.standard_normal(d))
    w5 = torch.from_numpy(rng.standard_normal((1, d)))
    b5 = torch.from_numpy(rng.standard_normal(1))
    layers = [(W1, b1), (w5, b5)]
    G = torch.from_numpy(rng.standard_normal((2, 128)) * 0.1)
    X = torch.from_numpy(rng.uniform(size=(2, 5, 2)))
    u, ux, uy, lap = sdnet.derivatives(layers, G, X)
    pre = (G @ W1[:, :128].T)[:, None, :] + X @ W1[:, 128:].T + b1
    t = torch.tanh(pre)
    s = 1 - t * t
    w = w5[0]
    ux_cf = (s * W1[:, 128] * w).sum(-1)
    uy_cf = (s * W1[:, 129] * w).sum(-1)
    lap_cf = (w * (-2 * t * s) * (W1[:, 128] ** 2 + W1[:, 129] ** 2)).sum(-1)
    assert torch.allclose(ux, ux_cf, rtol=0, atol=1e-12)
    assert torch.allclose(uy, uy_cf, rtol=0, atol=1e-12)
    assert torch.allclose(lap, lap_cf, rtol=0, atol=1e-12)


def test_laplacian_matches_finite_differences():
    d = 32
    layers = sdnet.unpack(_theta(d), d)
    rng = np.random.default_rng(3)
    G = torch.from_numpy(rng.standard_normal((3, 128)) * 0.5)
    X = torch.from_numpy(rng.uniform(0.2, 0.8, size=(3, 6, 2)))
    _, ux, uy, lap = sdnet.derivatives(layers, G, X)
    h = 1e-4

    def f(Y):
        return sdnet.forward(layers, G, Y)

    ex = torch.zeros_like(X); ex[..., 0] = h
    ey = torch.zeros_like(X); ey[..., 1] = h
    fd_lap = (f(X + ex) + f(X - ex) + f(X + ey) + f(X - ey) - 4 * f(X)) / h ** 2
    fd_ux = (f(X + ex) - f(X - ex)) / (2 * h)
    assert torch.max(torch.abs(fd_lap - lap)) < 1e-6 * max(1.0, lap.abs().max().item())
    assert torch.max(torch.abs(fd_ux - ux)) < 1e-8
