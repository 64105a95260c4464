"""SDNet N(x, g; theta) in float64 (oracle).

Sec. 3.1 describes SDNet as a stack of linear layers with smooth
activations fed with a discretised boundary function g (4N samples) and a
point x, through the input-split first layer of Sec. 3.2. The network here
is the plain form of it (no boundary embedding): four tanh hidden layers and
a scalar output, the first layer acting on [g, x, y]

    h1 = tanh(W1 [g; x; y] + b1),   h_{l+1} = tanh(W_{l+1} h_l + b_{l+1}),
    u  = w5 . h4 + b5.

The input-split form of Eq. 8 computes W1 [g; x] as the broadcast sum
g W1g^T (+) X W1x^T: the boundary part once per boundary condition and the
coordinate part once per point. ``forward_concat`` is Eq. 6 (the replicated
input matrix I = [G X]) and exists only so that tests can show the two agree.

Derivatives with respect to x (needed for the PDE loss, Eq. 3) are taken by
automatic differentiation, which is how the paper computes them (Sec. 5.2,
"Training Methodology").

Parameter layout (one flat vector):
W1 (d x 130, cols 0..127 boundary, 128 -> x, 129 -> y) | b1 | W2 | b2 | W3 |
b3 | W4 | b4 | w5 (d) | b5.
"""
from __future__ import annotations

import torch


def unpack(theta: torch.Tensor, width: int, depth: int = 4, n_boundary: int = 128):
    """Split the flat vector into [(W, b), ...] with W (out, in)."""
    d = width
    shapes = [(d, n_boundary + 2)] + [(d, d)] * (depth - 1) + [(1, d)]
    layers, off = [], 0
    for out_f, in_f in shapes:
        w = theta[off:off + out_f * in_f].reshape(out_f, in_f)
        off += out_f * in_f
        b = theta[off:off + out_f]
        off += out_f
        layers.append((w, b))
    assert off == theta.numel(), (off, theta.numel())
    return layers


def mlp_from_first(pre1: torch.Tensor, layers) -> torch.Tensor:
    """Given the first-layer pre-activation, finish the network."""
    h = torch.tanh(pre1)
    for w, b in layers[1:-1]:
        h = torch.tanh(h @ w.T + b)
    w5, b5 = layers[-1]
    return (h @ w5.T + b5)[..., 0]


def forward(layers, G: torch.Tensor, X: torch.Tensor, n_boundary: int = 128) -> torch.Tensor:
    """Input-split forward (Eq. 8).

    G: [B, 128] boundary vectors. X: [B, n, 2] per-condition points or
    [n, 2] points shared by every condition. Returns u: [B, n].
    """
    W1, b1 = layers[0]
    W1g, W1x = W1[:, :n_boundary], W1[:, n_boundary:]
    gproj = G @ W1g.T                       # once per boundary condition
    xproj = X @ W1x.T                       # once per point
    if X.dim() == 2:
        pre1 = gproj[:, None, :] + xproj[None, :, :] + b1
    else:
        pre1 = gproj[:, None, :] + xproj + b1
    return mlp_from_first(pre1, layers)


def forward_concat(layers, G: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    """Input-concat forward (Eq. 6): replicate g for every point."""
    B = G.shape[0]
    if X.dim() == 2:
        X = X[None].expand(B, -1, -1)
    n = X.shape[1]
    I = torch.cat([G[:, None, :].expand(B, n, G.shape[1]), X], dim=-1)
    W1, b1 = layers[0]
    return mlp_from_first(I @ W1.T + b1, layers)


def derivatives(layers, G: torch.Tensor, X: torch.Tensor, create_graph: bool = False):
    """(u, u_x, u_y, Laplacian u) at per-condition points X [B, n, 2].

    First and second derivatives with respect to the point coordinates come
    from autograd; the Laplacian is u_xx + u_yy.
    """
    X = X.detach().clone().requires_grad_(True)
    u = forward(layers, G, X)
    (gx,) = torch.autograd.grad(u.sum(), X, create_graph=True)
    ux, uy = gx[..., 0], gx[..., 1]
    (gxx,) = torch.autograd.grad(ux.sum(), X, create_graph=True)
    (gyy,) = torch.autograd.grad(uy.sum(), X, create_graph=create_graph)
    lap = gxx[..., 0] + gyy[..., 1]
    if not create_graph:
        return u.detach(), ux.detach(), uy.detach(), lap.detach()
    return u, ux, uy, lap
