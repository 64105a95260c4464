"""The paper's SDNet architecture in float64 (oracle): a 1-D convolutional
embedding of the boundary curve, the input-split first layer and GELU
layers (Sec. 3.1, Fig. 3; Sec. 3.2, Eq. 8).

Sec. 3.1 convolves the discretised boundary function, seen as a 1-D curve
along the boundary, into a high-dimensional embedding, applies the
input-split first layer to that embedding and the point x, and follows with
linear layers each followed by GELU. The paper gives neither the number of
convolutions nor their sizes; the reading used here:

* embedding: the 128 boundary samples (a closed curve, so the convolutions
  wrap around: circular padding) -> conv1d(1 -> C channels, kernel 5,
  padding 2) + bias -> GELU -> conv1d(C -> C, kernel 5, padding 2) + bias
  -> GELU -> flattened channel by channel, e[c * 128 + k], E = 128 C values;
* first layer: h1 = GELU(W1e e + W1x (x, y) + b1), W1 = [W1e | W1x] of
  shape d x (E + 2), evaluated in the input-split form of Eq. 8 (the
  embedding and W1e e + b1 once per boundary condition);
* three hidden layers h_{l+1} = GELU(W_{l+1} h_l + b_{l+1}) and the output
  u = w5 . h4 + b5;
* GELU(a) = a Phi(a) with Phi the standard normal distribution function
  (the exact form, Phi(a) = (1 + erf(a / sqrt 2)) / 2).

Parameter layout (one flat vector): Wc1 (C x 1 x 5) | bc1 (C) | Wc2 (C x C x
5) | bc2 (C) | W1 (d x (E + 2), columns 0..E-1 embedding, E -> x, E+1 -> y)
| b1 | W2 | b2 | W3 | b3 | W4 | b4 | w5 (d) | b5.

Derivatives with respect to x come from automatic differentiation, as in
``sdnet``.
"""
from __future__ import annotations

import math

import torch

KERNEL = 5
NB = 128


def param_count(width: int, channels: int) -> int:
    d, C = width, channels
    E = C * NB
    return C * KERNEL + C + C * C * KERNEL + C + d * (E + 2) + d + 3 * (d * d + d) + d + 1


def gelu(a: torch.Tensor) -> torch.Tensor:
    """a Phi(a), Phi(a) = (1 + erf(a / sqrt 2)) / 2."""
    return a * 0.5 * (1.0 + torch.erf(a / math.sqrt(2.0)))


def unpack(theta: torch.Tensor, width: int, channels: int):
    """(convs [(W (out, in, 5), b)], layers [(W (out, in), b)])."""
    d, C = width, channels
    E = C * NB
    off = 0

    def take(n, shape):
        nonlocal off
        t = theta[off:off + n].reshape(shape)
        off += n
        return t

    convs = []
    for cin in (1, C):
        w = take(C * cin * KERNEL, (C, cin, KERNEL))
        b = take(C, (C,))
        convs.append((w, b))
    layers = []
    for out_f, in_f in [(d, E + 2)] + [(d, d)] * 3 + [(1, d)]:
        w = take(out_f * in_f, (out_f, in_f))
        b = take(out_f, (out_f,))
        layers.append((w, b))
    assert off == theta.numel(), (off, theta.numel())
    return convs, layers


def conv_circular(h: torch.Tensor, w: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """h [B, Cin, 128] -> [B, Cout, 128]: out[o, k] = b[o] + sum_{i, t}
    w[o, i, t] h[i, (k + t - 2) mod 128]."""
    pad = KERNEL // 2
    hp = torch.cat([h[..., -pad:], h, h[..., :pad]], dim=-1)
    return torch.nn.functional.conv1d(hp, w) + b[None, :, None]


def embed(convs, G: torch.Tensor) -> torch.Tensor:
    """[B, 128] boundary vectors -> [B, E] embeddings."""
    h = G[:, None, :]
    for w, b in convs:
        h = gelu(conv_circular(h, w, b))
    return h.reshape(G.shape[0], -1)


def mlp_from_first(pre1: torch.Tensor, layers) -> torch.Tensor:
    h = gelu(pre1)
    for w, b in layers[1:-1]:
        h = gelu(h @ w.T + b)
    w5, b5 = layers[-1]
    return (h @ w5.T + b5)[..., 0]


def forward(params, G: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    """Input-split forward (Eq. 8) on the embedding. params = (convs,
    layers); G [B, 128]; X [B, n, 2] or shared [n, 2]. Returns [B, n]."""
    convs, layers = params
    e = embed(convs, G)
    W1, b1 = layers[0]
    E = e.shape[1]
    proj = e @ W1[:, :E].T + b1             # once per boundary condition
    xproj = X @ W1[:, E:].T                 # once per point
    pre1 = proj[:, None, :] + (xproj[None] if X.dim() == 2 else xproj)
    return mlp_from_first(pre1, layers)


def forward_concat(params, G: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    """Input-concat form (Eq. 6): [e, x, y] replicated for every point."""
    convs, layers = params
    e = embed(convs, G)
    B = G.shape[0]
    if X.dim() == 2:
        X = X[None].expand(B, -1, -1)
    n = X.shape[1]
    I = torch.cat([e[:, None, :].expand(B, n, e.shape[1]), X], dim=-1)
    W1, b1 = layers[0]
    return mlp_from_first(I @ W1.T + b1, layers)


def derivatives(params, G: torch.Tensor, X: torch.Tensor, create_graph: bool = False):
    """(u, u_x, u_y, Laplacian u) at per-condition points X [B, n, 2]; with
    create_graph the results stay differentiable in the parameters (for the
    PDE loss's gradient)."""
    X = X.detach().clone().requires_grad_(True)
    u = forward(params, G, X)
    (gx,) = torch.autograd.grad(u.sum(), X, create_graph=True)
    ux, uy = gx[..., 0], gx[..., 1]
    (gxx,) = torch.autograd.grad(ux.sum(), X, create_graph=True)
    (gyy,) = torch.autograd.grad(uy.sum(), X, create_graph=create_graph)
    lap = gxx[..., 0] + gyy[..., 1]
    if not create_graph:
        return u.detach(), ux.detach(), uy.detach(), lap.detach()
    return u, ux, uy, lap


def solver(theta: torch.Tensor, width: int, channels: int):
    """Subdomain solver for ``sweep``: the network at the local target
    coordinates t / 32."""
    params = unpack(theta, width, channels)

    def solve(G: torch.Tensor, tgts) -> torch.Tensor:
        X = torch.tensor([[i / 32.0, j / 32.0] for (i, j) in tgts], dtype=G.dtype)
        return forward(params, G, X)

    return solve
