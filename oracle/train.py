"""Physics-informed SDNet training step in float64 (oracle).

Alg. 1: a forward/backward pass over the data points, a second one over the
collocation points, gradients summed, then one optimiser step (the allreduce
of step 3 is the identity on one device).

Loss:
* data term: a mean squared error against known values at data points,
  L_data = mean_{b,k} (N(x_{b,k}, g_b) - y_{b,k})^2. The paper's data are
  solutions of each boundary value problem (Sec. 5.2, "Training
  Methodology"); without them the default is the boundary match: the data
  points are the 128 boundary nodes of the unit square and y_b = g_b, the
  boundary vector the network was given;
* PDE term (Eq. 3): L_pde = mean_{b,j} (Laplacian N(x_{b,j}, g_b))^2 over the
  collocation points.

Gradients come from automatic differentiation (the paper obtains the
second derivatives and the parameter gradient the same way, Sec. 5.2,
"Training Methodology").
Adam is the textbook update of Kingma and Ba with bias correction.
"""
from __future__ import annotations

import torch

from . import sdnet, sdnet_conv


def losses(theta: torch.Tensor, width: int, G: torch.Tensor, Xd: torch.Tensor,
           Xc: torch.Tensor, Yd: torch.Tensor | None = None):
    """(L_data, L_pde) as differentiable scalars.

    G: [B, 128]; Xd: data points, shared [nd, 2] or per condition
    [B, nd, 2]; Yd: data targets [B, nd], or None for the boundary match
    (then Xd are the 128 boundary nodes and the targets are G); Xc:
    [B, nc, 2] collocation points.
    """
    layers = sdnet.unpack(theta, width)
    u_d = sdnet.forward(layers, G, Xd)
    l_data = torch.mean((u_d - (G if Yd is None else Yd)) ** 2)
    _, _, _, lap = sdnet.derivatives(layers, G, Xc, create_graph=True)
    l_pde = torch.mean(lap ** 2)
    return l_data, l_pde


def gradient(theta: torch.Tensor, width: int, G, Xd, Xc, Yd=None):
    """Returns (L_data, L_pde, grad_data, grad_pde) in float64."""
    th = theta.detach().clone().requires_grad_(True)
    l_data, l_pde = losses(th, width, G, Xd, Xc, Yd)
    (g_data,) = torch.autograd.grad(l_data, th)
    (g_pde,) = torch.autograd.grad(l_pde, th)
    return l_data.item(), l_pde.item(), g_data, g_pde


def losses_conv(theta: torch.Tensor, width: int, channels: int, G: torch.Tensor, Xd: torch.Tensor,
                Xc: torch.Tensor, Yd: torch.Tensor | None = None):
    """(L_data, L_pde) of ``losses`` for the paper's network (``sdnet_conv``:
    convolutional boundary embedding and GELU layers, Sec. 3.1)."""
    params = sdnet_conv.unpack(theta, width, channels)
    u_d = sdnet_conv.forward(params, G, Xd)
    l_data = torch.mean((u_d - (G if Yd is None else Yd)) ** 2)
    _, _, _, lap = sdnet_conv.derivatives(params, G, Xc, create_graph=True)
    l_pde = torch.mean(lap ** 2)
    return l_data, l_pde


def gradient_conv(theta: torch.Tensor, width: int, channels: int, G, Xd, Xc, Yd=None):
    """Returns (L_data, L_pde, grad_data, grad_pde) of ``losses_conv``."""
    th = theta.detach().clone().requires_grad_(True)
    l_data, l_pde = losses_conv(th, width, channels, G, Xd, Xc, Yd)
    (g_data,) = torch.autograd.grad(l_data, th)
    (g_pde,) = torch.autograd.grad(l_pde, th)
    return l_data.item(), l_pde.item(), g_data, g_pde


def adam_update(theta, m, v, grad, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (step counts from 1). Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    theta = theta - lr * mhat / (torch.sqrt(vhat) + eps)
    return theta, m, v


def train_step(theta, m, v, step: int, width: int, G, Xd, Xc, Yd=None, **adam):
    """Alg. 1 then Adam: returns (theta, m, v, L_data, L_pde)."""
    l_data, l_pde, g_data, g_pde = gradient(theta, width, G, Xd, Xc, Yd)
    grad = g_data + g_pde
    theta, m, v = adam_update(theta, m, v, grad, step, **adam)
    return theta, m, v, l_data, l_pde
