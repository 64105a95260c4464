"""Sensitivity of the assembled solution to the boundary data (oracle).

The output of Alg. 2 on one device is the overlap-averaged assembly u_out
after K multiplicative sweeps started from the field u0 (Dirichlet ring plus
initial interior). Its adjoint maps a seed u_out_bar (one value per grid
point) to u0_bar = (d u_out / d u0)^T u_out_bar, the gradient of the scalar
J = sum over all grid points of u_out_bar * u_out. The values of u0_bar on
the outer ring are dJ/dg, the sensitivity to the Dirichlet data; the ring of
u_out is the ring of u0, so a seed on the ring passes straight through.

The default objective is J = sum over interior grid points of u_out^2, i.e.
the seed 2 u_out on the interior and 0 on the ring.

The derivative is taken by automatic differentiation through every sweep.
No checkpointing: the oracle keeps the whole graph, which is fine at the
sizes it is run on.
"""
from __future__ import annotations

import torch

from . import sweep as sw


def objective(u_out: torch.Tensor) -> torch.Tensor:
    return torch.sum(u_out[1:-1, 1:-1] ** 2)


def solve_adjoint(u0: torch.Tensor, ux: int, uy: int, solver, K: int, kind: str = "cross",
                  uout_bar: torch.Tensor | None = None):
    """Returns (J, u0_bar) for K sweeps followed by the assembly.

    Without ``uout_bar``: J = sum of squared interior values of u_out and
    u0_bar = dJ/du0. With it: J = <uout_bar, u_out> over the whole grid and
    u0_bar = (d u_out / d u0)^T uout_bar.
    """
    x = u0.detach().clone().requires_grad_(True)
    u = x
    for _ in range(K):
        u = sw.sweep(u, ux, uy, solver, kind)
    u_out = sw.assemble(u, ux, uy, solver)
    if uout_bar is None:
        J = objective(u_out)
    else:
        J = torch.sum(uout_bar.to(u_out.dtype) * u_out)
    (g,) = torch.autograd.grad(J, x)
    return J.item(), g
