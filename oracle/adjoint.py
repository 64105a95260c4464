"""Sensitivity of the assembled solution to the boundary data (oracle).

J(u0) = sum over interior grid points of u_out^2, where u_out is the
overlap-averaged assembly (Alg. 2, final phase) after K multiplicative
sweeps started from u0. The derivative dJ/du0 is taken by automatic
differentiation through every sweep; its values on the outer ring are
dJ/dg, the sensitivity to the Dirichlet data. No checkpointing: the oracle
keeps the whole graph, which is fine at the sizes it is run on.
"""
from __future__ import annotations

import torch

from . import sweep as sw


def objective(u_out: torch.Tensor) -> torch.Tensor:
    return torch.sum(u_out[1:-1, 1:-1] ** 2)


def solve_adjoint(u0: torch.Tensor, ux: int, uy: int, solver, K: int, kind: str = "cross"):
    """Returns (J, dJ/du0) for K sweeps followed by the assembly."""
    x = u0.detach().clone().requires_grad_(True)
    u = x
    for _ in range(K):
        u = sw.sweep(u, ux, uy, solver, kind)
    u_out = sw.assemble(u, ux, uy, solver)
    J = objective(u_out)
    (g,) = torch.autograd.grad(J, x)
    return J.item(), g
