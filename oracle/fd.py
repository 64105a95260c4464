"""Exact 5-point finite-difference solvers in float64 (oracle check mode).

The alternating Schwarz iteration (Sec. 2.3, Eq. 4) converges to the global
solution when each subdomain problem is solved exactly. Swapping SDNet for
the exact discrete subdomain solve therefore turns the Mosaic Flow sweep into
a classical multiplicative Schwarz method on the 5-point Laplacian, whose
fixed point is the global 5-point solution; for data that is exactly
discrete-harmonic (x^2 - y^2, xy, ...) it is that data itself.

* ``subdomain_operator``: H (961 x 128) mapping a 33 x 33 subdomain's
  boundary vector (the sweep's 128-point order) to the 5-point Dirichlet
  solution on its 31 x 31 interior, by sparse LU.
* ``operator_solver``: the sweep's solver interface backed by H.
* ``global_solve``: the 5-point Dirichlet solution of the whole domain.
"""
from __future__ import annotations

import functools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch

from . import geometry as geo


def _dirichlet_5pt(n_i: int, n_j: int):
    """Sparse matrix of -Laplacian_h (times h^2) on an n_i x n_j interior,
    unknowns ordered row by row (j outer, i inner)."""
    ex = np.ones(n_i)
    ey = np.ones(n_j)
    tx = sp.diags([-ex[:-1], 2 * ex, -ex[:-1]], [-1, 0, 1])
    ty = sp.diags([-ey[:-1], 2 * ey, -ey[:-1]], [-1, 0, 1])
    return (sp.kron(sp.identity(n_j), tx) + sp.kron(ty, sp.identity(n_i))).tocsc()


def _boundary_rhs(field: np.ndarray) -> np.ndarray:
    """Right-hand side from the Dirichlet ring of ``field`` (rows j, cols i)."""
    ny, nx = field.shape
    rhs = np.zeros((ny - 2, nx - 2))
    rhs[0, :] += field[0, 1:-1]
    rhs[-1, :] += field[-1, 1:-1]
    rhs[:, 0] += field[1:-1, 0]
    rhs[:, -1] += field[1:-1, -1]
    return rhs.reshape(-1)


@functools.lru_cache(maxsize=None)
def subdomain_operator_np() -> np.ndarray:
    """H [961, 128]: interior values (row by row) from the boundary vector."""
    n = geo.S - 1
    lu = spla.splu(_dirichlet_5pt(n, n))
    H = np.zeros((n * n, geo.NB))
    for k, (bi, bj) in enumerate(geo.boundary_local()):
        e = np.zeros((geo.S + 1, geo.S + 1))
        e[bj, bi] = 1.0
        H[:, k] = lu.solve(_boundary_rhs(e))
    return H


def subdomain_operator(kind: str = "interior") -> torch.Tensor:
    """Rows of H for the requested target set, as float64 tensor [T, 128]."""
    H = subdomain_operator_np()
    if kind == "interior":
        return torch.from_numpy(H.copy())
    n = geo.S - 1
    rows = [(tj - 1) * n + (ti - 1) for (ti, tj) in geo.targets(kind)]
    return torch.from_numpy(H[rows].copy())


def operator_solver():
    """Sweep solver backed by the exact 5-point subdomain solve."""
    H = torch.from_numpy(subdomain_operator_np())
    n = geo.S - 1

    def solve(G: torch.Tensor, tgts) -> torch.Tensor:
        rows = torch.tensor([(tj - 1) * n + (ti - 1) for (ti, tj) in tgts])
        return G @ H[rows].T.to(G.dtype)

    return solve


def global_solve(field: np.ndarray) -> np.ndarray:
    """5-point Dirichlet solution on the whole grid; the ring is kept."""
    field = np.asarray(field, dtype=np.float64)
    ny, nx = field.shape
    A = _dirichlet_5pt(nx - 2, ny - 2)
    sol = spla.spsolve(A, _boundary_rhs(field))
    out = field.copy()
    out[1:-1, 1:-1] = sol.reshape(ny - 2, nx - 2)
    return out
