"""Mosaic Flow predictor sweep in float64 (oracle).

Follows the paper's predictor (Sec. 2.4, Fig. 2; Sec. 4.1; Alg. 2 on one
device):

* a colour phase feeds every same-colour placement's boundary vector,
  gathered from the current global field, to the subdomain solver and writes
  the predictions at that placement's targets back into the field. All
  placements of the phase read the field as it was before the phase (they do
  not overlap, Sec. 4.1), so the phase is computed as a batch;
* a sweep (one iteration of Alg. 2's loop) runs the four colours in order;
* the loop stops after ``max_sweeps`` sweeps, or earlier when the relative
  change delta of the skeleton values drops below ``eps``;
* after the loop every placement predicts its full interior from the final
  field and the result is the average over all placements covering a point
  (Alg. 2, final phase). The outer ring keeps the Dirichlet data.

The subdomain solver is a callable ``solver(G, targets) -> [P, T]`` taking the
[P, 128] boundary vectors and a target list. ``sdnet_solver`` wraps the
network; ``fd.operator_solver`` wraps the exact 5-point solver used as the
check mode.
"""
from __future__ import annotations

import math

import torch

from . import geometry as geo
from . import sdnet


def sdnet_solver(theta: torch.Tensor, width: int):
    """Subdomain solver = SDNet at the local target coordinates t / 32."""
    layers = sdnet.unpack(theta, width)

    def solve(G: torch.Tensor, tgts) -> torch.Tensor:
        X = torch.tensor([[i / geo.S, j / geo.S] for (i, j) in tgts], dtype=G.dtype)
        return sdnet.forward(layers, G, X)

    return solve


def _gather_index(plist):
    """(row, col) index tensors [P, 128] of every listed placement's boundary."""
    bl = geo.boundary_local()
    jj = [[geo.HALF * b + bj for (bi, bj) in bl] for (a, b) in plist]
    ii = [[geo.HALF * a + bi for (bi, bj) in bl] for (a, b) in plist]
    return torch.tensor(jj), torch.tensor(ii)


def _target_index(plist, tgts):
    """(row, col) index tensors [P, T] of every listed placement's targets."""
    jj = [[geo.HALF * b + tj for (ti, tj) in tgts] for (a, b) in plist]
    ii = [[geo.HALF * a + ti for (ti, tj) in tgts] for (a, b) in plist]
    return torch.tensor(jj), torch.tensor(ii)


def gather(u: torch.Tensor, plist) -> torch.Tensor:
    """[P, 128] boundary vectors of the listed placements."""
    jj, ii = _gather_index(plist)
    return u[jj, ii]


def _scatter(u: torch.Tensor, plist, tgts, pred: torch.Tensor) -> torch.Tensor:
    """Write pred[p, t] at placement p's target t (functional, for autograd)."""
    jj, ii = _target_index(plist, tgts)
    out = u.clone()
    out[jj.reshape(-1), ii.reshape(-1)] = pred.reshape(-1)
    return out


def _average_into(u: torch.Tensor, plist, tgts, pred: torch.Tensor) -> torch.Tensor:
    """Every point covered by some prediction takes the mean of those
    predictions; other points keep u's value."""
    jj, ii = _target_index(plist, tgts)
    ny, nx = u.shape
    lin = (jj * nx + ii).reshape(-1)
    acc = torch.zeros(ny * nx, dtype=u.dtype).index_add(0, lin, pred.reshape(-1))
    cnt = torch.zeros(ny * nx, dtype=u.dtype).index_add(
        0, lin, torch.ones(lin.numel(), dtype=u.dtype))
    covered = cnt > 0
    safe = torch.where(covered, cnt, torch.ones_like(cnt))
    out = torch.where(covered, acc / safe, u.reshape(-1))
    return out.reshape(ny, nx)


def colour_phase(u: torch.Tensor, ux: int, uy: int, c: int, solver, kind: str = "cross"):
    """One batched colour phase: every placement of colour c reads u."""
    plist = geo.placements_of_colour(ux, uy, c)
    if not plist:
        return u
    tgts = geo.targets(kind)
    pred = solver(gather(u, plist), tgts)
    return _scatter(u, plist, tgts, pred)


def colour_phase_sequential(u: torch.Tensor, ux: int, uy: int, c: int, solver,
                            kind: str = "cross"):
    """The unbatched baseline: placements one at a time, each seeing the
    updates of the ones before it (Sec. 4.1)."""
    tgts = geo.targets(kind)
    for (a, b) in geo.placements_of_colour(ux, uy, c):
        pred = solver(gather(u, [(a, b)]), tgts)
        u = _scatter(u, [(a, b)], tgts, pred)
    return u


def sweep(u: torch.Tensor, ux: int, uy: int, solver, kind: str = "cross",
          sequential: bool = False):
    """One iteration of Alg. 2's loop: the four colour phases in order."""
    phase = colour_phase_sequential if sequential else colour_phase
    for c in range(4):
        u = phase(u, ux, uy, c, solver, kind)
    return u


def sweep_additive(u: torch.Tensor, ux: int, uy: int, solver, kind: str = "cross"):
    """Parallel (Lions-type, Sec. 2.3) variant: every placement reads the same
    field and each written point takes the mean of the predictions covering
    it."""
    tgts = geo.targets(kind)
    plist = geo.placements(ux, uy)
    pred = solver(gather(u, plist), tgts)
    return _average_into(u, plist, tgts, pred)


def skeleton_mask(ny: int, nx: int) -> torch.Tensor:
    return torch.tensor([[geo.is_skeleton(i, j) for i in range(nx)] for j in range(ny)])


def skeleton_values(u: torch.Tensor) -> torch.Tensor:
    """All field values on the skeleton (ring included), row by row."""
    return u[skeleton_mask(*u.shape)]


def delta(s_new: torch.Tensor, s_old: torch.Tensor) -> float:
    """Alg. 2 convergence measure ||s_i - s_{i-1}|| / ||s_{i-1}|| (L2);
    +inf when the old norm is zero."""
    den = torch.linalg.vector_norm(s_old).item()
    num = torch.linalg.vector_norm(s_new - s_old).item()
    return math.inf if den == 0.0 else num / den


def assemble(u: torch.Tensor, ux: int, uy: int, solver) -> torch.Tensor:
    """Final phase of Alg. 2: every placement predicts all 961 interior points
    from u; each interior grid point takes the mean over the placements that
    cover it. The outer ring keeps u's values."""
    tgts = geo.interior_targets()
    plist = geo.placements(ux, uy)
    pred = solver(gather(u, plist), tgts)
    return _average_into(u, plist, tgts, pred)


def assemble_at(u: torch.Tensor, ux: int, uy: int, solver, points) -> torch.Tensor:
    """The assembly (Alg. 2, final phase) at chosen interior grid points only:
    for each (j, i), the mean of SDNet's predictions there over every
    placement whose interior contains the point."""
    vals = []
    for (j, i) in points:
        preds = []
        for (a, b) in geo.placements(ux, uy):
            ti, tj = i - geo.HALF * a, j - geo.HALF * b
            if 0 < ti < geo.S and 0 < tj < geo.S:
                preds.append(solver(gather(u, [(a, b)]), [(ti, tj)])[0, 0])
        vals.append(torch.stack(preds).mean())
    return torch.stack(vals)


def solve(u0: torch.Tensor, ux: int, uy: int, solver, max_sweeps: int, eps: float = 0.0,
          check_every: int = 1, kind: str = "cross", mode: str = "multiplicative",
          trajectory: list | None = None, assemble_out: bool = True):
    """Alg. 2 on one device. Returns (u_K, u_out, sweeps_done, last_delta).

    delta is evaluated after sweep k whenever eps > 0 and k is a multiple of
    check_every, against the skeleton as it was before that sweep.
    """
    u = u0
    last = math.nan
    k = 0
    for k in range(1, max_sweeps + 1):
        check = eps > 0 and k % check_every == 0
        if check:
            s_old = skeleton_values(u)
        if mode == "multiplicative":
            u = sweep(u, ux, uy, solver, kind)
        else:
            u = sweep_additive(u, ux, uy, solver, kind)
        if trajectory is not None:
            trajectory.append(u.detach().clone())
        if check:
            last = delta(skeleton_values(u), s_old)
            if last < eps:
                break
    u_out = assemble(u, ux, uy, solver) if assemble_out else None
    return u, u_out, k, last
