"""Grid, placements, colours, boundary order and targets (oracle).

Follows Sec. 4.2 (the skeleton of subdomain boundaries is a Cartesian grid
with spacing m/2) and Sec. 4.1 (atomic subdomains that do not overlap are
predicted together). Readings where the paper is silent:

* 32 cells per unit, vertex-centred; a placement covers 33 x 33 vertices and
  placements sit every 16 cells (half a unit) in both directions.
* colour of placement (a, b) is (a mod 2) + 2 (b mod 2); a sweep runs colours
  0, 1, 2, 3 in that order.
* the 128-vector boundary input runs counter-clockwise from the placement's
  local (0, 0), 32 points per side, each side excluding its end corner.
* CROSS targets are the 61 interior points on the two centre lines (the
  per-iteration prediction set of Alg. 2), INTERIOR targets all 31 x 31
  interior points.
"""
from __future__ import annotations

S = 32          # cells per unit = cells per subdomain side
HALF = 16       # placement stride in cells
NB = 128        # boundary samples per subdomain


def grid_shape(ux: int, uy: int) -> tuple[int, int]:
    """(rows, cols) of the vertex grid for a ux x uy unit domain."""
    return S * uy + 1, S * ux + 1


def placements(ux: int, uy: int) -> list[tuple[int, int]]:
    """All placements (a, b); placement (a, b) covers columns 16a..16a+32 and
    rows 16b..16b+32."""
    return [(a, b) for b in range(2 * uy - 1) for a in range(2 * ux - 1)]


def colour(a: int, b: int) -> int:
    return (a % 2) + 2 * (b % 2)


def placements_of_colour(ux: int, uy: int, c: int) -> list[tuple[int, int]]:
    return [(a, b) for (a, b) in placements(ux, uy) if colour(a, b) == c]


def boundary_local() -> list[tuple[int, int]]:
    """Local (i, j) of the 128 boundary samples, counter-clockwise."""
    pts = []
    for k in range(S):
        pts.append((k, 0))
    for k in range(S):
        pts.append((S, k))
    for k in range(S):
        pts.append((S - k, S))
    for k in range(S):
        pts.append((0, S - k))
    return pts


def cross_targets() -> list[tuple[int, int]]:
    """Local (i, j) of the 61 centre-line interior points: the vertical line
    i = 16 (j = 1..31) then the horizontal line j = 16 without its centre."""
    pts = [(HALF, j) for j in range(1, S)]
    pts += [(i, HALF) for i in range(1, S) if i != HALF]
    return pts


def interior_targets() -> list[tuple[int, int]]:
    """Local (i, j) of all 31 x 31 interior points, row by row."""
    return [(i, j) for j in range(1, S) for i in range(1, S)]


def targets(kind: str) -> list[tuple[int, int]]:
    if kind == "cross":
        return cross_targets()
    if kind == "interior":
        return interior_targets()
    raise ValueError(kind)


def is_skeleton(i: int, j: int) -> bool:
    """A grid point lies on the skeleton when it is on a placement boundary
    line, i.e. either index is a multiple of the stride."""
    return i % HALF == 0 or j % HALF == 0
