"""Pins for the oracle's grid, placements, colours, boundary order and targets.

The placement and colour rules follow Sec. 4.1-4.2 of the paper (skeleton
spacing m/2, same-colour subdomains do not overlap). These tests check the
facts that the batched colour phase relies on by brute force.
"""
import numpy as np

import mf_inputs as mi
from oracle import geometry as geo


def _interior(a, b):
    return {(geo.HALF * a + i, geo.HALF * b + j) for i in range(1, 32) for j in range(1, 32)}


def _boundary(a, b):
    return {(geo.HALF * a + i, geo.HALF * b + j) for (i, j) in geo.boundary_local()}


def _targets(a, b, kind):
    return {(geo.HALF * a + i, geo.HALF * b + j) for (i, j) in geo.targets(kind)}


def test_colour_counts():
    # counts per colour follow from the number of even/odd placement indices
    for (ux, uy), want in {(2, 2): [4, 2, 2, 1], (16, 16): [256, 240, 240, 225],
                           (64, 64): [4096, 4032, 4032, 3969], (3, 5): [15, 10, 12, 8]}.items():
        got = [len(geo.placements_of_colour(ux, uy, c)) for c in range(4)]
        assert got == want
        assert sum(got) == (2 * ux - 1) * (2 * uy - 1)


def test_boundary_order():
    bl = geo.boundary_local()
    assert len(bl) == 128 and len(set(bl)) == 128
    assert bl[0] == (0, 0) and bl[32] == (32, 0) and bl[64] == (32, 32) and bl[96] == (0, 32)
    on_edge = [(i in (0, 32) or j in (0, 32)) for (i, j) in bl]
    assert all(on_edge)
    # consecutive samples are grid neighbours going counter-clockwise
    for k in range(128):
        (i0, j0), (i1, j1) = bl[k], bl[(k + 1) % 128]
        assert abs(i1 - i0) + abs(j1 - j0) == 1
        # cross product of (p - centre) and step is positive (CCW)
        assert (i0 - 16) * (j1 - j0) - (j0 - 16) * (i1 - i0) > 0


def test_generator_perimeter_matches_boundary_order():
    nodes = mi.unit_perimeter_nodes()
    want = np.array(geo.boundary_local(), dtype=np.float64) / 32.0
    np.testing.assert_array_equal(nodes, want)


def test_targets():
    cross = geo.cross_targets()
    inter = geo.interior_targets()
    assert len(cross) == 61 and len(set(cross)) == 61
    assert len(inter) == 961 and len(set(inter)) == 961
    assert all(i == 16 or j == 16 for (i, j) in cross)
    assert set(cross) <= set(inter)


def test_same_colour_independence():
    """Same-colour interiors are disjoint and no placement's targets touch a
    same-colour placement's boundary, so a colour phase depends only on the
    field before the phase (the basis of batching, Sec. 4.1)."""
    ux, uy = 4, 3
    for c in range(4):
        pl = geo.placements_of_colour(ux, uy, c)
        for p in pl:
            for q in pl:
                if p == q:
                    continue
                assert not (_interior(*p) & _interior(*q))
                assert not (_targets(*p, "interior") & _boundary(*q))


def test_skeleton_inside_placement_is_its_cross():
    """The only skeleton points strictly inside a placement are its centre
    lines, so CROSS and INTERIOR sweeps give the same skeleton trajectory."""
    a, b = 3, 2
    inside_skel = {(i, j) for (i, j) in _interior(a, b) if geo.is_skeleton(i, j)}
    assert inside_skel == _targets(a, b, "cross")
    # and every gathered boundary point is a skeleton point
    assert all(geo.is_skeleton(i, j) for (i, j) in _boundary(a, b))


def test_cover_count_closed_form():
    """count(i, j) = c(i) c(j), c(i) = 1 on stride lines or within half a unit
    of the ring, else 2 (the assembly's divisor)."""
    ux, uy = 3, 2
    nx, ny = 32 * ux + 1, 32 * uy + 1
    cnt = np.zeros((ny, nx), dtype=int)
    for (a, b) in geo.placements(ux, uy):
        for (i, j) in _interior(a, b):
            cnt[j, i] += 1

    def c1(i, n):
        return 1 if (i % 16 == 0 or i < 16 or i > n - 16) else 2

    for j in range(1, ny - 1):
        for i in range(1, nx - 1):
            assert cnt[j, i] == c1(i, nx - 1) * c1(j, ny - 1)
    assert cnt[0, :].sum() == 0 and cnt[:, 0].sum() == 0


def test_skeleton_counts():
    """Skeleton = grid points on a line i or j = 0 mod 16 (ring included):
    625, 32,769 and 512,001 points on the 2 x 2-, 16 x 16- and 64 x 64-unit
    grids, i.e. L (n + 1) * 2 - L^2 with L = n / 16 + 1 lines per axis."""
    from oracle import sweep as sw
    for units, want in ((2, 625), (16, 32769), (64, 512001)):
        n = 32 * units
        m = sw.skeleton_mask(n + 1, n + 1)
        assert int(m.sum()) == want, (units, int(m.sum()))
        L = n // 16 + 1
        assert want == 2 * L * (n + 1) - L * L


def test_skeleton_is_union_of_placement_boundaries():
    """Brute force on small domains: the skeleton mask (lines at multiples
    of the stride, Sec. 4.2) is exactly the set of grid points that are a
    boundary sample or a centre-cross target of some placement. From two
    units per side up the boundaries alone cover it; on a one-unit side the
    sole placement's centre line is a stride line that no boundary holds."""
    from oracle import sweep as sw
    for ux, uy in ((1, 1), (1, 3), (2, 2), (3, 2), (2, 5)):
        ny, nx = geo.grid_shape(ux, uy)
        bnd = np.zeros((ny, nx), dtype=bool)
        cross = np.zeros((ny, nx), dtype=bool)
        for (pa, pb) in geo.placements(ux, uy):
            for (bi, bj) in geo.boundary_local():
                bnd[geo.HALF * pb + bj, geo.HALF * pa + bi] = True
            for (ti, tj) in geo.cross_targets():
                cross[geo.HALF * pb + tj, geo.HALF * pa + ti] = True
        mask = sw.skeleton_mask(ny, nx).numpy()
        assert np.array_equal(bnd | cross, mask), (ux, uy)
        if ux >= 2 and uy >= 2:
            assert np.array_equal(bnd, mask), (ux, uy)
        else:
            assert not np.array_equal(bnd, mask), (ux, uy)
