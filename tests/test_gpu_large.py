"""GPU tests at sizes where one phase needs more than one kernel launch.

A launch covers at most 2^22 tiles (colour-phase kernel) or 2^22
placements (standalone gather/scatter), so that its work-items stay below
2^32; larger phases are split into several launches. These tests run phases
past that limit and check sampled outputs against the oracle:

* gather and scatter of colour 0 on a 2049 x 2048-unit field (65,537 x
  65,569 floats, 17 GB; 4,196,352 placements), bit-exact;
* the overlap-averaged assembly of a 600 x 600-unit domain with 32-row FP32
  tiles (10.8 M tiles per colour), relative L2 <= 1e-5 at sampled interior
  points. The oracle evaluates each sampled point on the 2 x 2-unit window
  that holds every placement covering it (the assembly at a point depends
  only on those placements).
"""
import numpy as np
import pytest
import torch

import mf_inputs as mi
from oracle import geometry as geo
from oracle import sweep as sw
from paper_2308_14258_amd import MF_CROSS, MF_FP32, Context, mf_colour_placements, mf_gather, mf_scatter, mf_solve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


def _pattern(j, i):
    """Integer-valued field pattern, exact in float32 (host or device ints)."""
    return (i * 7 + j * 13) % 1021


def _placement(q, c, ux):
    """Placement q of colour c in the oracle's enumeration order (checked below)."""
    na = ux - (c & 1)
    return (c & 1) + 2 * (q % na), (c >> 1) + 2 * (q // na)


def test_placement_closed_form_matches_the_oracle_order():
    for ux, uy in ((3, 4), (5, 2)):
        for c in range(4):
            pl = geo.placements_of_colour(ux, uy, c)
            assert [_placement(q, c, ux) for q in range(len(pl))] == pl


def test_gather_and_scatter_past_one_launch(ctx):
    ux, uy = 2049, 2048
    print(f"case: gather + scatter, {ux}x{uy} units (17 GB field)", flush=True)
    ny, nx = 32 * uy + 1, 32 * ux + 1
    n = mf_colour_placements((ux, uy), 0)
    assert n == ux * uy and n > (1 << 22)
    u = torch.empty(ny, nx, dtype=torch.float32, device="cuda")
    cols = torch.arange(nx, device="cuda", dtype=torch.int64)
    for r0 in range(0, ny, 4096):
        rows = torch.arange(r0, min(r0 + 4096, ny), device="cuda", dtype=torch.int64)[:, None]
        u[r0:r0 + rows.shape[0]] = _pattern(rows, cols).to(torch.float32)
    G = mf_gather(ctx, u, (ux, uy), 0)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    qs = sorted({0, 1, (1 << 22) - 1, 1 << 22, (1 << 22) + 1, n - 1, *rng.integers(0, n, 24).tolist()})
    bl = geo.boundary_local()
    Gs = G[torch.tensor(qs, device="cuda")].cpu().numpy()
    for row, q in zip(Gs, qs):
        a, b = _placement(q, 0, ux)
        want = [_pattern(geo.HALF * b + bj, geo.HALF * a + bi) for (bi, bj) in bl]
        np.testing.assert_array_equal(row, np.asarray(want, dtype=np.float32), err_msg=f"placement {q}")
    # scatter: target t of placement q takes -(q mod 997) - t / 64
    pred = -(torch.arange(n, device="cuda", dtype=torch.int64)[:, None] % 997).to(torch.float32) \
        - torch.arange(61, device="cuda", dtype=torch.float32)[None, :] / 64
    del G
    mf_scatter(ctx, pred, u, (ux, uy), 0, MF_CROSS)
    torch.cuda.synchronize()
    tg = geo.targets("cross")
    for q in qs:
        a, b = _placement(q, 0, ux)
        for t in (0, 15, 30, 31, 60):
            ti, tj = tg[t]
            got = u[geo.HALF * b + tj, geo.HALF * a + ti].item()
            assert got == -(q % 997) - t / 64, (q, t)
    # a point no colour-0 target touches keeps its value
    assert u[0, 5].item() == _pattern(0, 5)


def test_assembly_past_one_launch(ctx):
    ux = uy = 600
    width = 128
    print(f"case: FP32 assembly with 32-row tiles, {ux}x{uy} units, width {width}", flush=True)
    f = mi.random_interior_field(ux, uy, 21)
    params = mi.xavier_params(width, 4)
    u = torch.from_numpy(f).cuda()
    u_out = torch.empty_like(u)
    ctx.tile_rows(MF_FP32, 32)
    try:
        mf_solve(ctx, torch.from_numpy(params).cuda(), u, (ux, uy), 0, u_out=u_out)
        torch.cuda.synchronize()
    finally:
        ctx.tile_rows(MF_FP32, 0)
    rng = np.random.default_rng(8)
    ny, nx = f.shape
    pts = [(int(j), int(i)) for j, i in zip(rng.integers(1, ny - 1, 20), rng.integers(1, nx - 1, 20))]
    pts += [(1, 1), (ny - 2, nx - 2), (16 * 301, 16 * 377), (ny // 2 + 3, 16)]
    solver = sw.sdnet_solver(torch.from_numpy(params.astype(np.float64)), width)
    f64 = torch.from_numpy(f.astype(np.float64))
    want = []
    for (j, i) in pts:
        a0 = min(max(i // geo.HALF - 1, 0), 2 * ux - 4)
        b0 = min(max(j // geo.HALF - 1, 0), 2 * uy - 4)
        win = f64[geo.HALF * b0: geo.HALF * b0 + 65, geo.HALF * a0: geo.HALF * a0 + 65]
        want.append(float(sw.assemble_at(win, 2, 2, solver, [(j - geo.HALF * b0, i - geo.HALF * a0)])[0]))
    got = u_out.cpu().numpy().astype(np.float64)[[p[0] for p in pts], [p[1] for p in pts]]
    want = np.asarray(want)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    print(f"assembly past one launch: rel L2 at {len(pts)} points {err:.2e}", flush=True)
    assert err <= 1e-5
