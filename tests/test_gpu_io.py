"""GPU tests of the standalone boundary gather and target scatter (one colour
phase's data movement) through the C ABI.

Gather and scatter move float32 values without arithmetic, so they must match
the oracle's index-based gather and scatter bit for bit. The unfused phase
(gather -> sdnet_forward -> scatter) must match the fused colour phase of
mf_sweep to the float32 bar (relative L2 <= 1e-5 over the written points).
"""
import numpy as np
import pytest
import torch

import mf_inputs as mi
from oracle import geometry as geo
from oracle import sweep as sw
from paper_2308_14258_amd import (MF_CROSS, MF_FP32, MF_INTERIOR, Context, mf_colour_placements, mf_gather,
                                  mf_scatter, mf_sweep, mf_target_coords, sdnet_forward)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


def _field(ux, uy, seed):
    return mi.random_interior_field(ux, uy, seed).astype(np.float32)


@pytest.mark.parametrize("ux,uy", [(1, 1), (3, 5), (7, 2)])
def test_gather_is_the_oracle_gather(ctx, ux, uy):
    print(f"case: gather {ux}x{uy}", flush=True)
    f = _field(ux, uy, 11)
    u = torch.from_numpy(f).cuda()
    for c in range(4):
        plist = geo.placements_of_colour(ux, uy, c)
        G = mf_gather(ctx, u, (ux, uy), c)
        assert G.shape == (len(plist), 128)
        if plist:
            want = sw.gather(torch.from_numpy(f), plist).numpy()
            np.testing.assert_array_equal(G.cpu().numpy(), want)


def test_gather_on_a_padded_pitch(ctx):
    print("case: gather with row pitch 200 > 161", flush=True)
    ux, uy = 5, 3
    f = _field(ux, uy, 12)
    big = torch.full((f.shape[0], 200), float("nan"), device="cuda")
    big[:, :f.shape[1]] = torch.from_numpy(f).cuda()
    u = big[:, :f.shape[1]]
    assert u.stride(0) == 200
    for c in range(4):
        G = mf_gather(ctx, u, (ux, uy), c)
        want = sw.gather(torch.from_numpy(f), geo.placements_of_colour(ux, uy, c)).numpy()
        np.testing.assert_array_equal(G.cpu().numpy(), want)


@pytest.mark.parametrize("targets,kind", [(MF_CROSS, "cross"), (MF_INTERIOR, "interior")])
def test_scatter_is_the_oracle_scatter(ctx, targets, kind):
    print(f"case: scatter {kind} 4x3", flush=True)
    ux, uy = 4, 3
    f = _field(ux, uy, 13)
    T = 61 if targets == MF_CROSS else 961
    for c in range(4):
        plist = geo.placements_of_colour(ux, uy, c)
        pred = torch.from_numpy(np.random.default_rng(c).standard_normal((len(plist), T)).astype(np.float32))
        u = torch.from_numpy(f).cuda()
        mf_scatter(ctx, pred.cuda(), u, (ux, uy), c, targets)
        want = sw._scatter(torch.from_numpy(f), plist, geo.targets(kind), pred).numpy()
        np.testing.assert_array_equal(u.cpu().numpy(), want)


def test_empty_colour_is_a_no_op(ctx):
    print("case: 1x1 domain, colours 1-3 empty", flush=True)
    f = _field(1, 1, 14)
    u = torch.from_numpy(f).cuda()
    for c in (1, 2, 3):
        assert mf_colour_placements((1, 1), c) == 0
        assert mf_gather(ctx, u, (1, 1), c).shape == (0, 128)
        mf_scatter(ctx, torch.empty(0, 61, device="cuda"), u, (1, 1), c)
    np.testing.assert_array_equal(u.cpu().numpy(), f)


@pytest.mark.parametrize("width", [128, 256])
def test_unfused_phase_matches_the_fused_phase(ctx, width):
    print(f"case: unfused colour phases, width {width}, 6x5 units", flush=True)
    ux, uy = 6, 5
    params = torch.from_numpy(mi.xavier_params(width, 3)).cuda()
    f = mi.gp_field(ux, uy, 1.5, 4).astype(np.float32)
    X = mf_target_coords(MF_CROSS).cuda()
    fused = torch.from_numpy(f).cuda()
    unfused = fused.clone()
    for c in range(4):
        mf_sweep(ctx, params, fused, (ux, uy), colour=c, targets=MF_CROSS, prec=MF_FP32)
        G = mf_gather(ctx, unfused, (ux, uy), c)
        pred = sdnet_forward(ctx, params, G, X)
        mf_scatter(ctx, pred, unfused, (ux, uy), c, MF_CROSS)
    a = unfused.cpu().double().numpy()
    b = fused.cpu().double().numpy()
    m = sw.skeleton_mask(*f.shape).numpy()
    err = np.linalg.norm(a[m] - b[m]) / np.linalg.norm(b[m])
    print(f"unfused vs fused sweep rel L2 {err:.2e}", flush=True)
    assert err <= 1e-5
    np.testing.assert_array_equal(a[~m], b[~m])          # nothing off the skeleton is written


def test_gather_scatter_at_256x256_units(ctx):
    """The 8193 x 8193 field the bandwidth measurement uses (larger than the
    last-level cache): the gathers of colours 0 and 3 and a scatter, bit-exact
    (the other colours are covered at small sizes above)."""
    print("case: gather + scatter 256x256 units", flush=True)
    ux = uy = 256
    f = mi.random_interior_field(ux, uy, 15).astype(np.float32)
    u_cpu = torch.from_numpy(f)
    u = u_cpu.cuda()
    for c in (0, 3):
        plist = geo.placements_of_colour(ux, uy, c)
        G = mf_gather(ctx, u, (ux, uy), c)
        np.testing.assert_array_equal(G.cpu().numpy(), sw.gather(u_cpu, plist).numpy())
    c = 3
    plist = geo.placements_of_colour(ux, uy, c)
    pred = torch.from_numpy(np.random.default_rng(5).standard_normal((len(plist), 61)).astype(np.float32))
    mf_scatter(ctx, pred.cuda(), u, (ux, uy), c, MF_CROSS)
    want = sw._scatter(u_cpu, plist, geo.targets("cross"), pred)
    assert torch.equal(u.cpu(), want)


@pytest.mark.parametrize("ux,uy", [(1, 1), (3, 5), (7, 2), (9, 8)])
def test_skeleton_side_layout_gather_and_scatter(ctx, ux, uy):
    """Pack, gather from the side layout, scatter into it, unpack: the same
    boundary vectors as the oracle's gather and the same field as the
    oracle's CROSS scatter, bit for bit, colour by colour."""
    print(f"case: skeleton side layout {ux}x{uy}", flush=True)
    from paper_2308_14258_amd import SkeletonCols, mf_gather_skel, mf_scatter_skel, mf_skeleton_pack, mf_skeleton_unpack
    f = _field(ux, uy, 13)
    u = torch.from_numpy(f).cuda()
    cols = SkeletonCols(u, (ux, uy))
    mf_skeleton_pack(ctx, u, cols)
    ref = torch.from_numpy(f.astype(np.float64))
    rng = np.random.default_rng(ux * 31 + uy)
    for c in range(4):
        plist = geo.placements_of_colour(ux, uy, c)
        G = mf_gather_skel(ctx, u, cols, c)
        if plist:
            np.testing.assert_array_equal(G.cpu().numpy(), sw.gather(ref, plist).numpy().astype(np.float32))
        pred = rng.standard_normal((len(plist), 61)).astype(np.float32)
        mf_scatter_skel(ctx, torch.from_numpy(pred).cuda(), u, cols, c)
        if plist:
            ref = sw._scatter(ref, plist, geo.cross_targets(), torch.from_numpy(pred.astype(np.float64)))
    mf_skeleton_unpack(ctx, cols, u)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u.cpu().numpy(), ref.numpy().astype(np.float32))


def test_skeleton_side_layout_unfused_sweep_equals_mf_sweep(ctx):
    """gather (side layout) -> sdnet_forward -> scatter (side layout) for the
    four colours, then unpack: the fused sweep to the float32 bar, and the
    field-layout unfused sweep bit for bit."""
    print("case: skeleton side layout unfused sweep", flush=True)
    from paper_2308_14258_amd import SkeletonCols, mf_gather_skel, mf_scatter_skel, mf_skeleton_pack, mf_skeleton_unpack
    ux, uy = 6, 5
    params = torch.from_numpy(mi.random_params(256, seed=19)).cuda()
    f = mi.gp_field(ux, uy, 1.0, seed=20)
    X = mf_target_coords(MF_CROSS).cuda()
    a = torch.from_numpy(f).cuda()
    cols = SkeletonCols(a, (ux, uy))
    mf_skeleton_pack(ctx, a, cols)
    b = torch.from_numpy(f).cuda()
    for c in range(4):
        pa = sdnet_forward(ctx, params, mf_gather_skel(ctx, a, cols, c), X)
        mf_scatter_skel(ctx, pa.contiguous(), a, cols, c)
        pb = sdnet_forward(ctx, params, mf_gather(ctx, b, (ux, uy), c), X)
        mf_scatter(ctx, pb.contiguous(), b, (ux, uy), c, MF_CROSS)
    mf_skeleton_unpack(ctx, cols, a)
    fused = torch.from_numpy(f).cuda()
    mf_sweep(ctx, params, fused, (ux, uy))
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    m = sw.skeleton_mask(*f.shape).numpy()
    got, want = a.cpu().numpy()[m].astype(np.float64), fused.cpu().numpy()[m].astype(np.float64)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) <= 1e-5
