"""GPU parity of the paper's SDNet architecture (convolutional boundary
embedding, input-split first layer, GELU layers; Sec. 3.1, Fig. 3) through
the C ABI: sdnet_forward's value, gradient and Laplacian, and the sweep and
solve with it, against the float64 oracle (oracle/sdnet_conv.py). Bars as
for the tanh network: float32 relative L2 <= 1e-5 (Laplacian 1e-4)."""
import numpy as np
import pytest
import torch

import mf_inputs as mi
from oracle import sdnet_conv as sc
from oracle import sweep as sw
from paper_2308_14258_amd import MF_BF16, MF_INTERIOR, Batch, Context, MosaicError, mf_solve, mf_sweep
from paper_2308_14258_amd import sdnet_forward, sdnet_train_step
from paper_2308_14258_amd._lib import MF_EUNSUPPORTED

pytestmark = pytest.mark.gpu
C = 4


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _params(width, seed):
    return mi.xavier_conv_params(width, C, seed, bias_scale=0.1)


@pytest.mark.parametrize("width", [128, 256])
@pytest.mark.parametrize("per_bc", [False, True])
def test_forward_and_derivatives(ctx, width, per_bc):
    print(f"case: GELU sdnet_forward width={width} per_bc={per_bc}", flush=True)
    th = _params(width, 11)
    G = mi.gp_perimeter_batch(6, 0.5, seed=12)
    X = mi.collocation_points(6, 37, seed=13) if per_bc else mi.collocation_points(1, 37, seed=13)[0]
    p = torch.from_numpy(th).cuda()
    Gd, Xd = torch.from_numpy(G).cuda(), torch.from_numpy(np.ascontiguousarray(X)).cuda()
    U = sdnet_forward(ctx, p, Gd, Xd)
    U2, dU, lapU = sdnet_forward(ctx, p, Gd, Xd, derivatives=True)
    torch.cuda.synchronize()
    params = sc.unpack(torch.from_numpy(th.astype(np.float64)), width, C)
    X64 = torch.from_numpy(X.astype(np.float64))
    Xo = X64 if per_bc else X64[None].expand(6, -1, -1).contiguous()
    u, ux, uy, lap = sc.derivatives(params, torch.from_numpy(G.astype(np.float64)), Xo)
    errs = (_rel(U.cpu(), u), _rel(U2.cpu(), u), _rel(dU.cpu()[..., 0], ux), _rel(dU.cpu()[..., 1], uy),
            _rel(lapU.cpu(), lap))
    print(f"GELU forward rel L2 (u, u via derivs, ux, uy, lap): {errs}", flush=True)
    assert max(errs[:4]) <= 1e-5 and errs[4] <= 1e-4


@pytest.mark.parametrize("units,targets", [((3, 2), 0), ((2, 3), MF_INTERIOR)])
def test_one_sweep(ctx, units, targets):
    print(f"case: GELU sweep units={units} targets={targets}", flush=True)
    ux, uy = units
    th = _params(256, 21)
    f = mi.gp_field(ux, uy, 0.8, seed=22)
    u = torch.from_numpy(f).cuda()
    mf_sweep(ctx, torch.from_numpy(th).cuda(), u, units, targets=targets)
    torch.cuda.synchronize()
    solve = sc.solver(torch.from_numpy(th.astype(np.float64)), 256, C)
    want = sw.sweep(torch.from_numpy(f.astype(np.float64)), ux, uy, solve,
                    "interior" if targets == MF_INTERIOR else "cross").numpy()
    got = u.cpu().numpy().astype(np.float64)
    inner = (slice(1, -1), slice(1, -1))
    e = _rel(got[inner], want[inner])
    print(f"GELU one sweep rel L2 {e:.3e}", flush=True)
    assert e <= 1e-5
    np.testing.assert_array_equal(got[0], f[0])


def test_solve_with_assembly_and_chunked_phases(ctx):
    """3 sweeps + assembly on 2 x 2 units; then one sweep of a 40 x 30-unit
    domain whose colour phases span two row chunks (65,536 rows each)."""
    print("case: GELU solve 2x2 + chunked 40x30 sweep", flush=True)
    th = _params(128, 31)
    p = torch.from_numpy(th).cuda()
    solve = sc.solver(torch.from_numpy(th.astype(np.float64)), 128, C)
    f = mi.gp_field(2, 2, 0.8, seed=32)
    u = torch.from_numpy(f).cuda()
    u_out = torch.empty_like(u)
    mf_solve(ctx, p, u, (2, 2), 3, u_out=u_out)
    torch.cuda.synchronize()
    _, want, _, _ = sw.solve(torch.from_numpy(f.astype(np.float64)), 2, 2, solve, 3)
    e = _rel(u_out.cpu().numpy()[1:-1, 1:-1], want.numpy()[1:-1, 1:-1])
    print(f"GELU solve 2x2 u_out rel L2 {e:.3e}", flush=True)
    assert e <= 1e-5
    f = mi.gp_field(40, 30, 2.0, seed=33)
    u = torch.from_numpy(f).cuda()
    mf_sweep(ctx, p, u, (40, 30))
    torch.cuda.synchronize()
    want = sw.sweep(torch.from_numpy(f.astype(np.float64)), 40, 30, solve).numpy()
    mask = sw.skeleton_mask(*f.shape).numpy()
    e = _rel(u.cpu().numpy()[mask], want[mask])
    print(f"GELU chunked sweep 40x30 rel L2 skeleton {e:.3e}", flush=True)
    assert e <= 1e-5


def test_batch_equals_one_by_one(ctx):
    print("case: GELU batch", flush=True)
    sizes, fields = mi.batched_domains(4, 1, 4, 1.0, seed=5)
    p = torch.from_numpy(_params(256, 41)).cuda()
    batch = Batch(fields)
    out = torch.empty_like(batch.buf)
    mf_solve(ctx, p, batch, None, 2, u_out=out)
    for i, f in enumerate(fields):
        ux, uy = (int(v) for v in sizes[i])
        u = torch.from_numpy(f).cuda()
        uo = torch.empty_like(u)
        mf_solve(ctx, p, u, (ux, uy), 2, u_out=uo)
        torch.cuda.synchronize()
        assert torch.equal(batch.field(i), u), i
        assert torch.equal(batch.field(i, out), uo), i


def test_unsupported_forms_are_refused(ctx):
    p = torch.from_numpy(_params(128, 51)).cuda()
    u = torch.from_numpy(mi.gp_field(2, 2, 0.8, seed=52)).cuda()
    with pytest.raises(MosaicError) as e:
        mf_sweep(ctx, p, u, (2, 2), prec=MF_BF16)
    assert e.value.status == MF_EUNSUPPORTED
    G = torch.from_numpy(mi.gp_perimeter_batch(2, 0.5, seed=53)).cuda()
    Xb = torch.from_numpy(mi.unit_perimeter_nodes().astype(np.float32)).cuda()
    Xc = torch.from_numpy(mi.collocation_points(2, 4, seed=54)).cuda()
    z = torch.zeros_like(p)
    with pytest.raises(MosaicError) as e:
        sdnet_train_step(ctx, p, z, z.clone(), 1, G, Xb, Xc)
    assert e.value.status == MF_EUNSUPPORTED
