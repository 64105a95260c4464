"""GPU parity of the paper's SDNet architecture (convolutional boundary
embedding, input-split first layer, GELU layers; Sec. 3.1, Fig. 3) through
the C ABI: sdnet_forward's value, gradient and Laplacian, the sweep and
solve with it, and its training gradient (Alg. 1) and Adam steps, against
the float64 oracle (oracle/sdnet_conv.py, oracle/train.py). Bars as for the
tanh network: float32 relative L2 <= 1e-5 (Laplacian 1e-4, gradient 1e-4)."""
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


def _t64(a):
    return torch.from_numpy(np.asarray(a, dtype=np.float64))


@pytest.mark.parametrize("width,targets", [(128, "boundary"), (256, "boundary"), (128, "per_condition")])
def test_training_gradient_matches_the_oracle(ctx, width, targets):
    """Alg. 1 for the paper's network (sdnet_loss_grad): the data pass and the
    collocation pass with the GELU Taylor rules forward and backward, the
    first layer's gradient over the embedding, and the reverse through the
    two circular convolutions, against float64 autograd of the oracle's loss
    (oracle/train.py losses_conv): the losses to 1e-5 and the gradient to
    relative 1e-4, also tensor by tensor (convolutions included) to 1e-3."""
    print(f"case: GELU training gradient width={width} targets={targets}", flush=True)
    from oracle import optim, train
    from paper_2308_14258_amd import sdnet_loss_grad
    th = _params(width, 61)
    B, nc = 6, 24
    G = mi.gp_perimeter_batch(B, 0.5, seed=62)
    Xc = mi.collocation_points(B, nc, seed=63)
    if targets == "boundary":
        Xd, Yd = mi.unit_perimeter_nodes().astype(np.float32), None
    else:
        Xd = mi.collocation_points(B, 40, seed=64)
        Yd = np.random.default_rng(65).uniform(size=(B, 40)).astype(np.float32)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    loss, grad = sdnet_loss_grad(ctx, d(th), d(G), d(Xd), d(Xc), Yd=None if Yd is None else d(Yd))
    torch.cuda.synchronize()
    ld, lp, gd, gp = train.gradient_conv(_t64(th), width, C, _t64(G), _t64(Xd), _t64(Xc),
                                         None if Yd is None else _t64(Yd))
    want = (gd + gp).numpy()
    got = grad.cpu().numpy().astype(np.float64)
    L = loss.cpu().numpy().astype(np.float64)
    err = _rel(got, want)
    seg = optim.conv_segments(width, C)
    per = [_rel(got[a:b], want[a:b]) for a, b in zip(seg[:-1], seg[1:]) if np.linalg.norm(want[a:b]) > 0]
    print(f"GELU training width {width} ({targets}): loss {L[:2]} vs {ld:.6e} {lp:.6e}; gradient rel L2 "
          f"{err:.2e}, worst tensor {max(per):.2e}", flush=True)
    assert abs(L[0] - ld) <= 1e-5 * abs(ld) and abs(L[1] - lp) <= 1e-5 * abs(lp)
    assert err <= 1e-4
    assert max(per) <= 1e-3


def test_training_steps_track_the_oracle(ctx):
    """Twenty Alg. 1 + Adam steps of the paper's network (sdnet_train_step)
    against the same steps in float64: the loss curves agree to relative
    1e-3 and the loss falls."""
    print("case: GELU training, width 128, 4 x 12, 20 Adam steps", flush=True)
    from oracle import train
    width, B, nc, steps = 128, 4, 12, 20
    th = _params(width, 71)
    G = mi.gp_perimeter_batch(B, 0.5, seed=72)
    Xc = mi.collocation_points(B, nc, seed=73)
    Xb = mi.unit_perimeter_nodes().astype(np.float32)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    p = d(th)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    Gd, Xbd, Xcd = d(G), d(Xb), d(Xc)
    curve = []
    for t in range(1, steps + 1):
        curve.append(sdnet_train_step(ctx, p, m, v, t, Gd, Xbd, Xcd, lr=1e-3).clone())
    got = torch.stack(curve).cpu().numpy().astype(np.float64)[:, :2]
    x = _t64(th)
    mo, vo = torch.zeros_like(x), torch.zeros_like(x)
    want = []
    for t in range(1, steps + 1):
        ld, lp, gd, gp = train.gradient_conv(x, width, C, _t64(G), _t64(Xb), _t64(Xc))
        x, mo, vo = train.adam_update(x, mo, vo, gd + gp, t)
        want.append((ld, lp))
    want = np.array(want)
    rel = np.abs(got - want) / np.abs(want)
    print(f"GELU Adam curve: max rel diff {rel.max():.3e}; total {got[0].sum():.4e} -> {got[-1].sum():.4e}",
          flush=True)
    assert rel.max() <= 1e-3
    assert got[-1].sum() < got[0].sum()


@pytest.mark.parametrize("units,K,ce,targets", [((2, 2), 3, 2, "cross"), ((3, 2), 2, 1, "interior")])
def test_adjoint_matches_the_oracle(ctx, units, K, ce, targets):
    """mf_solve_adjoint for the paper's network (recomputed forward with the
    GELU rules, reverse value stream, and the boundary adjoint back through
    W1e and the two circular convolutions) against float64 autograd through
    the oracle's sweeps with the same network: relative 1e-4, J to 1e-5."""
    print(f"case: GELU adjoint units={units} K={K} ckpt={ce} targets={targets}", flush=True)
    from oracle import adjoint
    from paper_2308_14258_amd import MF_CROSS, mf_solve_adjoint
    ux, uy = units
    th = _params(128, 81)
    f = mi.gp_field(ux, uy, 0.6, seed=82)
    tg = MF_CROSS if targets == "cross" else MF_INTERIOR
    u0 = torch.from_numpy(f).cuda()
    ub, J = mf_solve_adjoint(ctx, torch.from_numpy(th).cuda(), u0, units, K, ce, tg)
    torch.cuda.synchronize()
    solver = sc.solver(torch.from_numpy(th.astype(np.float64)), 128, C)
    Jo, go = adjoint.solve_adjoint(torch.from_numpy(f.astype(np.float64)), ux, uy, solver, K, targets)
    err = _rel(ub.cpu().numpy(), go.numpy())
    print(f"GELU adjoint rel L2 {err:.3e}, J {J.item():.6e} vs {Jo:.6e}", flush=True)
    assert err <= 1e-4
    assert abs(J.item() - Jo) <= 1e-5 * abs(Jo)
