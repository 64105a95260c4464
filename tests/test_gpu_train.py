"""GPU parity of sdnet_train_step (Alg. 1 + Adam) and of sdnet_forward's
derivative outputs against the float64 oracle, through the C ABI.

Bars: the gradient matches the oracle's float64 autograd gradient and
float64 central finite differences of the oracle loss to relative 1e-4;
losses to 1e-5; value / first-derivative outputs to 1e-5 and the Laplacian
to 1e-4 (it is a small difference of float32 stream values). After 100 Adam
steps the trajectories of float32 and float64 need not agree to 1e-5 (Adam's
normalisation amplifies tiny gradient differences), so the loss curve is
held to relative 1e-3.
"""
import os

import numpy as np
import pytest
import torch

import mf_inputs as mi
from oracle import sdnet, train
from paper_2308_14258_amd import Context, physics_loss, sdnet_forward, sdnet_loss_grad, sdnet_train_step

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


def _batch(B, nc, seed=2):
    G = mi.gp_perimeter_batch(B, 0.5, seed)
    Xc = mi.collocation_points(B, nc, seed + 1)
    Xb = mi.unit_perimeter_nodes().astype(np.float32)
    return G, Xb, Xc


def _d(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _t64(a):
    return torch.from_numpy(np.asarray(a, dtype=np.float64))


def _gpu_grad(ctx, params, G, Xb, Xc):
    p = _d(params)
    grad = torch.empty_like(p)
    z = torch.zeros_like(p)
    loss = sdnet_train_step(ctx, p, z, z, 1, _d(G), _d(Xb), _d(Xc), grad_out=grad)
    torch.cuda.synchronize()
    return grad.cpu().numpy().astype(np.float64), loss.cpu().numpy().astype(np.float64)


def _groups(d):
    sizes = [("W1", d * 130), ("b1", d), ("W2", d * d), ("b2", d), ("W3", d * d), ("b3", d),
             ("W4", d * d), ("b4", d), ("w5", d), ("b5", 1)]
    off = 0
    for name, n in sizes:
        yield name, slice(off, off + n)
        off += n


@pytest.mark.parametrize("width", [128, 256])
def test_gradient_matches_oracle(ctx, width):
    print(f"case: train gradient width={width} B=8 nc=16", flush=True)
    params = mi.random_params(width, seed=13)
    G, Xb, Xc = _batch(8, 16)
    g, loss = _gpu_grad(ctx, params, G, Xb, Xc)
    ld, lp, gd, gp = train.gradient(_t64(params), width, _t64(G), _t64(Xb), _t64(Xc))
    want = (gd + gp).numpy()
    err = np.linalg.norm(g - want) / np.linalg.norm(want)
    print(f"gradient rel L2 {err:.3e}; loss {loss} vs {(ld, lp)}", flush=True)
    assert err <= 1e-4
    for name, sl in _groups(width):
        e = np.linalg.norm(g[sl] - want[sl]) / max(np.linalg.norm(want[sl]), 1e-30)
        assert e <= 1e-3, (name, e)
    assert abs(loss[0] - ld) <= 1e-5 * ld and abs(loss[1] - lp) <= 1e-5 * lp


@pytest.mark.parametrize("width,per_bc", [(128, True), (256, False)])
def test_gradient_with_data_targets_matches_oracle(ctx, width, per_bc):
    """The supervised data term (targets at data points, Sec. 5.2), with the
    data points per condition or shared and a count that is not the 128 of
    the boundary match: losses and gradient against the oracle."""
    print(f"case: train gradient with data targets width={width} per_bc={per_bc} B=6 nd=37 nc=16",
          flush=True)
    B, nd, nc = 6, 37, 16
    params = mi.random_params(width, seed=31)
    G, _, Xc = _batch(B, nc, seed=7)
    rng = np.random.default_rng(8)
    Xd = mi.collocation_points(B, nd, 9) if per_bc else mi.collocation_points(1, nd, 9)[0]
    Yd = rng.standard_normal((B, nd)).astype(np.float32)
    p = _d(params)
    grad = torch.empty_like(p)
    loss, _ = sdnet_loss_grad(ctx, p, _d(G), _d(Xd), _d(Xc), grad_out=grad, Yd=_d(Yd))
    torch.cuda.synchronize()
    g = grad.cpu().numpy().astype(np.float64)
    loss = loss.cpu().numpy().astype(np.float64)
    ld, lp, gd, gp = train.gradient(_t64(params), width, _t64(G), _t64(Xd), _t64(Xc), _t64(Yd))
    want = (gd + gp).numpy()
    err = np.linalg.norm(g - want) / np.linalg.norm(want)
    print(f"gradient rel L2 {err:.3e}; loss {loss} vs {(ld, lp)}", flush=True)
    assert err <= 1e-4
    assert abs(loss[0] - ld) <= 1e-5 * ld and abs(loss[1] - lp) <= 1e-5 * lp
    assert abs(loss[2] - (ld + lp)) <= 1e-5 * (ld + lp)


def test_gradient_matches_finite_differences(ctx):
    """4 conditions x 8 collocation points: directional derivatives of the
    float64 oracle loss by central differences."""
    print("case: train gradient vs FD, B=4 nc=8", flush=True)
    width = 128
    params = mi.random_params(width, seed=17)
    G, Xb, Xc = _batch(4, 8, seed=5)
    g, _ = _gpu_grad(ctx, params, G, Xb, Xc)
    th = _t64(params)

    def L(t):
        a, b = train.losses(t, width, _t64(G), _t64(Xb), _t64(Xc))
        return (a + b).item()

    rng = np.random.default_rng(0)
    h = 1e-5
    for _ in range(12):
        v = rng.standard_normal(th.numel())
        v /= np.linalg.norm(v)
        vt = _t64(v)
        fd = (L(th + h * vt) - L(th - h * vt)) / (2 * h)
        an = float(np.dot(g, v))
        assert abs(fd - an) <= 1e-4 * max(abs(fd), 1e-2 * np.linalg.norm(g)), (fd, an)


def test_adam_update(ctx):
    """One step with the update applied equals textbook Adam applied to the
    gradient the same call computes."""
    print("case: adam update", flush=True)
    width = 128
    params = mi.random_params(width, seed=19)
    G, Xb, Xc = _batch(8, 16, seed=7)
    g, _ = _gpu_grad(ctx, params, G, Xb, Xc)
    rng = np.random.default_rng(3)
    m0 = (rng.standard_normal(params.size) * 1e-3).astype(np.float32)
    v0 = (rng.uniform(size=params.size) * 1e-6).astype(np.float32)
    p, m, v = _d(params), _d(m0), _d(v0)
    sdnet_train_step(ctx, p, m, v, 5, _d(G), _d(Xb), _d(Xc), lr=1e-3)
    torch.cuda.synchronize()
    want_p, want_m, want_v = train.adam_update(_t64(params), _t64(m0), _t64(v0), _t64(g), 5)
    assert np.abs(p.cpu().numpy() - want_p.numpy()).max() <= 1e-6
    assert np.abs(m.cpu().numpy() - want_m.numpy()).max() <= 1e-6 * np.abs(want_m.numpy()).max()
    assert np.abs(v.cpu().numpy() - want_v.numpy()).max() <= 1e-5 * np.abs(want_v.numpy()).max()


@pytest.mark.skipif(not os.path.exists(os.path.join(HERE, "golden", "c3_train.npz")),
                    reason="c3_train.npz not generated")
def test_c3_full_batch_gradient_and_curve(ctx):
    """1024 conditions x 256 collocation points, width 128: the full-batch
    gradient at the initial parameters and 100 Adam steps."""
    print("case: C3 full batch, 100 Adam steps", flush=True)
    gold = np.load(os.path.join(HERE, "golden", "c3_train.npz"))
    w = mi.WORKLOADS["C3"]
    G = mi.gp_perimeter_batch(w["n_bc"], w["length"], w["bc_seed"])
    Xc = mi.collocation_points(w["n_bc"], w["n_colloc"], w["colloc_seed"])
    Xb = mi.unit_perimeter_nodes().astype(np.float32)
    params = mi.xavier_params(w["width"], 0)
    g, _ = _gpu_grad(ctx, params, G, Xb, Xc)
    err = np.linalg.norm(g - gold["grad0"]) / np.linalg.norm(gold["grad0"])
    print(f"C3 full-batch gradient rel L2 {err:.3e}", flush=True)
    assert err <= 1e-4
    p = _d(params)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    Gd, Xbd, Xcd = _d(G), _d(Xb), _d(Xc)
    losses = []
    for step in range(1, w["steps"] + 1):
        loss = sdnet_train_step(ctx, p, m, v, step, Gd, Xbd, Xcd)
        losses.append(loss.clone())
    curve = torch.stack(losses).cpu().numpy().astype(np.float64)[:, :2]
    rel = np.abs(curve - gold["curve"]) / np.abs(gold["curve"])
    print(f"C3 loss curve: max rel diff {rel.max():.3e}; final {curve[-1]} vs {gold['curve'][-1]}",
          flush=True)
    assert rel.max() <= 1e-3


@pytest.mark.parametrize("width", [128, 256])
@pytest.mark.parametrize("per_bc", [False, True])
def test_forward_derivatives(ctx, width, per_bc):
    print(f"case: forward derivatives width={width} per_bc={per_bc}", flush=True)
    params = mi.random_params(width, seed=23)
    rng = np.random.default_rng(width + per_bc)
    n_bc, n_pts = 9, 37
    G = rng.standard_normal((n_bc, 128)).astype(np.float32) * 0.5
    X = rng.uniform(size=(n_bc, n_pts, 2) if per_bc else (n_pts, 2)).astype(np.float32)
    U, dU, lapU = sdnet_forward(ctx, _d(params), _d(G), _d(X), derivatives=True)
    Xo = _t64(X) if per_bc else _t64(X)[None].expand(n_bc, -1, -1)
    u, ux, uy, lap = sdnet.derivatives(sdnet.unpack(_t64(params), width), _t64(G), Xo)

    def rel(a, b):
        return float(np.linalg.norm(a - b.numpy()) / np.linalg.norm(b.numpy()))

    U, dU, lapU = (t.cpu().numpy().astype(np.float64) for t in (U, dU, lapU))
    errs = (rel(U, u), rel(dU[..., 0], ux), rel(dU[..., 1], uy), rel(lapU, lap))
    print(f"forward derivative rel L2 (u, ux, uy, lap): {errs}", flush=True)
    assert errs[0] <= 1e-5 and errs[1] <= 1e-5 and errs[2] <= 1e-5 and errs[3] <= 1e-4


def test_autograd_function_gives_the_library_gradient(ctx):
    """physics_loss(...).backward() (torch.autograd.Function around the
    hand-written reverse pass) puts exactly the library's gradient into
    params.grad, scaled by the incoming gradient, and the value is
    L_data + L_pde; the gradient matches the float64 oracle."""
    print("case: autograd Function width=128 B=4 nc=8", flush=True)
    width = 128
    params = mi.random_params(width, seed=23)
    G, Xb, Xc = _batch(4, 8, seed=11)
    Gd, Xbd, Xcd = _d(G), _d(Xb), _d(Xc)
    p = _d(params).requires_grad_(True)
    L = physics_loss(ctx, p, Gd, Xbd, Xcd)
    (3.0 * L).backward()
    loss, grad = sdnet_loss_grad(ctx, _d(params), Gd, Xbd, Xcd)
    torch.cuda.synchronize()
    assert torch.equal(p.grad, 3.0 * grad)
    assert L.item() == loss[2].item()           # the library forms L_data + L_pde
    assert abs(L.item() - loss[:2].sum().item()) <= 1e-6 * abs(loss[:2].sum().item())
    ld, lp, gd, gp = train.gradient(_t64(params), width, _t64(G), _t64(Xb), _t64(Xc))
    want = (gd + gp).numpy()
    got = grad.cpu().numpy().astype(np.float64)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    print(f"autograd Function gradient rel L2 vs oracle {err:.3e}", flush=True)
    assert err <= 1e-4


def test_torch_adam_on_the_autograd_loss_tracks_the_fused_step(ctx):
    """Three steps of torch.optim.Adam driven by physics_loss follow the
    library's fused Adam step (sdnet_train_step) to float32 rounding."""
    print("case: torch Adam vs fused Adam, 3 steps", flush=True)
    width = 128
    params = mi.random_params(width, seed=29)
    G, Xb, Xc = _batch(4, 8, seed=13)
    Gd, Xbd, Xcd = _d(G), _d(Xb), _d(Xc)
    p = _d(params).requires_grad_(True)
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    q, m, v = _d(params), torch.zeros_like(p), torch.zeros_like(p)
    for k in range(1, 4):
        opt.zero_grad()
        physics_loss(ctx, p, Gd, Xbd, Xcd).backward()
        opt.step()
        sdnet_train_step(ctx, q, m, v, k, Gd, Xbd, Xcd, lr=1e-3)
    torch.cuda.synchronize()
    d = (p.detach() - q).norm() / (_d(params) - q).norm()
    print(f"torch Adam vs fused: relative difference of the update {d.item():.3e}", flush=True)
    assert d.item() <= 1e-4
