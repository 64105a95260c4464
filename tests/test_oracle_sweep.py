"""Pins for the oracle's sweep, delta test and assembly (Sec. 4.1, Alg. 2).

The exact 5-point subdomain solver stands in for SDNet: alternating Schwarz
with exact subdomain solves (Sec. 2.3, Eq. 4) has the global 5-point
solution as its fixed point, and polynomials such as x^2 - y^2 are exactly
discrete-harmonic, so the sweep must reproduce them.
"""
import math

import numpy as np
import pytest
import torch

import mf_inputs as mi
from oracle import fd, geometry as geo, sdnet, sweep as sw


HARMONIC = {
    "x2-y2": lambda x, y: x * x - y * y,
    "xy": lambda x, y: x * y,
    "one": lambda x, y: np.ones_like(x),
    "x": lambda x, y: x,
    "cubic": lambda x, y: x ** 3 - 3 * x * y * y,
}


def _field(arr):
    return torch.from_numpy(np.asarray(arr, dtype=np.float64))


def test_fd_operator_invariants():
    H = fd.subdomain_operator_np()
    assert H.shape == (961, 128)
    assert H.min() >= -1e-15                              # discrete maximum principle
    assert np.abs(H.sum(1) - 1).max() < 1e-13             # constants reproduced
    for k in (0, 32, 64, 96):                             # corners never enter the stencil
        assert np.abs(H[:, k]).max() == 0.0
    # rotating the subdomain by 90 degrees rotates the boundary vector by 32
    n = 31
    Hg = H.reshape(n, n, 128)                             # [j, i, k]
    rot = np.roll(np.arange(128), -32)                    # rot[k] = k + 32
    # rotation (i, j) -> (32 - j, i) maps local boundary sample k to k + 32
    for j in range(0, n, 5):
        for i in range(0, n, 5):
            ii, jj = n - 1 - j, i
            np.testing.assert_allclose(Hg[jj, ii, rot], Hg[j, i, :], atol=1e-14)


def test_fd_sweep_reproduces_x2_minus_y2():
    f = _field(mi.x2_minus_y2_field(2, 2))
    exact = mi.full_analytic(2, 2, HARMONIC["x2-y2"])
    u, u_out, k, _ = sw.solve(f, 2, 2, fd.operator_solver(), 50)
    assert k == 50
    assert np.abs(u.numpy() - exact)[sw.skeleton_mask(65, 65).numpy()].max() <= 1e-10
    assert np.abs(u_out.numpy() - exact).max() <= 1e-10


@pytest.mark.parametrize("name", ["xy", "one", "x", "cubic"])
def test_fd_sweep_reproduces_harmonic_polynomials(name):
    fn = HARMONIC[name]
    f = _field(mi.analytic_field(2, 3, fn))
    exact = mi.full_analytic(2, 3, fn)
    _, u_out, _, _ = sw.solve(f, 2, 3, fd.operator_solver(), 80)
    assert np.abs(u_out.numpy() - exact).max() <= 1e-10 * max(1.0, np.abs(exact).max())


def test_fd_sweep_converges_to_global_solve_gp_data():
    f = mi.gp_field(2, 2, length=0.7, seed=11)
    ref = fd.global_solve(f)
    _, u_out, _, _ = sw.solve(_field(f), 2, 2, fd.operator_solver(), 60)
    assert np.abs(u_out.numpy() - ref).max() <= 1e-10


def test_fd_additive_mode_converges():
    f = _field(mi.x2_minus_y2_field(2, 2))
    exact = mi.full_analytic(2, 2, HARMONIC["x2-y2"])
    _, u_out, _, _ = sw.solve(f, 2, 2, fd.operator_solver(), 60, mode="additive")
    assert np.abs(u_out.numpy() - exact).max() <= 1e-10


def test_single_placement_one_sweep_is_exact():
    f = mi.gp_field(1, 1, length=0.5, seed=3)
    ref = fd.global_solve(f)
    u = sw.sweep(_field(f), 1, 1, fd.operator_solver(), kind="interior")
    assert np.abs(u.numpy() - ref).max() <= 1e-13


def test_maximum_principle_every_phase():
    f = mi.gp_field(3, 2, length=0.8, seed=4)
    g = f[[0, -1], :].ravel().tolist() + f[:, [0, -1]].ravel().tolist()
    lo, hi = min(min(g), 0.0), max(max(g), 0.0)
    u = _field(f)
    solver = fd.operator_solver()
    for _ in range(10):
        for c in range(4):
            u = sw.colour_phase(u, 3, 2, c, solver)
            assert u.min().item() >= lo - 1e-13 and u.max().item() <= hi + 1e-13


def test_batched_phase_equals_sequential():
    """Sec. 4.1: batching same-colour placements does not change the result."""
    d = 32
    th = torch.from_numpy(mi.random_params(d, 9).astype(np.float64))
    solver = sw.sdnet_solver(th, d)
    u0 = _field(mi.random_interior_field(3, 3, seed=2))
    a = sw.sweep(u0, 3, 3, solver)
    b = sw.sweep(u0, 3, 3, solver, sequential=True)
    assert torch.linalg.vector_norm(a - b) <= 1e-15 * torch.linalg.vector_norm(b)


def test_cross_and_interior_give_same_skeleton():
    d = 32
    th = torch.from_numpy(mi.random_params(d, 8).astype(np.float64))
    solver = sw.sdnet_solver(th, d)
    u0 = _field(mi.gp_field(2, 2, 0.5, seed=5))
    uc = u0
    ui = u0
    for _ in range(3):
        uc = sw.sweep(uc, 2, 2, solver, "cross")
        ui = sw.sweep(ui, 2, 2, solver, "interior")
        sc, si = sw.skeleton_values(uc), sw.skeleton_values(ui)
        assert torch.linalg.vector_norm(sc - si) <= 1e-15 * torch.linalg.vector_norm(si)


def test_brute_force_two_placement_columns():
    """1 x 2 units (the paper's smallest batched case) by scalar loops with an
    independently built network."""
    d = 16
    th = torch.from_numpy(mi.random_params(d, 3).astype(np.float64))
    seq = torch.nn.Sequential(torch.nn.Linear(130, d), torch.nn.Tanh(),
                              torch.nn.Linear(d, d), torch.nn.Tanh(),
                              torch.nn.Linear(d, d), torch.nn.Tanh(),
                              torch.nn.Linear(d, d), torch.nn.Tanh(),
                              torch.nn.Linear(d, 1)).double()
    off = 0
    with torch.no_grad():
        for m in seq:
            if isinstance(m, torch.nn.Linear):
                for p in (m.weight, m.bias):
                    p.copy_(th[off:off + p.numel()].reshape(p.shape)); off += p.numel()
    f = mi.random_interior_field(1, 2, seed=6)
    u = f.astype(np.float64).copy()
    # placements (0,0),(0,1),(0,2); colours 0, 2, 0 -> phases 0 then 2
    for c in range(4):
        pl = [(a, b) for b in range(3) for a in range(1) if (a % 2) + 2 * (b % 2) == c]
        preds = []
        for (a, b) in pl:
            g = []
            for k in range(128):
                if k < 32:
                    i, j = k, 0
                elif k < 64:
                    i, j = 32, k - 32
                elif k < 96:
                    i, j = 32 - (k - 64), 32
                else:
                    i, j = 0, 32 - (k - 96)
                g.append(u[16 * b + j, 16 * a + i])
            vals = {}
            for (ti, tj) in [(16, j) for j in range(1, 32)] + [(i, 16) for i in range(1, 32) if i != 16]:
                inp = torch.tensor(g + [ti / 32.0, tj / 32.0])
                vals[(16 * a + ti, 16 * b + tj)] = seq(inp).item()
            preds.append(vals)
        for vals in preds:
            for (i, j), v in vals.items():
                u[j, i] = v
    got = sw.sweep(_field(f), 1, 2, sw.sdnet_solver(th, d)).numpy()
    assert np.abs(got - u).max() <= 1e-13


def test_resume_is_bitwise():
    d = 32
    th = torch.from_numpy(mi.random_params(d, 4).astype(np.float64))
    solver = sw.sdnet_solver(th, d)
    u0 = _field(mi.gp_field(2, 2, 0.5, seed=1))
    a, _, _, _ = sw.solve(u0, 2, 2, solver, 5, assemble_out=False)
    b, _, _, _ = sw.solve(u0, 2, 2, solver, 2, assemble_out=False)
    b, _, _, _ = sw.solve(b.clone(), 2, 2, solver, 3, assemble_out=False)
    assert torch.equal(a, b)


def test_delta_definition():
    assert sw.delta(torch.tensor([3.0, 9.0]), torch.tensor([3.0, 4.0])) == pytest.approx(1.0)
    assert sw.delta(torch.tensor([1.0]), torch.tensor([0.0])) == math.inf


def test_solve_stops_on_delta():
    f = _field(mi.x2_minus_y2_field(2, 2))
    u, _, k, last = sw.solve(f, 2, 2, fd.operator_solver(), 200, eps=1e-8, check_every=2)
    assert k < 200 and k % 2 == 0 and last < 1e-8
    # one check earlier the change was still above the threshold
    _, _, k2, last2 = sw.solve(f, 2, 2, fd.operator_solver(), k - 2, eps=1e-8, check_every=2)
    assert k2 == k - 2 and last2 >= 1e-8


def test_assembly_average_of_equal_predictions():
    """With every placement predicting the same exact solution, the
    overlap average returns it (the divisor is the cover count)."""
    f = _field(mi.analytic_field(3, 2, HARMONIC["xy"]))
    exact = _field(mi.full_analytic(3, 2, HARMONIC["xy"]))
    out = sw.assemble(exact, 3, 2, fd.operator_solver())
    assert torch.max(torch.abs(out - exact)) <= 1e-13
    assert torch.equal(out[0], f[0])


def test_assemble_at_matches_full_assembly():
    d = 16
    th = torch.from_numpy(mi.random_params(d, 12).astype(np.float64))
    solver = sw.sdnet_solver(th, d)
    u = _field(mi.random_interior_field(3, 2, seed=4))
    full = sw.assemble(u, 3, 2, solver)
    pts = [(1, 1), (16, 16), (17, 40), (32, 33), (63, 95), (20, 48)]
    part = sw.assemble_at(u, 3, 2, solver, pts)
    want = torch.stack([full[j, i] for (j, i) in pts])
    assert torch.max(torch.abs(part - want)) <= 1e-13
