"""Pins for the oracle's sensitivity dJ/du0 through K sweeps and the assembly.

With the exact 5-point subdomain solver the sweep is linear, so J is a
quadratic form in u0: central differences are exact up to rounding, and the
map M: u0 -> u_out satisfies <M v, w> = <v, M^T w>.
"""
import numpy as np
import torch

import mf_inputs as mi
from oracle import adjoint, fd, sweep as sw



def _J(u0, ux, uy, solver, K):
    u = u0
    for _ in range(K):
        u = sw.sweep(u, ux, uy, solver)
    return adjoint.objective(sw.assemble(u, ux, uy, solver)).item()


def test_linear_case_exact_directional_derivatives():
    solver = fd.operator_solver()
    u0 = torch.from_numpy(mi.gp_field(2, 1, 0.5, seed=8).astype(np.float64))
    J, g = adjoint.solve_adjoint(u0, 2, 1, solver, K=3)
    rng = np.random.default_rng(1)
    for _ in range(4):
        v = torch.from_numpy(rng.standard_normal(u0.shape))
        h = 1e-3
        fdv = (_J(u0 + h * v, 2, 1, solver, 3) - _J(u0 - h * v, 2, 1, solver, 3)) / (2 * h)
        assert abs(fdv - torch.sum(g * v).item()) <= 1e-9 * max(1.0, abs(fdv))


def test_linear_case_dot_product():
    solver = fd.operator_solver()
    shape = (33, 65)

    def M(u0):
        u = u0
        for _ in range(2):
            u = sw.sweep(u, 2, 1, solver)
        return sw.assemble(u, 2, 1, solver)

    rng = np.random.default_rng(2)
    v = torch.from_numpy(rng.standard_normal(shape))
    w = torch.from_numpy(rng.standard_normal(shape))
    x = v.clone().requires_grad_(True)
    Mv = M(x)
    (MTw,) = torch.autograd.grad(Mv, x, grad_outputs=w)
    lhs = torch.sum(Mv.detach() * w).item()
    rhs = torch.sum(v * MTw).item()
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_sdnet_case_directional_derivatives():
    d = 16
    th = torch.from_numpy(mi.random_params(d, 6).astype(np.float64))
    solver = sw.sdnet_solver(th, d)
    u0 = torch.from_numpy(mi.gp_field(1, 2, 0.5, seed=9).astype(np.float64))
    J, g = adjoint.solve_adjoint(u0, 1, 2, solver, K=2)
    rng = np.random.default_rng(3)
    for _ in range(4):
        v = torch.from_numpy(rng.standard_normal(u0.shape))
        h = 1e-5
        fdv = (_J(u0 + h * v, 1, 2, solver, 2) - _J(u0 - h * v, 1, 2, solver, 2)) / (2 * h)
        an = torch.sum(g * v).item()
        assert abs(fdv - an) <= 1e-6 * max(1.0, abs(an))


def test_linear_case_seeded_adjoint_equals_explicit_transpose():
    """u0_bar = M^T seed with M: u0 -> u_out built column by column (brute
    force: one forward run per grid point) for the exact linear solver."""
    solver = fd.operator_solver()
    ux, uy, K = 2, 1, 2
    shape = (33, 65)
    n = shape[0] * shape[1]

    def M(u0):
        u = u0
        for _ in range(K):
            u = sw.sweep(u, ux, uy, solver)
        return sw.assemble(u, ux, uy, solver)

    cols = np.empty((n, n))
    for k in range(n):
        e = torch.zeros(n, dtype=torch.float64)
        e[k] = 1.0
        cols[:, k] = M(e.reshape(shape)).reshape(-1).numpy()
    seed = np.random.default_rng(4).standard_normal(shape)
    u0 = torch.from_numpy(mi.gp_field(ux, uy, 0.5, seed=3).astype(np.float64))
    _, g = adjoint.solve_adjoint(u0, ux, uy, solver, K, uout_bar=torch.from_numpy(seed))
    want = (cols.T @ seed.reshape(-1)).reshape(shape)
    assert np.max(np.abs(g.numpy() - want)) <= 1e-12 * np.max(np.abs(want))


def test_sdnet_case_seeded_directional_derivatives():
    """<u0_bar, v> = d/dh <seed, u_out(u0 + h v)> by central differences."""
    d = 16
    th = torch.from_numpy(mi.random_params(d, 7).astype(np.float64))
    solver = sw.sdnet_solver(th, d)
    ux, uy, K = 2, 1, 2
    u0 = torch.from_numpy(mi.gp_field(ux, uy, 0.5, seed=10).astype(np.float64))
    rng = np.random.default_rng(5)
    seed = torch.from_numpy(rng.standard_normal(u0.shape))
    _, g = adjoint.solve_adjoint(u0, ux, uy, solver, K, uout_bar=seed)

    def J(u):
        for _ in range(K):
            u = sw.sweep(u, ux, uy, solver)
        return torch.sum(seed * sw.assemble(u, ux, uy, solver)).item()

    for _ in range(4):
        v = torch.from_numpy(rng.standard_normal(u0.shape))
        h = 1e-5
        fdv = (J(u0 + h * v) - J(u0 - h * v)) / (2 * h)
        an = torch.sum(g * v).item()
        assert abs(fdv - an) <= 1e-6 * max(1.0, abs(an))


def test_default_objective_is_the_seed_two_u_out():
    d = 16
    th = torch.from_numpy(mi.random_params(d, 8).astype(np.float64))
    solver = sw.sdnet_solver(th, d)
    u0 = torch.from_numpy(mi.gp_field(1, 2, 0.5, seed=11).astype(np.float64))
    _, g_default = adjoint.solve_adjoint(u0, 1, 2, solver, 2)
    u = u0
    for _ in range(2):
        u = sw.sweep(u, 1, 2, solver)
    u_out = sw.assemble(u, 1, 2, solver)
    seed = torch.zeros_like(u_out)
    seed[1:-1, 1:-1] = 2.0 * u_out[1:-1, 1:-1]
    _, g_seed = adjoint.solve_adjoint(u0, 1, 2, solver, 2, uout_bar=seed)
    assert torch.allclose(g_seed, g_default, rtol=1e-12, atol=1e-14)
