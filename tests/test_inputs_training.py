"""The SDNet training-data generator (Sec. 5.1): its exact subdomain
solutions are checked against the oracle's independently built 5-point
solver (sparse LU, a different method from the generator's sine-transform
diagonalisation) and against data that is exactly discrete-harmonic."""
import numpy as np

import mf_inputs as mi
from oracle import fd


def test_subdomain_solutions_equal_the_oracle_operator():
    G, _ = mi.sobol_gp_perimeter_batch(64, seed=11)
    U = mi.subdomain_solutions(G)
    want = G.astype(np.float64) @ fd.subdomain_operator_np().T
    assert np.max(np.abs(U[:, 1:-1, 1:-1].reshape(64, -1) - want)) <= 1e-12 * np.abs(want).max()
    jj, ii = mi.perimeter_grid_indices()
    np.testing.assert_array_equal(U[:, jj, ii], G.astype(np.float64))


def test_discrete_harmonic_data_is_reproduced():
    """x^2 - y^2 and x y are exactly discrete-harmonic for the 5-point
    stencil: the interior must equal them."""
    nodes = mi.unit_perimeter_nodes()
    x, y = nodes[:, 0], nodes[:, 1]
    j, i = np.meshgrid(np.arange(33), np.arange(33), indexing="ij")
    X, Y = i / 32.0, j / 32.0
    for f in (lambda a, b: a * a - b * b, lambda a, b: a * b, lambda a, b: 3 * a * a * b - b ** 3):
        U = mi.subdomain_solutions(f(x, y)[None])[0]
        assert np.max(np.abs(U - f(X, Y))) <= 1e-13


def test_sobol_hyperparameters_and_determinism():
    G1, h1 = mi.sobol_gp_perimeter_batch(256, seed=3)
    G2, h2 = mi.sobol_gp_perimeter_batch(256, seed=3)
    np.testing.assert_array_equal(G1, G2)
    assert h1[:, 0].min() >= 0.25 and h1[:, 0].max() <= 2.0
    assert h1[:, 1].min() >= 0.5 and h1[:, 1].max() <= 1.5
    # low-discrepancy coverage: every quarter of each (scaled) range is hit
    s1 = np.log(h1[:, 0] / 0.25) / np.log(8.0)
    s2 = h1[:, 1] - 0.5
    for s in (s1, s2):
        counts = np.histogram(s, bins=4, range=(0.0, 1.0))[0]
        assert counts.min() >= 48


def test_training_set_shapes_and_values():
    G, Xd, Yd, Xc, hyper = mi.training_set(8, 40, 16, seed=4)
    assert G.shape == (8, 128) and Xd.shape == (8, 40, 2) and Yd.shape == (8, 40) and Xc.shape == (8, 16, 2)
    U = mi.subdomain_solutions(G)
    ii = np.rint(Xd[..., 0] * 32).astype(int)
    jj = np.rint(Xd[..., 1] * 32).astype(int)
    for b in range(8):
        np.testing.assert_allclose(Yd[b], U[b, jj[b], ii[b]].astype(np.float32))
        assert len(set(zip(ii[b], jj[b]))) == 40
    assert Xc.min() >= 0.0 and Xc.max() <= 1.0


def test_learning_rate_schedule():
    """Linear warm-up over 0.1% of the iterations to the maximum, then linear
    decay to zero (Sec. 5.2's polynomial decay with exponent one)."""
    from paper_2308_14258_amd.sdnet_training import lr_at
    total = 10000
    assert lr_at(1, total, 1e-3) == 1e-3 / 10
    assert lr_at(10, total, 1e-3) == 1e-3
    lrs = [lr_at(i, total, 1e-3) for i in range(10, total + 1)]
    assert all(a >= b for a, b in zip(lrs, lrs[1:]))
    assert lr_at(total, total, 1e-3) == 1e-3 / (total - 10 + 1)
    assert abs(lr_at(5005, total, 1e-3) - 1e-3 * (total - 5005 + 1) / (total - 10 + 1)) < 1e-18
