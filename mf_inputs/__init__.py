"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module only draws random numbers and evaluates boundary functions. It
holds none of the Mosaic Flow arithmetic (no gather, no network, no sweep):
the oracle and the GPU path each implement that on their own and both read
the arrays produced here.

Conventions used by every generator:

* A domain of ``ux`` x ``uy`` units is a vertex-centred grid with 32 cells
  per unit, i.e. ``(32*uy + 1)`` rows by ``(32*ux + 1)`` columns, row-major,
  ``field[j, i]`` sitting at ``(x, y) = (i/32, j/32)`` in units.
* The outer ring holds the Dirichlet data; the interior starts at zero.
* SDNet parameters are one flat float32 vector laid out as
  ``W1 (d x 130) | b1 | W2 (d x d) | b2 | W3 | b3 | W4 | b4 | w5 (d) | b5``,
  every matrix row-major (out, in). Columns 0..127 of W1 act on the
  boundary vector, column 128 on x and column 129 on y.

Everything is rounded to float32 once and then treated as exact: the oracle
upcasts those float32 values to float64.
"""
from __future__ import annotations

import numpy as np

CELLS_PER_UNIT = 32
N_BOUNDARY = 128


def param_count(width: int, n_boundary: int = N_BOUNDARY) -> int:
    d = width
    return d * (n_boundary + 2) + d + 3 * (d * d + d) + d + 1


def xavier_params(width: int, seed: int = 0, n_boundary: int = N_BOUNDARY) -> np.ndarray:
    """Xavier-normal weights, zero biases, drawn layer by layer.

    The draws come from ``numpy.random.default_rng(seed).standard_normal`` in
    the order W1, W2, W3, W4, w5, each row-major (out, in), scaled by
    sqrt(2 / (fan_in + fan_out)).
    """
    d = width
    rng = np.random.default_rng(seed)
    shapes = [(d, n_boundary + 2), (d, d), (d, d), (d, d), (1, d)]
    mats = []
    for out_f, in_f in shapes:
        sigma = np.sqrt(2.0 / (in_f + out_f))
        mats.append(rng.standard_normal((out_f, in_f)) * sigma)
    parts = []
    for li, m in enumerate(mats):
        parts.append(m.reshape(-1))
        nb = m.shape[0]
        parts.append(np.zeros(nb))
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == param_count(width, n_boundary)
    return flat


def random_params(width: int, seed: int, scale: float = 1.0,
                  n_boundary: int = N_BOUNDARY) -> np.ndarray:
    """Xavier-normal weights with non-zero normal biases (scale * N(0, 0.1)).

    Used by tests so that every bias term is exercised.
    """
    flat = xavier_params(width, seed, n_boundary).astype(np.float64)
    rng = np.random.default_rng(seed + 1000)
    d = width
    off = 0
    sizes = [(d * (n_boundary + 2), d), (d * d, d), (d * d, d), (d * d, d), (d, 1)]
    for wsz, bsz in sizes:
        off += wsz
        flat[off:off + bsz] = 0.1 * rng.standard_normal(bsz)
        off += bsz
    return (flat * scale).astype(np.float32)


def conv_param_count(width: int, channels: int, n_boundary: int = N_BOUNDARY, kernel: int = 5) -> int:
    """Flat parameter count of the network with a convolutional boundary
    embedding: Wc1 (C x 1 x k) | bc1 | Wc2 (C x C x k) | bc2 | W1 (d x (C n_b + 2))
    | b1 | W2 | b2 | W3 | b3 | W4 | b4 | w5 | b5."""
    d, C = width, channels
    return C * kernel + C + C * C * kernel + C + d * (C * n_boundary + 2) + d + 3 * (d * d + d) + d + 1


def xavier_conv_params(width: int, channels: int, seed: int = 0, bias_scale: float = 0.0,
                       n_boundary: int = N_BOUNDARY, kernel: int = 5) -> np.ndarray:
    """Xavier-normal weights for the network with a convolutional boundary
    embedding, drawn from ``default_rng(seed).standard_normal`` in the order
    Wc1, Wc2, W1, W2, W3, W4, w5 (each in its row-major layout), scaled by
    sqrt(2 / (fan_in + fan_out)) (a convolution's fans are its channel counts
    times the kernel size). Biases are 0, or, with bias_scale > 0, normal
    with that standard deviation from ``default_rng(seed + 1000)`` in the
    same order (tests use that to exercise every bias)."""
    d, C = width, channels
    E = C * n_boundary
    rng = np.random.default_rng(seed)
    brng = np.random.default_rng(seed + 1000)
    parts = []
    for (shape, fan_in, fan_out) in [((C, 1, kernel), kernel, C * kernel),
                                     ((C, C, kernel), C * kernel, C * kernel),
                                     ((d, E + 2), E + 2, d), ((d, d), d, d), ((d, d), d, d), ((d, d), d, d),
                                     ((1, d), d, 1)]:
        parts.append((rng.standard_normal(shape) * np.sqrt(2.0 / (fan_in + fan_out))).reshape(-1))
        nb = shape[0]
        parts.append(bias_scale * brng.standard_normal(nb) if bias_scale > 0 else np.zeros(nb))
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == conv_param_count(width, channels, n_boundary, kernel)
    return flat


# ----------------------------------------------------------------------------
# Outer-ring enumeration (input side only: which grid points carry data).
# ----------------------------------------------------------------------------

def ring_indices(ux: int, uy: int) -> tuple[np.ndarray, np.ndarray]:
    """(j, i) index arrays of the outer ring, counter-clockwise from (0, 0)."""
    nx, ny = CELLS_PER_UNIT * ux, CELLS_PER_UNIT * uy
    ii, jj = [], []
    ii += list(range(0, nx)); jj += [0] * nx              # bottom, left->right
    ii += [nx] * ny; jj += list(range(0, ny))             # right, bottom->top
    ii += list(range(nx, 0, -1)); jj += [ny] * nx         # top, right->left
    ii += [0] * ny; jj += list(range(ny, 0, -1))          # left, top->bottom
    return np.asarray(jj), np.asarray(ii)


def _field_from_ring(ux: int, uy: int, values: np.ndarray) -> np.ndarray:
    f = np.zeros((CELLS_PER_UNIT * uy + 1, CELLS_PER_UNIT * ux + 1), dtype=np.float64)
    jj, ii = ring_indices(ux, uy)
    f[jj, ii] = values
    return f.astype(np.float32)


def analytic_field(ux: int, uy: int, fn) -> np.ndarray:
    """Ring = fn(x, y) evaluated in units (float64, then rounded); interior 0."""
    jj, ii = ring_indices(ux, uy)
    x = ii / CELLS_PER_UNIT
    y = jj / CELLS_PER_UNIT
    return _field_from_ring(ux, uy, fn(x, y))


def x2_minus_y2_field(ux: int, uy: int) -> np.ndarray:
    return analytic_field(ux, uy, lambda x, y: x * x - y * y)


def full_analytic(ux: int, uy: int, fn) -> np.ndarray:
    """fn evaluated at every grid vertex, float64 (for checks, not inputs)."""
    ny, nx = CELLS_PER_UNIT * uy + 1, CELLS_PER_UNIT * ux + 1
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    return fn(i / CELLS_PER_UNIT, j / CELLS_PER_UNIT)


def _se_cholesky_sample(pts: np.ndarray, length: float, variance: float,
                        z: np.ndarray, jitter: float = 1e-6) -> np.ndarray:
    diff = pts[:, None, :] - pts[None, :, :]
    r2 = np.sum(diff * diff, axis=-1)
    k = variance * np.exp(-r2 / (2.0 * length * length))
    k[np.diag_indices_from(k)] += jitter
    chol = np.linalg.cholesky(k)
    return chol @ z


def gp_ring_values(ux: int, uy: int, length: float, seed: int = 0,
                   variance: float = 1.0, rng: np.random.Generator | None = None) -> np.ndarray:
    """Squared-exponential GP sample on the outer ring.

    The covariance uses the Euclidean distance (in units) between ring
    points, so the sample is continuous around the corners. The sample is
    cholesky(K + 1e-6 I) @ z with z drawn from ``default_rng(seed)`` (or the
    given generator) in ring order.
    """
    jj, ii = ring_indices(ux, uy)
    pts = np.stack([ii / CELLS_PER_UNIT, jj / CELLS_PER_UNIT], axis=1)
    if rng is None:
        rng = np.random.default_rng(seed)
    z = rng.standard_normal(pts.shape[0])
    return _se_cholesky_sample(pts, length, variance, z)


def gp_field(ux: int, uy: int, length: float, seed: int = 0, variance: float = 1.0,
             rng: np.random.Generator | None = None) -> np.ndarray:
    vals = gp_ring_values(ux, uy, length, seed, variance, rng)
    return _field_from_ring(ux, uy, vals)


def expsin_field(ux: int, uy: int) -> np.ndarray:
    """e^x * sin(y) on domain-normalised coordinates, min-max scaled to [0, 1].

    x_hat = x / ux and y_hat = y / uy lie in [0, 1]; the ring values are then
    scaled so that their minimum is 0 and maximum is 1.
    """
    jj, ii = ring_indices(ux, uy)
    xh = ii / (CELLS_PER_UNIT * ux)
    yh = jj / (CELLS_PER_UNIT * uy)
    v = np.exp(xh) * np.sin(yh)
    v = (v - v.min()) / (v.max() - v.min())
    return _field_from_ring(ux, uy, v)


def random_interior_field(ux: int, uy: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Uniform(-scale, scale) everywhere (ring included): a generic test state."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(-scale, scale, size=(CELLS_PER_UNIT * uy + 1, CELLS_PER_UNIT * ux + 1))
    return f.astype(np.float32)


# ----------------------------------------------------------------------------
# Training batches: GP curves on the unit-square perimeter.
# ----------------------------------------------------------------------------

def unit_perimeter_nodes(n_per_side: int = 32) -> np.ndarray:
    """128 perimeter nodes of the unit square, counter-clockwise from (0,0).

    Side k of 4 holds n_per_side nodes and excludes its end corner:
    bottom (s, 0), right (1, s), top (1 - s, 1), left (0, 1 - s) with
    s = 0, 1/n, ..., (n-1)/n.
    """
    s = np.arange(n_per_side) / n_per_side
    bottom = np.stack([s, np.zeros_like(s)], 1)
    right = np.stack([np.ones_like(s), s], 1)
    top = np.stack([1.0 - s, np.ones_like(s)], 1)
    left = np.stack([np.zeros_like(s), 1.0 - s], 1)
    return np.concatenate([bottom, right, top, left], 0)


def gp_perimeter_batch(n_bc: int, length: float, seed: int, variance: float = 1.0) -> np.ndarray:
    """[n_bc x 128] float32 GP samples on the unit-square perimeter nodes."""
    pts = unit_perimeter_nodes()
    diff = pts[:, None, :] - pts[None, :, :]
    k = variance * np.exp(-np.sum(diff * diff, -1) / (2.0 * length * length))
    k[np.diag_indices_from(k)] += 1e-6
    chol = np.linalg.cholesky(k)
    z = np.random.default_rng(seed).standard_normal((n_bc, pts.shape[0]))
    return (z @ chol.T).astype(np.float32)


def collocation_points(n_bc: int, n_pts: int, seed: int) -> np.ndarray:
    """[n_bc x n_pts x 2] float32 points uniform in (0, 1)^2."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(n_bc, n_pts, 2)).astype(np.float32)


# ----------------------------------------------------------------------------
# Batched domains: sizes drawn from one stream, then per-domain GP data.
# ----------------------------------------------------------------------------

def batched_domains(n_domains: int = 48, lo: int = 4, hi: int = 48, length: float = 1.0,
                    seed: int = 7) -> tuple[np.ndarray, list[np.ndarray]]:
    """Sizes and GP ring data for a batch of independent domains.

    One ``default_rng(seed)`` stream draws the (units_x, units_y) pairs, each
    uniform on [lo, hi], then each domain's GP sample in domain order.
    """
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, size=(n_domains, 2))
    fields = [gp_field(int(ux), int(uy), length, rng=rng) for ux, uy in sizes]
    return sizes, fields


# ----------------------------------------------------------------------------
# Named workloads.
# ----------------------------------------------------------------------------

WORKLOADS = {
    "C1": dict(units=(2, 2), width=128, sweeps=50, data="x2-y2", prec="fp32"),
    "C2": dict(units=(16, 16), width=256, sweeps=200, data="gp", length=2.0, seed=1, prec="fp32"),
    "C3": dict(width=128, n_bc=1024, n_colloc=256, length=0.5, bc_seed=2, colloc_seed=3, steps=100),
    "C4": dict(units=(64, 64), width=256, sweeps=500, data="expsin", prec="bf16"),
    "C5": dict(n_domains=48, width=256, sweeps=20, length=1.0, seed=7, ckpt=5, prec="bf16"),
}


def workload_field(name: str) -> np.ndarray:
    w = WORKLOADS[name]
    ux, uy = w["units"]
    if w["data"] == "x2-y2":
        return x2_minus_y2_field(ux, uy)
    if w["data"] == "gp":
        return gp_field(ux, uy, w["length"], w["seed"])
    if w["data"] == "expsin":
        return expsin_field(ux, uy)
    raise ValueError(name)


# ----------------------------------------------------------------------------
# SDNet training data (Sec. 5.1 "Data Generation"): boundary conditions from
# Gaussian processes whose hyperparameters come from a Sobol sequence, and the
# solution of each subdomain problem, which the paper obtains with pyAMG.
# ----------------------------------------------------------------------------

def sobol_gp_perimeter_batch(n_bc: int, seed: int, length_range=(0.25, 2.0),
                             amplitude_range=(0.5, 1.5)) -> tuple[np.ndarray, np.ndarray]:
    """[n_bc x 128] GP samples on the unit-square perimeter nodes, each with
    its own squared-exponential hyperparameters, and those [n_bc x 2]
    (length scale, amplitude).

    A scrambled 2-D Sobol sequence (scipy.stats.qmc, seed) gives (s1, s2)
    per condition; the length scale is log-uniform over ``length_range``
    (l = l_lo (l_hi / l_lo)^s1) and the amplitude (standard deviation)
    uniform over ``amplitude_range``. The kernel uses the Euclidean distance
    between perimeter nodes, as ``gp_perimeter_batch`` does, and the sample
    is cholesky(K + 1e-6 I) z with z from default_rng(seed + 1).
    """
    import warnings

    from scipy.stats import qmc
    pts = unit_perimeter_nodes()
    diff = pts[:, None, :] - pts[None, :, :]
    r2 = np.sum(diff * diff, -1)
    with warnings.catch_warnings():   # balance is exact only for powers of two; any n is valid
        warnings.simplefilter("ignore", UserWarning)
        s = qmc.Sobol(d=2, scramble=True, seed=seed).random(n_bc)
    lo, hi = length_range
    ell = lo * (hi / lo) ** s[:, 0]
    amp = amplitude_range[0] + (amplitude_range[1] - amplitude_range[0]) * s[:, 1]
    z = np.random.default_rng(seed + 1).standard_normal((n_bc, pts.shape[0]))
    out = np.empty((n_bc, pts.shape[0]))
    eye = 1e-6 * np.eye(pts.shape[0])
    for b in range(n_bc):
        chol = np.linalg.cholesky(amp[b] ** 2 * np.exp(-r2 / (2.0 * ell[b] ** 2)) + eye)
        out[b] = chol @ z[b]
    return out.astype(np.float32), np.stack([ell, amp], 1)


def perimeter_grid_indices(cells: int = CELLS_PER_UNIT) -> tuple[np.ndarray, np.ndarray]:
    """(j, i) grid indices of the 128 perimeter nodes on a (cells+1)^2 grid,
    in the boundary-vector order of ``unit_perimeter_nodes``."""
    p = np.rint(unit_perimeter_nodes(cells) * cells).astype(np.int64)
    return p[:, 1], p[:, 0]


def subdomain_solutions(G: np.ndarray, cells: int = CELLS_PER_UNIT) -> np.ndarray:
    """[B x (cells+1) x (cells+1)] float64 grids: ring = the boundary vectors
    G [B x 4 cells] (corners included), interior = the solution of the
    5-point discrete Laplace equation with that Dirichlet ring.

    Training targets for the data loss (the paper solves each boundary value
    problem with pyAMG; here the 5-point system on the square is solved
    exactly by diagonalisation: the discrete sine transform (type I) turns
    the operator 4 u - (the four neighbours) into multiplication by
    4 sin^2(p pi / 2n) + 4 sin^2(q pi / 2n), n = cells)."""
    from scipy.fft import dstn, idstn
    G = np.asarray(G, dtype=np.float64)
    B = G.shape[0]
    n = cells
    U = np.zeros((B, n + 1, n + 1))
    jj, ii = perimeter_grid_indices(cells)
    U[:, jj, ii] = G
    rhs = np.zeros((B, n - 1, n - 1))
    rhs[:, 0, :] += U[:, 0, 1:-1]
    rhs[:, -1, :] += U[:, -1, 1:-1]
    rhs[:, :, 0] += U[:, 1:-1, 0]
    rhs[:, :, -1] += U[:, 1:-1, -1]
    k = np.arange(1, n)
    s2 = 4.0 * np.sin(k * np.pi / (2.0 * n)) ** 2
    lam = s2[:, None] + s2[None, :]
    U[:, 1:-1, 1:-1] = idstn(dstn(rhs, type=1, axes=(1, 2)) / lam, type=1, axes=(1, 2))
    return U


def training_set(n_bc: int, n_data: int, n_colloc: int, seed: int, cells: int = CELLS_PER_UNIT):
    """A seeded SDNet training set of n_bc boundary conditions
    (``sobol_gp_perimeter_batch``), each with n_data data points drawn
    without replacement from its (cells+1)^2 grid nodes (coordinates in
    [0, 1]^2) and their exact values (``subdomain_solutions``), and n_colloc
    collocation points uniform in (0, 1)^2. Returns float32 arrays
    G [n_bc, 128], Xd [n_bc, n_data, 2], Yd [n_bc, n_data],
    Xc [n_bc, n_colloc, 2] and the hyperparameters [n_bc, 2]."""
    G, hyper = sobol_gp_perimeter_batch(n_bc, seed)
    U = subdomain_solutions(G, cells)
    rng = np.random.default_rng(seed + 2)
    nodes = (cells + 1) ** 2
    idx = np.stack([rng.choice(nodes, n_data, replace=False) for _ in range(n_bc)])
    jj, ii = idx // (cells + 1), idx % (cells + 1)
    Xd = np.stack([ii / cells, jj / cells], -1)
    Yd = np.take_along_axis(U.reshape(n_bc, -1), idx, 1)
    Xc = rng.uniform(0.0, 1.0, size=(n_bc, n_colloc, 2))
    f32 = np.float32
    return G, Xd.astype(f32), Yd.astype(f32), Xc.astype(f32), hyper
