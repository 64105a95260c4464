"""A trained SDNet (paper_2308_14258_amd/weights/sdnet_laplace_d256.npz,
written by paper_2308_14258_amd.sdnet_training on one MI355X: width 256,
tanh, 18,432 Sobol-sampled GP boundary conditions with exact subdomain
solutions, 3000 epochs) and the predictor's accuracy with it, through the
C ABI (Sec. 5.1-5.3, Fig. 1, Table 4).

Ground truth is the oracle's global 5-point solve of the same Dirichlet
data (tests/golden/mfp_global.npz); the network's weights are used by the
GPU only. Measured when these bars were set: validation MSE 3.7e-3; 4x4
units, MAE 1.8e-3 against the global solve (float64 oracle with the same
weights); 64x64 units, MAE 0.0441 after 2000 sweeps in float32."""
import os

import numpy as np
import pytest
import torch

import mf_inputs as mi
from paper_2308_14258_amd import MF_BF16, MF_FP16, MF_FP32, Context, mf_solve, sdnet_forward
from paper_2308_14258_amd.sdnet_training import WEIGHTS_DIR, grid_nodes, load_trained

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def net():
    params, width, cfg, hist = load_trained(os.path.join(WEIGHTS_DIR, "sdnet_laplace_d256.npz"))
    assert width == 256 and params.size == mi.param_count(256)
    return torch.from_numpy(params).cuda(), hist


def test_validation_error(ctx, net):
    """Held-out boundary conditions (the training set's generator with
    another seed) at all 33 x 33 grid nodes against the exact subdomain
    solutions."""
    print("case: trained network validation", flush=True)
    p, hist = net
    G, _ = mi.sobol_gp_perimeter_batch(1024, seed=99)
    U = sdnet_forward(ctx, p, torch.from_numpy(G).cuda(), torch.from_numpy(grid_nodes()).cuda())
    want = mi.subdomain_solutions(G).reshape(1024, -1)
    mse = float(np.mean((U.cpu().numpy().astype(np.float64) - want) ** 2))
    print(f"trained network: MSE on 1024 new conditions {mse:.3e} (training log: {hist['val_mse'][-1]:.3e})",
          flush=True)
    assert mse <= 6e-3


@pytest.mark.parametrize("prec,bar", [(MF_FP32, 5e-3), (MF_BF16, 5e-2), (MF_FP16, 1e-2)])
def test_fig1_analogue_mae(ctx, net, prec, bar):
    """4 x 4 units (129 x 129 grid), GP ring data (length 1, seed 31): MAE of
    the assembly after 100 sweeps against the global solve. Float32 is held
    to 5e-3 (measured 1.8e-3); BF16, whose rounding of the network's inputs
    and activations alone moves each prediction by ~1e-2, to the paper's
    MAE target of 0.05 (measured 1.8e-2); FP16, which rounds the hidden
    layers' operands 8x more finely, to 1e-2."""
    print(f"case: trained MFP 4x4 prec={prec}", flush=True)
    p, _ = net
    g = np.load(os.path.join(HERE, "golden", "mfp_global.npz"))
    f = mi.gp_field(4, 4, 1.0, seed=31)
    u = torch.from_numpy(f).cuda()
    uo = torch.empty_like(u)
    mf_solve(ctx, p, u, (4, 4), 100, prec=prec, u_out=uo)
    torch.cuda.synchronize()
    err = np.abs(uo.cpu().numpy().astype(np.float64) - g["u4"])[1:-1, 1:-1]
    print(f"4x4 units prec={prec}: MAE {err.mean():.4e}, max {err.max():.3e}", flush=True)
    assert err.mean() <= bar


def test_table4_analogue_mae(ctx, net):
    """64 x 64 units (2049 x 2049 grid, 16,129 placements), GP ring data
    (length 2, seed 41): float32 MAE against the global solve at 65,536
    sampled points, after 500 and 2000 sweeps; the 16-bit forms reported, FP16
    held below BF16 (its finer operand rounding drifts less)."""
    print("case: trained MFP 64x64", flush=True)
    p, _ = net
    g = np.load(os.path.join(HERE, "golden", "mfp_global.npz"))
    f = mi.gp_field(64, 64, 2.0, seed=41)
    res = {}
    for prec in (MF_FP32, MF_BF16, MF_FP16):
        u = torch.from_numpy(f).cuda()
        uo = torch.empty_like(u)
        done = 0
        for k in (500, 2000):
            mf_solve(ctx, p, u, (64, 64), k - done, prec=prec, u_out=uo)
            done = k
            torch.cuda.synchronize()
            res[(prec, k)] = float(np.mean(np.abs(uo.cpu().numpy()[g["sample_j"], g["sample_i"]] - g["u64_sample"])))
    print(f"64x64 units MAE: fp32 {res[(MF_FP32, 500)]:.4f} @500, {res[(MF_FP32, 2000)]:.4f} @2000; "
          f"bf16 {res[(MF_BF16, 500)]:.4f} @500, {res[(MF_BF16, 2000)]:.4f} @2000; "
          f"fp16 {res[(MF_FP16, 500)]:.4f} @500, {res[(MF_FP16, 2000)]:.4f} @2000", flush=True)
    assert res[(MF_FP32, 2000)] <= 0.05
    assert res[(MF_FP32, 2000)] <= res[(MF_FP32, 500)]
    assert np.isfinite(res[(MF_BF16, 2000)])
    assert res[(MF_FP16, 2000)] < res[(MF_BF16, 2000)]


@pytest.fixture(scope="module")
def gelu_net():
    params, width, cfg, hist = load_trained(os.path.join(WEIGHTS_DIR, "sdnet_laplace_gelu_c4_d256.npz"))
    assert width == 256 and cfg["channels"] == 4 and params.size == mi.conv_param_count(256, 4)
    return torch.from_numpy(params).cuda(), hist


def test_papers_network_trained(ctx, gelu_net):
    """The paper's network (convolutional embedding with 4 channels, GELU,
    width 256; weights/sdnet_laplace_gelu_c4_d256.npz, trained like the tanh
    network with the same data, 3000 epochs): held-out MSE (measured 1.3e-3,
    below the tanh network's 3.7e-3), the 4 x 4-unit problem after 100
    sweeps (MAE 2.8e-3) and the 64 x 64-unit problem at its best, 300 sweeps
    (MAE 0.070). Unlike the tanh network's, its iteration on 64 x 64 units
    does not settle: the MAE grows again after 300 sweeps (0.40 at 2000), so
    only the early value is held to a bar."""
    print("case: trained paper network (conv + GELU)", flush=True)
    p, hist = gelu_net
    G, _ = mi.sobol_gp_perimeter_batch(1024, seed=99)
    U = sdnet_forward(ctx, p, torch.from_numpy(G).cuda(), torch.from_numpy(grid_nodes()).cuda())
    want = mi.subdomain_solutions(G).reshape(1024, -1)
    mse = float(np.mean((U.cpu().numpy().astype(np.float64) - want) ** 2))
    g = np.load(os.path.join(HERE, "golden", "mfp_global.npz"))
    u = torch.from_numpy(mi.gp_field(4, 4, 1.0, seed=31)).cuda()
    uo = torch.empty_like(u)
    mf_solve(ctx, p, u, (4, 4), 100, u_out=uo)
    torch.cuda.synchronize()
    mae4 = float(np.abs(uo.cpu().numpy().astype(np.float64) - g["u4"])[1:-1, 1:-1].mean())
    u = torch.from_numpy(mi.gp_field(64, 64, 2.0, seed=41)).cuda()
    uo = torch.empty_like(u)
    mf_solve(ctx, p, u, (64, 64), 300, u_out=uo)
    torch.cuda.synchronize()
    mae64 = float(np.mean(np.abs(uo.cpu().numpy()[g["sample_j"], g["sample_i"]] - g["u64_sample"])))
    print(f"paper's network: MSE on 1024 new conditions {mse:.3e} (training log {hist['val_mse'][-1]:.3e}); "
          f"4x4 MAE {mae4:.4e}; 64x64 MAE after 300 sweeps {mae64:.4f}", flush=True)
    assert mse <= 2.5e-3
    assert mae4 <= 5e-3
    assert mae64 <= 0.08
