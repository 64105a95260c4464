"""GPU parity of sdnet_forward (Sec. 2.2: N(x, g; theta)) against the
float64 oracle network, through the C ABI."""
import numpy as np
import pytest
import torch

import mf_inputs as mi
from oracle import sdnet
from paper_2308_14258_amd import MF_BF16, MF_FP16, MF_FP32, Context, sdnet_forward

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("width", [128, 256])
@pytest.mark.parametrize("shape", [(1, 1), (7, 61), (33, 5), (300, 97)])
@pytest.mark.parametrize("per_bc", [False, True])
def test_forward_matches_oracle(ctx, width, shape, per_bc):
    n_bc, n_pts = shape
    print(f"case: forward width={width} shape={shape} per_bc={per_bc}", flush=True)
    params = mi.random_params(width, seed=11)
    rng = np.random.default_rng(n_bc * 1000 + n_pts)
    G = rng.standard_normal((n_bc, 128)).astype(np.float32)
    X = rng.uniform(size=(n_bc, n_pts, 2) if per_bc else (n_pts, 2)).astype(np.float32)
    U = sdnet_forward(ctx, torch.from_numpy(params).cuda(), torch.from_numpy(G).cuda(),
                      torch.from_numpy(X).cuda(), MF_FP32)
    layers = sdnet.unpack(torch.from_numpy(params.astype(np.float64)), width)
    want = sdnet.forward(layers, torch.from_numpy(G.astype(np.float64)),
                         torch.from_numpy(X.astype(np.float64))).numpy()
    assert U.shape == (n_bc, n_pts)
    assert _rel(U.cpu().numpy(), want) <= 1e-5


@pytest.mark.parametrize("prec,tol", [(MF_BF16, 2e-2), (MF_FP16, 5e-3)])
@pytest.mark.parametrize("width", [128, 256])
def test_forward_bf16_error(ctx, width, prec, tol):
    print(f"case: forward prec {prec} width={width}", flush=True)
    params = mi.xavier_params(width, 0)
    rng = np.random.default_rng(5)
    G = rng.standard_normal((64, 128)).astype(np.float32)
    X = rng.uniform(size=(61, 2)).astype(np.float32)
    U = sdnet_forward(ctx, torch.from_numpy(params).cuda(), torch.from_numpy(G).cuda(),
                      torch.from_numpy(X).cuda(), prec)
    layers = sdnet.unpack(torch.from_numpy(params.astype(np.float64)), width)
    want = sdnet.forward(layers, torch.from_numpy(G.astype(np.float64)),
                         torch.from_numpy(X.astype(np.float64))).numpy()
    err = _rel(U.cpu().numpy(), want)
    print(f"forward prec {prec} width {width}: rel L2 {err:.3e}", flush=True)
    assert err <= tol


def test_forward_empty(ctx):
    params = torch.from_numpy(mi.xavier_params(128, 0)).cuda()
    U = sdnet_forward(ctx, params, torch.zeros(0, 128, device="cuda", dtype=torch.float32),
                      torch.zeros(5, 2, device="cuda", dtype=torch.float32))
    assert U.shape == (0, 5)
