"""Train an SDNet for the Laplace equation on one GPU (Sec. 5.1-5.2).

Data (Sec. 5.1, ``mf_inputs.training_set``): boundary conditions drawn from
Gaussian processes whose length scale and amplitude come from a Sobol
sequence; for each, the exact 5-point solution of the subdomain problem
(the paper solves these with pyAMG) at randomly chosen grid nodes of the
33 x 33 subdomain (data loss) and random collocation points (Laplacian
loss). 90% of the conditions train, 10% validate.

Optimisation (Sec. 5.2): each iteration is one call of the library's
``sdnet_train_step`` (Alg. 1 on one device: data pass, collocation pass,
summed gradient, then the fused Adam update); the learning rate rises
linearly to its maximum over the first 0.1% of the iterations and then
decays linearly (polynomial decay with exponent one) to zero. Weight decay
is zero.

Validation: ``sdnet_forward`` at all 33 x 33 grid nodes of the held-out
conditions against their exact solutions (mean squared error).

    python -m paper_2308_14258_amd.sdnet_training --width 256 --epochs 500 --out weights.npz

With --optimizer lamb each iteration is ``sdnet_loss_grad`` (the same Alg. 1
passes) followed by ``sdnet_lamb_step`` (LAMB with the per-tensor trust
ratio and the gradient clipped to norm 1, the optimiser the paper names for
large batches) at the library's schedule (``lr_at``).

With --channels C (1..8) the network is the paper's (Sec. 3.1): a circular
convolutional embedding of the boundary with C channels and GELU layers;
without it, the tanh network. The weights file holds the flat float32
parameter vector in the library's layout, the width, the training
configuration and the loss history.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WEIGHTS_DIR = os.path.join(HERE, "weights")


def lr_at(it: int, total: int, lr_max: float, warmup_frac: float = 1e-3) -> float:
    """Linear warm-up over the first warmup_frac of the iterations, then
    linear decay to zero at the last iteration (it counts from 1)."""
    warm = max(1, int(round(warmup_frac * total)))
    if it <= warm:
        return lr_max * it / warm
    return lr_max * max(0.0, (total - it + 1) / (total - warm + 1))


def grid_nodes(cells: int = 32) -> np.ndarray:
    """[(cells+1)^2, 2] coordinates (i / cells, j / cells), row by row."""
    j, i = np.meshgrid(np.arange(cells + 1), np.arange(cells + 1), indexing="ij")
    return np.stack([i.reshape(-1) / cells, j.reshape(-1) / cells], 1).astype(np.float32)


def train(width: int = 256, n_bc: int = 20480, n_data: int = 128, n_colloc: int = 128, batch: int = 512,
          epochs: int = 500, lr: float = 1e-3, seed: int = 0, val_every: int = 25, log=print, channels: int = 0,
          optimizer: str = "adam"):
    """Returns (params [float32 numpy], history dict)."""
    import torch

    import mf_inputs as mi
    from paper_2308_14258_amd import (Context, lr_at as sched_lr, lr_schedule, sdnet_forward, sdnet_lamb_step,
                                      sdnet_loss_grad, sdnet_train_step)

    t0 = time.perf_counter()
    G, Xd, Yd, Xc, hyper = mi.training_set(n_bc, n_data, n_colloc, seed)
    n_val = n_bc // 10
    n_tr = (n_bc - n_val) // batch * batch
    Gv = G[n_bc - n_val:]
    Uv = mi.subdomain_solutions(Gv).reshape(n_val, -1).astype(np.float32)
    gen_s = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    d = {k: torch.from_numpy(np.ascontiguousarray(a)).to(dev) for k, a in
         (("G", G[:n_tr]), ("Xd", Xd[:n_tr]), ("Yd", Yd[:n_tr]), ("Xc", Xc[:n_tr]), ("Gv", Gv), ("Uv", Uv),
          ("Xv", grid_nodes()))}
    ctx = Context(0)
    init = mi.xavier_conv_params(width, channels, seed) if channels else mi.xavier_params(width, seed)
    p = torch.from_numpy(init).to(dev)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    loss = torch.empty(3, device=dev)
    steps_per_epoch = n_tr // batch
    total = steps_per_epoch * epochs
    hist = {"epoch": [], "loss_data": [], "loss_pde": [], "val_mse": [], "seconds": []}
    grad = torch.empty_like(p)
    sched = lr_schedule(lr, total, warmup_frac=1e-3)

    def validate():
        U = sdnet_forward(ctx, p, d["Gv"], d["Xv"])
        return float(((U - d["Uv"]) ** 2).mean().item())

    it = 0
    t1 = time.perf_counter()
    for ep in range(1, epochs + 1):
        acc = torch.zeros(3, device=dev)
        for s in range(steps_per_epoch):
            it += 1
            sl = slice(s * batch, (s + 1) * batch)
            if optimizer == "lamb":
                sdnet_loss_grad(ctx, p, d["G"][sl], d["Xd"][sl], d["Xc"][sl], loss=loss, grad_out=grad,
                                Yd=d["Yd"][sl])
                sdnet_lamb_step(ctx, p, m, v, grad, it, lr=sched_lr(sched, it), max_grad_norm=1.0)
            else:
                sdnet_train_step(ctx, p, m, v, it, d["G"][sl], d["Xd"][sl], d["Xc"][sl], lr=lr_at(it, total, lr),
                                 loss=loss, Yd=d["Yd"][sl])
            acc += loss
        if ep % val_every == 0 or ep == epochs or ep == 1:
            acc = (acc / steps_per_epoch).cpu().numpy()
            val = validate()
            hist["epoch"].append(ep)
            hist["loss_data"].append(float(acc[0]))
            hist["loss_pde"].append(float(acc[1]))
            hist["val_mse"].append(val)
            hist["seconds"].append(time.perf_counter() - t1)
            log(f"epoch {ep}: L_data {acc[0]:.3e} L_pde {acc[1]:.3e} val MSE {val:.3e} "
                f"({time.perf_counter() - t1:.0f} s)")
    torch.cuda.synchronize()
    hist["train_s"] = time.perf_counter() - t1
    hist["data_generation_s"] = gen_s
    hist["iterations"] = total
    out = p.cpu().numpy()
    ctx.close()
    return out, hist


def save(path: str, params: np.ndarray, width: int, config: dict, hist: dict) -> None:
    np.savez_compressed(path, params=params.astype(np.float32), width=np.int32(width),
                        config=json.dumps(config), history=json.dumps(hist))


def load_trained(path: str):
    """(params [float32], width, config, history) from a weights file written
    by ``save`` (plain arrays and JSON text; nothing is unpickled)."""
    z = np.load(path, allow_pickle=False)
    return (z["params"], int(z["width"]), json.loads(str(z["config"])), json.loads(str(z["history"])))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--width", type=int, default=256)
    ap.add_argument("--n-bc", type=int, default=20480)
    ap.add_argument("--n-data", type=int, default=128)
    ap.add_argument("--n-colloc", type=int, default=128)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--epochs", type=int, default=500)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--val-every", type=int, default=25)
    ap.add_argument("--channels", type=int, default=0, help="embedding channels (0: the tanh network)")
    ap.add_argument("--optimizer", choices=["adam", "lamb"], default="adam")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    cfg = {k: getattr(a, k) for k in ("width", "n_bc", "n_data", "n_colloc", "batch", "epochs", "lr", "seed",
                                      "channels", "optimizer")}
    params, hist = train(a.width, a.n_bc, a.n_data, a.n_colloc, a.batch, a.epochs, a.lr, a.seed, a.val_every,
                         log=lambda s: print(s, flush=True), channels=a.channels, optimizer=a.optimizer)
    save(a.out, params, a.width, cfg, hist)
    print(json.dumps({"out": a.out, "val_mse": hist["val_mse"][-1], "train_s": hist["train_s"]}), flush=True)


if __name__ == "__main__":
    main()
