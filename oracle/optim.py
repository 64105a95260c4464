"""The large-batch optimiser and learning-rate schedule of the SDNet training
(Sec. 5.2, "Hyperparameters") in float64 (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper trains with LAMB (You et al., "Large Batch Optimization for Deep
Learning: Training BERT in 76 minutes", ICLR 2020), a learning rate that
warms up linearly over a fraction of the iterations and then decays
polynomially (exponent one: linearly) to zero, and, when the batch grows by
a factor k on k times more devices, scales the peak learning rate by sqrt(k)
and the warm-up fraction by k.

LAMB, one step t (counting from 1), for every parameter tensor ("layer") s:

    m = beta1 m + (1 - beta1) g,   v = beta2 v + (1 - beta2) g^2
    u = (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps) + lambda w
    r_s = ||w_s|| / ||u_s||        (1 when either norm is zero)
    w_s = w_s - lr r_s u_s

with the scaling function phi of the LAMB paper taken as the identity.
Readings where the paper is silent (it names NVIDIA Apex's FusedLAMB and
its settings, not the update):

* the gradient may first be scaled as a whole by min(1, max_grad_norm /
  ||g||) (global-norm clipping; max_grad_norm = 0: off);
* the trust ratio is applied to every tensor (LAMB as published) or, with
  trust_without_decay off, only when weight decay is non-zero; the paper's
  weight decay is zero, so in that mode its update is Adam on the clipped
  gradient;
* the tensors ("layers") are the weight matrices and bias vectors of the
  parameter layout, each on its own.

The schedule, for total iterations T and W = ceil(warmup_frac T) warm-up
iterations: lr(t) = max_lr t / W for t <= W, then end_lr + (max_lr - end_lr)
(1 - (t - W) / (T - W))^power up to t = T, end_lr afterwards.

Pins (tests/test_oracle_optim.py): without the trust ratio LAMB is
torch.optim.Adam, and with clipping it is Adam on the gradient that
torch.nn.utils.clip_grad_norm_ scales; the trust ratio makes every tensor's
step exactly lr ||w_s|| long; with eps = 0 the step does not change when the
gradient is scaled; tensors do not interact; the schedule's warm-up is
torch's LinearLR and its decay torch's PolynomialLR. ``scaled_schedule`` is
parity unpinned: the paper states the two rules without a worked value.
"""
from __future__ import annotations

import math

import torch

from . import sdnet_conv


def tanh_segments(width: int, n_boundary: int = 128):
    """Tensor boundaries of the tanh network's flat vector (``sdnet``):
    begin offsets of W1, b1, W2, b2, W3, b3, W4, b4, w5, b5 and the end."""
    d = width
    begins, off = [0], 0
    for out_f, in_f in [(d, n_boundary + 2)] + [(d, d)] * 3 + [(1, d)]:
        off += out_f * in_f
        begins.append(off)
        off += out_f
        begins.append(off)
    return begins


def conv_segments(width: int, channels: int):
    """Tensor boundaries of the convolutional-embedding network's flat vector
    (``sdnet_conv``): the two convolutions' kernels and biases, then the
    layers of the tanh layout with the embedding in place of the boundary."""
    d, C = width, channels
    sizes = [C * 1 * sdnet_conv.KERNEL, C, C * C * sdnet_conv.KERNEL, C]
    E = C * sdnet_conv.NB
    for out_f, in_f in [(d, E + 2)] + [(d, d)] * 3 + [(1, d)]:
        sizes += [out_f * in_f, out_f]
    begins = [0]
    for n in sizes:
        begins.append(begins[-1] + n)
    return begins


def lamb_update(theta, m, v, grad, step: int, segments, lr: float, beta1: float = 0.9,
                beta2: float = 0.999, eps: float = 1e-6, weight_decay: float = 0.0,
                max_grad_norm: float = 0.0, trust_without_decay: bool = True):
    """One LAMB step on the flat vectors; segments = tensor boundaries
    (begin offsets and the end). Returns new (theta, m, v)."""
    g = grad
    if max_grad_norm > 0.0:
        norm = torch.sqrt(torch.sum(g * g))
        if norm > max_grad_norm:
            g = g * (max_grad_norm / norm)
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    u = mhat / (torch.sqrt(vhat) + eps) + weight_decay * theta
    new = theta.clone()
    use_trust = trust_without_decay or weight_decay != 0.0
    for a, b in zip(segments[:-1], segments[1:]):
        w_s, u_s = theta[a:b], u[a:b]
        r = 1.0
        if use_trust:
            wn = torch.sqrt(torch.sum(w_s * w_s)).item()
            un = torch.sqrt(torch.sum(u_s * u_s)).item()
            if wn > 0.0 and un > 0.0:
                r = wn / un
        new[a:b] = w_s - lr * r * u_s
    return new, m, v


def warmup_steps(total_steps: int, warmup_frac: float) -> int:
    return int(math.ceil(warmup_frac * total_steps))


def lr_at(step: int, total_steps: int, max_lr: float, warmup_frac: float, power: float = 1.0,
          end_lr: float = 0.0) -> float:
    """Learning rate of iteration `step` (from 1): linear warm-up, then
    polynomial decay to end_lr at total_steps."""
    W = warmup_steps(total_steps, warmup_frac)
    if step <= W:
        return max_lr * step / W
    if step >= total_steps:
        return end_lr
    frac = 1.0 - (step - W) / (total_steps - W)
    return end_lr + (max_lr - end_lr) * frac ** power


def scaled_schedule(max_lr: float, warmup_frac: float, batch_factor: float):
    """The multi-device rules: peak learning rate times sqrt(k), warm-up
    fraction times k (at most 1), for a batch k times larger."""
    return max_lr * math.sqrt(batch_factor), min(1.0, warmup_frac * batch_factor)


def lamb_train_step(theta, m, v, step: int, width: int, G, Xd, Xc, Yd=None, **lamb):
    """Alg. 1 (both passes, gradients summed; the allreduce is the identity
    on one device), then one LAMB step: returns (theta, m, v, L_data, L_pde)."""
    from . import train
    l_data, l_pde, g_data, g_pde = train.gradient(theta, width, G, Xd, Xc, Yd)
    theta, m, v = lamb_update(theta, m, v, g_data + g_pde, step, tanh_segments(width), **lamb)
    return theta, m, v, l_data, l_pde

