"""CPU float64 oracle for the Mosaic Flow sweep and the SDNet training step.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports this package:
only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may use it. It shares no code with the HIP library; the
only common inputs are the seeded arrays from ``mf_inputs``.

The oracle is written from the paper's statement of the method (arXiv
2308.14258) in plain PyTorch CPU float64 operations, one step at a time, with
no blocking, fusion or reordering beyond what the definitions state:

* ``geometry``  -- grid, overlapping placements, colours, boundary vector
  order, target sets (Sec. 4.2 "Domain Parallelization", Fig. 2).
* ``sdnet``     -- the subdomain network N(x, g; theta) with the input-split
  first layer (Sec. 3.2, Eqs. 5-8) and its derivatives by autograd.
* ``sdnet_conv`` -- the paper's architecture: a circular 1-D convolutional
  embedding of the boundary curve, the input-split first layer and GELU
  layers (Sec. 3.1, Fig. 3; Sec. 3.2, Eq. 8).
* ``sweep``     -- batched colour phases, sweeps, the delta test and the
  overlap-averaged final assembly (Sec. 4.1, Alg. 2).
* ``fd``        -- exact 5-point subdomain solver and global 5-point solve,
  used as the check mode that swaps SDNet for a known linear solver
  (Sec. 2.3, Eq. 4).
* ``train``     -- boundary-match + PDE loss (Eq. 3), its gradient, and Adam
  (Alg. 1).
* ``adjoint``   -- d J / d g through K sweeps and the assembly.
* ``optim``     -- LAMB, the warm-up + polynomial-decay learning rate and the
  multi-device scaling rules of the training (Sec. 5.2, "Hyperparameters").

Every function states which passage it follows. Pins that tie the oracle to
facts outside itself live in ``tests/test_oracle_*.py``.
"""
from . import adjoint, fd, geometry, optim, sdnet, sdnet_conv, sweep, train  # noqa: F401
