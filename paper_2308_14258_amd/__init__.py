"""Mosaic Flow on MI355X: the predictor sweep and SDNet training step as
hand-written HIP kernels behind a C ABI (include/mosaic.h).

The Python layer only marshals arguments: torch tensors provide device
memory and the current stream; every step runs in libmosaic.so.
"""
from ._lib import (MF_ADDITIVE, MF_BF16, MF_CROSS, MF_FP16, MF_FP32, MF_INTERIOR, MF_MULTIPLICATIVE,  # noqa: F401
                   MF_GELU, MF_TANH, MF_TILE_PERSIST, MF_TILE_ROWSPLIT, MF_TILE_STREAM, MF_TILE_WIDE,
                   MosaicError, load)
from .api import (Batch, Context, PhysicsLoss, mf_autotune, mf_colour_placements, mf_gather,  # noqa: F401
                  mf_scatter, mf_solve, mf_solve_adjoint, mf_solve_mixed, mf_sweep, mf_sweep_noalloc, mf_sweep_operator, mf_target_coords,
                  physics_loss, sdnet_forward, sdnet_loss_grad, sdnet_train_step, SkeletonCols,
                  mf_skeleton_pack, mf_skeleton_unpack, mf_gather_skel, mf_scatter_skel, param_segments,
                  sdnet_lamb_step, lr_schedule, lr_at, lr_schedule_scaled)
