"""Write the stored expected values used by the GPU parity tests.

Every value here comes from the float64 oracle (``oracle/``) run on the
seeded inputs of ``mf_inputs``; nothing is read from the HIP path.

    python tests/golden/make_golden.py [name ...]

c2_fp32.npz -- 16 x 16 units, width 256, GP ring data (length 2, seed 1),
    Xavier weights seed 0, 200 CROSS sweeps then the assembly. Holds the
    skeleton after 20 and 200 sweeps and u_out at 8192 sampled interior
    points (seed 123).
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import mf_inputs as mi  # noqa: E402
from oracle import sweep as sw  # noqa: E402


def _sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]


def c2():
    w = mi.WORKLOADS["C2"]
    ux, uy = w["units"]
    field = mi.workload_field("C2")
    params = mi.xavier_params(w["width"], seed=0)
    solver = sw.sdnet_solver(torch.from_numpy(params.astype(np.float64)), w["width"])
    u = torch.from_numpy(field.astype(np.float64))
    t0 = time.time()
    skel20 = None
    for k in range(1, w["sweeps"] + 1):
        u = sw.sweep(u, ux, uy, solver)
        if k == 20:
            skel20 = sw.skeleton_values(u).numpy()
        if k % 20 == 0:
            print(f"c2: sweep {k} ({time.time() - t0:.0f} s)", flush=True)
    skel = sw.skeleton_values(u).numpy()
    u_out = sw.assemble(u, ux, uy, solver).numpy()
    rng = np.random.default_rng(123)
    ny, nx = u_out.shape
    jj = rng.integers(1, ny - 1, 8192)
    ii = rng.integers(1, nx - 1, 8192)
    np.savez_compressed(os.path.join(HERE, "c2_fp32.npz"), skel20=skel20, skel200=skel,
                        sample_j=jj.astype(np.int32), sample_i=ii.astype(np.int32),
                        u_out_sample=u_out[jj, ii], field_sha=_sha(field), params_sha=_sha(params))
    print(f"c2: done in {time.time() - t0:.0f} s", flush=True)


JOBS = {"c2": c2}

if __name__ == "__main__":
    torch.set_num_threads(os.cpu_count() or 1)
    for name in (sys.argv[1:] or list(JOBS)):
        JOBS[name]()
