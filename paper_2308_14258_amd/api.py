"""Thin Python binding over libmosaic's C ABI.

Each function has the name of the C entry point it calls and only marshals
arguments: torch tensors supply device pointers (and the workspace), the
current torch stream is passed as the HIP stream. No computation happens
here.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import (MF_BF16, MF_GELU, MF_CROSS, MF_FP32, MF_MAX_SEGMENTS, MF_MULTIPLICATIVE, MF_TANH, Adam,
                   DomainDesc, Lamb, LrSchedule, SdnetDesc, check, load)


def _gelu_count(d: int, C: int) -> int:
    return 5 * C + C + 5 * C * C + C + d * (128 * C + 2) + d + 3 * (d * d + d) + d + 1


def net_of(params: torch.Tensor):
    """(width, activation, embedding channels) of a flat parameter vector:
    the tanh network (no embedding) or the convolutional-embedding GELU
    network with 1..8 channels, at width 128 or 256."""
    n = params.numel()
    for d in (128, 256):
        if 3 * d * d + 135 * d + 1 == n:
            return d, MF_TANH, 0
        for C in range(1, 9):
            if _gelu_count(d, C) == n:
                return d, MF_GELU, C
    raise ValueError(f"parameter vector of {n} floats matches no supported network")


def width_of(params: torch.Tensor) -> int:
    return net_of(params)[0]


def sdnet_desc(width: int, activation: int = MF_TANH, embed_channels: int = 0) -> SdnetDesc:
    return SdnetDesc(width, 4, 128, activation, embed_channels)


def desc_of(params: torch.Tensor) -> SdnetDesc:
    return sdnet_desc(*net_of(params))


def domain_desc(u: torch.Tensor, units) -> DomainDesc:
    ux, uy = units
    return DomainDesc(int(ux), int(uy), 32, 16, int(u.stride(0)), 0)


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need_cuda_f32(t: torch.Tensor, name: str):
    if not (t.is_cuda and t.dtype == torch.float32):
        raise TypeError(f"{name} must be a float32 CUDA tensor")


def _need_field(u: torch.Tensor, units):
    _need_cuda_f32(u, "field")
    ux, uy = units
    if u.dim() != 2 or u.shape != (32 * uy + 1, 32 * ux + 1) or u.stride(1) != 1:
        raise ValueError(f"field must be [{32 * uy + 1}, {32 * ux + 1}] with unit column stride")


class Context:
    """One mf_ctx plus a cached device workspace."""

    def __init__(self, device: int = 0):
        lib = load()
        ptr = ctypes.c_void_p()
        check(lib.mf_ctx_create(device, ctypes.byref(ptr)), "mf_ctx_create")
        self.ptr = ptr
        self.device = device
        self._ws = None

    def workspace(self, nbytes: int) -> torch.Tensor:
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def tile_rows(self, prec: int, rows: int) -> None:
        """Force the colour-phase tile height for one precision (0 = automatic)."""
        check(load().mf_ctx_tile_rows(self.ptr, prec, rows), "mf_ctx_tile_rows")

    def graphs(self, enable: bool) -> None:
        check(load().mf_ctx_graphs(self.ptr, 1 if enable else 0), "mf_ctx_graphs")

    def timing(self, enable: bool) -> None:
        check(load().mf_ctx_timing(self.ptr, 1 if enable else 0), "mf_ctx_timing")

    def timing_read(self):
        """(launches, total_ms, rows) of the timed colour-phase launches."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        rows = ctypes.c_int64()
        check(load().mf_ctx_timing_read(self.ptr, ctypes.byref(n), ctypes.byref(ms),
                                        ctypes.byref(rows)), "mf_ctx_timing_read")
        return n.value, ms.value, rows.value

    def close(self):
        if self.ptr:
            load().mf_ctx_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _sweep_ws(ctx: Context, params: torch.Tensor, dom, prec: int, n_domains: int = 1, targets: int = MF_CROSS,
              mode: int = MF_MULTIPLICATIVE) -> torch.Tensor:
    n = ctypes.c_size_t()
    check(load().mf_workspace_size(ctypes.byref(desc_of(params)), _dom_arg(dom), n_domains, prec,
                                   targets, mode, ctypes.byref(n)), "mf_workspace_size")
    return ctx.workspace(n.value)


def _dom_arg(dom):
    return dom if isinstance(dom, ctypes.Array) else ctypes.byref(dom)


class Batch:
    """Independent domains packed into one flat float32 device buffer.

    ``fields`` are [32 uy + 1, 32 ux + 1] arrays; each domain is stored
    row-major with its own pitch (the row length) at its offset.
    """

    def __init__(self, fields, device="cuda:0"):
        self.units = []
        offs = []
        off = 0
        for f in fields:
            ny, nx = f.shape
            self.units.append(((nx - 1) // 32, (ny - 1) // 32))
            offs.append(off)
            off += ny * nx
        self.offsets = offs
        self.buf = torch.empty(off, dtype=torch.float32, device=device)
        for f, o in zip(fields, offs):
            t = torch.as_tensor(f, dtype=torch.float32)
            self.buf[o:o + t.numel()].copy_(t.reshape(-1))
        arr = (DomainDesc * len(fields))()
        for i, ((ux, uy), o) in enumerate(zip(self.units, offs)):
            arr[i] = DomainDesc(ux, uy, 32, 16, 32 * ux + 1, o)
        self.descs = arr

    def __len__(self):
        return len(self.units)

    def field(self, i, buf=None):
        ux, uy = self.units[i]
        ny, nx = 32 * uy + 1, 32 * ux + 1
        b = self.buf if buf is None else buf
        return b[self.offsets[i]:self.offsets[i] + ny * nx].view(ny, nx)


def _field_and_domains(u, units):
    """(device pointer owner, domain descriptor(s), count) for a single 2-D
    field with units (ux, uy), or a Batch."""
    if isinstance(u, Batch):
        return u.buf, u.descs, len(u)
    _need_field(u, units)
    return u, domain_desc(u, units), 1


def mf_sweep(ctx: Context, params: torch.Tensor, u, units=None, colour: int = -1,
             targets: int = MF_CROSS, prec: int = MF_FP32, mode: int = MF_MULTIPLICATIVE):
    """One colour phase (0..3) or one sweep (-1) of u in place (u: a 2-D
    field with units (ux, uy), or a Batch of domains)."""
    _need_cuda_f32(params, "params")
    buf, dom, nd = _field_and_domains(u, units)
    width = width_of(params)
    ws = _sweep_ws(ctx, params, dom, prec, nd, targets, mode)
    check(load().mf_sweep(ctx.ptr, ctypes.byref(desc_of(params)), _ptr(params), _ptr(buf),
                          _dom_arg(dom), nd, colour, targets, mode, prec, _ptr(ws), ws.numel(),
                          _stream()), "mf_sweep")


def mf_sweep_noalloc(ctx: Context, params: torch.Tensor, u, units=None, colour: int = -1,
                     targets: int = MF_CROSS, prec: int = MF_FP32):
    """mf_sweep (multiplicative) with the library's static device scratch in
    place of a workspace: no device memory is allocated by this call."""
    _need_cuda_f32(params, "params")
    buf, dom, nd = _field_and_domains(u, units)
    width = width_of(params)
    check(load().mf_sweep_noalloc(ctx.ptr, ctypes.byref(desc_of(params)), _ptr(params), _ptr(buf),
                                  _dom_arg(dom), nd, colour, targets, prec, _stream()),
          "mf_sweep_noalloc")


def mf_autotune(ctx: Context, params: torch.Tensor, u, units=None,
                targets: int = MF_CROSS, prec: int = MF_FP32, trials: int = 3) -> int:
    """Time every tile shape on u (which advances; a 2-D field with units
    (ux, uy), or a Batch) and keep the fastest for later calls on the same
    domain (or domain list). Returns the chosen shape code."""
    _need_cuda_f32(params, "params")
    buf, dom, nd = _field_and_domains(u, units)
    ws = _sweep_ws(ctx, params, dom, prec, nd, targets)
    rows = ctypes.c_int32(0)
    check(load().mf_autotune(ctx.ptr, ctypes.byref(desc_of(params)), _ptr(params), _ptr(buf),
                             _dom_arg(dom), nd, targets, prec, trials, _ptr(ws), ws.numel(),
                             _stream(), ctypes.byref(rows)), "mf_autotune")
    return rows.value


def mf_solve(ctx: Context, params: torch.Tensor, u, units, max_sweeps: int,
             eps: float = 0.0, check_every: int = 1, targets: int = MF_CROSS,
             prec: int = MF_FP32, u_out=None, flags: int = 0,
             mode: int = MF_MULTIPLICATIVE, report: bool = False):
    """Alg. 2 on one GPU; u is updated in place, u_out receives the assembly.
    u is a 2-D field with units (ux, uy), or a Batch (then units is ignored
    and u_out, if given, is a flat buffer laid out like u.buf).
    Returns (sweeps_done, last_delta) when report is True (synchronises)."""
    _need_cuda_f32(params, "params")
    buf, dom, nd = _field_and_domains(u, units)
    if u_out is not None:
        if nd == 1:
            _need_field(u_out, units)
            if u_out.stride(0) != u.stride(0):
                raise ValueError("u_out must have the same pitch as u")
        elif u_out.numel() != buf.numel():
            raise ValueError("u_out must match the batch buffer")
    width = width_of(params)
    ws = _sweep_ws(ctx, params, dom, prec, nd, targets, mode)
    done = ctypes.c_int32(-1)
    last = ctypes.c_float(float("nan"))
    check(load().mf_solve(ctx.ptr, ctypes.byref(desc_of(params)), _ptr(params), _ptr(buf),
                          _dom_arg(dom), nd, targets, mode, prec, max_sweeps, eps, check_every,
                          flags, _ptr(u_out), ctypes.byref(done) if report else None,
                          ctypes.byref(last) if report else None, _ptr(ws), ws.numel(),
                          _stream()), "mf_solve")
    return (done.value, last.value) if report else None


def mf_solve_mixed(ctx: Context, params: torch.Tensor, u, units, max_sweeps: int, refresh_every: int = 20,
                   prec: int = MF_BF16, targets: int = MF_CROSS, u_out=None, assembly_prec: int = MF_FP32):
    """Sweeps in 16 bits (prec MF_BF16 or MF_FP16) with a float32 correction
    refreshed every refresh_every sweeps, then the assembly into u_out
    (optional) in assembly_prec (MF_FP32 or prec). u is a 2-D field with
    units (ux, uy), or a Batch."""
    _need_cuda_f32(params, "params")
    buf, dom, nd = _field_and_domains(u, units)
    if u_out is not None:
        if nd == 1:
            _need_field(u_out, units)
            if u_out.stride(0) != u.stride(0):
                raise ValueError("u_out must have the same pitch as u")
        elif u_out.numel() != buf.numel():
            raise ValueError("u_out must match the batch buffer")
    n = ctypes.c_size_t()
    lib = load()
    check(lib.mf_mixed_ws_size(ctypes.byref(desc_of(params)), _dom_arg(dom), nd, targets, prec, ctypes.byref(n)),
          "mf_mixed_ws_size")
    ws = ctx.workspace(n.value)
    check(lib.mf_solve_mixed(ctx.ptr, ctypes.byref(desc_of(params)), _ptr(params), _ptr(buf), _dom_arg(dom), nd,
                             targets, prec, max_sweeps, refresh_every, assembly_prec, _ptr(u_out), _ptr(ws),
                             ws.numel(),
                             _stream()), "mf_solve_mixed")


def mf_solve_adjoint(ctx: Context, params: torch.Tensor, u0, units, K: int, ckpt_every: int = 5,
                     targets: int = MF_CROSS, u_out=None, J: torch.Tensor | None = None,
                     u0_bar=None, uout_bar=None):
    """u0_bar = (d u_out / d u0)^T uout_bar through K sweeps and the assembly.
    Without uout_bar the seed is that of J = sum of squared interior values
    of u_out; with it, J = <uout_bar, u_out> over every grid point. u0 is a
    2-D field (units (ux, uy)) or a Batch (then u_out / u0_bar / uout_bar
    are flat buffers like u0.buf). Returns (u0_bar, J)."""
    _need_cuda_f32(params, "params")
    buf, dom, nd = _field_and_domains(u0, units)
    if uout_bar is not None:
        _need_cuda_f32(uout_bar, "uout_bar")
        if uout_bar.numel() != buf.numel() or (nd == 1 and uout_bar.stride(0) != buf.stride(0)):
            raise ValueError("uout_bar must be laid out like u0")
    width = width_of(params)
    if u0_bar is None:
        u0_bar = torch.zeros_like(buf)
    if J is None:
        J = torch.zeros(1, dtype=torch.float32, device=buf.device)
    n = ctypes.c_size_t()
    lib = load()
    check(lib.mf_adjoint_ws_size(ctypes.byref(desc_of(params)), _dom_arg(dom), nd, targets, K,
                                 ckpt_every, ctypes.byref(n)), "mf_adjoint_ws_size")
    ws = ctx.workspace(n.value)
    check(lib.mf_solve_adjoint(ctx.ptr, ctypes.byref(desc_of(params)), _ptr(params), _ptr(buf),
                               _dom_arg(dom), nd, targets, K, ckpt_every, _ptr(uout_bar), _ptr(u_out),
                               _ptr(J), _ptr(u0_bar), _ptr(ws), ws.numel(), _stream()),
          "mf_solve_adjoint")
    return u0_bar, J


def mf_sweep_operator(ctx: Context, Hop: torch.Tensor, u: torch.Tensor, units, colour: int = -1,
                      targets: int = MF_CROSS, u_out: torch.Tensor | None = None):
    """Sweep (colour -1), phase (0..3) or assembly (4) with a linear solver."""
    _need_field(u, units)
    _need_cuda_f32(Hop, "Hop")
    if u_out is not None:
        _need_field(u_out, units)
    if Hop.dim() != 2 or Hop.shape[1] != 128:
        raise ValueError("Hop must be [T, 128]")
    dom = domain_desc(u, units)
    Hop = Hop.contiguous()
    check(load().mf_sweep_operator(ctx.ptr, _ptr(Hop), Hop.shape[0], targets, _ptr(u), _ptr(u_out),
                                   ctypes.byref(dom), colour, _stream()), "mf_sweep_operator")


def mf_colour_placements(units, colour: int) -> int:
    """Number of placements of a colour (0..3) in a ux x uy domain."""
    ux, uy = units
    n = load().mf_colour_placements(ctypes.byref(DomainDesc(int(ux), int(uy), 32, 16, 32 * int(ux) + 1, 0)),
                                    colour)
    if n < 0:
        check(_lib.MF_EINVAL, "mf_colour_placements")
    return int(n)


def mf_target_coords(targets: int = MF_CROSS) -> torch.Tensor:
    """[T, 2] local (x, y) of the target set in the library's order (host tensor)."""
    T = 61 if targets == MF_CROSS else 961
    X = torch.empty(T, 2, dtype=torch.float32)
    check(load().mf_target_coords(targets, _ptr(X)), "mf_target_coords")
    return X


def mf_gather(ctx: Context, u: torch.Tensor, units, colour: int, G: torch.Tensor | None = None):
    """[P_c, 128] boundary vectors of every placement of one colour."""
    _need_field(u, units)
    n = mf_colour_placements(units, colour)
    if G is None:
        G = torch.empty(n, 128, device=u.device, dtype=torch.float32)
    elif not (G.is_cuda and G.dtype == torch.float32 and G.is_contiguous() and G.shape == (n, 128)):
        raise ValueError(f"G must be a contiguous float32 CUDA tensor of shape ({n}, 128)")
    dom = domain_desc(u, units)
    check(load().mf_gather(ctx.ptr, _ptr(u), ctypes.byref(dom), colour, _ptr(G) if n else None, _stream()),
          "mf_gather")
    return G


def mf_scatter(ctx: Context, pred: torch.Tensor, u: torch.Tensor, units, colour: int,
               targets: int = MF_CROSS) -> None:
    """Write pred [P_c, T] at the targets of every placement of one colour."""
    _need_field(u, units)
    _need_cuda_f32(pred, "pred")
    T = 61 if targets == MF_CROSS else 961
    n = mf_colour_placements(units, colour)
    if not (pred.is_contiguous() and pred.shape == (n, T)):
        raise ValueError(f"pred must be contiguous of shape ({n}, {T})")
    dom = domain_desc(u, units)
    check(load().mf_scatter(ctx.ptr, _ptr(pred) if n else None, targets, _ptr(u), ctypes.byref(dom), colour,
                            _stream()), "mf_scatter")


class SkeletonCols:
    """The transposed skeleton columns of one field (the side layout of
    mf_gather_skel / mf_scatter_skel): cols[c, j] = u[j, 16 c]."""

    def __init__(self, u: torch.Tensor, units):
        _need_field(u, units)
        self.units = (int(units[0]), int(units[1]))
        self.dom = domain_desc(u, units)
        n = load().mf_skeleton_cols_size(ctypes.byref(self.dom))
        if n < 0:
            check(_lib.MF_EINVAL, "mf_skeleton_cols_size")
        self.buf = torch.empty(int(n), dtype=torch.float32, device=u.device)


def mf_skeleton_pack(ctx: Context, u: torch.Tensor, cols: SkeletonCols) -> None:
    check(load().mf_skeleton_pack(ctx.ptr, _ptr(u), ctypes.byref(cols.dom), _ptr(cols.buf), _stream()),
          "mf_skeleton_pack")


def mf_skeleton_unpack(ctx: Context, cols: SkeletonCols, u: torch.Tensor) -> None:
    check(load().mf_skeleton_unpack(ctx.ptr, _ptr(cols.buf), _ptr(u), ctypes.byref(cols.dom), _stream()),
          "mf_skeleton_unpack")


def mf_gather_skel(ctx: Context, u: torch.Tensor, cols: SkeletonCols, colour: int, G: torch.Tensor | None = None):
    """[P_c, 128] boundary vectors of one colour from the side layout."""
    n = mf_colour_placements(cols.units, colour)
    if G is None:
        G = torch.empty(n, 128, device=u.device, dtype=torch.float32)
    check(load().mf_gather_skel(ctx.ptr, _ptr(u), _ptr(cols.buf), ctypes.byref(cols.dom), colour,
                                _ptr(G) if n else None, _stream()), "mf_gather_skel")
    return G


def mf_scatter_skel(ctx: Context, pred: torch.Tensor, u: torch.Tensor, cols: SkeletonCols, colour: int) -> None:
    """CROSS predictions [P_c, 61] of one colour into the side layout."""
    _need_cuda_f32(pred, "pred")
    n = mf_colour_placements(cols.units, colour)
    if not (pred.is_contiguous() and pred.shape == (n, 61)):
        raise ValueError(f"pred must be contiguous of shape ({n}, 61)")
    check(load().mf_scatter_skel(ctx.ptr, _ptr(pred) if n else None, _ptr(u), _ptr(cols.buf),
                                 ctypes.byref(cols.dom), colour, _stream()), "mf_scatter_skel")


def sdnet_forward(ctx: Context, params: torch.Tensor, G: torch.Tensor, X: torch.Tensor,
                  prec: int = MF_FP32, derivatives: bool = False):
    """U [n_bc, n_pts] (and dU [n_bc, n_pts, 2], lapU [n_bc, n_pts])."""
    _need_cuda_f32(params, "params")
    _need_cuda_f32(G, "G")
    _need_cuda_f32(X, "X")
    G = G.contiguous()
    X = X.contiguous()
    width = width_of(params)
    n_bc = G.shape[0]
    x_per_bc = 1 if X.dim() == 3 else 0
    n_pts = X.shape[1] if x_per_bc else X.shape[0]
    U = torch.empty(n_bc, n_pts, device=G.device, dtype=torch.float32)
    dU = torch.empty(n_bc, n_pts, 2, device=G.device, dtype=torch.float32) if derivatives else None
    lapU = torch.empty(n_bc, n_pts, device=G.device, dtype=torch.float32) if derivatives else None
    n = ctypes.c_size_t()
    lib = load()
    check(lib.sdnet_forward_ws_size(ctypes.byref(desc_of(params)), n_bc, n_pts,
                                    1 if derivatives else 0, prec, ctypes.byref(n)),
          "sdnet_forward_ws_size")
    ws = ctx.workspace(n.value)
    check(lib.sdnet_forward(ctx.ptr, ctypes.byref(desc_of(params)), _ptr(params), _ptr(G), n_bc,
                            _ptr(X), n_pts, x_per_bc, _ptr(U), _ptr(dU), _ptr(lapU), prec, _ptr(ws),
                            ws.numel(), _stream()), "sdnet_forward")
    return (U, dU, lapU) if derivatives else U


def _data_args(G: torch.Tensor, Xd: torch.Tensor, Yd):
    """(Xd, nd, xd_per_bc, Yd) for the training entry points: Xd is shared
    [nd, 2] or per condition [B, nd, 2]; Yd is [B, nd] or None (boundary
    match, targets G)."""
    _need_cuda_f32(Xd, "Xd")
    per_bc = 1 if Xd.dim() == 3 else 0
    nd = Xd.shape[1] if per_bc else Xd.shape[0]
    if Xd.shape[-1] != 2 or (per_bc and Xd.shape[0] != G.shape[0]):
        raise ValueError("Xd must be [nd, 2] or [B, nd, 2]")
    if Yd is not None:
        _need_cuda_f32(Yd, "Yd")
        if tuple(Yd.shape) != (G.shape[0], nd):
            raise ValueError(f"Yd must be [{G.shape[0]}, {nd}]")
        Yd = Yd.contiguous()
    return Xd.contiguous(), nd, per_bc, Yd


def _train_ws(ctx: Context, params: torch.Tensor, B: int, nd: int, nc: int) -> torch.Tensor:
    n = ctypes.c_size_t()
    check(load().sdnet_train_ws_size(ctypes.byref(desc_of(params)), B, nd, nc, ctypes.byref(n)),
          "sdnet_train_ws_size")
    return ctx.workspace(n.value)


def sdnet_train_step(ctx: Context, params: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
                     step: int, G: torch.Tensor, Xd: torch.Tensor, Xc: torch.Tensor,
                     lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                     loss: torch.Tensor | None = None, grad_out: torch.Tensor | None = None,
                     Yd: torch.Tensor | None = None):
    """One Alg. 1 iteration + Adam. Xd: data points ([nd, 2] shared or
    [B, nd, 2]); Yd: their targets [B, nd], or None for the boundary match
    (Xd = the 128 perimeter nodes, targets G). Returns the device loss
    tensor [3] = (L_data, L_pde, L_data + L_pde)."""
    for t, name in ((params, "params"), (m, "m"), (v, "v"), (G, "G"), (Xc, "Xc")):
        _need_cuda_f32(t, name)
    width = width_of(params)
    B, nc = Xc.shape[0], Xc.shape[1]
    Xd, nd, per_bc, Yd = _data_args(G, Xd, Yd)
    if loss is None:
        loss = torch.empty(3, device=G.device, dtype=torch.float32)
    ws = _train_ws(ctx, params, B, nd, nc)
    hp = Adam(lr, beta1, beta2, eps)
    check(load().sdnet_train_step(ctx.ptr, ctypes.byref(desc_of(params)), _ptr(params), _ptr(m),
                                  _ptr(v), step, ctypes.byref(hp), _ptr(G.contiguous()), B, _ptr(Xd), nd,
                                  per_bc, _ptr(Yd), _ptr(Xc.contiguous()), nc, _ptr(loss),
                                  _ptr(grad_out), _ptr(ws), ws.numel(), _stream()),
          "sdnet_train_step")
    return loss


def sdnet_loss_grad(ctx: Context, params: torch.Tensor, G: torch.Tensor, Xd: torch.Tensor,
                    Xc: torch.Tensor, loss: torch.Tensor | None = None,
                    grad_out: torch.Tensor | None = None, Yd: torch.Tensor | None = None):
    """(L_data, L_pde, L_data + L_pde) of Alg. 1 at `params` and the
    gradient of L_data + L_pde from the library's hand-written reverse pass,
    with no parameter update (C entry point sdnet_loss_grad). Returns
    (loss [3], grad), both device tensors."""
    for t, name in ((params, "params"), (G, "G"), (Xc, "Xc")):
        _need_cuda_f32(t, name)
    width = width_of(params)
    B, nc = Xc.shape[0], Xc.shape[1]
    Xd, nd, per_bc, Yd = _data_args(G, Xd, Yd)
    if loss is None:
        loss = torch.empty(3, device=G.device, dtype=torch.float32)
    if grad_out is None:
        grad_out = torch.empty_like(params)
    _need_cuda_f32(grad_out, "grad_out")
    ws = _train_ws(ctx, params, B, nd, nc)
    check(load().sdnet_loss_grad(ctx.ptr, ctypes.byref(desc_of(params)), _ptr(params), _ptr(G.contiguous()), B,
                                 _ptr(Xd), nd, per_bc, _ptr(Yd), _ptr(Xc.contiguous()), nc, _ptr(loss),
                                 _ptr(grad_out), _ptr(ws), ws.numel(), _stream()),
          "sdnet_loss_grad")
    return loss, grad_out


def param_segments(desc_or_params) -> list:
    """Tensor boundaries of an SDNet's flat parameter vector (C entry point
    mf_param_segments): the first index of W1, b1, W2, ..., w5, b5 (the GELU
    network's two convolutions first) and, last, the parameter count."""
    d = desc_or_params if isinstance(desc_or_params, SdnetDesc) else desc_of(desc_or_params)
    begin = (ctypes.c_int64 * (MF_MAX_SEGMENTS + 1))()
    n = ctypes.c_int32()
    check(load().mf_param_segments(ctypes.byref(d), begin, MF_MAX_SEGMENTS, ctypes.byref(n)), "mf_param_segments")
    return list(begin[:n.value + 1])


def sdnet_lamb_step(ctx: Context, params: torch.Tensor, m: torch.Tensor, v: torch.Tensor, grad: torch.Tensor,
                    step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-6,
                    weight_decay: float = 0.0, max_grad_norm: float = 0.0, trust_without_decay: bool = True,
                    segments=None) -> None:
    """One LAMB step on params, m and v in place from grad (C entry point
    sdnet_lamb_step). segments: tensor boundaries (default: the SDNet layout
    of params, param_segments)."""
    for t, name in ((params, "params"), (m, "m"), (v, "v"), (grad, "grad")):
        _need_cuda_f32(t, name)
        if t.numel() != params.numel() or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with {params.numel()} elements")
    seg = param_segments(params) if segments is None else [int(x) for x in segments]
    if seg[-1] != params.numel():
        raise ValueError("segments must end at the parameter count")
    arr = (ctypes.c_int64 * len(seg))(*seg)
    hp = Lamb(lr, beta1, beta2, eps, weight_decay, max_grad_norm, 1 if trust_without_decay else 0)
    check(load().sdnet_lamb_step(ctx.ptr, _ptr(params), _ptr(m), _ptr(v), _ptr(grad), arr, len(seg) - 1, step,
                                 ctypes.byref(hp), _stream()), "sdnet_lamb_step")


def lr_schedule(max_lr: float, total_steps: int, warmup_frac: float = 0.001, power: float = 1.0,
                end_lr: float = 0.0) -> LrSchedule:
    """Linear warm-up then polynomial decay (the paper's defaults: 0.1%
    warm-up, exponent 1, decay to 0)."""
    return LrSchedule(max_lr, warmup_frac, power, end_lr, total_steps)


def lr_at(sched: LrSchedule, step: int) -> float:
    """The schedule's learning rate at iteration step (from 1; C entry point
    mf_lr_at)."""
    lr = ctypes.c_double()
    check(load().mf_lr_at(ctypes.byref(sched), step, ctypes.byref(lr)), "mf_lr_at")
    return lr.value


def lr_schedule_scaled(sched: LrSchedule, batch_factor: float) -> LrSchedule:
    """Peak learning rate times sqrt(k) and warm-up fraction times k for a
    batch k times larger (C entry point mf_lr_schedule_scaled)."""
    out = LrSchedule()
    check(load().mf_lr_schedule_scaled(ctypes.byref(sched), batch_factor, ctypes.byref(out)),
          "mf_lr_schedule_scaled")
    return out


class PhysicsLoss(torch.autograd.Function):
    """L = L_data + L_pde (Alg. 1: data term plus the squared Laplacian
    residual of Eq. 3) as a differentiable function of the flat parameter
    vector. The forward and the backward are one call of the library's
    training kernels (Taylor-mode forward, hand-written reverse pass), which
    also forms the sum; the backward returns the saved gradient scaled by
    the incoming one, so the loss composes with torch optimisers and other
    loss terms."""

    @staticmethod
    def forward(fctx, params, G, Xd, Xc, mf_ctx, Yd=None):
        loss, grad = sdnet_loss_grad(mf_ctx, params.detach(), G, Xd, Xc, Yd=Yd)
        fctx.save_for_backward(grad)
        return loss[2]

    @staticmethod
    def backward(fctx, g):
        (grad,) = fctx.saved_tensors
        return g * grad, None, None, None, None, None


def physics_loss(ctx: Context, params: torch.Tensor, G: torch.Tensor, Xd: torch.Tensor,
                 Xc: torch.Tensor, Yd: torch.Tensor | None = None) -> torch.Tensor:
    """Scalar L_data + L_pde whose .backward() runs the hand-written reverse pass."""
    return PhysicsLoss.apply(params, G, Xd, Xc, ctx, Yd)


__all__ = ["Batch", "Context", "PhysicsLoss", "SkeletonCols", "mf_skeleton_pack", "mf_skeleton_unpack",
           "mf_gather_skel", "mf_scatter_skel", "mf_autotune", "mf_solve_adjoint", "mf_sweep",
           "mf_sweep_noalloc", "mf_solve",
           "mf_sweep_operator", "mf_colour_placements", "mf_target_coords", "mf_gather", "mf_scatter", "physics_loss", "sdnet_forward", "sdnet_loss_grad", "sdnet_train_step",
           "width_of", "sdnet_desc", "domain_desc", "_lib"]
