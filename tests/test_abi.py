"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/mosaic.h, and rejects bad arguments on the host before
touching a device."""
import ctypes
import os
import re

import pytest

from paper_2308_14258_amd import _lib
from paper_2308_14258_amd._lib import (MF_BF16, MF_CROSS, MF_EDEVICE, MF_EINVAL, MF_ENOMEM,
                                       MF_INTERIOR,
                                       MF_ESHAPE, MF_EUNSUPPORTED, MF_FP32, MF_OK, DomainDesc,
                                       SdnetDesc)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "mosaic.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return set(re.findall(r"^\s*(?:mf_status|void|int64_t|int32_t|const char\*)\s+(\w+)\s*\(", txt, re.M))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def _has_gpu():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert {"mf_sweep", "mf_solve", "sdnet_forward", "sdnet_train_step"} <= names
    for n in names:
        assert hasattr(lib, n), n
    assert names == set(_lib._SIG), names ^ set(_lib._SIG)


def test_param_count(lib):
    assert lib.mf_param_count(ctypes.byref(SdnetDesc(128, 4, 128, 0))) == 66433
    assert lib.mf_param_count(ctypes.byref(SdnetDesc(256, 4, 128, 0))) == 231169
    assert lib.mf_param_count(ctypes.byref(SdnetDesc(100, 4, 128, 0))) == -1
    assert lib.mf_param_count(None) == -1


def _dom(ux=2, uy=2, pitch=None, cpu=32, stride=16):
    return DomainDesc(ux, uy, cpu, stride, pitch if pitch is not None else 32 * ux + 1, 0)


def test_workspace_size(lib):
    n = ctypes.c_size_t()
    d = SdnetDesc(256, 4, 128, 0)
    assert lib.mf_workspace_size(ctypes.byref(d), ctypes.byref(_dom(16, 16)), 1, MF_FP32, 0, 0,
                                 ctypes.byref(n)) == MF_OK
    fp32 = n.value
    assert fp32 >= 3 * 256 * 256 * 4 + 32769 * 4
    assert lib.mf_workspace_size(ctypes.byref(d), ctypes.byref(_dom(16, 16)), 1, MF_BF16, 0, 0,
                                 ctypes.byref(n)) == MF_OK
    assert n.value < fp32
    assert lib.mf_workspace_size(ctypes.byref(d), ctypes.byref(_dom(0, 2)), 1, MF_FP32, 0, 0,
                                 ctypes.byref(n)) == MF_ESHAPE
    assert b"units" in lib.mf_last_error()
    assert lib.mf_workspace_size(ctypes.byref(d), ctypes.byref(_dom(2, 2, cpu=16)), 1, MF_FP32, 0, 0,
                                 ctypes.byref(n)) == MF_ESHAPE
    assert lib.mf_workspace_size(ctypes.byref(d), ctypes.byref(_dom()), 1, 7, 0, 0,
                                 ctypes.byref(n)) == MF_EINVAL
    assert lib.mf_workspace_size(ctypes.byref(d), ctypes.byref(_dom()), 1, MF_FP32, 0, 0, None) == MF_EINVAL
    # target set and sweep mode: unknown values are rejected; the additive
    # mode adds one field-sized buffer (the next field) to the workspace
    assert lib.mf_workspace_size(ctypes.byref(d), ctypes.byref(_dom()), 1, MF_FP32, 2, 0,
                                 ctypes.byref(n)) == MF_EINVAL
    assert lib.mf_workspace_size(ctypes.byref(d), ctypes.byref(_dom()), 1, MF_FP32, 0, 2,
                                 ctypes.byref(n)) == MF_EINVAL
    assert lib.mf_workspace_size(ctypes.byref(d), ctypes.byref(_dom(16, 16)), 1, MF_FP32, 1, 1,
                                 ctypes.byref(n)) == MF_OK
    assert n.value >= fp32 + 513 * 513 * 4


@pytest.mark.skipif(_has_gpu(), reason="checks the no-GPU path")
def test_ctx_create_without_gpu(lib):
    p = ctypes.c_void_p()
    assert lib.mf_ctx_create(0, ctypes.byref(p)) == MF_EDEVICE
    assert not p.value
    assert len(lib.mf_last_error()) > 0


FAKE = 1 << 20       # a 256-byte aligned non-null address that is never dereferenced


def _sweep(lib, *, ctx=None, desc=None, params=FAKE, u=FAKE, dom=None, nd=1, colour=-1,
           targets=MF_CROSS, mode=0, prec=MF_FP32, ws=FAKE, ws_bytes=1 << 30):
    desc = desc or SdnetDesc(128, 4, 128, 0)
    dom = dom or _dom()
    return lib.mf_sweep(ctx, ctypes.byref(desc), ctypes.c_void_p(params) if params else None,
                        ctypes.c_void_p(u) if u else None, ctypes.byref(dom), nd, colour, targets,
                        mode, prec, ctypes.c_void_p(ws) if ws else None, ws_bytes, None)


def test_sweep_argument_errors(lib):
    assert _sweep(lib) == MF_EINVAL and b"ctx" in lib.mf_last_error()   # all else valid
    assert _sweep(lib, params=0) == MF_EINVAL and b"params" in lib.mf_last_error()
    assert _sweep(lib, u=FAKE + 2) == MF_EINVAL and b"aligned" in lib.mf_last_error()
    assert _sweep(lib, desc=SdnetDesc(64, 4, 128, 0)) == MF_ESHAPE
    assert _sweep(lib, desc=SdnetDesc(128, 3, 128, 0)) == MF_ESHAPE
    assert _sweep(lib, desc=SdnetDesc(128, 4, 128, 5)) == MF_EINVAL
    assert _sweep(lib, dom=_dom(2, 2, pitch=64)) == MF_ESHAPE and b"pitch" in lib.mf_last_error()
    assert _sweep(lib, dom=_dom(2, 2, stride=8)) == MF_ESHAPE
    assert _sweep(lib, nd=0) == MF_ESHAPE
    two = (DomainDesc * 2)(_dom(), _dom())             # same offsets: overlapping
    assert lib.mf_sweep(None, ctypes.byref(SdnetDesc(128, 4, 128, 0)), ctypes.c_void_p(FAKE),
                        ctypes.c_void_p(FAKE), two, 2, -1, MF_CROSS, 0, MF_FP32,
                        ctypes.c_void_p(FAKE), 1 << 30, None) == MF_EINVAL
    assert b"overlap" in lib.mf_last_error()
    two[1].field_offset = 65 * 65
    assert lib.mf_sweep(None, ctypes.byref(SdnetDesc(128, 4, 128, 0)), ctypes.c_void_p(FAKE),
                        ctypes.c_void_p(FAKE), two, 2, -1, MF_CROSS, 0, MF_FP32,
                        ctypes.c_void_p(FAKE), 1 << 30, None) == MF_EINVAL
    assert b"ctx" in lib.mf_last_error()               # a valid batch gets as far as the ctx
    assert _sweep(lib, colour=4) == MF_EINVAL
    assert _sweep(lib, targets=3) == MF_EINVAL
    assert _sweep(lib, mode=1) == MF_EINVAL and b"ctx" in lib.mf_last_error()   # additive is valid
    assert _sweep(lib, mode=1, colour=2) == MF_EINVAL and b"additive" in lib.mf_last_error()
    assert _sweep(lib, mode=2) == MF_EINVAL
    assert _sweep(lib, prec=2) == MF_EINVAL and b"ctx" in lib.mf_last_error()   # MF_FP16 is valid
    assert _sweep(lib, prec=3) == MF_EINVAL and b"precision" in lib.mf_last_error()
    assert _sweep(lib, ws=0) == MF_EINVAL
    assert _sweep(lib, ws=FAKE + 64) == MF_EINVAL
    assert _sweep(lib, ws_bytes=1024) == MF_ENOMEM and b"needed" in lib.mf_last_error()


def test_solve_argument_errors(lib):
    d = SdnetDesc(128, 4, 128, 0)
    dom = _dom()

    def solve(max_sweeps=10, eps=0.0, check_every=1, flags=0, u_out=None, u=FAKE):
        return lib.mf_solve(None, ctypes.byref(d), ctypes.c_void_p(FAKE), ctypes.c_void_p(u),
                            ctypes.byref(dom), 1, MF_CROSS, 0, MF_FP32, max_sweeps, eps,
                            check_every, flags, ctypes.c_void_p(u_out) if u_out else None, None,
                            None, ctypes.c_void_p(FAKE), 1 << 30, None)

    assert solve() == MF_EINVAL and b"ctx" in lib.mf_last_error()
    assert solve(max_sweeps=-1) == MF_EINVAL
    assert solve(eps=-1.0) == MF_EINVAL
    assert solve(eps=float("nan")) == MF_EINVAL
    assert solve(eps=1e-3, check_every=0) == MF_EINVAL
    assert solve(flags=8) == MF_EINVAL
    assert solve(u_out=FAKE) == MF_EINVAL and b"alias" in lib.mf_last_error()


def test_forward_argument_errors(lib):
    d = SdnetDesc(256, 4, 128, 0)
    n = ctypes.c_size_t()
    assert lib.sdnet_forward_ws_size(ctypes.byref(d), 1000, 7, 0, MF_FP32, ctypes.byref(n)) == MF_OK
    assert n.value >= 1000 * 256 * 4
    f = ctypes.c_void_p(FAKE)
    assert lib.sdnet_forward(None, ctypes.byref(d), f, f, 10, f, 5, 0, f, None, None, MF_FP32, f,
                             n.value, None) == MF_EINVAL
    assert lib.sdnet_forward(None, ctypes.byref(d), f, f, -1, f, 5, 0, f, None, None, MF_FP32, f,
                             n.value, None) == MF_ESHAPE
    assert lib.sdnet_forward(None, ctypes.byref(d), f, f, 10, f, 5, 2, f, None, None, MF_FP32, f,
                             n.value, None) == MF_EINVAL
    assert lib.sdnet_forward(None, ctypes.byref(d), f, f, 10, f, 5, 0, f, None, None, MF_FP32, f,
                             16, None) == MF_ENOMEM


def test_operator_argument_errors(lib):
    f = ctypes.c_void_p(FAKE)
    dom = _dom()
    op = lib.mf_sweep_operator
    assert op(None, f, 61, MF_CROSS, f, None, ctypes.byref(dom), -1, None) == MF_EINVAL
    assert b"ctx" in lib.mf_last_error()
    assert op(None, f, 961, MF_CROSS, f, None, ctypes.byref(dom), -1, None) == MF_ESHAPE
    assert op(None, f, 61, MF_INTERIOR, f, None, ctypes.byref(dom), -1, None) == MF_ESHAPE
    assert op(None, f, 61, MF_CROSS, f, f, ctypes.byref(dom), 4, None) == MF_EINVAL
    assert b"INTERIOR" in lib.mf_last_error()
    assert op(None, None, 61, MF_CROSS, f, None, ctypes.byref(dom), -1, None) == MF_EINVAL


def test_train_and_loss_grad_argument_errors(lib):
    d = SdnetDesc(128, 4, 128, 0)
    f = ctypes.c_void_p(FAKE)
    big = 1 << 40

    def train(m=f, v=f, step=1, grad=None, B=4, hp=True, nd=128, per_bc=0, Yd=None):
        adam = _lib.Adam(1e-3, 0.9, 0.999, 1e-8)
        return lib.sdnet_train_step(None, ctypes.byref(d), f, m, v, step,
                                    ctypes.byref(adam) if hp else None, f, B, f, nd, per_bc, Yd, f, 8, f,
                                    grad, f, big, None)

    assert train() == MF_EINVAL and b"ctx" in lib.mf_last_error()      # all else valid
    assert train(m=None) == MF_EINVAL and b"m is NULL" in lib.mf_last_error()
    assert train(step=0) == MF_EINVAL
    assert train(hp=False) == MF_EINVAL
    assert train(B=0) == MF_ESHAPE
    assert train(nd=0, Yd=f) == MF_ESHAPE
    assert train(m=None, v=None, hp=False, grad=f) == MF_EINVAL and b"ctx" in lib.mf_last_error()
    # without targets the data term is the boundary match: nd must be 128
    assert train(nd=64) == MF_ESHAPE and b"nd must be 128" in lib.mf_last_error()
    assert train(nd=64, per_bc=1, Yd=f) == MF_EINVAL and b"ctx" in lib.mf_last_error()
    assert train(per_bc=2) == MF_EINVAL and b"xd_per_bc" in lib.mf_last_error()

    def loss_grad(grad=f, ws_bytes=big):
        return lib.sdnet_loss_grad(None, ctypes.byref(d), f, f, 4, f, 128, 0, None, f, 8, f, grad, f, ws_bytes,
                                   None)

    assert loss_grad() == MF_EINVAL and b"ctx" in lib.mf_last_error()
    assert loss_grad(grad=None) == MF_EINVAL and b"grad_out is NULL" in lib.mf_last_error()
    assert loss_grad(ws_bytes=1024) == MF_ENOMEM


def test_colour_placements_and_target_coords(lib):
    from oracle import geometry as geo
    for ux, uy in ((16, 16), (1, 1), (3, 5), (64, 64)):
        dom = _dom(ux, uy)
        for c in range(4):
            want = len(geo.placements_of_colour(ux, uy, c))
            assert lib.mf_colour_placements(ctypes.byref(dom), c) == want, (ux, uy, c)
    assert [lib.mf_colour_placements(ctypes.byref(_dom(16, 16)), c) for c in range(4)] == [256, 240, 240, 225]
    assert lib.mf_colour_placements(ctypes.byref(_dom(2, 2)), 4) == -1
    assert lib.mf_colour_placements(ctypes.byref(_dom(0, 2)), 0) == -1
    assert lib.mf_colour_placements(None, 0) == -1
    for targets, kind in ((MF_CROSS, "cross"), (MF_INTERIOR, "interior")):
        want = [(i / 32.0, j / 32.0) for (i, j) in geo.targets(kind)]
        X = (ctypes.c_float * (2 * len(want)))()
        assert lib.mf_target_coords(targets, X) == MF_OK
        got = [(X[2 * t], X[2 * t + 1]) for t in range(len(want))]
        assert got == want
    assert lib.mf_target_coords(2, X) == MF_EINVAL
    assert lib.mf_target_coords(MF_CROSS, None) == MF_EINVAL


def test_gather_scatter_argument_errors(lib):
    f = ctypes.c_void_p(FAKE)
    dom = _dom(3, 2)
    assert lib.mf_gather(None, f, ctypes.byref(dom), 0, f, None) == MF_EINVAL
    assert b"ctx" in lib.mf_last_error()                              # all else valid
    assert lib.mf_gather(None, f, ctypes.byref(dom), 4, f, None) == MF_EINVAL
    assert lib.mf_gather(None, None, ctypes.byref(dom), 0, f, None) == MF_EINVAL
    assert lib.mf_gather(None, f, ctypes.byref(dom), 0, None, None) == MF_EINVAL
    assert b"G is NULL" in lib.mf_last_error()
    assert lib.mf_gather(None, f, ctypes.byref(_dom(3, 2, pitch=64)), 0, f, None) == MF_ESHAPE
    one = _dom(1, 1)                                                   # colour 3 is empty: nothing to do
    assert lib.mf_gather(None, f, ctypes.byref(one), 3, None, None) == MF_OK
    assert lib.mf_scatter(None, f, MF_CROSS, f, ctypes.byref(dom), 1, None) == MF_EINVAL
    assert b"ctx" in lib.mf_last_error()
    assert lib.mf_scatter(None, f, 2, f, ctypes.byref(dom), 1, None) == MF_EINVAL
    assert lib.mf_scatter(None, None, MF_INTERIOR, f, ctypes.byref(dom), 1, None) == MF_EINVAL
    assert lib.mf_scatter(None, f, MF_CROSS, f, ctypes.byref(dom), -1, None) == MF_EINVAL
    assert lib.mf_scatter(None, None, MF_CROSS, f, ctypes.byref(one), 1, None) == MF_OK


def _noalloc(lib, *, ctx=None, desc=None, params=FAKE, u=FAKE, dom=None, nd=1, colour=-1,
             targets=MF_CROSS, prec=MF_FP32):
    desc = desc or SdnetDesc(128, 4, 128, 0)
    dom = dom if dom is not None else _dom()
    dom_arg = dom if isinstance(dom, ctypes.Array) else ctypes.byref(dom)
    return lib.mf_sweep_noalloc(ctx, ctypes.byref(desc), ctypes.c_void_p(params) if params else None,
                                ctypes.c_void_p(u) if u else None, dom_arg, nd, colour, targets, prec,
                                None)


def test_sweep_noalloc_argument_errors(lib):
    assert _noalloc(lib) == MF_EINVAL and b"ctx" in lib.mf_last_error()   # all else valid
    assert _noalloc(lib, params=0) == MF_EINVAL and b"params" in lib.mf_last_error()
    assert _noalloc(lib, u=FAKE + 2) == MF_EINVAL and b"aligned" in lib.mf_last_error()
    assert _noalloc(lib, desc=SdnetDesc(64, 4, 128, 0)) == MF_ESHAPE
    assert _noalloc(lib, colour=4) == MF_EINVAL
    assert _noalloc(lib, targets=3) == MF_EINVAL
    assert _noalloc(lib, prec=3) == MF_EINVAL
    # the static scratch holds the width-256 fp32 network (924,928 bytes) plus
    # 56 bytes per domain of a batch: 2,207 one-unit domains fit, 2,300 do not
    for n, want in ((2207, MF_EINVAL), (2300, MF_ENOMEM)):
        many = (DomainDesc * n)()
        for i in range(n):
            many[i] = DomainDesc(1, 1, 32, 16, 33, 33 * 33 * i)
        st = _noalloc(lib, desc=SdnetDesc(256, 4, 128, 0), dom=many, nd=n)
        assert st == want, (n, st, lib.mf_last_error())
    assert b"static scratch" in lib.mf_last_error()
    many = (DomainDesc * 2300)()
    for i in range(2300):
        many[i] = DomainDesc(1, 1, 32, 16, 33, 33 * 33 * i)
    assert _noalloc(lib, desc=SdnetDesc(256, 4, 128, 0), dom=many, nd=2300, prec=MF_BF16) == MF_EINVAL


def test_fault_inject_spec_parsing(lib):
    k, c = ctypes.c_int32(-1), ctypes.c_int32(-1)
    assert lib.mf_fault_inject_parse(b"3:2", ctypes.byref(k), ctypes.byref(c)) == 1
    assert (k.value, c.value) == (3, 2)
    for bad in (b"", b"0:1", b"3:4", b"3", b"3:1x", b"a:b", None):
        assert lib.mf_fault_inject_parse(bad, ctypes.byref(k), ctypes.byref(c)) == 0, bad
        assert (k.value, c.value) == (0, 0)


def test_gelu_network_descriptor(lib):
    """The convolutional-embedding GELU network: parameter count, descriptor
    checks, the forms it does not run, and its training workspace."""
    from paper_2308_14258_amd._lib import MF_EUNSUPPORTED
    import mf_inputs as mi
    for d in (128, 256):
        for C in (1, 4, 8):
            g = SdnetDesc(d, 4, 128, 1, C)
            assert lib.mf_param_count(ctypes.byref(g)) == mi.conv_param_count(d, C)
    assert lib.mf_param_count(ctypes.byref(SdnetDesc(256, 4, 128, 1, 0))) == -1
    assert lib.mf_param_count(ctypes.byref(SdnetDesc(256, 4, 128, 1, 9))) == -1
    assert lib.mf_param_count(ctypes.byref(SdnetDesc(256, 4, 128, 0, 4))) == -1
    n = ctypes.c_size_t()
    g = SdnetDesc(256, 4, 128, 1, 4)
    assert lib.mf_workspace_size(ctypes.byref(g), ctypes.byref(_dom(16, 16)), 1, MF_FP32, 0, 0,
                                 ctypes.byref(n)) == MF_OK
    assert n.value >= 2 * 65536 * 256 * 4
    assert lib.mf_workspace_size(ctypes.byref(g), ctypes.byref(_dom(16, 16)), 1, MF_BF16, 0, 0,
                                 ctypes.byref(n)) == MF_EUNSUPPORTED
    assert lib.mf_workspace_size(ctypes.byref(g), ctypes.byref(_dom(16, 16)), 1, MF_FP32, 0, 1,
                                 ctypes.byref(n)) == MF_EUNSUPPORTED
    assert lib.sdnet_train_ws_size(ctypes.byref(g), 4, 128, 8, ctypes.byref(n)) == MF_OK   # trains too
    t = ctypes.c_size_t()
    assert lib.sdnet_train_ws_size(ctypes.byref(SdnetDesc(256, 4, 128, 0)), 4, 128, 8, ctypes.byref(t)) == MF_OK
    assert n.value > t.value   # layer 1's saved pre-activations, the embeddings and convolution partials
    assert lib.mf_adjoint_ws_size(ctypes.byref(g), ctypes.byref(_dom(2, 2)), 1, 0, 2, 1,
                                  ctypes.byref(n)) == MF_OK   # the adjoint takes it too
    assert lib.sdnet_forward_ws_size(ctypes.byref(g), 4, 10, 1, MF_FP32, ctypes.byref(n)) == MF_OK


def test_solve_mixed_argument_errors(lib):
    from paper_2308_14258_amd._lib import MF_FP16
    d = SdnetDesc(128, 4, 128, 0)
    dom = _dom()
    n = ctypes.c_size_t(0)

    def call(prec=MF_BF16, refresh=10, sweeps=5, u_out=None, desc=d, ws=FAKE, ws_bytes=1 << 34, asm=MF_FP32):
        return lib.mf_solve_mixed(None, ctypes.byref(desc), ctypes.c_void_p(FAKE), ctypes.c_void_p(FAKE),
                                  ctypes.byref(dom), 1, MF_CROSS, prec, sweeps, refresh, asm,
                                  ctypes.c_void_p(u_out) if u_out else None, ctypes.c_void_p(ws) if ws else None,
                                  ws_bytes, None)
    assert call() == MF_EINVAL and b"ctx" in lib.mf_last_error()              # all else valid
    assert call(prec=MF_FP16) == MF_EINVAL and b"ctx" in lib.mf_last_error()
    assert call(prec=MF_FP32) == MF_EINVAL and b"MF_BF16 or MF_FP16" in lib.mf_last_error()
    assert call(refresh=0) == MF_EINVAL and b"refresh_every" in lib.mf_last_error()
    assert call(asm=MF_BF16) == MF_EINVAL and b"ctx" in lib.mf_last_error()    # the sweeps' precision
    assert call(asm=MF_FP16) == MF_EINVAL and b"assembly_prec" in lib.mf_last_error()
    assert call(sweeps=-1) == MF_EINVAL
    assert call(u_out=FAKE) == MF_EINVAL and b"alias" in lib.mf_last_error()
    assert call(ws_bytes=1024) == MF_ENOMEM
    assert call(desc=SdnetDesc(128, 4, 128, 1, 4)) != MF_OK                    # the GELU network: not supported
    assert lib.mf_mixed_ws_size(ctypes.byref(d), ctypes.byref(dom), 1, MF_CROSS, MF_BF16, ctypes.byref(n)) == MF_OK
    # three prepared networks, one field copy and four correction fields
    nf = 65 * 65
    assert n.value >= 5 * nf * 4


def test_param_segments_match_the_oracle_layouts(lib):
    """mf_param_segments (host) gives the tensors of the oracle's layouts."""
    from oracle import optim
    n = ctypes.c_int32()
    for desc, want in ((SdnetDesc(128, 4, 128, 0), optim.tanh_segments(128)),
                       (SdnetDesc(256, 4, 128, 0), optim.tanh_segments(256)),
                       (SdnetDesc(128, 4, 128, 1, 4), optim.conv_segments(128, 4))):
        begin = (ctypes.c_int64 * 65)()
        assert lib.mf_param_segments(ctypes.byref(desc), begin, 64, ctypes.byref(n)) == MF_OK
        assert list(begin[:n.value + 1]) == want
        assert begin[n.value] == lib.mf_param_count(ctypes.byref(desc))
    begin = (ctypes.c_int64 * 5)()
    assert lib.mf_param_segments(ctypes.byref(SdnetDesc(128, 4, 128, 0)), begin, 4, ctypes.byref(n)) == MF_ESHAPE
    assert n.value == 10


def test_lr_schedule_matches_the_oracle(lib):
    """mf_lr_at / mf_lr_schedule_scaled (host) against the oracle's
    schedule, over warm-up, decay and the end, for several settings."""
    from oracle import optim
    lr = ctypes.c_double()
    for T, frac, lr0, power, end in ((50000, 0.001, 1e-3, 1.0, 0.0), (400, 0.05, 2e-3, 2.0, 1e-5),
                                     (10, 0.0, 1e-3, 1.0, 0.0), (7, 1.0, 1e-3, 0.5, 0.0)):
        sc = _lib.LrSchedule(lr0, frac, power, end, T)
        for step in sorted({1, 2, 3, 5, 9, 10, 11, 49, 50, 51, 100, 200, 399, 400, 401, T - 1, T, T + 1, 25000}):
            if step < 1:
                continue
            assert lib.mf_lr_at(ctypes.byref(sc), step, ctypes.byref(lr)) == MF_OK
            assert lr.value == pytest.approx(optim.lr_at(step, T, lr0, frac, power, end), rel=1e-12, abs=1e-300)
    out = _lib.LrSchedule()
    sc = _lib.LrSchedule(1e-3, 0.001, 1.0, 0.0, 50000)
    for k in (1.0, 2.0, 8.0, 2000.0):
        assert lib.mf_lr_schedule_scaled(ctypes.byref(sc), k, ctypes.byref(out)) == MF_OK
        want_lr, want_frac = optim.scaled_schedule(1e-3, 0.001, k)
        assert out.max_lr == pytest.approx(want_lr, rel=1e-15) and out.warmup_frac == pytest.approx(want_frac)
        assert out.total_steps == 50000 and out.power == 1.0
    assert lib.mf_lr_at(ctypes.byref(sc), 0, ctypes.byref(lr)) == MF_EINVAL
    bad = _lib.LrSchedule(1e-3, 1.5, 1.0, 0.0, 100)
    assert lib.mf_lr_at(ctypes.byref(bad), 1, ctypes.byref(lr)) == MF_EINVAL
    bad = _lib.LrSchedule(1e-3, 0.1, 0.0, 0.0, 100)
    assert lib.mf_lr_at(ctypes.byref(bad), 1, ctypes.byref(lr)) == MF_EINVAL
    assert lib.mf_lr_schedule_scaled(ctypes.byref(sc), 0.0, ctypes.byref(out)) == MF_EINVAL


def test_lamb_step_argument_errors(lib):
    FAKE = 1 << 40
    hp = _lib.Lamb(1e-3, 0.9, 0.999, 1e-6, 0.0, 1.0, 1)

    def call(seg=(0, 10, 20), n=None, step=1, h=hp, ptr=FAKE):
        arr = (ctypes.c_int64 * len(seg))(*seg)
        return lib.sdnet_lamb_step(None, ctypes.c_void_p(ptr), ctypes.c_void_p(FAKE), ctypes.c_void_p(FAKE),
                                   ctypes.c_void_p(FAKE), arr, len(seg) - 1 if n is None else n, step,
                                   ctypes.byref(h), None)
    assert call() == MF_EINVAL and b"ctx" in lib.mf_last_error()              # all else valid
    assert call(seg=(1, 10)) == MF_EINVAL and b"seg_begin[0]" in lib.mf_last_error()
    assert call(seg=(0, 10, 5)) == MF_EINVAL and b"decreases" in lib.mf_last_error()
    assert call(seg=(0, 0)) == MF_EINVAL and b"no parameters" in lib.mf_last_error()
    assert call(seg=(0, 0, 7)) == MF_EINVAL and b"ctx" in lib.mf_last_error()   # empty tensors are allowed
    assert call(n=0) == MF_EINVAL and b"n_segments" in lib.mf_last_error()
    assert call(seg=tuple(range(66)), n=65) == MF_EINVAL and b"n_segments" in lib.mf_last_error()
    assert call(step=0) == MF_EINVAL
    assert call(ptr=0) == MF_EINVAL and b"params" in lib.mf_last_error()
    assert call(h=_lib.Lamb(1e-3, 1.0, 0.999, 1e-6, 0.0, 0.0, 1)) == MF_EINVAL
    assert call(h=_lib.Lamb(1e-3, 0.9, 0.999, 1e-6, -1.0, 0.0, 1)) == MF_EINVAL
    assert call(h=_lib.Lamb(1e-3, 0.9, 0.999, 1e-6, 0.0, 0.0, 2)) == MF_EINVAL
