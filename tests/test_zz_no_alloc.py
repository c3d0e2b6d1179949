"""The allocation-free recovery entry point (dsi_recover_noalloc) through the C
ABI: on two calls in a row, the second with a smaller batch (and, for BF16, a
second network of another image size), its output equals dsi_recover's bit for
bit -- the same kernels on the same inputs, only the workspace differs -- and a
batch beyond the fixed workspace fails with DSI_E_SHAPE, leaving the output
untouched."""
import ctypes

import numpy as np
import pytest

from cases import make_case

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def _noalloc(ctx, net, y, B):
    import torch

    from paper_1701_03891_amd import _lib
    out = torch.full((B, net.n1, net.n2), 3.0, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = _lib.lib().dsi_recover_noalloc(ctx.h, net.h, ctypes.c_void_p(y.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), B, s)
    return st, out


@pytest.mark.parametrize("prec,B", [("bf16", 48), ("f32", 32), ("fp8", 48)])
def test_noalloc_equals_recover(prec, B):
    import torch

    import paper_1701_03891_amd as P
    from paper_1701_03891_amd import _lib
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = P.Context(0)
    case = make_case(64, 64, 1024, B, cfg_id=71, bias_std=0.02)
    net = ctx.prepare(64, 64, 1024, case.torch_params(), prec=prec)
    if prec == "fp8":
        net.set_act_scales([2.0 ** -6, 1.0, 2.0 ** -7, 1.0])
    assert net.workspace_size(B) <= _lib.NOALLOC_SCRATCH_BYTES
    y = _t(case.y)
    ref = net.recover(y)
    st, out = _noalloc(ctx, net, y, B)
    assert st == _lib.DSI_OK, _lib.dsi_last_error()
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    # second call, smaller batch: the fixed workspace keeps the first call's contents
    b2 = 5
    y2 = y[7:7 + b2].contiguous()
    st, out2 = _noalloc(ctx, net, y2, b2)
    assert st == _lib.DSI_OK, _lib.dsi_last_error()
    assert torch.equal(out2, net.recover(y2))
    if prec == "bf16":
        # a second network (32 x 32, M = 256) on the same fixed workspace
        c2 = make_case(32, 32, 256, 3, cfg_id=72, bias_std=0.02)
        net2 = ctx.prepare(32, 32, 256, c2.torch_params(), prec="bf16")
        y3 = _t(c2.y)
        st, out3 = _noalloc(ctx, net2, y3, 3)
        assert st == _lib.DSI_OK, _lib.dsi_last_error()
        assert torch.equal(out3, net2.recover(y3))
        net2.free()
    # beyond the fixed workspace: a clear error before any launch, output untouched
    big = 1
    while net.workspace_size(big) <= _lib.NOALLOC_SCRATCH_BYTES:
        big *= 2
    ybig = torch.zeros((big, 1024), device="cuda")
    st, outb = _noalloc(ctx, net, ybig, big)
    assert st == _lib.DSI_E_SHAPE
    assert "fixed workspace" in _lib.dsi_last_error()
    torch.cuda.synchronize()
    assert torch.all(outb == 3.0)
    net.free()
    ctx.close()
