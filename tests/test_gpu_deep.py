"""Deeper and wider networks (Sec. 5 leaves larger DeepInverse networks to future
work) on the matrix-core kernels in BF16: stacks of 11 x 11 layers whose hidden
widths are 32 or 64 channels, any depth, against the FP64 oracle with both
parity gates of ``cases.check_recovery`` (norm-wise 2e-2 per image; per pixel
8 sigma of the oracle's BF16 rounding-error model for that network)."""
import numpy as np
import pytest

from cases import check_recovery, make_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dsi():
    import torch

    import paper_1701_03891_amd as P
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = P.Context(0)
    yield P, ctx
    ctx.close()


def _recover(ctx, case, prec="bf16"):
    import torch
    net = ctx.prepare(case.n1, case.n2, case.M, case.torch_params(), prec=prec, C=case.C, k=case.k,
                      bias_per_pixel=case.bias_per_pixel, relu_last=case.relu_last)
    out = net.recover(torch.tensor(case.y, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64).reshape(case.B, -1)
    net.free()
    return got


@pytest.mark.parametrize("C,n1,n2,M,B,bpp", [
    ((1, 64, 64, 32, 1), 64, 64, 1024, 16, True),     # one more 64 -> 64 layer
    ((1, 64, 64, 32, 1), 40, 48, 500, 3, False),      # ragged tiles, per-channel biases
    ((1, 32, 32, 1), 45, 50, 700, 3, True),           # narrower, width not a multiple of 8
    ((1, 32, 64, 64, 32, 64, 1), 24, 40, 300, 2, True),  # L = 6, every layer kind
])
def test_deep_bf16_recovery(dsi, C, n1, n2, M, B, bpp):
    P, ctx = dsi
    L = len(C) - 1
    case = make_case(n1, n2, M, B, cfg_id=90 + L, C=C, k=(11,) * L, bias_per_pixel=bpp, bias_std=0.03)
    check_recovery(case, _recover(ctx, case), "bf16", label=f"C={C} {n1}x{n2}")


def test_deep_bf16_trains_only_in_fp32(dsi):
    """BF16 training needs the paper's architecture: the other stacks train in FP32 (direct
    kernels); their BF16 training calls are refused with DSI_E_DTYPE."""
    import torch

    from paper_1701_03891_amd import _lib
    P, ctx = dsi
    case = make_case(16, 16, 64, 2, cfg_id=97, C=(1, 64, 64, 32, 1), k=(11,) * 4)
    net = ctx.prepare(16, 16, 64, case.torch_params(), prec="bf16", C=case.C, k=case.k)
    y = torch.tensor(case.y, dtype=torch.float32, device="cuda")
    x = torch.tensor(case.x, dtype=torch.float32, device="cuda")
    with pytest.raises(P.DsiError) as e:
        net.loss_grad(y, x, case.torch_params())
    assert e.value.status == _lib.DSI_E_DTYPE
    net.free()
    # other filter sizes or widths stay on FP32 / FP64
    bad = make_case(16, 16, 64, 2, cfg_id=97, C=(1, 48, 32, 1), k=(11,) * 3)
    with pytest.raises(P.DsiError) as e:
        ctx.prepare(16, 16, 64, bad.torch_params(), prec="bf16", C=bad.C, k=bad.k)
    assert e.value.status == _lib.DSI_E_DTYPE
