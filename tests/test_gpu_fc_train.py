"""Training the fully connected layer too (Sec. 4 lists W_fc among the
parameters Omega that backpropagation learns; it is initialised with Phi^T).

dL/dW_fc[p][m] = sum_b dL/dx~[b][p] y[b][m] against the oracle's FP64
gradient: FP32 <= 1e-5, FP64 checking path <= 1e-6, BF16 <= 2e-2 on the
same forward state (the GPU's saved activations, differentiated by the
oracle in FP64).
"""
import numpy as np
import pytest

from cases import make_case

pytestmark = pytest.mark.gpu

GTOL = {"f32": 1e-5, "bf16": 2e-2, "f64": 1e-6}


@pytest.fixture(scope="module")
def dsi():
    import torch

    import paper_1701_03891_amd as P
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = P.Context(0)
    yield P, ctx
    ctx.close()


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def _rel(a, ref):
    a = np.asarray(a, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return np.linalg.norm(a - ref) / max(np.linalg.norm(ref), 1e-300)


def _prepare(ctx, case, prec):
    return ctx.prepare(case.n1, case.n2, case.M, case.torch_params(), prec=prec, C=case.C, k=case.k,
                       bias_per_pixel=case.bias_per_pixel, relu_last=case.relu_last, fc_trainable=True)


@pytest.mark.parametrize("prec,shape", [("f32", (40, 48, 500, 3)), ("f64", (16, 16, 64, 3)),
                                        ("f32", (16, 16, 64, 3))])
def test_fc_gradient_matches_oracle(dsi, prec, shape):
    """Paper net on a ragged 40x48 image (M = 500) in FP32; the tiny net on the
    generic kernels in FP32 and FP64."""
    import oracle
    P, ctx = dsi
    n1, n2, M, B = shape
    tiny = n1 == 16
    kw = dict(C=(1, 4, 2, 1), k=(5, 5, 5)) if tiny else {}
    case = make_case(n1, n2, M, B, cfg_id=61, bias_std=0.05, **kw)
    params = case.torch_params()
    net = _prepare(ctx, case, prec)
    loss, g, _ = net.loss_grad(_t(case.y), _t(case.x), params)
    G = oracle.backward(case.oracle_net(), case.phi.T, case.w, case.oracle_bias(), case.y, case.x,
                        want_gwfc=True)
    e = _rel(g.w_fc.cpu().numpy(), G.wfc)
    print(prec, shape, f"gW_fc rel err {e:.2e}")
    assert e <= GTOL[prec]
    assert abs(loss.item() - G.loss) <= GTOL[prec] * abs(G.loss)
    net.free()


@pytest.mark.parametrize("shape", [(32, 32, 256, 4), (45, 50, 500, 37), (64, 64, 1024, 64)])
def test_fc_gradient_bf16_same_state(dsi, shape):
    """BF16 networks compute dW_fc on the BF16 matrix cores from packed dx~^T and y^T: pixel
    and measurement counts that are not multiples of a 32-row tile and batches that are not
    multiples of a 16-deep k-step exercise the packing tails and the GEMM's edges."""
    import torch

    import oracle
    P, ctx = dsi
    n1, n2, M, B = shape
    case = make_case(n1, n2, M, B, cfg_id=62, bias_std=0.05)
    params = case.torch_params()
    net = _prepare(ctx, case, "bf16")
    y, B = _t(case.y), case.B
    xh, saved = net.forward_train(y)
    acts = [net.saved_activation(saved, B, l).cpu().numpy().astype(np.float64) for l in range(4)]
    g_out = (2.0 / B) * (xh.reshape(B, -1).cpu().numpy().astype(np.float64) - case.x)
    g, _ = net.backward(_t(g_out).reshape(B, n1, n2), saved, params)
    torch.cuda.synchronize()
    H = oracle.backward_acts(case.oracle_net(), case.phi.T, case.w, case.y,
                             [[acts[l][b] for l in range(4)] for b in range(B)], g_out, want_gwfc=True)
    e = _rel(g.w_fc.cpu().numpy(), H.wfc)
    print(f"bf16 {shape} gW_fc same-state rel err {e:.2e}")
    assert e <= GTOL["bf16"]
    net.free()


def test_grads_without_fc_buffer_rejected(dsi):
    """A trainable FC layer needs somewhere to put its gradient."""
    from paper_1701_03891_amd import _lib
    P, ctx = dsi
    case = make_case(16, 16, 64, 2, cfg_id=63)
    params = case.torch_params()
    net = _prepare(ctx, case, "f32")
    g = P.NetParams.grads_like(params, with_fc=False)
    with pytest.raises(P.DsiError) as e:
        _lib.dsi_loss_grad(ctx.h, net.h, _ptr(_t(case.y)), _ptr(_t(case.x)), 2, g.grads_to_c(), None,
                           None, None)
    assert e.value.status == _lib.DSI_E_NULL
    opt = P.AdamState.zeros_like(params)  # no m_fc / v_fc
    with pytest.raises(P.DsiError) as e:
        net.train_step(params, opt, _t(case.y), _t(case.x))
    assert e.value.status == _lib.DSI_E_NULL
    net.free()


def _ptr(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_train_step_updates_fc_with_adam(dsi, prec):
    """One step moves W_fc exactly as the oracle's Adam does with the same gradient;
    further steps keep lowering the loss, and the recovery uses the new W_fc."""
    import torch

    import oracle
    P, ctx = dsi
    case = make_case(24, 24, 150, 4, cfg_id=64, bias_std=0.02)
    params = case.torch_params()
    net = _prepare(ctx, case, prec)
    opt = P.AdamState.zeros_like(params, with_fc=True)
    y, x = _t(case.y), _t(case.x)
    lr = 1e-3
    wfc0 = params.w_fc.cpu().numpy().astype(np.float64)
    _, g, _ = net.loss_grad(y, x, params)
    gfc = g.w_fc.cpu().numpy().astype(np.float64)
    loss0 = net.train_step(params, opt, y, x, lr=lr)
    th, _, _ = oracle.adam(wfc0, gfc, np.zeros_like(wfc0), np.zeros_like(wfc0), 1, lr=lr)
    got = params.w_fc.cpu().numpy().astype(np.float64)
    assert np.abs(got - th).max() <= 1e-6 * lr + 2e-7
    assert np.abs(got - wfc0).max() > 0.5 * lr
    # the net now recovers with the updated W_fc: same as a fresh net prepared from params
    fresh = ctx.prepare(24, 24, 150, params, prec=prec)
    assert torch.equal(net.recover(y), fresh.recover(y))
    fresh.free()
    losses = [loss0.item()]
    for _ in range(30):
        losses.append(net.train_step(params, opt, y, x, lr=lr).item())
    print(prec, "loss with trainable FC", losses[0], "->", losses[-1])
    assert losses[-1] < 0.7 * losses[0]
    net.free()
