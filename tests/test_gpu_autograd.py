"""The autograd bridge (DeepInverseFn / DeepInverse) and activation recomputation,
through the C ABI.

* torch.autograd.grad through the module against the FP64 oracle's
  backpropagation (Sec. 4) on the GPU's own forward state: FP32 <= 1e-5, BF16
  <= 2e-2 per tensor (dy included); end to end against the oracle's own forward
  state within that plus 3 sqrt(fraction of ReLU units whose activity differs).
* recompute = 1 (only the proxy and the output kept, hidden layers recomputed in
  the backward pass) gives bit-identical gradients to recompute = 0 when the
  batch is one chunk, and the same sums reassociated (<= 1e-6 per tensor) when a
  small recompute budget splits it into chunks.
* a small saved-state budget makes the module select recompute.
"""
import numpy as np
import pytest
import torch

import oracle
from cases import make_case

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def _rel(a, ref):
    a = np.asarray(a, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return np.linalg.norm(a - ref) / max(np.linalg.norm(ref), 1e-300)


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1701_03891_amd.autograd import DeepInverse
    return DeepInverse


def _module(DeepInverse, case, prec, **kw):
    return DeepInverse(case.n1, case.n2, case.M, case.phi.T, case.w, case.b, prec=prec, C=case.C, k=case.k,
                       bias_per_pixel=case.bias_per_pixel, relu_last=case.relu_last, **kw)


def _grads(mod, case, want_y=True):
    y = _t(case.y).requires_grad_(want_y)
    x = _t(case.x).reshape(case.B, case.n1, case.n2)
    xh = mod(y)
    loss = ((xh - x) ** 2).sum() / case.B          # Sec. 4: sum over pixels, mean over the batch
    params = [*mod.w, *mod.b] + ([y] if want_y else [])
    g = torch.autograd.grad(loss, params)
    L = len(mod.w)
    return loss.item(), [t.cpu().numpy() for t in g[:L]], [t.cpu().numpy() for t in g[L:2 * L]], \
        (g[2 * L].cpu().numpy() if want_y else None)


def _oracle(case):
    G = oracle.backward(case.oracle_net(), case.phi.T, case.w, case.oracle_bias(), case.y, case.x, want_gy=True)
    gb = [oracle.crop_full(G.b[l], case.k[l]) if case.bias_per_pixel else G.b[l] for l in range(len(case.k))]
    return G.loss, G.w, gb, G.y


def _same_state_oracle(mod, case):
    """The oracle's FP64 backpropagation on the forward state the module's network
    produces (its saved activations, through the C ABI), with the module's loss
    gradient dL/dxhat = (2/B)(xhat - x), and the fraction of hidden units whose
    activity differs from the oracle's own FP64 forward pass."""
    net, B, L = mod.net, case.B, len(case.k)
    xh, saved = net.forward_train(_t(case.y))
    acts = [net.saved_activation(saved, B, l).cpu().numpy().astype(np.float64) for l in range(L + 1)]
    g_out = (2.0 / B) * (xh.reshape(B, -1).cpu().numpy().astype(np.float64) - case.x)
    H = oracle.backward_acts(case.oracle_net(), case.phi.T, case.w, case.y,
                             [[acts[l][b] for l in range(L + 1)] for b in range(B)], g_out, want_gy=True)
    gb = [oracle.crop_full(H.b[l], case.k[l]) if case.bias_per_pixel else H.b[l] for l in range(L)]
    _, ref = oracle.forward(case.oracle_net(), case.phi.T, case.w, case.oracle_bias(), case.y, return_acts=True)
    f = max(float(np.mean((acts[l] > 0) != (np.stack([r[l] for r in ref]) > 0))) for l in range(1, L))
    return H.w, gb, H.y, f


@pytest.mark.parametrize("prec,shape", [("f32", (40, 48, 500, 3, (1, 64, 32, 1), (11, 11, 11))),
                                        ("f32", (16, 16, 64, 3, (1, 4, 2, 1), (5, 5, 5))),
                                        ("bf16", (40, 48, 500, 3, (1, 64, 32, 1), (11, 11, 11)))])
def test_autograd_matches_oracle(mods, prec, shape):
    """torch.autograd.grad of L = (1/B) sum ||xhat - x||^2 through the module: every
    gradient (dy included) against the oracle's backpropagation on the same forward
    state (FP32 1e-5, BF16 2e-2 per tensor), and against the oracle end to end within
    that tolerance plus 3 sqrt(f), f the fraction of hidden units whose ReLU activity
    differs between the GPU's and the oracle's forward pass (a flipped unit changes
    one whole term of the gradient sums)."""
    n1, n2, M, B, C, k = shape
    case = make_case(n1, n2, M, B, cfg_id=81, C=C, k=k, bias_std=0.05)
    mod = _module(mods, case, prec)
    loss, gw, gb, gy = _grads(mod, case)
    tol = {"f32": 1e-5, "bf16": 2e-2}[prec]
    hw, hb, hy, f = _same_state_oracle(mod, case)
    errs = {"y": _rel(gy, hy)}
    for l in range(len(hw)):
        errs[f"w{l}"], errs[f"b{l}"] = _rel(gw[l], hw[l]), _rel(gb[l], hb[l])
    print(f"autograd {prec} {shape[:4]} same state:", " ".join(f"{a}={v:.2e}" for a, v in errs.items()))
    assert max(errs.values()) <= tol, errs
    lr, wr, br, yr = _oracle(case)
    e2e = {"y": _rel(gy, yr)}
    for l in range(len(wr)):
        e2e[f"w{l}"], e2e[f"b{l}"] = _rel(gw[l], wr[l]), _rel(gb[l], br[l])
    bound = tol + 3.0 * np.sqrt(f)
    print(f"autograd {prec} end to end (flipped {f:.2e}, bound {bound:.2e}): loss={abs(loss - lr) / lr:.2e}",
          " ".join(f"{a}={v:.2e}" for a, v in e2e.items()))
    assert max(e2e.values()) <= bound, e2e
    assert abs(loss - lr) / lr <= tol
    mod.close()


@pytest.mark.parametrize("prec", ["bf16", "f32"])
def test_recompute_bitwise_and_chunked(mods, prec):
    """64x64, batch 24: recompute (one chunk) gives the saved-activation gradients bit
    for bit; a recompute budget of about five images' workspace splits the batch into
    chunks, whose gradients agree to FP32 reassociation."""
    case = make_case(64, 64, 1024, 24, cfg_id=83, bias_std=0.02)
    mod = _module(mods, case, prec, recompute=False)
    ref = _grads(mod, case)
    mod.recompute = True
    rc = _grads(mod, case)
    assert mod.last_recompute is True
    assert rc[0] == ref[0]
    for a, b in zip(rc[1] + rc[2] + [rc[3]], ref[1] + ref[2] + [ref[3]]):
        assert np.array_equal(a, b)
    # saved state: proxy + output only
    assert mod.net.saved_bytes(24, recompute=True) * 5 < mod.net.saved_bytes(24, recompute=False)
    # chunks of a few images
    per_image = mod.net.saved_bytes(1, recompute=False)
    mod.ctx.set_recompute_budget(6 * per_image)
    ch = _grads(mod, case)
    mod.ctx.set_recompute_budget(0)
    errs = [_rel(a, b) for a, b in zip(ch[1] + ch[2] + [ch[3]], ref[1] + ref[2] + [ref[3]])]
    print(prec, "chunked recompute vs saved: max rel diff", max(errs))
    assert max(errs) <= 1e-6
    assert np.array_equal(ch[3], ref[3])        # dy is per image: unchanged by chunking
    mod.close()


def test_small_budget_selects_recompute(mods):
    case = make_case(32, 32, 256, 8, cfg_id=84, bias_std=0.02)
    mod = _module(mods, case, "bf16", saved_budget_bytes=1 << 10)
    g_rc = _grads(mod, case)
    assert mod.last_recompute is True
    mod.saved_budget_bytes = 1 << 40
    g_sv = _grads(mod, case)
    assert mod.last_recompute is False
    for a, b in zip(g_rc[1] + g_rc[2], g_sv[1] + g_sv[2]):
        assert np.array_equal(a, b)
    mod.close()


def test_module_trains_with_torch_adam_and_repacks(mods):
    """The module under torch.optim.Adam: parameters change in place, the next forward
    re-packs the network from them (its output equals a freshly prepared network's),
    and the loss falls."""
    import paper_1701_03891_amd as P
    case = make_case(24, 24, 150, 8, cfg_id=85, bias_std=0.02)
    mod = _module(mods, case, "bf16")
    opt = torch.optim.Adam([*mod.w, *mod.b], lr=1e-3)
    y, x = _t(case.y), _t(case.x).reshape(8, 24, 24)
    losses = []
    for _ in range(30):
        opt.zero_grad()
        loss = ((mod(y) - x) ** 2).sum() / 8
        loss.backward()
        opt.step()
        losses.append(loss.item())
    print("module + torch Adam: loss", losses[0], "->", losses[-1])
    assert losses[-1] < 0.7 * losses[0]
    with torch.no_grad():
        out = mod(y)
    fresh = mod.ctx.prepare(24, 24, 150, P.NetParams(mod.w_fc.data, [t.data for t in mod.w], [t.data for t in mod.b]),
                            prec="bf16")
    assert torch.equal(out, fresh.recover(y))
    fresh.free()
    mod.close()
