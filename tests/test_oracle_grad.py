"""Pins of the oracle's backpropagation (Sec. 4: L minimised by backprop).

* P12: central finite differences in FP64 on the tiny net (16x16, M = 64,
  1->4->2->1 channels, 5x5 filters), every parameter of a random subset.
* Library routine: torch autograd in float64 on the CPU, on a small paper-like net.
* P18: forward against an independent numpy/scipy implementation.
"""
import numpy as np
import pytest
import scipy.signal

import synth

TINY = dict(n=16, M=64, C=(1, 4, 2, 1), k=(5, 5, 5))


def _tiny(orc, bias_full, relu_last=False, seed=0):
    n, M, C, k = TINY["n"], TINY["M"], TINY["C"], TINY["k"]
    net = orc.Net(n, n, M, C=C, k=k, bias_full=bias_full, relu_last=relu_last)
    p = synth.he_init(synth.Arch(C, k), n, n, bias_per_pixel=bias_full, cfg_id=50 + seed, bias_std=0.1)
    bs = [orc.full_bias_from_cropped(p.b[l], k[l], border=0.3) if bias_full else p.b[l] for l in range(3)]
    phi = synth.make_phi(M, n * n, cfg_id=50 + seed)
    x = synth.piecewise_smooth_images(3, n, cfg_id=50 + seed).reshape(3, -1)
    y = orc.measure(phi, x)
    return net, phi, p.w, bs, x, y


def _loss(orc, net, wfc, ws, bs, y, x):
    return orc.loss(orc.forward(net, wfc, ws, bs, y), x)[0]


@pytest.mark.parametrize("bias_full,relu_last", [(True, False), (False, False), (True, True)])
def test_p12_finite_differences_tiny_net(orc, bias_full, relu_last):
    net, phi, ws, bs, x, y = _tiny(orc, bias_full, relu_last)
    wfc = phi.T.copy()
    G = orc.backward(net, wfc, ws, bs, y, x, want_gy=True, want_gwfc=True)
    assert G.loss == pytest.approx(_loss(orc, net, wfc, ws, bs, y, x), rel=1e-14)
    g = synth.rng(77, int(bias_full) + 2 * int(relu_last))
    checked = 0

    def fd(get, set_, idx):
        th = get()[idx]
        h = 1e-6 * max(1.0, abs(th))
        set_(idx, th + h)
        lp = _loss(orc, net, wfc, ws, bs, y, x)
        set_(idx, th - h)
        lm = _loss(orc, net, wfc, ws, bs, y, x)
        set_(idx, th)
        return (lp - lm) / (2 * h)

    def close(a, ref, scale):
        return abs(a - ref) <= 1e-6 * max(abs(ref), 1e-3 * scale)

    for l in range(3):
        gw_scale = np.abs(G.w[l]).max()
        for _ in range(12):
            idx = tuple(int(g.integers(0, s)) for s in ws[l].shape)

            def set_w(i, v, l=l):
                ws[l][i] = v
            num = fd(lambda l=l: ws[l], set_w, idx)
            assert close(G.w[l][idx], num, gw_scale), (l, idx, G.w[l][idx], num)
            checked += 1
        gb_scale = np.abs(G.b[l]).max()
        for _ in range(8):
            idx = tuple(int(g.integers(0, s)) for s in bs[l].shape)

            def set_b(i, v, l=l):
                bs[l][i] = v
            num = fd(lambda l=l: bs[l], set_b, idx)
            assert close(G.b[l][idx], num, gb_scale), (l, idx, G.b[l][idx], num)
            checked += 1
    for _ in range(6):
        idx = (int(g.integers(0, y.shape[0])), int(g.integers(0, y.shape[1])))

        def set_y(i, v):
            y[i] = v
        num = fd(lambda: y, set_y, idx)
        assert close(G.y[idx], num, np.abs(G.y).max())
        idx2 = (int(g.integers(0, wfc.shape[0])), int(g.integers(0, wfc.shape[1])))

        def set_f(i, v):
            wfc[i] = v
        num = fd(lambda: wfc, set_f, idx2)
        assert close(G.wfc[idx2], num, np.abs(G.wfc).max())
        checked += 2
    assert checked >= 70
    if bias_full:
        # the crop S passes no gradient to the padding borders of the full-grid bias
        for l in range(3):
            gbf = G.b[l]
            r = (net.k[l] - 1) // 2
            inner = gbf[:, r:-r, r:-r].copy()
            gbf2 = gbf.copy()
            gbf2[:, r:-r, r:-r] = 0
            assert np.all(gbf2 == 0) and np.abs(inner).max() > 0


def test_backward_matches_torch_autograd(orc):
    """Library routine: torch autograd (float64, CPU) on a small paper-shaped net."""
    import torch
    import torch.nn.functional as F

    n1, n2, M, B = 12, 14, 50, 2
    C, k = (1, 6, 3, 1), (11, 11, 11)
    net = orc.Net(n1, n2, M, C=C, k=k, bias_full=True)
    p = synth.he_init(synth.Arch(C, k), n1, n2, True, cfg_id=60, bias_std=0.05)
    bs = [orc.full_bias_from_cropped(p.b[l], 11) for l in range(3)]
    phi = synth.make_phi(M, n1 * n2, cfg_id=60)
    x = synth.piecewise_smooth_images(B, n1, n2, cfg_id=60).reshape(B, -1)
    y = orc.measure(phi, x)
    G = orc.backward(net, phi.T, p.w, bs, y, x, want_gy=True)

    tw = [torch.tensor(w, requires_grad=True) for w in p.w]
    tb = [torch.tensor(b, requires_grad=True) for b in p.b]
    ty = torch.tensor(y, requires_grad=True)
    a = (ty @ torch.tensor(phi)).reshape(B, 1, n1, n2)
    for l in range(3):
        a = F.conv2d(a, tw[l], padding=5) + tb[l][None]
        if l < 2:
            a = torch.relu(a)
    loss = ((a.reshape(B, -1) - torch.tensor(x)) ** 2).sum() / B
    loss.backward()
    assert G.loss == pytest.approx(loss.item(), rel=1e-12)
    for l in range(3):
        np.testing.assert_allclose(G.w[l], tw[l].grad.numpy(), rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(orc.crop_full(G.b[l], 11), tb[l].grad.numpy(), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(G.y, ty.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_p18_forward_vs_independent_numpy(orc):
    """Forward of the paper's layer shapes on a small image against scipy/numpy loops."""
    n1, n2, M, B = 13, 11, 60, 2
    C, k = (1, 5, 3, 1), (11, 11, 11)
    net = orc.Net(n1, n2, M, C=C, k=k, bias_full=True)
    p = synth.he_init(synth.Arch(C, k), n1, n2, True, cfg_id=61, bias_std=0.1)
    bs = [orc.full_bias_from_cropped(p.b[l], 11, border=5.0) for l in range(3)]
    phi = synth.make_phi(M, n1 * n2, cfg_id=61)
    y = synth.normal_values((B, M), 1.0, 61, 9)
    xhat = orc.forward(net, phi.T, p.w, bs, y)
    for bi in range(B):
        a = (phi.T @ y[bi]).reshape(1, n1, n2)
        for l in range(3):
            z = np.stack([sum(scipy.signal.correlate2d(a[ci], p.w[l][co, ci], mode="same")
                              for ci in range(C[l])) for co in range(C[l + 1])]) + p.b[l]
            a = np.maximum(z, 0) if l < 2 else z
        np.testing.assert_allclose(xhat[bi], a.reshape(-1), rtol=1e-11, atol=1e-12)


def test_backward_from_given_activations_equals_backward(orc):
    """orc_backward_acts on the oracle's own forward activations reproduces orc_backward
    bit for bit (so the FD and autograd pins above carry over to it)."""
    for bias_full, relu_last in ((True, False), (False, True)):
        net, phi, ws, bs, x, y = _tiny(orc, bias_full, relu_last, seed=3)
        G = orc.backward(net, phi.T, ws, bs, y, x, want_gy=True)
        xhat, acts = orc.forward(net, phi.T, ws, bs, y, return_acts=True)
        _, g = orc.loss(xhat, x)
        H = orc.backward_acts(net, phi.T, ws, y, acts, g, want_gy=True)
        for l in range(3):
            assert np.array_equal(H.w[l], G.w[l])
            assert np.array_equal(H.b[l], G.b[l])
        assert np.array_equal(H.y, G.y)
