"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties one part of the oracle to something other than itself: a closed
form, an invariant, a library routine (scipy, numpy, torch CPU in float64) or
brute force on tiny inputs.  The paper (Mousavi & Baraniuk, arXiv 1701.03891)
prints no worked numeric example, so there are no printed values to match.
"""
import math

import numpy as np
import pytest
import scipy.fft
import scipy.signal

import synth

R = 5  # (k - 1) / 2 for the paper's 11x11 filters


def _zero_bias(C, n1, n2, k, full=True):
    return np.zeros((C, n1 + k - 1, n2 + k - 1)) if full else np.zeros(C)


# ------------------------------------------------------------- Eq. (1) pins
def test_p1_centred_delta_is_identity(orc):
    """A centred delta filter maps every channel to itself (ReLU on non-negative input)."""
    x = synth.uniform_values((2, 3, 9, 13), 0.0, 1.0, 101, 5)
    w = np.zeros((3, 3, 11, 11))
    for c in range(3):
        w[c, c, R, R] = 1.0
    out = orc.conv_layer(x, w, _zero_bias(3, 9, 13, 11), relu=True)
    assert np.array_equal(out, x)


@pytest.mark.parametrize("u0,v0", [(2, 7), (0, 0), (10, 10), (5, 0), (9, 3)])
def test_p2_offcentre_delta_shifts(orc, u0, v0):
    """Delta at (u0, v0): out[i][j] = in[i+u0-5][j+v0-5], zeros entering (correlation)."""
    n1, n2 = 12, 15
    x = synth.normal_values((1, 1, n1, n2), 1.0, 102, 5)
    w = np.zeros((1, 1, 11, 11))
    w[0, 0, u0, v0] = 1.0
    out = orc.conv_layer(x, w, np.zeros(1), bias_full=False, relu=False)[0, 0]
    ref = np.zeros((n1, n2))
    for i in range(n1):
        for j in range(n2):
            ii, jj = i + u0 - R, j + v0 - R
            if 0 <= ii < n1 and 0 <= jj < n2:
                ref[i, j] = x[0, 0, ii, jj]
    assert np.array_equal(out, ref)


def test_p3_ones_counts_padding(orc):
    """All-ones filter on an all-ones image counts the in-range taps (zero padding 5)."""
    n1, n2 = 16, 23
    x = np.ones((1, 1, n1, n2))
    w = np.ones((1, 1, 11, 11))
    out = orc.conv_layer(x, w, np.zeros(1), bias_full=False, relu=False)[0, 0]
    i = np.arange(n1)[:, None]
    j = np.arange(n2)[None, :]
    cnt = (np.minimum(i, R) + np.minimum(n1 - 1 - i, R) + 1) * (np.minimum(j, R) + np.minimum(n2 - 1 - j, R) + 1)
    assert np.array_equal(out, cnt.astype(float))
    assert out[0, 0] == 36 and out[8, 11] == 121 and out[0, 11] == 66


@pytest.mark.parametrize("k", [3, 5, 11])
def test_p4_matches_scipy_correlate2d(orc, k):
    """Sum over input channels of scipy.signal.correlate2d(mode='same'), plus bias, ReLU."""
    B, Cin, Cout, n1, n2 = 2, 3, 4, 14, 17
    x = synth.normal_values((B, Cin, n1, n2), 1.0, 103, 5)
    w = synth.normal_values((Cout, Cin, k, k), 0.3, 103, 6)
    b = synth.normal_values((Cout, n1, n2), 0.5, 103, 7)
    bf = orc.full_bias_from_cropped(b, k, border=synth.normal_values((Cout, n1 + k - 1, n2 + k - 1), 9.0, 103, 8))
    out = orc.conv_layer(x, w, bf, bias_full=True, relu=True)
    for bi in range(B):
        for co in range(Cout):
            z = sum(scipy.signal.correlate2d(x[bi, ci], w[co, ci], mode="same") for ci in range(Cin))
            ref = np.maximum(z + b[co], 0.0)
            np.testing.assert_allclose(out[bi, co], ref, rtol=1e-13, atol=1e-13)


def test_p4_matches_torch_conv2d(orc):
    """Library routine: torch.nn.functional.conv2d (a cross-correlation) in float64 on the CPU."""
    import torch
    import torch.nn.functional as F

    B, Cin, Cout, n1, n2 = 2, 5, 3, 20, 20
    x = synth.normal_values((B, Cin, n1, n2), 1.0, 104, 5)
    w = synth.normal_values((Cout, Cin, 11, 11), 0.1, 104, 6)
    b = synth.normal_values((Cout,), 0.1, 104, 7)
    out = orc.conv_layer(x, w, b, bias_full=False, relu=False)
    ref = F.conv2d(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b), padding=5).numpy()
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-12)


def _layer_matrix(w, n1, n2):
    """Explicit (Cout n1 n2) x (Cin n1 n2) matrix of a zero-padded 'same' correlation.

    Built from the definition by iterating over (output pixel, tap) pairs, not by
    calling any convolution routine."""
    Cout, Cin, k, _ = w.shape
    r = (k - 1) // 2
    T = np.zeros((Cout * n1 * n2, Cin * n1 * n2))
    for co in range(Cout):
        for i in range(n1):
            for j in range(n2):
                row = (co * n1 + i) * n2 + j
                for ci in range(Cin):
                    for u in range(k):
                        for v in range(k):
                            ii, jj = i + u - r, j + v - r
                            if 0 <= ii < n1 and 0 <= jj < n2:
                                T[row, (ci * n1 + ii) * n2 + jj] += w[co, ci, u, v]
    return T


def test_p5_dense_brute_force_8x8(orc):
    """Brute force on 8x8: the layer equals its explicit dense matrix times the input."""
    n = 8
    for (cin, cout, k, seed) in [(1, 3, 11, 1), (3, 2, 11, 2), (2, 2, 5, 3)]:
        x = synth.normal_values((1, cin, n, n), 1.0, 105, seed)
        w = synth.normal_values((cout, cin, k, k), 0.2, 106, seed)
        b = synth.normal_values((cout, n, n), 0.3, 107, seed)
        out = orc.conv_layer(x, w, orc.full_bias_from_cropped(b, k), relu=False)[0]
        ref = (_layer_matrix(w, n, n) @ x.reshape(-1)).reshape(cout, n, n) + b
        np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-13)


def test_p6_linear_regime_is_a_matrix_product(orc):
    """W, b, Phi, y >= 0 keeps every ReLU inactive: the net is a product of matrices."""
    n, M = 8, 20
    net = orc.Net(n, n, M, C=(1, 3, 2, 1), k=(5, 3, 5), bias_full=True, relu_last=True)
    phi = synth.uniform_values((M, n * n), 0.0, 1.0, 108, 0)
    y = synth.uniform_values((2, M), 0.0, 1.0, 108, 1)
    ws = [synth.uniform_values((net.C[l + 1], net.C[l], net.k[l], net.k[l]), 0.0, 0.2, 108, 2 + l) for l in range(3)]
    bs_c = [synth.uniform_values((net.C[l + 1], n, n), 0.0, 0.1, 108, 6 + l) for l in range(3)]
    bs = [orc.full_bias_from_cropped(bs_c[l], net.k[l]) for l in range(3)]
    xhat = orc.forward(net, phi.T, ws, bs, y)
    for bi in range(2):
        a = phi.T @ y[bi]
        for l in range(3):
            a = _layer_matrix(ws[l], n, n) @ a + bs_c[l].reshape(-1)
        np.testing.assert_allclose(xhat[bi], a, rtol=1e-12)


def _paper_like_net(orc, n1, n2, M, C=(1, 8, 4, 1), k=(11, 11, 11), seed=0, bias_std=0.05):
    net = orc.Net(n1, n2, M, C=C, k=k, bias_full=True)
    arch = synth.Arch(C, k)
    p = synth.he_init(arch, n1, n2, bias_per_pixel=True, cfg_id=seed, bias_std=bias_std)
    bs = [orc.full_bias_from_cropped(p.b[l], k[l],
                                     border=synth.normal_values(net.full_bias_shape(l), 1.0, seed, 40 + l))
          for l in range(len(k))]
    phi = synth.make_phi(M, n1 * n2, cfg_id=seed)
    return net, phi, p, bs


def test_p7_positive_homogeneity(orc):
    """Zero biases: M(a y) = a M(y) for a > 0; bitwise for a = 2^k in FP64."""
    n, M = 12, 40
    net, phi, p, _ = _paper_like_net(orc, n, n, M, seed=3)
    bs = [np.zeros(net.full_bias_shape(l)) for l in range(3)]
    y = synth.normal_values((3, M), 1.0, 109, 1)
    base = orc.forward(net, phi.T, p.w, bs, y)
    assert np.abs(base).max() > 0
    for a in (0.25, 2.0, 8.0):
        assert np.array_equal(orc.forward(net, phi.T, p.w, bs, a * y), a * base)
    np.testing.assert_allclose(orc.forward(net, phi.T, p.w, bs, 3.7 * y), 3.7 * base, rtol=1e-13, atol=1e-14)


def test_p8_batch_independence_and_permutation(orc):
    n, M = 10, 30
    net, phi, p, bs = _paper_like_net(orc, n, n, M, seed=4)
    y = synth.normal_values((5, M), 1.0, 110, 1)
    full = orc.forward(net, phi.T, p.w, bs, y)
    perm = np.array([3, 0, 4, 2, 1])
    assert np.array_equal(orc.forward(net, phi.T, p.w, bs, y[perm]), full[perm])
    for bi in range(5):
        assert np.array_equal(orc.forward(net, phi.T, p.w, bs, y[bi:bi + 1])[0], full[bi])


def test_border_bias_is_discarded_by_crop(orc):
    """Eq. (1): S drops the padding borders, so border bias values never reach the output."""
    n, M = 10, 30
    net, phi, p, bs = _paper_like_net(orc, n, n, M, seed=5)
    y = synth.normal_values((2, M), 1.0, 111, 1)
    a = orc.forward(net, phi.T, p.w, bs, y)
    bs2 = [orc.full_bias_from_cropped(orc.crop_full(b, 11), 11, border=-123.0) for b in bs]
    assert np.array_equal(orc.forward(net, phi.T, p.w, bs2, y), a)
    # the per-channel form equals a constant per-pixel bias
    net_c = orc.Net(n, n, M, C=net.C, k=net.k, bias_full=False)
    bc = [synth.normal_values((net.C[l + 1],), 0.1, 111, 5 + l) for l in range(3)]
    bf = [np.broadcast_to(bc[l][:, None, None], net.full_bias_shape(l)).copy() for l in range(3)]
    np.testing.assert_array_equal(orc.forward(net_c, phi.T, p.w, bc, y), orc.forward(net, phi.T, p.w, bf, y))


# -------------------------------------------------------- Sec. 1 / Sec. 4 FC
def test_p9_adjointness_and_numpy(orc):
    M, N, B = 37, 91, 3
    phi = synth.make_phi(M, N, cfg_id=7)
    x = synth.normal_values((B, N), 1.0, 112, 1)
    y = synth.normal_values((B, M), 1.0, 112, 2)
    Phix = orc.measure(phi, x)
    Pty = orc.proxy(phi.T, y)
    np.testing.assert_allclose(Phix, x @ phi.T, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(Pty, y @ phi, rtol=1e-13, atol=1e-13)
    for b in range(B):
        lhs, rhs = np.dot(Phix[b], y[b]), np.dot(x[b], Pty[b])
        assert abs(lhs - rhs) <= 1e-13 * (np.abs(x[b]).sum() * np.abs(y[b]).sum())


def test_p10_orthonormal_rows_exact_projection(orc):
    M, N = 24, 64
    phi = synth.make_phi_orthonormal_rows(M, N, cfg_id=8)
    # Phi Phi^T = I, column by column through the oracle
    G = orc.measure(phi, phi)           # row m of phi measured by phi: (Phi Phi^T)[m, :]
    np.testing.assert_allclose(G, np.eye(M), atol=1e-14)
    # x in the row space is reproduced exactly by Phi^T Phi
    c = synth.normal_values((4, M), 1.0, 113, 1)
    x = orc.proxy(phi.T, c)
    np.testing.assert_allclose(orc.proxy(phi.T, orc.measure(phi, x)), x, atol=1e-13)
    # P = Phi^T Phi is idempotent on arbitrary signals
    z = synth.normal_values((3, N), 1.0, 113, 2)
    Pz = orc.proxy(phi.T, orc.measure(phi, z))
    np.testing.assert_allclose(orc.proxy(phi.T, orc.measure(phi, Pz)), Pz, atol=1e-13)


def test_p11_gaussian_phi_is_isotropic_on_average(orc):
    """E[Phi^T Phi] = I for iid N(0, 1/M) entries (loose, statistical)."""
    M, N, S = 16, 12, 400
    acc = np.zeros((N, N))
    for s in range(S):
        phi = synth.make_phi(M, N, cfg_id=1000 + s)
        acc += orc.proxy(phi.T, phi.T.copy()).T  # column n: Phi^T Phi e_n
    acc /= S
    assert np.abs(acc - np.eye(N)).max() < 0.1


# ---------------------------------------------------------- Sec. 4 training
def test_p13_loss_closed_form(orc):
    B, N = 3, 50
    x = synth.normal_values((B, N), 1.0, 114, 1)
    c = 0.25
    L, g = orc.loss(x + c, x)
    assert L == pytest.approx(N * c * c, rel=1e-14)
    np.testing.assert_allclose(g, np.full((B, N), 2 * c / B), rtol=1e-14)


def test_p14_adam_first_step(orc):
    g = np.array([1e-3, -2.0, 0.0, 5e-9, -7.5])
    theta = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    lr = 1e-3
    t1, m, v = orc.adam(theta, g, np.zeros(5), np.zeros(5), 1, lr=lr)
    np.testing.assert_allclose(t1 - theta, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)
    assert t1[2] == theta[2]
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-12)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)
    # second step with the same gradient keeps the step size lr * sign(g) (bias correction)
    t2, _, _ = orc.adam(t1, g, m, v, 2, lr=lr)
    big = np.abs(g) > 1e-3
    np.testing.assert_allclose((t2 - t1)[big], -lr * np.sign(g[big]), rtol=1e-6)


def test_p15_psnr_and_success_closed_forms(orc):
    N = 64
    x = synth.uniform_values((2, N), 0.0, 1.0, 115, 1)
    c = 0.05
    ps = orc.psnr(x + c, x)
    np.testing.assert_allclose(ps, 20 * np.log10(x.max(axis=1) / c), rtol=1e-12)
    # success indicator is inclusive at the 0.1 threshold
    xx = np.ones((1, 100))
    ok = np.ones((1, 100))
    ok[0, :10] = 1.0 - 1.0  # ||d||^2 = 10, ||x||^2 = 100 -> ratio exactly 0.1
    assert orc.success(ok, xx)[0] == 1
    ok[0, 10] = 0.999
    assert orc.success(ok, xx)[0] == 0
    assert orc.relerr(np.array([3.0, 4.0]), np.array([0.0, 0.0]))[0] == 5.0


# ----------------------------------------------------- ISTA-DCT reference
def test_p16_dct_orthonormal_and_scipy(orc):
    for n in (8, 32, 13):
        C = orc.dct_matrix(n)
        np.testing.assert_allclose(C @ C.T, np.eye(n), atol=1e-14)
    C1, C2 = orc.dct_matrix(8), orc.dct_matrix(12)
    X = synth.normal_values((8, 12), 1.0, 116, 1)
    np.testing.assert_allclose(C1 @ X @ C2.T, scipy.fft.dctn(X, norm="ortho"), atol=1e-13)
    K = C1 @ np.ones((8, 12)) @ C2.T
    assert abs(K[0, 0] - math.sqrt(96)) < 1e-13
    K[0, 0] = 0
    assert np.abs(K).max() < 1e-13


def test_spectral_norm_matches_svd(orc):
    phi = synth.make_phi(20, 50, cfg_id=9)
    sv = np.linalg.svd(phi, compute_uv=False)[0]
    est = orc.spectral_norm(phi, iters=3000)
    assert est <= sv * (1 + 1e-14) and est == pytest.approx(sv, rel=1e-9)


@pytest.mark.parametrize("seed", range(3))
def test_p17_ista_recovers_sparse_exactly_small(orc, seed):
    n, M, K = 8, 32, 4
    # the pixels synth returns are rounded to fp32; exact sparsity needs the unrounded image
    _, s_true = synth.dct_sparse_images(1, n, K, cfg_id=200 + seed, return_coeffs=True)
    x = scipy.fft.idctn(s_true[0], norm="ortho")[None]
    phi = synth.make_phi(M, n * n, cfg_id=200 + seed)
    y = orc.measure(phi, x.reshape(1, -1))[0]
    xr, s, ns = orc.ista_dct(phi, y, n, n)
    assert ns == K
    assert np.linalg.norm(xr - x.reshape(-1)) / np.linalg.norm(x) < 1e-10
    np.testing.assert_allclose(s, s_true[0], atol=1e-10)


def test_p17_ista_recovers_sparse_exactly_32(orc):
    """32x32 images, M = 256, K = 40 DCT-sparse (the paper's K << N regime, Sec. 1)."""
    n, M, K = 32, 256, 40
    _, s_true = synth.dct_sparse_images(1, n, K, cfg_id=300, return_coeffs=True)
    x = scipy.fft.idctn(s_true[0], norm="ortho")[None]
    phi = synth.make_phi(M, n * n, cfg_id=300)
    y = orc.measure(phi, x.reshape(1, -1))[0]
    xr, s, ns = orc.ista_dct(phi, y, n, n, stages=12, iters=300)
    assert np.linalg.norm(xr - x.reshape(-1)) / np.linalg.norm(x) < 1e-9


def test_p17_ista_batch_recovers_each_sparse_signal_and_is_batch_independent(orc):
    """The batched ISTA (several measurement vectors in one call, sharing the passes over
    Phi) recovers every K-sparse signal of the batch exactly (P17 per image), and each
    image's result is bit for bit the one it gets alone and in another batch (P8's
    invariant: images are independent)."""
    n, M, K, B = 8, 32, 4, 5
    phi = synth.make_phi(M, n * n, cfg_id=210)
    xs, ys = [], []
    for q in range(B):
        _, s_true = synth.dct_sparse_images(1, n, K, cfg_id=220 + q, return_coeffs=True)
        x = scipy.fft.idctn(s_true[0], norm="ortho").reshape(-1)
        xs.append(x)
        ys.append(orc.measure(phi, x[None])[0])
    Y = np.stack(ys)
    X, S, ns = orc.ista_dct_batch(phi, Y, n, n)
    for q in range(B):
        assert ns[q] == K
        assert np.linalg.norm(X[q] - xs[q]) / np.linalg.norm(xs[q]) < 1e-10
        x1, s1, n1 = orc.ista_dct(phi, Y[q], n, n)
        assert np.array_equal(x1, X[q]) and np.array_equal(s1, S[q]) and n1 == ns[q]
    X2, _, _ = orc.ista_dct_batch(phi, Y[[4, 1, 3]], n, n)
    assert np.array_equal(X2, X[[4, 1, 3]])


def test_noise_reaches_the_requested_snr(orc):
    """Sec. 5 / Table 3 noise model: the added noise has exactly the requested SNR and direction."""
    y = synth.normal_values((3, 40), 1.0, 117, 1)
    e = synth.normal_values((3, 40), 1.0, 117, 2)
    yn = orc.add_noise(y, e, 20.0)
    d = yn - y
    snr = 10 * np.log10((y ** 2).sum(axis=1) / (d ** 2).sum(axis=1))
    np.testing.assert_allclose(snr, 20.0, atol=1e-12)
    for b in range(3):   # d is a positive multiple of e
        c = np.dot(d[b], e[b]) / np.dot(e[b], e[b])
        assert c > 0
        np.testing.assert_allclose(d[b], c * e[b], atol=1e-14)
    assert np.array_equal(orc.add_noise(y, np.zeros_like(e), 20.0), y)
