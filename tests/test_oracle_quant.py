"""Pins of the oracle's reduced-precision forward pass.

The BF16 and FP8 variants of the network (BF16 operands; OCP e4m3 operands with
power-of-two per-tensor scales) round their operands at fixed points and sum
exactly otherwise.  These tests tie the oracle's rounding and its quantised
forward pass to things other than themselves: torch's own float32 -> bfloat16
and float32 -> float8_e4m3fn conversions (library routines), brute-force
enumeration of every e4m3 code, reduction to the already pinned FP64 forward
pass, and delta networks whose output exposes one rounded operand.  The error
model (the per-pixel standard deviation of the rounding error) is pinned by the
distribution of the actual rounding errors.
"""
import numpy as np
import pytest
import torch

import synth

R = 5


def _f32_bits_sample(n, seed, lo_exp=-140, hi_exp=20):
    """float32 values spread over many binades (subnormals included), both signs."""
    g = synth.rng(seed, 5)
    e = g.integers(lo_exp, hi_exp, n)
    m = g.uniform(1.0, 2.0, n)
    v = np.ldexp(m, e) * np.where(g.random(n) < 0.5, -1.0, 1.0)
    return v.astype(np.float32).astype(np.float64)


def _bf16_torch(v):
    return torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()


def _e4m3_torch(v):
    c = np.clip(v, -448.0, 448.0)
    return torch.tensor(c, dtype=torch.float32).to(torch.float8_e4m3fn).to(torch.float64).numpy()


# ------------------------------------------------------------ formats
def test_bf16_rounding_matches_torch(orc):
    v = _f32_bits_sample(20000, 1)
    # exact ties: a BF16 value plus half its spacing, and the values next to them
    base = _bf16_torch(_f32_bits_sample(2000, 2, -120, 30))
    half = np.abs(base) * 0.0
    for q, b in enumerate(base):
        e = np.frexp(abs(b))[1] - 1
        half[q] = np.ldexp(1.0, max(e, -126) - 8)
    ties = np.concatenate([base + half, base - half, base + 0.75 * half]).astype(np.float32).astype(np.float64)
    v = np.concatenate([v, ties, [0.0, -0.0, 1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8]])
    got = orc.round_fmt(v, orc.Q_BF16)
    assert np.array_equal(got, _bf16_torch(v))


def test_e4m3_rounding_matches_torch(orc):
    g = synth.rng(3, 5)
    v = np.concatenate([g.uniform(-500, 500, 5000), g.uniform(-1, 1, 5000), g.uniform(-0.02, 0.02, 5000),
                        g.uniform(-2 ** -8, 2 ** -8, 3000)]).astype(np.float32).astype(np.float64)
    got = orc.round_fmt(v, orc.Q_E4M3)
    assert np.array_equal(got, _e4m3_torch(v))


def _e4m3_values():
    """Every finite non-negative e4m3fn value in code order (codes 0x00..0x7e), decoded by torch."""
    return torch.arange(0, 127, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float64).numpy()


def test_e4m3_every_code_and_every_midpoint(orc):
    """Brute force over the format: each value is a fixed point, each midpoint between
    neighbours goes to the neighbour with the even code (even last significand bit),
    points just off a midpoint go to the nearer neighbour, and beyond 448 it saturates."""
    vals = _e4m3_values()
    assert vals[-1] == 448.0 and vals[1] == 2.0 ** -9 and vals[8] == 2.0 ** -6
    for sgn in (1.0, -1.0):
        assert np.array_equal(orc.round_fmt(sgn * vals, orc.Q_E4M3), sgn * vals)
        mid = 0.5 * (vals[:-1] + vals[1:])
        even = np.where(np.arange(len(vals) - 1) % 2 == 0, vals[:-1], vals[1:])
        assert np.array_equal(orc.round_fmt(sgn * mid, orc.Q_E4M3), sgn * even)
        gap = vals[1:] - vals[:-1]
        assert np.array_equal(orc.round_fmt(sgn * (mid - gap / 8), orc.Q_E4M3), sgn * vals[:-1])
        assert np.array_equal(orc.round_fmt(sgn * (mid + gap / 8), orc.Q_E4M3), sgn * vals[1:])
        assert np.array_equal(orc.round_fmt(sgn * np.array([448.0, 464.0, 500.0, 1e6]), orc.Q_E4M3),
                              sgn * np.full(4, 448.0))


def test_quantize_applies_the_scale(orc):
    v = synth.uniform_values((1000,), -3.0, 3.0, 4, 5)
    for s in (2.0 ** -8, 2.0 ** -3, 1.0, 8.0):
        assert np.array_equal(orc.quantize(v, orc.Q_E4M3, s), s * _e4m3_torch(v / s))
        assert np.array_equal(orc.quantize(v, orc.Q_BF16, s), s * _bf16_torch(v / s))
    assert np.array_equal(orc.quantize(v, orc.Q_NONE, 1.0), v)


# ------------------------------------------------------------ quantised forward pass
def _net(orc, n1, n2, M, C, k, seed, bias_std=0.05):
    phi = synth.make_phi(M, n1 * n2, cfg_id=seed)
    p = synth.he_init(synth.Arch(C, k), n1, n2, bias_per_pixel=True, cfg_id=seed, bias_std=bias_std)
    net = orc.Net(n1, n2, M, C=C, k=k, bias_full=True)
    b = [orc.full_bias_from_cropped(p.b[l], k[l], border=0.3) for l in range(len(k))]
    return net, phi.T.copy(), p.w, b


def test_forward_q_without_rounding_is_the_forward_pass(orc):
    net, wfc, w, b = _net(orc, 12, 10, 40, (1, 6, 3, 1), (5, 3, 7), 11)
    y = synth.normal_values((3, 40), 1.0, 11, 6)
    ref = orc.forward(net, wfc, w, b, y)
    assert np.array_equal(orc.forward_q(net, wfc, w, b, y, orc.Quant()), ref)


def test_forward_q_is_exact_on_representable_values(orc):
    """Small integers are BF16 values, and with delta filters every sum stays a small
    integer: the BF16 forward pass then equals the FP64 one exactly; a non-representable
    input breaks the equality."""
    n1 = n2 = 8
    M, N = 5, 64
    g = synth.rng(12, 5)
    wfc = g.integers(-3, 4, (N, M)).astype(np.float64)
    y = g.integers(-3, 4, (2, M)).astype(np.float64)
    C, k = (1, 2, 2, 1), (3, 3, 3)
    w = [np.zeros((C[l + 1], C[l], 3, 3)) for l in range(3)]
    w[0][0, 0, 1, 1], w[0][1, 0, 1, 1] = 1.0, -1.0
    w[1][0, 0, 1, 1], w[1][0, 1, 1, 1], w[1][1, 0, 1, 1], w[1][1, 1, 1, 1] = 1.0, -1.0, -1.0, 1.0
    w[2][0, 0, 1, 1], w[2][0, 1, 1, 1] = 2.0, -2.0
    b = [np.zeros((C[l + 1], n1 + 2, n2 + 2)) for l in range(3)]
    net = orc.Net(n1, n2, M, C=C, k=k, bias_full=True)
    ref = orc.forward(net, wfc, w, b, y)
    assert np.array_equal(orc.forward_q(net, wfc, w, b, y, orc.Quant.bf16()), ref)
    assert np.array_equal(ref, 2.0 * (wfc @ y.T).T)      # the delta network is 2 x~
    wfc2 = wfc.copy()
    wfc2[0, 0] = 1.0 + 2.0 ** -10
    y2 = y.copy()
    y2[0, 0] = 1.0
    assert not np.array_equal(orc.forward_q(net, wfc2, w, b, y2, orc.Quant.bf16()), orc.forward(net, wfc2, w, b, y2))


def _delta_net(orc, n1, n2, M, w1=1.0):
    """1 -> 2 -> 2 -> 1 network of 3x3 delta filters, zero biases, whose output is w1 * x~:
    channel 0 carries the positive part, channel 1 the negative part, so signed values
    survive the ReLUs."""
    C, k = (1, 2, 2, 1), (3, 3, 3)
    w = [np.zeros((C[l + 1], C[l], 3, 3)) for l in range(3)]
    w[0][0, 0, 1, 1], w[0][1, 0, 1, 1] = w1, -w1
    w[1][0, 0, 1, 1], w[1][1, 1, 1, 1] = 1.0, 1.0
    w[2][0, 0, 1, 1], w[2][0, 1, 1, 1] = 1.0, -1.0
    b = [np.zeros((C[l + 1], n1 + 2, n2 + 2)) for l in range(3)]
    return orc.Net(n1, n2, M, C=C, k=k, bias_full=True), w, b


def test_delta_network_exposes_each_rounding_point(orc):
    """With y a unit vector, the output of the delta network is one column of W_fc after
    every rounding point it passes: the FC weights (bf16 / e4m3 with scale s_fc), the
    proxy x~, conv layer 1's output, conv layer 2's output -- each against torch."""
    n1, n2, M = 6, 7, 4
    N = n1 * n2
    g = synth.rng(13, 5)
    col = g.uniform(-3.0, 3.0, N)
    col[:8] = [1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 2 ** -130, 0.0, 3e-3, -2.5e-3, 7.0]
    wfc = np.zeros((N, M))
    wfc[:, 2] = col.astype(np.float32)
    y = np.zeros((1, M))
    y[0, 2] = 1.0
    net, w, b = _delta_net(orc, n1, n2, M)
    got = orc.forward_q(net, wfc, w, b, y, orc.Quant.bf16())[0]
    assert np.array_equal(got, _bf16_torch(wfc[:, 2]))
    # FP8: only W_fc rounds (x~ = s_fc q(W / s_fc) is a BF16 value, conv layer 1 passes it
    # unchanged when its scale is s_fc, conv layer 2 is exact)
    s_fc = 2.0 ** -6
    got8 = orc.forward_q(net, wfc, w, b, y, orc.Quant.fp8(1.0, s_fc, s_fc, 2.0 ** -8))[0]
    assert np.array_equal(got8, s_fc * _e4m3_torch(wfc[:, 2] / s_fc))
    # conv layer 1's output rounds to e4m3 with its own scale: w1 = 1.375 moves every value
    s_a1 = 2.0 ** -4
    net, w, b = _delta_net(orc, n1, n2, M, w1=1.375)
    got8 = orc.forward_q(net, wfc, w, b, y, orc.Quant.fp8(1.0, s_fc, s_a1, 2.0 ** -8))[0]
    xt = s_fc * _e4m3_torch(wfc[:, 2] / s_fc)
    a1 = 1.375 * xt      # exact: 4 x 3 significand bits
    assert np.array_equal(got8, s_a1 * _e4m3_torch(a1 / s_a1))
    # the proxy rounds its sum: two columns of W_fc, each rounded, added exactly, rounded
    y2 = np.zeros((1, M))
    y2[0, 1], y2[0, 2] = 1.0, 2.0 ** -9
    wfc2 = wfc.copy()
    wfc2[:, 1] = g.uniform(-3.0, 3.0, N).astype(np.float32)
    # (conv layer 1 scales by 1 + 2^-7, so rounding x~ and rounding conv layer 1's
    # output are two different roundings)
    net, w, b = _delta_net(orc, n1, n2, M, w1=1.0078125)
    got = orc.forward_q(net, wfc2, w, b, y2, orc.Quant.bf16())[0]
    xt = _bf16_torch(_bf16_torch(wfc2[:, 1]) + 2.0 ** -9 * _bf16_torch(wfc2[:, 2]))
    assert np.array_equal(got, _bf16_torch(1.0078125 * xt))
    assert not np.array_equal(got, _bf16_torch(1.0078125 * (_bf16_torch(wfc2[:, 1]) + 2.0 ** -9 * _bf16_torch(wfc2[:, 2]))))
    # the measurement vector rounds too: y = 1.1 is stored as 1.125 in e4m3
    y[0, 2] = 1.1
    net, w, b = _delta_net(orc, n1, n2, M)
    got8 = orc.forward_q(net, wfc, w, b, y, orc.Quant.fp8(1.0, s_fc, 2.0 ** -3, 2.0 ** -8))[0]
    xt = _bf16_torch(s_fc * _e4m3_torch(wfc[:, 2] / s_fc) * 1.125)
    assert np.array_equal(got8, 2.0 ** -3 * _e4m3_torch(xt / 2.0 ** -3))


# ------------------------------------------------------------ error model
@pytest.mark.parametrize("variant", ["bf16", "fp8"])
def test_error_model_matches_the_rounding_errors(orc, variant):
    """The modelled per-pixel standard deviation sigma of the rounding error against the
    exact forward pass describes the actual errors of the quantised pass: over ~10^4
    pixels the normalised error e / sigma has standard deviation between 0.6 and 1.1
    (the uniform-error model is exact per rounding; correlations are ignored) and no
    pixel exceeds 6 sigma.  A model that dropped a source of error would give a
    standard deviation above 1.1 (checked in the mutation tests)."""
    n1, n2, M, B = 16, 16, 96, 40
    net, wfc, w, b = _net(orc, n1, n2, M, (1, 16, 8, 1), (11, 11, 11), 14, bias_std=0.02)
    x = synth.piecewise_smooth_images(B, n1, n2, cfg_id=14).reshape(B, -1)
    y = synth.as_f32_exact(orc.measure(wfc.T, x))
    ref = orc.forward(net, wfc, w, b, y)
    if variant == "bf16":
        q = orc.Quant.bf16()
    else:
        xt = orc.proxy(wfc, y)
        s_y = 2.0 ** np.ceil(np.log2(np.abs(y).max() / 448))
        s_fc = 2.0 ** np.ceil(np.log2(np.abs(wfc).max() / 448))
        s_w2 = 2.0 ** np.ceil(np.log2(np.abs(w[1]).max() / 448))
        a1 = orc.conv_layer(xt.reshape(B, 1, n1, n2), w[0], b[0])
        s_a1 = 2.0 ** np.ceil(np.log2(np.abs(a1).max() / 448))
        q = orc.Quant.fp8(s_y, s_fc, s_a1, s_w2)
    q.acc_fp32 = False          # the oracle sums exactly: model the operand roundings only
    got, sig = orc.forward_q(net, wfc, w, b, y, q, want_sigma=True)
    z = (got - ref) / sig
    print(variant, "std(e/sigma)", z.std(), "max |e/sigma|", np.abs(z).max(), "median rel sigma",
          np.median(sig / np.sqrt((ref ** 2).mean(axis=1, keepdims=True))))
    assert 0.6 <= z.std() <= 1.1
    assert np.abs(z).max() <= 6.0


def test_error_model_fp32_accumulation_term(orc):
    """The FP32 running-sum term: sums of n random-sign terms accumulated in float32 in
    order have an error variance below the model's (n / 24) 2^-46 sum(t^2) and above a
    tenth of it."""
    g = synth.rng(15, 5)
    n, trials = 2000, 400
    t = g.standard_normal((trials, n)).astype(np.float32)
    exact = t.astype(np.float64).sum(axis=1)
    acc = np.zeros(trials, dtype=np.float32)
    for q in range(n):
        acc = (acc + t[:, q]).astype(np.float32)
    err = acc.astype(np.float64) - exact
    model = n / 24.0 * 2.0 ** -46 * (t.astype(np.float64) ** 2).sum(axis=1)
    ratio = (err ** 2).mean() / model.mean()
    print("fp32 running sum: empirical / model variance", ratio)
    assert 0.1 <= ratio <= 1.0
    # and the oracle's model uses that coefficient: a one-layer network with a single
    # output and n inputs reports sigma^2 = (n+1)/24 2^-46 sum (w a)^2 for FP32
    net = orc.Net(1, 1, 4, C=(1, 1), k=(1,), bias_full=False)
    wfc = np.array([[1.0, 2.0, -1.0, 0.5]])
    yv = np.array([[1.0, 1.0, 1.0, 1.0]])
    w = [np.array([[[[3.0]]]])]
    out, sig = orc.forward_q(net, wfc, w, [np.zeros(1)], yv, orc.Quant(acc_fp32=True), want_sigma=True)
    xt = 2.5
    v0 = 4 / 24 * 2.0 ** -46 * (1 + 4 + 1 + 0.25)
    v1 = 9 * v0 + 2 / 24 * 2.0 ** -46 * 9 * xt ** 2
    assert out[0, 0] == 7.5
    assert np.isclose(sig[0, 0] ** 2, v1, rtol=1e-12, atol=0.0)
