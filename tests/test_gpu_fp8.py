"""FP8 e4m3 recovery path (proxy GEMM and conv layer 2 on FP8 MFMA with
power-of-two per-tensor scales, conv layers 1 and 3 in BF16, FP32
accumulation) against the FP64 oracle, through the C ABI.

FP8 keeps three mantissa bits, so its error is stated, not held to the BF16
bound: the norm-wise gate is 1e-1 per image against FP64 (observed values are
printed), and the per-pixel gate bounds each pixel by SIGMA_GATE times the
oracle's modelled rounding-error standard deviation of the FP8 variant (with
the net's own scales).  The parity tests set static activation scales large
enough that nothing in their batch saturates; calibration is tested on its own.
The encodings themselves are pinned bit for bit: a network of delta filters
passes each quantised value to the output unchanged.  Static scales make each
image's result independent of the rest of its batch, which is checked bit for
bit.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from cases import check_recovery, fp8_scales_from_oracle, make_case, oracle_ref, relerr_per_image

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dsi():
    import paper_1701_03891_amd as P
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = P.Context(0)
    yield P, ctx
    ctx.close()


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def _calib_y(case, B=32):
    """Measurements of a separate seeded calibration batch (same Phi)."""
    xc = synth.piecewise_smooth_images(B, case.n1, case.n2, cfg_id=900, stream=synth.STREAM_CALIB)
    return synth.as_f32_exact(oracle.measure(case.phi, xc.reshape(B, -1)))


def _fp8_net(ctx, case, calibrate=False):
    net = ctx.prepare(case.n1, case.n2, case.M, case.torch_params(), prec="fp8",
                      bias_per_pixel=case.bias_per_pixel, relu_last=case.relu_last)
    if calibrate:
        net.calibrate(_t(_calib_y(case)))
    else:
        net.set_act_scales(fp8_scales_from_oracle(case))
    return net


def test_fp8_scales_are_powers_of_two(dsi):
    P, ctx = dsi
    case = make_case(32, 32, 256, 4, cfg_id=41, bias_std=0.02)
    net = _fp8_net(ctx, case, calibrate=True)
    sc = net.scales()
    for v in (sc[0], sc[1], sc[2], sc[4]):
        assert v > 0 and math.log2(v) == int(math.log2(v)), sc
    # weight scales: the largest magnitude lands in (224, 448]
    amax_fc = np.abs(case.phi).max()
    assert 224 < amax_fc / sc[0] <= 448
    amax_w2 = np.abs(case.w[1]).max()
    assert 224 < amax_w2 / sc[1] <= 448
    # the calibration batch's y lands in (224, 448] of its scale
    assert 224 < np.abs(_calib_y(case)).max() / sc[2] <= 448
    net.free()


@pytest.mark.parametrize("n1,n2,M,B,cfg", [(32, 32, 256, 8, 42), (40, 48, 500, 3, 43), (5, 7, 3, 2, 47),
                                           (45, 50, 700, 3, 48)])
def test_fp8_recover_small(dsi, n1, n2, M, B, cfg):
    """32x32 (M = 256), ragged 40x48 (M = 500, K padded to 512), 5x7 (smaller than the
    filters), 45x50 (width not a multiple of 8)."""
    P, ctx = dsi
    case = make_case(n1, n2, M, B, cfg_id=cfg, bias_std=0.02)
    net = _fp8_net(ctx, case)
    got = net.recover(_t(case.y)).cpu().numpy().astype(np.float64).reshape(case.B, -1)
    check_recovery(case, got, "fp8", scales=net.scales(), label=f"{n1}x{n2}")
    net.free()


def test_fp8_c2_full_size(dsi):
    """64x64, M = 1024, batch 256: every image against the oracle."""
    P, ctx = dsi
    case = make_case(64, 64, 1024, 256, cfg_id=44, bias_std=0.02)
    net = _fp8_net(ctx, case)
    got = net.recover(_t(case.y)).cpu().numpy().astype(np.float64).reshape(256, -1)
    check_recovery(case, got, "fp8", scales=net.scales(), label="C2 64x64 B=256")
    ref = oracle_ref(case)
    dps = oracle.psnr(ref, case.x) - oracle.psnr(got, case.x)
    print(f"fp8 64x64: dPSNR {dps.mean():.4f} dB (max {np.abs(dps).max():.4f}; random weights)")
    net.free()


def test_fp8_calibrated_batch_independence(dsi):
    """Scales calibrated on a separate batch; each image's result is the same alone and in
    its batch of 256 (static scales), and the error stays within the FP8 norm-wise gate."""
    P, ctx = dsi
    case = make_case(64, 64, 1024, 256, cfg_id=44, bias_std=0.02)
    net = _fp8_net(ctx, case, calibrate=True)
    y = _t(case.y)
    full = net.recover(y).cpu().numpy().reshape(256, -1)
    idx = np.array([0, 77, 200, 255])
    err = relerr_per_image(full[idx].astype(np.float64), oracle_ref(case, idx))
    print(f"fp8 calibrated: max rel err {err.max():.3e}")
    assert err.max() <= 1e-1
    for i in (0, 77, 255):
        alone = net.recover(y[i:i + 1].contiguous()).cpu().numpy().reshape(1, -1)
        assert np.array_equal(alone[0], full[i])
    net.free()


def test_fp8_c4_128x128(dsi):
    """128x128 (N = 16384), M = 4096 dense FC (4096 x 16384), batch 64: every image."""
    P, ctx = dsi
    case = make_case(128, 128, 4096, 64, cfg_id=45, bias_std=0.02)
    net = _fp8_net(ctx, case)
    got = net.recover(_t(case.y)).cpu().numpy().astype(np.float64).reshape(64, -1)
    check_recovery(case, got, "fp8", scales=net.scales(), label="C4 128x128 B=64")
    net.free()


# ------------------------------------------------------------ encodings, bit for bit
def _e4m3(v):
    """OCP e4m3fn value of float32 v after clamping to +-448 (torch's conversion)."""
    c = np.clip(np.asarray(v, dtype=np.float64), -448.0, 448.0)
    return torch.tensor(c, dtype=torch.float32).to(torch.float8_e4m3fn).to(torch.float64).numpy()


def _bf16(v):
    return torch.tensor(np.asarray(v, dtype=np.float64), dtype=torch.float32).to(torch.bfloat16).to(
        torch.float64).numpy()


def _e4m3_grid():
    """Every finite non-negative e4m3 value (codes 0x00..0x7e)."""
    return torch.arange(0, 127, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float64).numpy()


def _code_column(N, seed):
    """N FC weights (one W_fc column) covering the e4m3 format at scale 1: every value,
    every midpoint between neighbours (ties), points a quarter-gap off each midpoint,
    subnormals and values below half the smallest subnormal, both signs, 448 (so the
    per-tensor weight scale is exactly 1), rest random."""
    v = _e4m3_grid()
    mid = 0.5 * (v[:-1] + v[1:])
    gap = v[1:] - v[:-1]
    pts = np.concatenate([v, mid, mid - gap / 4, mid + gap / 4, [2.0 ** -10, 2.0 ** -11, 3 * 2.0 ** -11]])
    pts = np.concatenate([pts, -pts])
    g = synth.rng(seed, 5)
    rest = g.uniform(-448.0, 448.0, N - len(pts)) * np.exp2(-g.integers(0, 14, N - len(pts)))
    col = np.concatenate([pts, rest]).astype(np.float32).astype(np.float64)
    col[0] = 448.0
    return col[g.permutation(N)]


def _delta_params(n, M, w1, cols):
    """The paper's 1 -> 64 -> 32 -> 1 architecture with delta filters and zero biases:
    conv layer 1 maps x~ to +w1 x~ (channel 0) and -w1 x~ (channel 1), conv layer 2
    copies channels 0 and 1, conv layer 3 outputs channel 0 minus channel 1.  The
    network's output is then sign(x~) times conv layer 2's stored input, so every
    rounding point of the path reaches the output unchanged."""
    N = n * n
    wfc = np.zeros((N, M))
    for m, c in cols.items():
        wfc[:, m] = c
    w = [np.zeros((64, 1, 11, 11)), np.zeros((32, 64, 11, 11)), np.zeros((1, 32, 11, 11))]
    w[0][0, 0, 5, 5], w[0][1, 0, 5, 5] = w1, -w1
    w[1][0, 0, 5, 5], w[1][1, 1, 5, 5] = 1.0, 1.0
    w[2][0, 0, 5, 5], w[2][0, 1, 5, 5] = 1.0, -1.0
    b = [np.zeros(64), np.zeros(32), np.zeros(1)]
    return wfc, w, b


def _recover_delta(P, ctx, n, M, wfc, w, b, y, prec, act_scales=None):
    from paper_1701_03891_amd import NetParams
    params = NetParams(_t(wfc), [_t(a) for a in w], [_t(a) for a in b])
    net = ctx.prepare(n, n, M, params, prec=prec, bias_per_pixel=False)
    if act_scales is not None:
        net.set_act_scales(act_scales)
    out = net.recover(_t(y)).cpu().numpy().astype(np.float64).reshape(y.shape[0], -1)
    sc = net.scales()
    net.free()
    return out, sc


def test_e4m3_encodings_bit_exact(dsi):
    """FP8 e4m3 rounding at every quantisation point, bit for bit against torch's
    float32 -> float8_e4m3fn conversion (after clamping to +-448) and against the
    oracle's quantised forward pass:
      * the software encoder of the weights (W_fc, scale 1): image 0, y = e_0, w1 = 1,
        s_a1 = 1, so conv layer 1's output x~ = q(W_fc[:, 0]) is an e4m3 value and
        passes its own rounding unchanged;
      * the encoder of y (static scale s_y = 2^-3, saturating): images 1-3 carry
        y = c e_1 with c / s_y on a tie, off a tie and above 448;
      * the hardware conversion of conv layer 1's output (clamp, then
        round-to-nearest-even): images 4-7 with w1 = 1.375 or 1 and several s_a1, so
        w1 x~ needs up to 11 significand bits and lands on ties, in the subnormal range
        (s_a1 = 2^4) and beyond 448 s_a1 (s_a1 = 2^-6)."""
    P, ctx = dsi
    n, M = 64, 8
    N = n * n
    cols = {0: _code_column(N, 61), 1: _code_column(N, 62)}
    cases = [  # (y entries {m: value}, w1, s_a1)
        ({0: 1.0}, 1.0, 1.0),
        ({1: 1.0625 * 2 ** -3}, 1.0, 1.0),        # 1.0625 = tie between 1 and 1.125 -> 1
        ({1: 1.1 * 2 ** -3}, 1.0, 1.0),            # -> 1.125
        ({1: 600.0 * 2 ** -3}, 1.0, 2.0 ** 9),     # y saturates at 448 s_y
        ({0: 1.0}, 1.375, 1.0),
        ({0: 1.0}, 1.375, 2.0 ** 4),              # many conv-1 outputs in the subnormal range
        ({1: 1.0}, 1.0078125, 2.0 ** -6),          # many beyond 448 s_a1: saturate
        ({1: 1.0}, 1.375, 0.5),
    ]
    s_y = 2.0 ** -3
    for i, (ye, w1, s_a1) in enumerate(cases):
        y = np.zeros((1, M))
        for m, c in ye.items():
            y[0, m] = c
        wfc, w, b = _delta_params(n, M, w1, cols)
        got, sc = _recover_delta(P, ctx, n, M, wfc, w, b, y, "fp8", act_scales=[s_y, 1.0, s_a1, 1.0])
        assert sc[0] == 1.0 and sc[1] == 2.0 ** -8, sc
        # expected, from torch's conversions: x~ = bf16(q(W) q(y)) (one product of two
        # 4-bit significands, exact), z1 = w1 x~ (exact in FP32), a1 = s_a1 q(relu(+-z1) / s_a1),
        # conv layer 2 copies it (W2 = 1 = 256 s_w2, exact), output a1[0] - a1[1]
        m, c = next(iter(ye.items()))
        xt = _bf16(_e4m3(wfc[:, m]) * s_y * _e4m3(c / s_y))
        z1 = w1 * xt
        exp = s_a1 * (_e4m3(np.maximum(z1, 0) / s_a1) - _e4m3(np.maximum(-z1, 0) / s_a1))
        bad = np.flatnonzero(got[0] != exp)
        assert bad.size == 0, (i, bad[:5], got[0][bad[:5]], exp[bad[:5]])
        # and the oracle's quantised forward pass (pinned to torch on the CPU) agrees
        net_o = oracle.Net(n, n, M, bias_full=False)
        q = oracle.Quant.fp8(s_y, 1.0, s_a1, 2.0 ** -8)
        ref = oracle.forward_q(net_o, wfc, w, b, y, q)
        assert np.array_equal(got[0], ref[0]), i
        if i == 0:
            assert np.array_equal(got[0], _e4m3(wfc[:, 0]))
    # the columns cover ties, subnormals and saturation of the a1 conversion
    z = _bf16(_e4m3(cols[0]) * 1.375)
    assert np.any(np.abs(z) / 2.0 ** 4 < 2.0 ** -6) and np.any(np.abs(_bf16(_e4m3(cols[1]))) / 2.0 ** -6 > 448)


def test_bf16_encodings_bit_exact(dsi):
    """BF16 rounding at every point of the BF16 path, bit for bit against torch's
    float32 -> bfloat16 conversion: W_fc and y (software round-to-nearest-even), the
    proxy's product (two 8-bit significands, rounded once), conv layer 1's output
    (w1 = 1 + 2^-7 moves every value), through the same delta network."""
    P, ctx = dsi
    n, M = 64, 8
    N = n * n
    g = synth.rng(63, 5)
    col = g.uniform(-3.0, 3.0, N) * np.exp2(-g.integers(0, 20, N))
    col[:6] = [1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 2 ** -100, 0.0, 1 + 2 ** -9]
    col = col.astype(np.float32).astype(np.float64)
    for yv, w1 in ((1.0, 1.0), (1.0 + 2 ** -8 + 2 ** -12, 1.0), (0.7, 1.0078125)):
        y = np.zeros((1, M))
        y[0, 3] = np.float32(yv)
        wfc, w, b = _delta_params(n, M, w1, {3: col})
        got, _ = _recover_delta(P, ctx, n, M, wfc, w, b, y, "bf16")
        xt = _bf16(_bf16(col) * _bf16(y[0, 3]))
        exp = _bf16(w1 * xt)
        bad = np.flatnonzero(got[0] != exp)
        assert bad.size == 0, (yv, bad[:5], got[0][bad[:5]], exp[bad[:5]])
        net_o = oracle.Net(n, n, M, bias_full=False)
        assert np.array_equal(got[0], oracle.forward_q(net_o, wfc, w, b, y, oracle.Quant.bf16())[0])


def test_fp8_rejects_training_and_other_archs(dsi):
    P, ctx = dsi
    from paper_1701_03891_amd import _lib
    case = make_case(16, 16, 64, 2, cfg_id=46)
    net = ctx.prepare(16, 16, 64, case.torch_params(), prec="fp8")
    params = case.torch_params()
    with pytest.raises(P.DsiError) as e:
        net.loss_grad(_t(case.y), _t(case.x), params)
    assert e.value.status == _lib.DSI_E_DTYPE
    net.free()
    tiny = make_case(16, 16, 64, 2, cfg_id=46, C=(1, 4, 2, 1), k=(5, 5, 5))
    with pytest.raises(P.DsiError):
        ctx.prepare(16, 16, 64, tiny.torch_params(), prec="fp8", C=tiny.C, k=tiny.k)
