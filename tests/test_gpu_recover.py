"""GPU parity of the recovery path (measurement, proxy, Eq. (1) conv stack)
against the FP64 oracle, through the C ABI.

Every recovered image passes two gates (``cases.check_recovery``): the
norm-wise relative error per image (FP32 <= 1e-5, BF16 <= 2e-2; the FP64
checking precision returns xhat through the float32 interface, so 1e-7), and
a per-pixel bound of SIGMA_GATE times the oracle's modelled rounding-error
standard deviation of that pixel for the precision variant.  Full-size
configurations check every image of the batch.
"""
import numpy as np
import pytest

from cases import check_recovery, make_case, relerr_per_image

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


def _recover(P, ctx, case, prec):
    import torch
    params = case.torch_params()
    net = ctx.prepare(case.n1, case.n2, case.M, params, prec=prec, C=case.C, k=case.k,
                      bias_per_pixel=case.bias_per_pixel, relu_last=case.relu_last)
    y = torch.tensor(case.y, dtype=torch.float32, device="cuda")
    xh = net.recover(y)
    torch.cuda.synchronize()
    out = xh.cpu().numpy().astype(np.float64).reshape(case.B, -1)
    net.free()
    return out


# ---------------------------------------------------------------- Sec. 1
@pytest.mark.parametrize("M,n1,n2,B", [(256, 32, 32, 8), (77, 40, 48, 3), (50, 13, 11, 5), (1024, 64, 64, 64)])
def test_measure_parity(dsi, M, n1, n2, B):
    import torch

    import oracle
    import synth
    P, ctx = dsi
    N = n1 * n2
    phi = synth.make_phi(M, N, cfg_id=M + N)
    x = synth.piecewise_smooth_images(B, n1, n2, cfg_id=M + N).reshape(B, N)
    ref = oracle.measure(phi, x)
    y = ctx.measure(torch.tensor(phi, dtype=torch.float32, device="cuda"),
                    torch.tensor(x, dtype=torch.float32, device="cuda"))
    got = y.cpu().numpy().astype(np.float64)
    assert relerr_per_image(got, ref).max() <= 1e-5
    # per element: an FP32 sum of N products, |error| <= N 2^-24 sum |phi x| (worst case)
    bound = N * 2.0 ** -24 * (np.abs(x) @ np.abs(phi).T) + 2.0 ** -24 * np.abs(ref)
    assert np.all(np.abs(got - ref) <= bound)


def test_measure_empty_batch_is_noop(dsi):
    import torch
    P, ctx = dsi
    phi = torch.ones((4, 16), device="cuda")
    x = torch.ones((0, 16), device="cuda")
    y = ctx.measure(phi, x)
    assert y.shape == (0, 4)


# ---------------------------------------------------------------- Sec. 4
@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_recover_c1_dct_sparse(dsi, prec):
    """32x32 DCT-sparse signals (K = 40), M = 256, batch 8, He-init, ReLU after layers 1-2."""
    P, ctx = dsi
    case = make_case(32, 32, 256, 8, cfg_id=1, signal="dct", bias_std=0.0)
    check_recovery(case, _recover(P, ctx, case, prec), prec, label="C1")


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("bias_per_pixel", [True, False])
def test_recover_ragged_tiles(dsi, prec, bias_per_pixel):
    """40x48 images (ragged against 32-wide and 16/32-high tiles), M = 500 (padded K), batch 3."""
    P, ctx = dsi
    case = make_case(40, 48, 500, 3, cfg_id=2, bias_per_pixel=bias_per_pixel, bias_std=0.05)
    check_recovery(case, _recover(P, ctx, case, prec), prec, label=f"ragged bias_pp={bias_per_pixel}")


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_recover_width_not_multiple_of_8(dsi, prec):
    """45x50 images: a width that is not a multiple of 8 takes conv layer 1's unaligned
    halo staging in BF16; 45 rows and 50 columns are ragged against every tile; M = 700,
    batch 4."""
    P, ctx = dsi
    case = make_case(45, 50, 700, 4, cfg_id=14, bias_std=0.05)
    check_recovery(case, _recover(P, ctx, case, prec), prec, label="45x50")


@pytest.mark.parametrize("bias_per_pixel", [True, False])
def test_recover_conv3_row_bands_and_column_tiles(dsi, bias_per_pixel):
    """70 x 152 images: BF16 conv3 works on images wider than 128 columns in 64-row bands of
    70 output columns, so this is a full and a 6-row band, and two full and one 12-column
    tile (each reading 5 columns beyond its edges); batch 2, M = 600."""
    P, ctx = dsi
    case = make_case(70, 152, 600, 2, cfg_id=13, bias_per_pixel=bias_per_pixel, bias_std=0.05)
    check_recovery(case, _recover(P, ctx, case, "bf16"), "bf16", label=f"70x152 bias_pp={bias_per_pixel}")


@pytest.mark.parametrize("bias_per_pixel", [True, False])
def test_recover_conv3_whole_rows_ragged_band(dsi, bias_per_pixel):
    """100 x 90 images: BF16 conv3 gives images up to 128 columns wide 8 waves over the whole
    row (here 90 columns and 38 past the edge) in 32-row bands, so this is three full bands
    and a 4-row one; batch 3, M = 900."""
    P, ctx = dsi
    case = make_case(100, 90, 900, 3, cfg_id=15, bias_per_pixel=bias_per_pixel, bias_std=0.05)
    check_recovery(case, _recover(P, ctx, case, "bf16"), "bf16", label=f"100x90 bias_pp={bias_per_pixel}")


def test_recover_uneven_tiles_per_block(dsi):
    """BF16 conv2 runs one block per CU over every G-th tile: 40x48 images, batch 100 give
    400 tiles, so some blocks run two tiles (prefetching the second's first slice) and
    others one."""
    P, ctx = dsi
    case = make_case(40, 48, 500, 100, cfg_id=12, bias_std=0.05)
    check_recovery(case, _recover(P, ctx, case, "bf16"), "bf16", label="uneven tiles")


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_recover_image_smaller_than_filter(dsi, prec):
    """5x7 images, smaller than the 11x11 filters (taps reach the zero padding); M = 3; batch 2."""
    P, ctx = dsi
    case = make_case(5, 7, 3, 2, cfg_id=3, bias_std=0.1)
    check_recovery(case, _recover(P, ctx, case, prec), prec, label="5x7")


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_recover_relu_last_and_m_above_n(dsi, prec):
    """relu_last = 1 (ReLU in every layer, as Sec. 4 states) and M > N (allowed)."""
    P, ctx = dsi
    case = make_case(16, 16, 300, 2, cfg_id=4, relu_last=True, bias_std=0.05)
    check_recovery(case, _recover(P, ctx, case, prec), prec, label="relu_last")


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_recover_c2_full_size(dsi, prec):
    """64x64, M = 1024, batch 256 in the benchmark's launch configuration; every image
    against the oracle."""
    P, ctx = dsi
    case = make_case(64, 64, 1024, 256, cfg_id=5, bias_std=0.02)
    check_recovery(case, _recover(P, ctx, case, prec), prec, label="C2 64x64 B=256")


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_recover_c4_128x128(dsi, prec):
    """128x128 (N = 16384), M = 4096 (FC 16384 x 4096), batch 64: every image."""
    P, ctx = dsi
    case = make_case(128, 128, 4096, 64, cfg_id=45, bias_std=0.02)
    check_recovery(case, _recover(P, ctx, case, prec), prec, label="C4 128x128 B=64")


# ------------------------------------------------ any shape (direct kernels)
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_recover_generic_tiny_net(dsi, prec):
    """16x16, M = 64, 1 -> 4 -> 2 -> 1 with 5x5 filters (the tiny net of the gradient checks)."""
    P, ctx = dsi
    case = make_case(16, 16, 64, 3, cfg_id=6, C=(1, 4, 2, 1), k=(5, 5, 5), bias_std=0.1)
    check_recovery(case, _recover(P, ctx, case, prec), prec, label="tiny net")


def test_recover_generic_deeper_net(dsi):
    """A deeper, narrower stack (L = 5, mixed filter sizes): the direct-kernel path."""
    P, ctx = dsi
    case = make_case(20, 18, 90, 2, cfg_id=7, C=(1, 8, 6, 4, 3, 1), k=(3, 7, 5, 3, 9), bias_std=0.1)
    check_recovery(case, _recover(P, ctx, case, "f32"), "f32", label="L=5")


# -------------------------------------------------------------- error paths
def test_error_paths(dsi):
    import torch

    from paper_1701_03891_amd import _lib
    P, ctx = dsi
    case = make_case(16, 16, 64, 2, cfg_id=8)
    params = case.torch_params()
    # BF16 on a non-paper architecture
    tiny = make_case(16, 16, 64, 2, cfg_id=8, C=(1, 4, 2, 1), k=(5, 5, 5))
    with pytest.raises(P.DsiError) as e:
        ctx.prepare(16, 16, 64, tiny.torch_params(), prec="bf16", C=tiny.C, k=tiny.k)
    assert e.value.status == _lib.DSI_E_DTYPE
    # even filter size
    with pytest.raises(P.DsiError) as e:
        ctx.prepare(16, 16, 64, tiny.torch_params(), prec="f32", C=tiny.C, k=(5, 4, 5))
    assert e.value.status == _lib.DSI_E_SHAPE
    net = ctx.prepare(16, 16, 64, params, prec="bf16")
    y = torch.tensor(case.y, dtype=torch.float32, device="cuda")
    out = torch.full((2, 16, 16), 7.0, device="cuda")
    # misaligned y: status DSI_E_ALIGN and the output untouched
    buf = torch.zeros(2 * 64 + 1, device="cuda")
    st = _lib.lib().dsi_recover(ctx.h, net.h, buf.data_ptr() + 4, out.data_ptr(), 2, None)
    assert st == _lib.DSI_E_ALIGN
    st = _lib.lib().dsi_recover(ctx.h, net.h, None, out.data_ptr(), 2, None)
    assert st == _lib.DSI_E_NULL
    st = _lib.lib().dsi_recover(ctx.h, net.h, y.data_ptr(), out.data_ptr(), -1, None)
    assert st == _lib.DSI_E_SHAPE
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)
    # B = 0 is a no-op
    assert _lib.lib().dsi_recover(ctx.h, net.h, None, None, 0, None) == _lib.DSI_OK
    net.free()


def test_measure_noisy_parity(dsi):
    """Noisy measurements at 20 dB (Sec. 5, Table 3) against the oracle's noise model."""
    import torch

    import oracle
    import synth
    P, ctx = dsi
    M, n, B = 410, 64, 6
    phi = synth.make_phi(M, n * n, cfg_id=51)
    x = synth.piecewise_smooth_images(B, n, cfg_id=51).reshape(B, -1)
    e = synth.normal_values((B, M), 1.0, 51, 7)
    ref = oracle.add_noise(oracle.measure(phi, x), e, 20.0)
    t = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")  # noqa: E731
    got = ctx.measure_noisy(t(phi), t(x), t(e), 20.0).cpu().numpy().astype(np.float64)
    assert relerr_per_image(got, ref).max() <= 1e-5


@pytest.mark.parametrize("prec", ["bf16", "f32", "fp8"])
def test_stage_timing_per_pass(dsi, prec):
    """Stage timing records one set of events per forward pass and does not change the result:
    the per-pass query returns the passes' four stage times, at most max_passes of them, and
    forgets every recorded event."""
    import torch

    from paper_1701_03891_amd import _lib
    P, ctx = dsi
    case = make_case(32, 32, 256, 4, cfg_id=31, bias_std=0.05)
    net = ctx.prepare(32, 32, 256, case.torch_params(), prec=prec)
    y = torch.tensor(case.y, dtype=torch.float32, device="cuda")
    ref = net.recover(y).clone()
    _lib.dsi_stage_times(ctx.h)
    _lib.dsi_set_stage_timing(ctx.h, 1)
    outs = [net.recover(y) for _ in range(3)]
    _lib.dsi_set_stage_timing(ctx.h, 0)
    rows, calls = _lib.dsi_stage_times_each(ctx.h, 4, 2)
    assert calls == 3 and len(rows) == 2
    # four stage times, then the time to the next pass's first event (not before this pass ends)
    assert all(len(r) == 5 and all(t > 0 for t in r) and r[4] >= sum(r[:4]) - 1e-6 for r in rows)
    assert all(torch.equal(o, ref) for o in outs)
    # conv layer 2 alone: only its time and the period between passes
    _lib.dsi_set_stage_timing_mask(ctx.h, 1 << 2)
    outs = [net.recover(y) for _ in range(2)]
    _lib.dsi_set_stage_timing_mask(ctx.h, 0)
    rows, calls = _lib.dsi_stage_times_each(ctx.h, 4, 4)
    assert calls == 2 and len(rows) == 2
    assert rows[0][2] > 0 and rows[0][4] >= rows[0][2] and rows[1][2] > 0 and rows[1][4] == 0
    assert rows[0][0] == rows[0][1] == rows[0][3] == 0 and rows[1][0] == rows[1][1] == rows[1][3] == 0
    assert all(torch.equal(o, ref) for o in outs)
    net.recover(y)
    torch.cuda.synchronize()
    assert _lib.dsi_stage_times_each(ctx.h, 4, 2) == ([], 0)
    assert _lib.dsi_stage_times(ctx.h, 4)[1] == 0
    net.free()
