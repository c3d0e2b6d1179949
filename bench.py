"""Benchmark of the DeepInverse recovery path on one MI355X.

Workload (the configuration the headline metric is quoted on): 64 x 64 images
(N = 4096), M = 1024 measurements (M/N = 0.25), batch 256, the paper's
1 -> 64 -> 32 -> 1 network with 11 x 11 filters; synthetic piecewise-smooth
images, Gaussian Phi, weights trained first (He-initialised, then Adam steps on
the same kind of images).  A step is one recovery (dsi_recover: proxy GEMM,
three conv layers) of one batch whose measurements are already resident in HBM.
Before the warm-up steps the batch is recovered for SETTLE_S seconds while the
GPU's clock ramps up.

Prints ONE JSON line: images/s of the BF16 path (value), the FP32 path beside
it, per-batch latency percentiles, per-stage times, the roofline of the
dominant kernel (conv layer 2) and the FP64 CPU oracle's rate on a sample of
the same workload (which also gives the error and PSNR loss of the BF16 and
FP32 outputs against FP64 on that sample).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SETTLE_S = 0.1          # seconds of recoveries before the warm-up steps (clock ramp)
METRIC = "images recovered/s (64×64, M/N=0.25) bf16 vs fp32; p99 latency; ΔPSNR vs FP64"
PEAK_BF16_TFLOPS = 2500.0   # MI355X dense BF16 MFMA
PEAK_FP32_TFLOPS = 157.3
# HBM bytes per launch of conv layer 2 (BF16, batch 256) from the rocprofv3
# FETCH_SIZE / WRITE_SIZE runs summarised in profiles/recover_64x64_b256_kernels.md,
# fetch scaled by 1.9997 and write by 1.0 (a 256 MiB copy reads back as 128 MiB
# fetched, 256 MiB written).  Valid only for the conv_mid kernel source it was
# measured on; any change to that source makes the figure null.
CONV2_TRAFFIC = {"src_sha256_16": "199179caa758133e", "bytes": (159.22 + 64.00) * 2**20}
N1 = N2 = 64
M = 1024
BATCH = 256


def conv2_flops(B, N):
    """Algorithmic flops of conv layer 2 (64 -> 32 channels, 11 x 11) per launch."""
    return 2.0 * 64 * 32 * 121 * N * B


def path_flops(B, N, M):
    """2MN + 2 k^2 N (C0C1 + C1C2 + C2C3) per image (proxy + three conv layers)."""
    return B * (2.0 * M * N + 2.0 * 121 * N * (64 + 64 * 32 + 32))


def conv2_traffic():
    """Measured HBM bytes of conv layer 2 if its kernel source is the one profiled, else None."""
    import hashlib
    path = os.path.join(ROOT, "paper_1701_03891_amd", "csrc", "conv_mfma.hip")
    src = open(path).read()
    a = src.index("// ===================================================================== conv_mid")
    b = src.index("// =================================================================== conv_first")
    h = hashlib.sha256(src[a:b].encode()).hexdigest()[:16]
    return CONV2_TRAFFIC["bytes"] if h == CONV2_TRAFFIC["src_sha256_16"] else None


def make_inputs(ctx, P, torch, cfg_id=2):
    import synth
    N = N1 * N2
    phi = synth.make_phi(M, N, cfg_id=cfg_id)
    x = synth.piecewise_smooth_images(BATCH, N1, N2, cfg_id=cfg_id).reshape(BATCH, N)
    prm = synth.he_init(synth.PAPER_ARCH, N1, N2, bias_per_pixel=True, cfg_id=cfg_id)
    dev = "cuda:0"
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)  # noqa: E731
    params = P.NetParams(t(phi.T), [t(w) for w in prm.w], [t(b) for b in prm.b])
    phi_d, x_d = t(phi), t(x)
    y = ctx.measure(phi_d, x_d)          # measurements resident in HBM
    return phi, x, prm, params, x_d, y


def time_path(ctx, net, y, steps, warmup, torch):
    """Times `steps` recoveries of the batch y back to back.  The total comes from two events
    around the loop.  Inside it the library records timing-only events (they write no caches
    back, unlike a default event) around conv layer 2 alone, the dominant kernel whose launch
    time the roofline uses; the per-batch latencies are the times from one pass's first event
    to the next pass's.  The four-stage breakdown comes from a second set of `steps` passes
    with every stage boundary timed (each boundary event costs the pass about 1 us).

    Before the `warmup` steps the batch is recovered for SETTLE_S seconds: the GPU raises its
    clock over the first ~20 ms of sustained matrix work (conv layer 2 ran ~410 us per launch in
    the first passes after a pause, ~350 us from about the 60th on), and the timed steps are
    to see the clock a server under load runs at."""
    from paper_1701_03891_amd import _lib
    B = y.shape[0]
    names = ["proxy_gemm", "conv1", "conv2", "conv3"]
    xh = torch.empty((B, N1, N2), dtype=torch.float32, device=y.device)
    t_settle = time.perf_counter()
    settle = 0
    while time.perf_counter() - t_settle < SETTLE_S:
        for _ in range(8):
            net.recover(y, xh)
        settle += 8
        torch.cuda.synchronize()
    for _ in range(warmup):
        net.recover(y, xh)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    _lib.dsi_stage_times(ctx.h)   # drop anything recorded before
    _lib.dsi_set_stage_timing_mask(ctx.h, 1 << names.index("conv2"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        net.recover(y, xh)
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    _lib.dsi_set_stage_timing_mask(ctx.h, 0)
    total_ms = e0.elapsed_time(e1)
    rows, calls = _lib.dsi_stage_times_each(ctx.h, 4, steps)
    assert calls == steps, f"{calls} timed passes recorded for {steps} steps"
    rows = np.array(rows)
    per = rows[:-1, 4] if steps > 1 else np.array([total_ms])   # one step: its own time
    conv2_ms = float(rows[:, 2].mean())
    # the breakdown: every stage timed, outside the timed region
    _lib.dsi_set_stage_timing(ctx.h, 1)
    for _ in range(steps):
        net.recover(y, xh)
    torch.cuda.synchronize()
    _lib.dsi_set_stage_timing(ctx.h, 0)
    rows, calls = _lib.dsi_stage_times_each(ctx.h, 4, steps)
    rows = np.array(rows)
    stages = {name: float(rows[:, q].mean()) for q, name in enumerate(names)}
    return dict(total_ms=total_ms, wall_s=wall, per_step_ms=per, conv2_ms=conv2_ms, stages=stages, xhat=xh,
                settle_passes=settle)


def time_recover(net, y, n1, n2, steps, warmup, torch, settle_s=SETTLE_S):
    """Average ms per dsi_recover of the batch y (events on the current stream), after
    settle_s seconds of recoveries while the clock ramps up and `warmup` more."""
    B = y.shape[0]
    xh = torch.empty((B, n1, n2), dtype=torch.float32, device=y.device)
    t_settle = time.perf_counter()
    while time.perf_counter() - t_settle < settle_s:
        for _ in range(8):
            net.recover(y, xh)
        torch.cuda.synchronize()
    for _ in range(warmup):
        net.recover(y, xh)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        net.recover(y, xh)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, xh


def c4_leg(ctx, P, torch, steps, warmup):
    """128 x 128 images, M = 4096 (a 16384 x 4096 FC layer), batch 64, He-initialised:
    FP8 (static power-of-two scales) and BF16 recovery rates."""
    import synth
    n, Mc, B = 128, 4096, 64
    dev = "cuda:0"
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)  # noqa: E731
    phi = synth.make_phi(Mc, n * n, cfg_id=4)
    x = synth.piecewise_smooth_images(B, n, n, cfg_id=4).reshape(B, -1)
    prm = synth.he_init(synth.PAPER_ARCH, n, n, bias_per_pixel=True, cfg_id=4)
    params = P.NetParams(t(phi.T), [t(w) for w in prm.w], [t(b) for b in prm.b])
    phi_d = t(phi)
    y = ctx.measure(phi_d, t(x))
    xc = synth.piecewise_smooth_images(32, n, n, cfg_id=901, stream=synth.STREAM_CALIB).reshape(32, -1)
    yc = ctx.measure(phi_d, t(xc))
    out = {"workload": "128x128 images, M=4096 (FC 16384x4096), batch 64, He-init, piecewise-smooth"}
    xh = {}
    for prec in ("fp8", "bf16"):
        net = ctx.prepare(n, n, Mc, params, prec=prec)
        if prec == "fp8":
            net.calibrate(yc)
        net.reserve(B)
        ms, xr = time_recover(net, y, n, n, steps, warmup, torch)
        out[prec] = {"images_per_s": B / (ms / 1e3), "ms_per_batch": ms}
        xh[prec] = xr.cpu().numpy().reshape(B, -1)
        net.free()
    del params, phi_d
    return out, {"phi": phi, "x": x, "prm": prm, "y": y.cpu().numpy().astype(np.float64), "xhat": xh}


def c1_leg(ctx, P, torch, steps, warmup):
    """32 x 32 DCT-sparse signals (K = 40), M = 256: recovery time per image of the network
    (He-init; its run time does not depend on the weights) at batch 8 and batch 256."""
    import synth
    n, Mc = 32, 256
    dev = "cuda:0"
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)  # noqa: E731
    phi = synth.make_phi(Mc, n * n, cfg_id=1)
    x = synth.dct_sparse_images(256, n, 40, cfg_id=1).reshape(256, -1)
    prm = synth.he_init(synth.PAPER_ARCH, n, n, bias_per_pixel=True, cfg_id=1)
    params = P.NetParams(t(phi.T), [t(w) for w in prm.w], [t(b) for b in prm.b])
    y = ctx.measure(t(phi), t(x))
    net = ctx.prepare(n, n, Mc, params, prec="bf16")
    net.reserve(256)
    out = {"workload": "32x32 DCT-sparse (K=40), M=256, BF16"}
    for B in (8, 256):
        ms, _ = time_recover(net, y[:B].contiguous(), n, n, steps, warmup, torch)
        out[f"batch{B}"] = {"ms_per_batch": ms, "us_per_image": ms * 1e3 / B}
    net.free()
    return out, {"phi": phi, "x": x, "y": y.cpu().numpy().astype(np.float64)}


SWEEP_N = 32                                       # image side of the M/N sweep
SWEEP_RATIOS = (0.01, 0.05, 0.10, 0.20, 0.25, 0.50)


def sweep_leg(ctx, P, torch, n_test=2000, train_steps=2000, log=None):
    """Recovery quality and run time over M/N (Sec. 5, Figs. 2-3 and Table 1 analogue) on
    32 x 32 piecewise-smooth images: per ratio, a network trained from He-init (BF16,
    Adam) on its own Phi, then success rate (phi, Sec. 5) and mean PSNR over n_test
    fresh Monte Carlo images, and the recovery time per image."""
    import synth
    n = SWEEP_N
    N = n * n
    dev = "cuda:0"
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)  # noqa: E731
    pool = synth.piecewise_smooth_images(8192, n, n, cfg_id=30, stream=11).reshape(8192, -1)
    xtest = synth.piecewise_smooth_images(n_test, n, n, cfg_id=31).reshape(n_test, -1)
    xp_d, xt_d = t(pool), t(xtest)
    out, data = {}, {}
    for q, r in enumerate(SWEEP_RATIOS):
        Mr = synth.m_for_ratio(r, N)
        phi = synth.make_phi(Mr, N, cfg_id=40 + q)
        prm = synth.he_init(synth.PAPER_ARCH, n, n, bias_per_pixel=True, cfg_id=40 + q)
        params = P.NetParams(t(phi.T), [t(w) for w in prm.w], [t(b) for b in prm.b])
        phi_d = t(phi)
        yp, yt = ctx.measure(phi_d, xp_d), ctx.measure(phi_d, xt_d)
        net = ctx.prepare(n, n, Mr, params, prec="bf16")
        net.reserve(256, train=True)
        opt = P.AdamState.zeros_like(params)
        g = synth.rng(40 + q, 12)
        for st in range(train_steps):
            idx = torch.tensor(g.choice(8192, size=128, replace=False), device=dev)
            net.train_step(params, opt, yp[idx].contiguous(), xp_d[idx].contiguous(), lr=3e-4)
        net.update(params)
        xh = torch.empty((n_test, n, n), dtype=torch.float32, device=dev)
        for b0 in range(0, n_test, 256):
            net.recover(yt[b0:b0 + 256].contiguous(), xh[b0:b0 + 256])
        m = ctx.metrics(xh.reshape(n_test, -1), xt_d).cpu().numpy()
        ms1, _ = time_recover(net, yt[:1].contiguous(), n, n, 50, 5, torch)
        ms256, _ = time_recover(net, yt[:256].contiguous(), n, n, 20, 3, torch)
        out[f"{r:.2f}"] = {"M": Mr, "success_rate": float(m[:, 3].mean()), "psnr_mean_db": float(m[:, 1].mean()),
                           "ms_per_image_batch1": ms1, "images_per_s_batch256": 256 / (ms256 / 1e3)}
        if log:
            log(f"sweep M/N {r:.2f}: success {m[:, 3].mean():.3f}, PSNR {m[:, 1].mean():.2f} dB, "
                f"{ms1 * 1e3:.0f} us per image alone")
        data[f"{r:.2f}"] = {"phi": phi, "y": yt[:100].cpu().numpy().astype(np.float64)}
        net.free()
    out["workload"] = (f"32x32 piecewise-smooth images, Gaussian Phi per ratio, network trained "
                       f"{train_steps} Adam steps (lr 3e-4, batch 128) per ratio, {n_test} test images")
    return out, {"x": xtest[:100], "ratios": data}


def cpu_sweep(sw, n_img=100):
    """ISTA-DCT (the classical sparsity-regularised solver) on the first n_img test images
    of every ratio of the sweep (one batched oracle call per ratio, its threads over the
    host's cores): success rate, PSNR, time per image."""
    import oracle
    out = {}
    x = sw["x"][:n_img]
    for key, d in sw["ratios"].items():
        t0 = time.perf_counter()
        xh, _, _ = oracle.ista_dct_batch(d["phi"], d["y"][:n_img], SWEEP_N, SWEEP_N)
        dt = time.perf_counter() - t0
        out[key] = {"success_rate": float(oracle.success(xh, x).mean()),
                    "psnr_mean_db": float(oracle.psnr(xh, x).mean()),
                    "seconds_per_image": dt / n_img, "images": n_img,
                    "note": "wall time of the batch on the host's threads, divided by the images"}
    return out


def train_network(ctx, P, torch, phi, params, steps, batch=128, lr=3e-4, pool=4096, Mx=M):
    """Adam training of the network (Sec. 4: MSE loss, backpropagation) on a pool of
    synthetic piecewise-smooth 64x64 images (a different seed from the benchmark
    batch), BF16 compute with FP32 master weights, through dsi_train_step.
    Updates `params` in place; returns the training statistics."""
    import synth
    dev = "cuda:0"
    xs = synth.piecewise_smooth_images(pool, N1, N2, cfg_id=3, stream=11).reshape(pool, -1)
    xd = torch.tensor(xs, dtype=torch.float32, device=dev)
    yd = ctx.measure(torch.tensor(np.ascontiguousarray(phi), dtype=torch.float32, device=dev), xd)
    net = ctx.prepare(N1, N2, Mx, params, prec="bf16")
    net.reserve(batch, train=True)
    opt = P.AdamState.zeros_like(params)
    g = synth.rng(3, 12)
    idx = [torch.tensor(g.choice(pool, size=batch, replace=False), device=dev) for _ in range(steps)]
    losses = []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for s in range(steps):
        loss = net.train_step(params, opt, yd[idx[s]].contiguous(), xd[idx[s]].contiguous(), lr=lr)
        if s % 50 == 0 or s == steps - 1:
            losses.append(loss)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / max(steps, 1)
    net.free()
    L = [float(v.item()) for v in losses]
    return {"steps": steps, "batch": batch, "lr": lr, "M": Mx, "ms_per_step": ms, "images_per_s": batch / (ms / 1e3),
            "loss_first": L[0], "loss_last": L[-1], "precision": "bf16 compute, fp32 master weights"}


T3_M = 410          # M/N = 0.10 at 64 x 64 (Sec. 5, Table 3)
T3_SNR_DB = 20.0


def table3_leg(ctx, P, torch, train_steps, n_test=256):
    """Noisy measurements (Sec. 5, Table 3 analogue) at 64 x 64, M/N = 0.10 (M = 410):
    a network trained from He-init on its own Phi (noiseless training data, BF16,
    Adam), then mean PSNR over n_test fresh images from noiseless y = Phi x and from
    y = Phi x + e at 20 dB SNR per measurement vector (dsi_measure_noisy, the noise
    draw e seeded)."""
    import synth
    dev = "cuda:0"
    N = N1 * N2
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)  # noqa: E731
    phi = synth.make_phi(T3_M, N, cfg_id=6)
    prm = synth.he_init(synth.PAPER_ARCH, N1, N2, bias_per_pixel=True, cfg_id=6)
    params = P.NetParams(t(phi.T), [t(w) for w in prm.w], [t(b) for b in prm.b])
    train = train_network(ctx, P, torch, phi, params, train_steps, Mx=T3_M)
    x = synth.piecewise_smooth_images(n_test, N1, N2, cfg_id=6).reshape(n_test, -1)
    e = synth.normal_values((n_test, T3_M), 1.0, 6, 7)
    phi_d, x_d = t(phi), t(x)
    ys = {"noiseless": ctx.measure(phi_d, x_d), "snr20db": ctx.measure_noisy(phi_d, x_d, t(e), T3_SNR_DB)}
    net = ctx.prepare(N1, N2, T3_M, params, prec="bf16")
    out = {"workload": f"64x64 piecewise-smooth images, M={T3_M} (M/N=0.10), network trained {train_steps} "
                       f"Adam steps on noiseless measurements; {n_test} test images, noise at "
                       f"{T3_SNR_DB:.0f} dB SNR per measurement vector",
           "training": train}
    host = {"phi": phi, "x": x}
    for k, y in ys.items():
        xh = net.recover(y)
        m = ctx.metrics(xh.reshape(n_test, -1), x_d).cpu().numpy()
        out[k] = {"network_psnr_mean_db": float(m[:, 1].mean()), "network_success_rate": float(m[:, 3].mean())}
        host[k] = y.cpu().numpy().astype(np.float64)
    out["psnr_drop_db_network"] = out["noiseless"]["network_psnr_mean_db"] - out["snr20db"]["network_psnr_mean_db"]
    net.free()
    return out, host


def cpu_table3(t3, n_img=32):
    """ISTA-DCT on the first n_img test images of the noisy-measurement leg, from the
    noiseless and from the 20 dB measurements: mean PSNR (and time per image)."""
    import oracle
    out = {"images": n_img}
    x = t3["x"][:n_img]
    for k in ("noiseless", "snr20db"):
        t0 = time.perf_counter()
        xh, _, _ = oracle.ista_dct_batch(t3["phi"], t3[k][:n_img], N1, N2)
        dt = time.perf_counter() - t0
        out[k] = {"ista_psnr_mean_db": float(oracle.psnr(xh, x).mean()),
                  "ista_success_rate": float(oracle.success(xh, x).mean()), "seconds": dt}
    out["psnr_drop_db_ista"] = out["noiseless"]["ista_psnr_mean_db"] - out["snr20db"]["ista_psnr_mean_db"]
    return out


def calibration_y(ctx, P, torch, phi, B=64):
    """Measurements of a separate seeded calibration batch (FP8 static activation scales)."""
    import synth
    xc = synth.piecewise_smooth_images(B, N1, N2, cfg_id=900, stream=synth.STREAM_CALIB).reshape(B, -1)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda:0")  # noqa: E731
    return ctx.measure(t(phi), t(xc))


def cpu_baseline(phi, x, prm, y_host, xhs, n_img, c4=None, c1=None):
    """The FP64 oracle on the first n_img images of the batch, on this host's cores
    (and on one core for a few images); with c4 / c1, the 128 x 128 FP8 accuracy
    on two sampled images and the classical ISTA-DCT solver's time on one C1 signal."""
    import oracle
    threads = min(16, os.cpu_count() or 1)
    net = oracle.Net(N1, N2, M, bias_full=True)
    bfull = [oracle.full_bias_from_cropped(prm.b[l], 11) for l in range(3)]
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.forward(net, phi.T, prm.w, bfull, y_host[:4])
    dt1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    t0 = time.perf_counter()
    ref = oracle.forward(net, phi.T, prm.w, bfull, y_host[:n_img])
    dt = time.perf_counter() - t0
    xs = x[:n_img]
    ps64 = oracle.psnr(ref, xs)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), model)
    except OSError:
        pass
    out = {"value": n_img / dt, "unit": "images/s", "cores": threads, "kind": "oracle",
           "host": {"cpu_model": model, "logical_cpus": os.cpu_count()},
           "sample": f"{n_img} of the 256 images of the batch (64x64, M=1024), FP64 C oracle, "
                     f"{dt:.1f} s on {threads} threads",
           "single_core": {"value": 4 / dt1, "unit": "images/s", "sample": f"4 images, {dt1:.1f} s on 1 thread"}}
    acc = {}
    for name, xh in xhs.items():
        xh = xh[:n_img].reshape(n_img, -1).astype(np.float64)
        rel = oracle.relerr(xh, ref)
        dps = ps64 - oracle.psnr(xh, xs)
        acc[name] = {"max_relerr_vs_fp64": float(rel.max()), "dpsnr_mean_db": float(dps.mean()),
                     "dpsnr_max_abs_db": float(np.abs(dps).max()),
                     "psnr_mean_db": float(oracle.psnr(xh, xs).mean()),
                     "success_rate": float(oracle.success(xh, xs).mean())}
    acc["fp64"] = {"psnr_mean_db": float(ps64.mean()), "success_rate": float(oracle.success(ref, xs).mean())}
    if c4 is not None:
        n = 128
        net4 = oracle.Net(n, n, 4096, bias_full=True)
        b4 = [oracle.full_bias_from_cropped(c4["prm"].b[l], 11) for l in range(3)]
        idx = np.array([0, 63])
        t0 = time.perf_counter()
        ref4 = oracle.forward(net4, c4["phi"].T, c4["prm"].w, b4, c4["y"][idx])
        dt4 = time.perf_counter() - t0
        x4 = c4["x"][idx]
        a4 = {"sample": f"images 0 and 63 of the 128x128 batch, FP64 oracle {dt4:.1f} s"}
        for name, xh in c4["xhat"].items():
            xh = xh[idx].astype(np.float64)
            a4[name] = {"max_relerr_vs_fp64": float(oracle.relerr(xh, ref4).max()),
                        "dpsnr_mean_db": float((oracle.psnr(ref4, x4) - oracle.psnr(xh, x4)).mean())}
        acc["c4_128x128"] = a4
    if c1 is not None:
        # the classical sparsity-regularised solver (ISTA in the 2-D DCT basis, 12 x 300
        # iterations with continuation, then a least-squares debias) on one signal
        t0 = time.perf_counter()
        xi, _, _ = oracle.ista_dct(c1["phi"], c1["y"][0], 32, 32)
        dti = time.perf_counter() - t0
        out["ista_dct"] = {"seconds_per_image": dti, "threads": 1,
                           "relerr_vs_truth": float(oracle.relerr(xi[None], c1["x"][:1])[0]),
                           "sample": "one 32x32 DCT-sparse signal (K=40), M=256"}
    return out, acc


def profile_leg(ctx, P, torch, leg, steps, warmup):
    """One workload and precision alone (for rocprofv3 runs): prepare, SETTLE_S seconds of
    recoveries while the clock ramps up, then warmup + steps recoveries of one batch, each
    stage's time from the library's HIP events."""
    import synth
    cfg, prec = leg.split(":")
    if cfg == "train":
        # training steps (forward, loss, backward, Adam, repack) at 64x64, batch 128, M = 1024
        phi = synth.make_phi(M, N1 * N2, cfg_id=3)
        prm = synth.he_init(synth.PAPER_ARCH, N1, N2, bias_per_pixel=True, cfg_id=3)
        t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda:0")  # noqa: E731
        params = P.NetParams(t(phi.T), [t(w) for w in prm.w], [t(b) for b in prm.b])
        # 125 more steps first (~0.1 s) while the clock ramps up
        st = train_network(ctx, P, torch, phi, params, 125 + warmup + steps, batch=128, pool=1024)
        print(json.dumps({"profile_leg": leg, "training": st}))
        return
    if cfg == "c2":
        n, Mx, B, cid = N1, M, BATCH, 2
    elif cfg == "c4":
        n, Mx, B, cid = 128, 4096, 64, 4
    else:
        raise SystemExit(f"unknown profiling leg {leg}")
    dev = "cuda:0"
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)  # noqa: E731
    phi = synth.make_phi(Mx, n * n, cfg_id=cid)
    x = synth.piecewise_smooth_images(B, n, n, cfg_id=cid).reshape(B, -1)
    prm = synth.he_init(synth.PAPER_ARCH, n, n, bias_per_pixel=True, cfg_id=cid)
    params = P.NetParams(t(phi.T), [t(w) for w in prm.w], [t(b) for b in prm.b])
    y = ctx.measure(t(phi), t(x))
    net = ctx.prepare(n, n, Mx, params, prec=prec)
    if prec == "fp8":
        xc = synth.piecewise_smooth_images(32, n, n, cfg_id=900 + cid, stream=synth.STREAM_CALIB).reshape(32, -1)
        net.calibrate(ctx.measure(t(phi), t(xc)))
    net.reserve(B)
    xh = torch.empty((B, n, n), dtype=torch.float32, device=dev)
    t_settle = time.perf_counter()   # recoveries while the clock ramps up
    while time.perf_counter() - t_settle < SETTLE_S:
        for _ in range(8):
            net.recover(y, xh)
        torch.cuda.synchronize()
    for _ in range(warmup):
        net.recover(y, xh)
    torch.cuda.synchronize()
    from paper_1701_03891_amd import _lib
    _lib.dsi_stage_times(ctx.h)
    _lib.dsi_set_stage_timing(ctx.h, 1)
    for _ in range(steps):
        net.recover(y, xh)
    torch.cuda.synchronize()
    _lib.dsi_set_stage_timing(ctx.h, 0)
    ms, calls = _lib.dsi_stage_times(ctx.h, 4)
    print(json.dumps({"profile_leg": leg, "batch": B, "image": [n, n], "M": Mx, "steps": calls,
                      "stage_ms": dict(zip(["proxy_gemm", "conv1", "conv2", "conv3"],
                                           [v / max(calls, 1) for v in ms]))}))
    net.free()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-images", type=int, default=256, help="images in the oracle's timed sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving (latency under load) leg")
    ap.add_argument("--train-steps", type=int, default=2000,
                    help="Adam steps on synthetic images before timing (0: He-init weights)")
    ap.add_argument("--serve-requests", type=int, default=10000, help="measured requests per load point")
    ap.add_argument("--serve-qps", type=str, default="2000,8000,64000",
                    help="offered loads (requests/s); the highest should exceed capacity")
    ap.add_argument("--no-extra", action="store_true", help="skip the 128x128 FP8 and 32x32 legs")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the M/N sweep (32x32: a trained network per ratio, 2000 test images, "
                         "ISTA-DCT on 100 of them)")
    ap.add_argument("--no-noise", action="store_true",
                    help="skip the noisy-measurement leg (64x64, M/N = 0.10, 20 dB; ISTA-DCT on 32 images)")
    ap.add_argument("--profile", type=str, default="",
                    help="profiling mode: run only one workload leg, c2:bf16 | c2:f32 | c2:fp8 (64x64, "
                         "B=256) or c4:bf16 | c4:fp8 (128x128, M=4096, B=64), warmup + steps recoveries on "
                         "He-init weights, or train:bf16 (warmup + steps BF16 training steps, 64x64, B=128), "
                         "and print its timing (not the benchmark line)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library and this benchmark run on one GPU; --gpus {args.gpus} is not supported "
              "(images are independent, so N GPUs would each run this benchmark on their own batch)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1701_03891_amd as P

    ctx = P.Context(0)
    if args.copy_mib:
        src = torch.ones(args.copy_mib * (1 << 18), dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.profile:
        profile_leg(ctx, P, torch, args.profile, args.steps, args.warmup)
        ctx.close()
        return
    phi, x, prm, params, x_d, y = make_inputs(ctx, P, torch)
    N = N1 * N2
    train = None
    if args.train_steps > 0:
        train = train_network(ctx, P, torch, phi, params, args.train_steps)
        # the oracle and every precision below use the trained FP32 parameters
        prm.w = [w.cpu().numpy().astype(np.float64) for w in params.w]
        prm.b = [b.cpu().numpy().astype(np.float64) for b in params.b]
    res = {}
    for prec in ("bf16", "f32", "fp8"):
        net = ctx.prepare(N1, N2, M, params, prec=prec)
        if prec == "fp8":
            net.calibrate(calibration_y(ctx, P, torch, phi))
        net.reserve(BATCH)
        r = time_path(ctx, net, y, args.steps, args.warmup, torch)
        r["xhat_host"] = r["xhat"].cpu().numpy()
        res[prec] = r
        net.free()

    sw = sw_data = None
    if not args.no_sweep:
        sw, sw_data = sweep_leg(ctx, P, torch, log=lambda m: print(m, file=sys.stderr, flush=True))
    t3 = t3_data = None
    if not args.no_noise:
        t3, t3_data = table3_leg(ctx, P, torch, max(args.train_steps, 500))
        print(f"noisy measurements: network PSNR {t3['noiseless']['network_psnr_mean_db']:.2f} -> "
              f"{t3['snr20db']['network_psnr_mean_db']:.2f} dB", file=sys.stderr, flush=True)
    c4 = c4_data = c1 = c1_data = None
    if not args.no_extra:
        c4, c4_data = c4_leg(ctx, P, torch, 20, 3)
        c1, c1_data = c1_leg(ctx, P, torch, 50, 5)

    b = res["bf16"]
    ms_step = b["total_ms"] / args.steps
    value = BATCH * args.steps / (b["total_ms"] / 1e3)
    f = res["f32"]
    f_ms = f["total_ms"] / args.steps
    c2_ms = b["conv2_ms"]
    achieved = conv2_flops(BATCH, N) / (c2_ms / 1e3) / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "images/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle": {"seconds": SETTLE_S, "bf16_passes": b["settle_passes"],
                   "what": "untimed recoveries before the warm-up steps while the GPU clock ramps up"},
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "DeepInverse recovery, 64x64 images, M=1024 (M/N=0.25), batch 256, "
                               "1->64->32->1 conv 11x11, weights trained on synthetic images"
                               if train else "DeepInverse recovery, 64x64 images, M=1024 (M/N=0.25), batch 256, "
                               "1->64->32->1 conv 11x11, He-init",
                   "global_batch": BATCH, "image": [N1, N2], "M": M, "parallelism": "single GPU"},
        "fp32": {"value": BATCH * args.steps / (f_ms * args.steps / 1e3), "ms_per_step": f_ms,
                 "stages_ms": f["stages"]},
        "fp8": {"value": BATCH * args.steps / (res["fp8"]["total_ms"] / 1e3),
                "ms_per_step": res["fp8"]["total_ms"] / args.steps, "stages_ms": res["fp8"]["stages"]},
        "speedup_bf16_vs_fp32": f_ms / ms_step,
        "latency_ms_per_batch": {"p50": float(np.percentile(b["per_step_ms"], 50)),
                                 "p99": float(np.percentile(b["per_step_ms"], 99)),
                                 "fp32_p99": float(np.percentile(f["per_step_ms"], 99))},
        "stages_ms": b["stages"],
        "stages_ms_from": "a second set of passes with every stage boundary timed",
        "path_tflops": path_flops(BATCH, N, M) / (ms_step / 1e3) / 1e12,
        "roofline": {"kernel": "conv_mid (conv layer 2, 64->32, 11x11)", "bound": "mfma",
                     "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_BF16_TFLOPS, "traffic": conv2_traffic(),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                     "launch_us": c2_ms * 1e3,
                     "launch_us_from": "timing-only HIP events around conv layer 2 in the timed steps"},
        "cpu_baseline": None,
        "training": train,
        "c4_128x128": c4,
        "c1_32x32": c1,
        "sweep_mn": sw,
        "noisy_measurements": t3,
    }
    if not args.no_cpu:
        y_host = y.cpu().numpy().astype(np.float64)
        cb, acc = cpu_baseline(phi, x, prm, y_host, {k: res[k]["xhat_host"] for k in res}, args.cpu_images,
                               c4=c4_data, c1=c1_data)
        out["cpu_baseline"] = cb
        out["accuracy_vs_fp64_on_sample"] = acc
        if sw_data is not None:
            out["sweep_mn_ista_dct"] = cpu_sweep(sw_data)
            print("sweep: ISTA-DCT done", file=sys.stderr, flush=True)
        if t3_data is not None:
            out["noisy_measurements"]["ista_dct"] = cpu_table3(t3_data)
            print("noisy measurements: ISTA-DCT done", file=sys.stderr, flush=True)
        if c1 is not None and "ista_dct" in cb:
            out["c1_32x32"]["ista_over_network_time_per_image"] = (
                cb["ista_dct"]["seconds_per_image"] / (c1["batch8"]["us_per_image"] * 1e-6))
    ctx.close()
    if not args.no_serve:
        from paper_1701_03891_amd import serve
        qps = [float(q) for q in args.serve_qps.split(",") if q]
        sv = serve.sweep_serving(qps, n_req=args.serve_requests, slots=4, budget_gib=16.0, warmup=1000,
                                 at_fraction=0.7, log=lambda m: print(m, file=sys.stderr, flush=True))
        sv["workload"] = ("Poisson arrivals, 1-32 images per request, 9 networks "
                          "(32/64/128 px x M/N 0.10/0.25/0.50), BF16, 4 streams, HIP graphs; "
                          f"{args.serve_requests} measured requests per load after 1000 warm-up")
        out["serving"] = sv
    print(json.dumps(out))


if __name__ == "__main__":
    main()
