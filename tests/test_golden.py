"""The constants the paper states (tests/golden/paper_constants.txt, each line citing its
section) against the oracle, the input generators and the package."""
import os

import numpy as np

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    vals = {}
    with open(os.path.join(HERE, "golden", "paper_constants.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, value = line.split()[:2]
                vals[name] = value
    return vals


def test_architecture_matches_the_paper():
    g = _golden()
    chans = tuple(int(c) for c in g["channels"].split(","))
    k = int(g["filter_size"])
    assert synth.PAPER_ARCH.C == chans and synth.PAPER_ARCH.k == (k,) * (len(chans) - 1)
    import paper_1701_03891_amd as P
    assert P.PAPER_C == chans and P.PAPER_K == (k,) * (len(chans) - 1)
    # He-init draws weights of the paper's shapes: [Cout][Cin][k][k] per layer
    prm = synth.he_init(synth.PAPER_ARCH, int(g["train_image_size"]), int(g["train_image_size"]),
                        bias_per_pixel=False, cfg_id=0)
    assert [w.shape for w in prm.w] == [(chans[l + 1], chans[l], k, k) for l in range(len(chans) - 1)]


def test_success_threshold_matches_the_paper():
    """phi = 1 exactly when ||xhat - x||^2 / ||x||^2 <= the paper's threshold (inclusive)."""
    thr = float(_golden()["success_threshold"])
    x = np.ones((1, 100))
    # squared relative error r: xhat = x + sqrt(r) on one pixel of 100 ones -> r = e^2 / 100
    for r, want in [(thr * 0.999, 1), (thr * 1.001, 0), (0.0, 1), (1.0, 0)]:
        xhat = x.copy()
        xhat[0, 0] += np.sqrt(r * 100.0)
        assert oracle.success(xhat, x)[0] == want, r
    # the oracle's default threshold is the paper's
    xhat = x.copy()
    xhat[0, 0] += np.sqrt(thr * 1.001 * 100.0)
    assert oracle.success(xhat, x)[0] == oracle.success(xhat, x, thr=thr)[0] == 0


def test_noise_experiment_constants():
    """The noisy-measurement experiment adds noise at the paper's SNR (checked on the
    oracle's noise model: the realised per-image SNR is the requested one)."""
    g = _golden()
    snr = float(g["noise_snr_db"])
    assert snr == 20.0 and float(g["noise_undersampling"]) == 0.1
    M, B = 410, 4
    y = synth.normal_values((B, M), 1.0, 77, 1)
    e = synth.normal_values((B, M), 1.0, 77, 2)
    yn = oracle.add_noise(y, e, snr)
    got = 10 * np.log10((y ** 2).sum(1) / ((yn - y) ** 2).sum(1))
    assert np.allclose(got, snr, atol=1e-9)


def test_sweep_uses_the_papers_monte_carlo_count():
    """The M/N sweep (Figs. 2-3 analogue) scores as many test images per ratio as the paper's
    Monte Carlo samples."""
    import inspect

    import bench
    n = int(_golden()["monte_carlo_samples"])
    assert inspect.signature(bench.sweep_leg).parameters["n_test"].default == n
