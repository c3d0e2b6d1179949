"""Seeded test cases shared by the GPU parity tests, and the parity gates.

Inputs come from ``synth`` only; expected values come from ``oracle`` only.
The GPU side receives the same fp32-exact inputs and nothing the oracle
computed except the measurement vectors y (an input of the recovery path).

Two gates hold for every recovered image (``check_recovery``):

* norm-wise: ||xhat_b - ref_b||_2 / ||ref_b||_2 <= TOL_NORM[prec] per image,
  ref the FP64 oracle on the same inputs (the tolerances of the path's
  precision variants);
* per pixel: |xhat[b][p] - ref[b][p]| <= SIGMA_GATE * sigma[b][p] + 2^-22 |ref[b][p]|,
  where sigma is the oracle's first-order model of that pixel's rounding-error
  standard deviation for the precision variant (``oracle.forward_q`` with
  ``want_sigma``: every operand rounding the variant performs and FP32
  accumulation, propagated through the layers).  The second term is the FP32
  rounding of the output itself.  The model is pinned against the actual
  rounding-error distribution on the CPU (std of e / sigma 0.93-0.98, no pixel
  beyond 6 sigma in 10^4-10^6 pixels), so one wrong pixel -- an error of the
  pixel's own magnitude, hundreds of sigma -- fails the gate even where the
  image's norm-wise error stays small.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import oracle
import synth

TOL_NORM = {"f32": 1e-5, "bf16": 2e-2, "fp8": 1e-1, "f64": 1e-7}
SIGMA_GATE = 8.0


@dataclass
class Case:
    n1: int
    n2: int
    M: int
    B: int
    C: tuple
    k: tuple
    bias_per_pixel: bool
    relu_last: bool
    phi: np.ndarray      # [M][N]
    x: np.ndarray        # [B][N] ground truth
    y: np.ndarray        # [B][M] fp32-exact measurements
    w: list              # [Cout][Cin][k][k]
    b: list              # [Cout][n1][n2] or [Cout]

    @property
    def N(self):
        return self.n1 * self.n2

    def oracle_net(self):
        return oracle.Net(self.n1, self.n2, self.M, C=self.C, k=self.k, bias_full=self.bias_per_pixel,
                          relu_last=self.relu_last)

    def oracle_bias(self, border=0.7):
        """Biases on the full grid of Eq. (1) (random borders, which the crop S discards)."""
        if not self.bias_per_pixel:
            return self.b
        return [oracle.full_bias_from_cropped(self.b[l], self.k[l], border=border) for l in range(len(self.k))]

    def oracle_forward(self, idx=None):
        y = self.y if idx is None else self.y[idx]
        return oracle.forward(self.oracle_net(), self.phi.T, self.w, self.oracle_bias(), y)

    def torch_params(self, device="cuda"):
        import torch

        from paper_1701_03891_amd import NetParams
        t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=device)  # noqa: E731
        return NetParams(t(self.phi.T), [t(w) for w in self.w], [t(b) for b in self.b])


def make_case(n1, n2, M, B, cfg_id, C=(1, 64, 32, 1), k=(11, 11, 11), bias_per_pixel=True,
              relu_last=False, signal="smooth", bias_std=0.05, K=40) -> Case:
    N = n1 * n2
    phi = synth.make_phi(M, N, cfg_id=cfg_id)
    if signal == "dct":
        x = synth.dct_sparse_images(B, n1, K, cfg_id=cfg_id).reshape(B, N)
    else:
        x = synth.piecewise_smooth_images(B, n1, n2, cfg_id=cfg_id).reshape(B, N)
    y = synth.as_f32_exact(oracle.measure(phi, x))
    p = synth.he_init(synth.Arch(C, k), n1, n2, bias_per_pixel=bias_per_pixel, cfg_id=cfg_id,
                      bias_std=bias_std)
    return Case(n1, n2, M, B, tuple(C), tuple(k), bias_per_pixel, relu_last, phi, x, y, p.w, p.b)


def relerr_per_image(a, ref):
    a = np.asarray(a, dtype=np.float64).reshape(ref.shape[0], -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(ref.shape[0], -1)
    return oracle.relerr(a, ref)


# ------------------------------------------------------------------ parity gates
_REF = {}


def _key(case):
    return (case.n1, case.n2, case.M, case.B, case.C, case.k, case.bias_per_pixel, case.relu_last,
            float(case.y[0, 0]), float(case.w[0].ravel()[0]), float(case.b[0].ravel()[0]))


def oracle_ref(case, idx=None):
    """FP64 forward of every image (cached per case), or of the images idx."""
    k = _key(case)
    if k not in _REF:
        _REF.clear()            # one case at a time: full-size references are large
        _REF[k] = case.oracle_forward()
    ref = _REF[k]
    return ref if idx is None else ref[idx]


def pow2_scale(amax):
    """Smallest power of two s with amax / s <= 448 (the e4m3 range)."""
    return float(2.0 ** np.ceil(np.log2(amax / 448.0)))


def fp8_scales_from_oracle(case, margin=1.05):
    """Static activation scales {s_y, s_x~, s_a1, s_a2} large enough that no value of this
    batch saturates: y from the inputs, conv layer 1's output from the FP64 forward pass
    (with a margin for the rounding of its inputs)."""
    _, acts = oracle.forward(case.oracle_net(), case.phi.T, case.w, case.oracle_bias(), case.y,
                             return_acts=True)
    a1max = max(float(a[1].max()) for a in acts)
    return [pow2_scale(margin * np.abs(case.y).max()), 1.0, pow2_scale(margin * a1max), 1.0]


def quant_for(prec, scales=None, L=3):
    """The oracle's model of a precision variant of an L-layer network.  scales: the FP8
    net's {W_fc, W2, s_y, s_x~, s_a1, s_a2} (Net.scales())."""
    if prec == "f32":
        return oracle.Quant.fp32(L)
    if prec == "bf16":
        return oracle.Quant.bf16(L)
    if prec == "fp8":
        s_fc, s_w2, s_y, _, s_a1 = (float(v) for v in scales[:5])
        return oracle.Quant.fp8(s_y, s_fc, s_a1, s_w2)
    raise ValueError(prec)


def check_recovery(case, got, prec, idx=None, scales=None, label=""):
    """Both parity gates on recovered images got [len(idx) or B][N] (float64 copy of the
    GPU output).  Returns (max norm-wise error, max |error| / allowed)."""
    got = np.asarray(got, dtype=np.float64).reshape(len(idx) if idx is not None else case.B, -1)
    ref = oracle_ref(case, idx)
    norm = relerr_per_image(got, ref)
    rms = np.sqrt((ref ** 2).mean(axis=1, keepdims=True)) + 1e-300
    if prec == "f64":
        # FP64 arithmetic, output rounded to float32 once
        allowed = 2.0 ** -23 * np.abs(ref) + 1e-12 * rms
    else:
        y = case.y if idx is None else case.y[idx]
        _, sig = oracle.forward_q(case.oracle_net(), case.phi.T, case.w, case.oracle_bias(), y,
                                  quant_for(prec, scales, len(case.k)), want_sigma=True)
        allowed = SIGMA_GATE * sig + 2.0 ** -22 * np.abs(ref) + 1e-12 * rms
    ratio = np.abs(got - ref) / allowed
    worst = np.unravel_index(np.argmax(ratio), ratio.shape)
    print(f"{label} {prec}: {got.shape[0]} images, max norm-wise err {norm.max():.3e} (tol {TOL_NORM[prec]}), "
          f"max |err|/allowed {ratio.max():.3f} at image {worst[0]} pixel {worst[1]}"
          + (f" ({ratio.max() * SIGMA_GATE:.2f} sigma)" if prec != "f64" else ""))
    assert np.all(np.isfinite(got))
    assert norm.max() <= TOL_NORM[prec], (label, prec, norm.max())
    assert ratio.max() <= 1.0, (label, prec, ratio.max(), worst)
    return norm.max(), ratio.max()
