"""Seeded test cases shared by the GPU parity tests.

Inputs come from ``synth`` only; expected values come from ``oracle`` only.
The GPU side receives the same fp32-exact inputs and nothing the oracle
computed except the measurement vectors y (an input of the recovery path).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import oracle
import synth


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
