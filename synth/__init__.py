"""Seeded synthetic inputs shaped like the DeepInverse workloads.

This module only draws inputs: measurement matrices, ground-truth signals,
initial weights and biases. It holds none of the recovery method's
arithmetic (no measurement, no proxy, no convolution, no loss), so both the
FP64 oracle and the GPU library can be fed from it without sharing code.

Every generator is driven by ``numpy.random.default_rng`` seeded with a
``SeedSequence([cfg_id, stream])`` pair.  Streams: 0 = measurement matrix,
1 = signals, 2 = weights, 3 = arrivals (serving), 4 = calibration,
5 and up = test-specific draws.

All arrays are returned in float64 but hold values that are exactly
representable in float32 (``as_f32_exact``), so the oracle and the FP32 GPU
inputs see identical numbers.

Paper context (Mousavi & Baraniuk, "Learning to Invert", arXiv 1701.03891):
  * y = Phi x with Phi an M x N matrix, M << N (Sec. 1).
  * x = Psi s with K << N nonzero coefficients in a basis Psi (Sec. 1).
  * three 11x11 convolutional layers with 64, 32 and 1 filters (Sec. 5).
  * training and test images are 64x64 ImageNet crops (Sec. 5); ImageNet is
    not available here, so piecewise-smooth images in [0, 1] of that shape
    stand in for it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

STREAM_PHI = 0
STREAM_SIGNAL = 1
STREAM_WEIGHTS = 2
STREAM_ARRIVALS = 3
STREAM_CALIB = 4


def rng(cfg_id: int, stream: int) -> np.random.Generator:
    """Generator for (configuration id, stream id)."""
    return np.random.default_rng(np.random.SeedSequence([int(cfg_id), int(stream)]))


def as_f32_exact(a) -> np.ndarray:
    """Round to float32 and return as float64 (values exactly representable in fp32)."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def m_for_ratio(ratio: float, n_pix: int) -> int:
    """Number of measurements for an undersampling ratio M/N, rounded half up."""
    return int(math.floor(ratio * n_pix + 0.5))


# --------------------------------------------------------------------------
# measurement matrices (Sec. 1: an arbitrary, non-blocky M x N matrix)
# --------------------------------------------------------------------------
def make_phi(M: int, N: int, cfg_id: int = 0, stream: int = STREAM_PHI) -> np.ndarray:
    """Phi with iid N(0, 1/M) entries, shape [M][N] row-major."""
    g = rng(cfg_id, stream)
    return as_f32_exact(g.standard_normal((M, N)) / math.sqrt(M))


def make_phi_orthonormal_rows(M: int, N: int, cfg_id: int = 0, stream: int = STREAM_PHI) -> np.ndarray:
    """Phi with orthonormal rows (Phi Phi^T = I), from the QR factors of a Gaussian.

    Kept in float64 (not rounded) because its use is to pin exact projection
    identities of the oracle.
    """
    if M > N:
        raise ValueError("orthonormal rows need M <= N")
    g = rng(cfg_id, stream)
    q, r = np.linalg.qr(g.standard_normal((N, M)))
    q = q * np.sign(np.diag(r))[None, :]
    return np.ascontiguousarray(q.T)


# --------------------------------------------------------------------------
# signals
# --------------------------------------------------------------------------
def dct_sparse_images(B: int, n: int, K: int, cfg_id: int = 0, stream: int = STREAM_SIGNAL,
                      return_coeffs: bool = False):
    """B images of n x n pixels, each K-sparse in the orthonormal 2-D DCT-II basis.

    K positions are drawn uniformly without replacement over all n*n
    coefficients (DC included); the values are N(0, 1).  Pixels are the
    orthonormal inverse 2-D DCT (scipy's ``idctn(norm='ortho')``).
    """
    import scipy.fft

    g = rng(cfg_id, stream)
    N = n * n
    coeffs = np.zeros((B, n, n))
    for b in range(B):
        pos = g.choice(N, size=K, replace=False)
        vals = g.standard_normal(K)
        flat = coeffs[b].reshape(-1)
        flat[pos] = vals
    imgs = np.stack([scipy.fft.idctn(coeffs[b], norm="ortho") for b in range(B)])
    imgs = as_f32_exact(imgs)
    if return_coeffs:
        return imgs, coeffs
    return imgs


def piecewise_smooth_images(B: int, n1: int, n2: int | None = None, cfg_id: int = 0,
                            stream: int = STREAM_SIGNAL, sigma: float = 1.5) -> np.ndarray:
    """B piecewise-smooth images of n1 x n2 pixels with values in [0, 1].

    Each image: background 0; U{3..8} shapes, each a rectangle or an ellipse
    with probability 1/2, painted in order with an intensity U[0, 1].
    Rectangles are axis-aligned with sorted uniform integer bounds.  Ellipses
    have a centre U[0, n)^2, semi-axes U[n/16, n/4] and an angle U[0, pi).
    Then a separable Gaussian blur (sigma 1.5, truncated at 4 sigma, reflected
    borders) and a clip to [0, 1].
    """
    import scipy.ndimage

    if n2 is None:
        n2 = n1
    g = rng(cfg_id, stream)
    out = np.zeros((B, n1, n2))
    ii, jj = np.meshgrid(np.arange(n1) + 0.5, np.arange(n2) + 0.5, indexing="ij")
    nmin = min(n1, n2)
    for b in range(B):
        img = np.zeros((n1, n2))
        for _ in range(int(g.integers(3, 9))):
            val = g.uniform(0.0, 1.0)
            if g.uniform() < 0.5:
                r0, r1 = np.sort(g.integers(0, n1 + 1, size=2))
                c0, c1 = np.sort(g.integers(0, n2 + 1, size=2))
                img[r0:r1, c0:c1] = val
            else:
                ci, cj = g.uniform(0, n1), g.uniform(0, n2)
                a, bb = g.uniform(nmin / 16, nmin / 4, size=2)
                th = g.uniform(0, math.pi)
                di, dj = ii - ci, jj - cj
                p = (di * math.cos(th) + dj * math.sin(th)) / a
                q = (-di * math.sin(th) + dj * math.cos(th)) / bb
                img[p * p + q * q <= 1.0] = val
        img = scipy.ndimage.gaussian_filter(img, sigma=sigma, truncate=4.0, mode="reflect")
        out[b] = np.clip(img, 0.0, 1.0)
    return as_f32_exact(out)


# --------------------------------------------------------------------------
# network parameters (Sec. 4 architecture, Sec. 5 sizes)
# --------------------------------------------------------------------------
@dataclass
class Arch:
    """Channel counts C[0..L] and odd filter sizes k[0..L-1] of the conv stack."""

    C: tuple = (1, 64, 32, 1)
    k: tuple = (11, 11, 11)

    @property
    def L(self) -> int:
        return len(self.k)


PAPER_ARCH = Arch((1, 64, 32, 1), (11, 11, 11))
TINY_ARCH = Arch((1, 4, 2, 1), (5, 5, 5))


@dataclass
class Params:
    """Weights [Cout][Cin][k][k] and biases ([Cout] or [Cout][n1][n2]) per layer."""

    w: list = field(default_factory=list)
    b: list = field(default_factory=list)


def he_init(arch: Arch, n1: int, n2: int, bias_per_pixel: bool = True, cfg_id: int = 0,
            stream: int = STREAM_WEIGHTS, bias_std: float = 0.0) -> Params:
    """He-normal weights (std sqrt(2 / (Cin k^2))); biases N(0, bias_std^2) (0 by default)."""
    g = rng(cfg_id, stream)
    p = Params()
    for l in range(arch.L):
        cin, cout, k = arch.C[l], arch.C[l + 1], arch.k[l]
        std = math.sqrt(2.0 / (cin * k * k))
        p.w.append(as_f32_exact(g.standard_normal((cout, cin, k, k)) * std))
        shape = (cout, n1, n2) if bias_per_pixel else (cout,)
        p.b.append(as_f32_exact(g.standard_normal(shape) * bias_std))
    return p


def uniform_values(shape, lo: float, hi: float, cfg_id: int, stream: int) -> np.ndarray:
    """Uniform draws rounded to fp32, for test inputs of arbitrary shape."""
    return as_f32_exact(rng(cfg_id, stream).uniform(lo, hi, size=shape))


def normal_values(shape, std: float, cfg_id: int, stream: int) -> np.ndarray:
    """Normal draws rounded to fp32, for test inputs of arbitrary shape."""
    return as_f32_exact(rng(cfg_id, stream).standard_normal(shape) * std)


def poisson_arrivals(n: int, qps: float, cfg_id: int = 0, stream: int = STREAM_ARRIVALS):
    """Arrival times (s) of n requests of a Poisson process at rate qps."""
    g = rng(cfg_id, stream)
    return np.cumsum(g.exponential(1.0 / qps, size=n))
