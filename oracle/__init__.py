"""FP64 CPU oracle for DeepInverse -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls it, and it shares no code
with the GPU library: the arithmetic lives in ``orc.c`` (plain C, double
precision), this file only marshals numpy arrays into it.

Every function cites the passage of the paper (Mousavi & Baraniuk, arXiv
1701.03891) it follows; see ``orc.h`` for layouts.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liborc.so")
_SRC = [os.path.join(_HERE, "orc.c")]
_lib = None

_D = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile orc.c into liborc.so with gcc (-O3, OpenMP, no fast-math, no FMA contraction: every
    floating-point operation is rounded as written, in the order written)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        cmd = ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-Wall", "-o", tmp] + _SRC + ["-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(tmp, _SO)
    return _SO


class _Net(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int), ("n2", ctypes.c_int), ("M", ctypes.c_int),
                ("L", ctypes.c_int), ("C", ctypes.c_int * 9), ("k", ctypes.c_int * 8),
                ("bias_full", ctypes.c_int), ("relu_last", ctypes.c_int)]


def lib():
    """The loaded oracle library (ORC_LIB_PATH overrides the path, for mutation tests)."""
    global _lib
    if _lib is None:
        path = os.environ.get("ORC_LIB_PATH")
        if not path:
            if not os.path.exists(_SO):
                build(force=False)
            path = _SO
        L = ctypes.CDLL(path)
        i, d, l_ = ctypes.c_int, ctypes.c_double, ctypes.c_long
        P = ctypes.c_void_p
        sig = {
            "orc_measure": (None, [P, P, P, i, i, i]),
            "orc_proxy": (None, [P, P, P, i, i, i]),
            "orc_add_noise": (None, [P, P, i, i, d]),
            "orc_conv_layer": (None, [P, i, i, i, P, i, i, P, i, i, P, P]),
            "orc_acts_per_image": (l_, [P]),
            "orc_forward": (None, [P, P, P, P, P, i, P, P]),
            "orc_loss": (d, [P, P, i, i, P]),
            "orc_backward": (d, [P, P, P, P, P, P, i, P, P, P, P]),
            "orc_adam": (None, [P, P, P, P, l_, l_, d, d, d, d]),
            "orc_backward_acts": (None, [P, P, P, P, P, P, i, P, P, P, P]),
            "orc_psnr": (d, [P, P, i]),
            "orc_relerr": (d, [P, P, i]),
            "orc_success": (i, [P, P, i, d]),
            "orc_dct_matrix": (None, [i, P]),
            "orc_spectral_norm": (d, [P, i, i, i]),
            "orc_ista_dct": (i, [P, P, i, i, i, i, i, d, P, P]),
            "orc_ista_dct_batch": (None, [P, P, i, i, i, i, i, i, d, P, P, P]),
            "orc_round": (d, [d, i]),
            "orc_quantize": (None, [P, P, l_, i, d]),
            "orc_forward_q": (None, [P, P, P, P, P, i, P, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _ptr_array(arrs):
    arr = (ctypes.c_void_p * len(arrs))()
    for q, a in enumerate(arrs):
        arr[q] = a.ctypes.data
    return arr


def set_threads(n: int) -> None:
    """Number of OpenMP threads the oracle uses (images are split across them)."""
    os.environ["OMP_NUM_THREADS"] = str(int(n))
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
    except OSError:
        pass


# ---------------------------------------------------------------- network
@dataclass
class Net:
    """Conv-stack description (Sec. 4): channels C[0..L] and odd filter sizes k."""

    n1: int
    n2: int
    M: int
    C: tuple = (1, 64, 32, 1)
    k: tuple = (11, 11, 11)
    bias_full: bool = True
    relu_last: bool = False

    @property
    def L(self):
        return len(self.k)

    def _c(self) -> _Net:
        s = _Net()
        s.n1, s.n2, s.M, s.L = self.n1, self.n2, self.M, self.L
        for q, c in enumerate(self.C):
            s.C[q] = c
        for q, kk in enumerate(self.k):
            s.k[q] = kk
        s.bias_full, s.relu_last = int(self.bias_full), int(self.relu_last)
        return s

    def full_bias_shape(self, l):
        return (self.C[l + 1], self.n1 + self.k[l] - 1, self.n2 + self.k[l] - 1)


def full_bias_from_cropped(b: np.ndarray, k: int, border: float | np.ndarray = 0.0) -> np.ndarray:
    """Embed a per-pixel bias [C][n1][n2] into the full (n+k-1) grid that Eq. (1) uses.

    The crop S discards the border entries, so their value (``border``) can be
    anything; tests set it to random values to show that.
    """
    C, n1, n2 = b.shape
    r = (k - 1) // 2
    out = np.empty((C, n1 + k - 1, n2 + k - 1))
    out[...] = border
    out[:, r:r + n1, r:r + n2] = b
    return out


def crop_full(bf: np.ndarray, k: int) -> np.ndarray:
    """Inverse of ``full_bias_from_cropped``: the window the crop S keeps."""
    r = (k - 1) // 2
    C, f1, f2 = bf.shape
    return bf[:, r:f1 - r, r:f2 - r].copy()


# ---------------------------------------------------------------- Sec. 1, 4
def measure(phi, x):
    """y = Phi x (Sec. 1). phi [M][N], x [B][N] -> y [B][M]."""
    phi, x = _c(phi), _c(x)
    B, N = x.shape
    M = phi.shape[0]
    y = np.empty((B, M))
    lib().orc_measure(_p(phi), _p(x), _p(y), B, M, N)
    return y


def add_noise(y, e, snr_db):
    """y + s e per row with ||y||^2 / ||s e||^2 = 10^(snr_db/10) (Sec. 5, Table 3: noisy measurements)."""
    y, e = _c(y).copy(), _c(e)
    B, M = y.shape
    lib().orc_add_noise(_p(y), _p(e), B, M, float(snr_db))
    return y


def proxy(wfc, y):
    """Signal proxy x~ = Phi^T y by the fixed fully connected layer (Sec. 4). wfc [N][M]."""
    wfc, y = _c(wfc), _c(y)
    B, M = y.shape
    N = wfc.shape[0]
    xt = np.empty((B, N))
    lib().orc_proxy(_p(wfc), _p(y), _p(xt), B, M, N)
    return xt


def conv_layer(x, w, b, bias_full=True, relu=True, return_zfull=False):
    """One layer of Eq. (1) on each image of a batch.

    x [B][Cin][n1][n2], w [Cout][Cin][k][k], b [Cout][n1+k-1][n2+k-1] (bias_full)
    or [Cout].  Returns out [B][Cout][n1][n2] (and the full pre-activation).
    """
    x, w, b = _c(x), _c(w), _c(b)
    B, Cin, n1, n2 = x.shape
    Cout, _, k, _ = w.shape
    out = np.empty((B, Cout, n1, n2))
    zf = np.empty((B, Cout, n1 + k - 1, n2 + k - 1))
    for bi in range(B):
        lib().orc_conv_layer(_p(x[bi]), Cin, n1, n2, _p(w), Cout, k, _p(b), int(bias_full),
                             int(relu), _p(zf[bi]), _p(out[bi]))
    return (out, zf) if return_zfull else out


def _params_c(net: Net, w, b):
    ws = [_c(a) for a in w]
    bs = [_c(a) for a in b]
    for l in range(net.L):
        exp_w = (net.C[l + 1], net.C[l], net.k[l], net.k[l])
        exp_b = net.full_bias_shape(l) if net.bias_full else (net.C[l + 1],)
        if ws[l].shape != exp_w or bs[l].shape != exp_b:
            raise ValueError(f"layer {l}: w {ws[l].shape} (want {exp_w}), b {bs[l].shape} (want {exp_b})")
    return ws, bs


def forward(net: Net, wfc, w, b, y, return_acts=False):
    """xhat = M(y, Omega) (Sec. 4): proxy, then Eq. (1) for every layer.

    w[l] [Cout][Cin][k][k]; b[l] full-grid [Cout][n1+k-1][n2+k-1] (bias_full)
    or [Cout].  Returns xhat [B][N] (and per-image activations a_0..a_L).
    """
    wfc, y = _c(wfc), _c(y)
    ws, bs = _params_c(net, w, b)
    B = y.shape[0]
    N = net.n1 * net.n2
    xhat = np.empty((B, N))
    cn = net._c()
    acts = None
    if return_acts:
        per = lib().orc_acts_per_image(ctypes.byref(cn))
        acts = np.empty((B, per))
    lib().orc_forward(ctypes.byref(cn), _p(wfc), _ptr_array(ws), _ptr_array(bs), _p(y), B,
                      _p(xhat), _p(acts) if acts is not None else None)
    if not return_acts:
        return xhat
    out = []
    for bi in range(B):
        off, a = 0, []
        for l in range(net.L + 1):
            sz = net.C[l] * N
            a.append(acts[bi, off:off + sz].reshape(net.C[l], net.n1, net.n2))
            off += sz
        out.append(a)
    return xhat, out


# ------------------------------------------------ reduced-precision operands
Q_NONE, Q_BF16, Q_E4M3 = 0, 1, 2


class _Q(ctypes.Structure):
    _fields_ = [("fmt", ctypes.c_int), ("scale", ctypes.c_double)]


class _Quant(ctypes.Structure):
    _fields_ = [("y", _Q), ("wfc", _Q), ("xt", _Q), ("w", _Q * 8), ("a", _Q * 8),
                ("acc_fp32", ctypes.c_int)]


@dataclass
class Quant:
    """Where a reduced-precision forward pass rounds its operands: each point is
    (format, scale), a value v being stored as round(v / scale) * scale.  Points:
    y, the FC weights W_fc, the proxy x~, the weights w[l] of conv layer l and the
    output a[l] of conv layer l.  acc_fp32 adds FP32 accumulation to the error model."""

    y: tuple = (Q_NONE, 1.0)
    wfc: tuple = (Q_NONE, 1.0)
    xt: tuple = (Q_NONE, 1.0)
    w: list = field(default_factory=lambda: [(Q_NONE, 1.0)] * 8)
    a: list = field(default_factory=lambda: [(Q_NONE, 1.0)] * 8)
    acc_fp32: bool = False

    def _c(self) -> _Quant:
        q = _Quant()
        for name in ("y", "wfc", "xt"):
            f, sc = getattr(self, name)
            setattr(q, name, _Q(int(f), float(sc)))
        for l in range(8):
            q.w[l] = _Q(int(self.w[l][0]), float(self.w[l][1]))
            q.a[l] = _Q(int(self.a[l][0]), float(self.a[l][1]))
        q.acc_fp32 = int(self.acc_fp32)
        return q

    @staticmethod
    def fp32(L=3) -> "Quant":
        """FP32 operands, FP32 accumulation (no operand rounding: the inputs are FP32 values)."""
        return Quant(acc_fp32=True)

    @staticmethod
    def bf16(L=3) -> "Quant":
        """BF16 variant: y, W_fc and every conv weight are rounded to BF16 before use, the
        proxy x~ and every hidden layer's output after it is computed; sums in FP32 and
        the network's output is FP32."""
        b = (Q_BF16, 1.0)
        return Quant(y=b, wfc=b, xt=b, w=[b] * L + [(Q_NONE, 1.0)] * (8 - L),
                     a=[b] * (L - 1) + [(Q_NONE, 1.0)] * (9 - L), acc_fp32=True)

    @staticmethod
    def fp8(s_y, s_fc, s_a1, s_w2) -> "Quant":
        """FP8 variant of the paper's network: the proxy layer and conv layer 2 take e4m3
        operands with power-of-two per-tensor scales (y: s_y, W_fc: s_fc, conv layer 1's
        output: s_a1, W2: s_w2); conv layers 1 and 3 take BF16 operands, x~ and conv
        layer 2's output are stored in BF16; sums in FP32."""
        b, e = (Q_BF16, 1.0), Q_E4M3
        none = (Q_NONE, 1.0)
        return Quant(y=(e, s_y), wfc=(e, s_fc), xt=b, w=[b, (e, s_w2), b] + [none] * 5,
                     a=[(e, s_a1), b] + [none] * 6, acc_fp32=True)


def round_fmt(x, fmt):
    """Round each value to the nearest value of format fmt (ties to even; e4m3 saturating)."""
    x = np.asarray(x, dtype=np.float64)
    return np.vectorize(lambda v: lib().orc_round(float(v), int(fmt)), otypes=[np.float64])(x)


def quantize(x, fmt, scale=1.0):
    """round(x / scale) * scale elementwise."""
    x = _c(x)
    out = np.empty_like(x)
    lib().orc_quantize(_p(x), _p(out), x.size, int(fmt), float(scale))
    return out


def forward_q(net: Net, wfc, w, b, y, quant: Quant, want_sigma=False):
    """The forward map (Sec. 4, Eq. 1) with operands rounded at the points of ``quant``
    (exact sums).  With ``want_sigma`` also returns the modelled standard deviation of
    each output pixel's error against the exact map (see orc.h)."""
    wfc, y = _c(wfc), _c(y)
    ws, bs = _params_c(net, w, b)
    B = y.shape[0]
    N = net.n1 * net.n2
    xhat = np.empty((B, N))
    sig = np.empty((B, N)) if want_sigma else None
    cn, cq = net._c(), quant._c()
    lib().orc_forward_q(ctypes.byref(cn), _p(wfc), _ptr_array(ws), _ptr_array(bs), _p(y), B,
                        ctypes.byref(cq), _p(xhat), _p(sig) if sig is not None else None)
    return (xhat, sig) if want_sigma else xhat


def loss(xhat, x):
    """L = (1/B) sum_b ||xhat_b - x_b||^2 (Sec. 4) and dL/dxhat."""
    xhat, x = _c(xhat), _c(x)
    B, N = x.shape
    g = np.empty_like(x)
    L = lib().orc_loss(_p(xhat), _p(x), B, N, _p(g))
    return L, g


@dataclass
class Grads:
    loss: float
    w: list = field(default_factory=list)
    b: list = field(default_factory=list)
    y: np.ndarray | None = None
    wfc: np.ndarray | None = None


def backward(net: Net, wfc, w, b, y, x, want_gy=False, want_gwfc=False) -> Grads:
    """Loss (Sec. 4) and its gradient for every parameter, by backpropagation."""
    wfc, y, x = _c(wfc), _c(y), _c(x)
    ws, bs = _params_c(net, w, b)
    B = y.shape[0]
    gw = [np.empty_like(a) for a in ws]
    gb = [np.empty_like(a) for a in bs]
    gy = np.empty_like(y) if want_gy else None
    gwfc = np.empty_like(wfc) if want_gwfc else None
    cn = net._c()
    L = lib().orc_backward(ctypes.byref(cn), _p(wfc), _ptr_array(ws), _ptr_array(bs), _p(y),
                           _p(x), B, _ptr_array(gw), _ptr_array(gb),
                           _p(gy) if gy is not None else None,
                           _p(gwfc) if gwfc is not None else None)
    return Grads(L, gw, gb, gy, gwfc)


def backward_acts(net: Net, wfc, w, y, acts, g_out, want_gy=False, want_gwfc=False) -> Grads:
    """Backpropagation (Sec. 4) from GIVEN activations: acts[b] = [a_0, ..., a_L]
    (each [C_l][n1][n2]), g_out = dL/dxhat [B][N].  ReLU masks come from the
    given post-activations, so a network whose forward pass ran elsewhere
    (e.g. in reduced precision) can be differentiated exactly in FP64."""
    wfc, y, g_out = _c(wfc), _c(y), _c(g_out)
    ws = [_c(a) for a in w]
    B = y.shape[0]
    flat = np.ascontiguousarray(np.stack([np.concatenate([np.asarray(a, dtype=np.float64).ravel()
                                                           for a in acts[b]]) for b in range(B)]))
    gw = [np.empty_like(a) for a in ws]
    gb = [np.empty(net.full_bias_shape(l) if net.bias_full else (net.C[l + 1],)) for l in range(net.L)]
    gy = np.empty_like(y) if want_gy else None
    gwfc = np.empty_like(wfc) if want_gwfc else None
    cn = net._c()
    lib().orc_backward_acts(ctypes.byref(cn), _p(wfc), _ptr_array(ws), _p(y), _p(flat), _p(g_out), B,
                            _ptr_array(gw), _ptr_array(gb), _p(gy) if gy is not None else None,
                            _p(gwfc) if gwfc is not None else None)
    return Grads(float("nan"), gw, gb, gy, gwfc)


def adam(theta, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba, bias-corrected); updates theta, m, v in place copies."""
    theta, g, m, v = _c(theta).copy(), _c(g), _c(m).copy(), _c(v).copy()
    lib().orc_adam(_p(theta), _p(g), _p(m), _p(v), theta.size, int(t), lr, beta1, beta2, eps)
    return theta, m, v


def psnr(xhat, x):
    """Per-image PSNR = 10 log10(max(x)^2 / MSE) (Sec. 5 footnote)."""
    xhat, x = np.atleast_2d(_c(xhat)), np.atleast_2d(_c(x))
    return np.array([lib().orc_psnr(_p(_c(xhat[q])), _p(_c(x[q])), x.shape[1])
                     for q in range(x.shape[0])])


def relerr(a, ref):
    """Per-image norm-wise relative error ||a - ref|| / ||ref||."""
    a, ref = np.atleast_2d(_c(a)), np.atleast_2d(_c(ref))
    return np.array([lib().orc_relerr(_p(_c(a[q])), _p(_c(ref[q])), ref.shape[1])
                     for q in range(ref.shape[0])])


def success(xhat, x, thr=0.1):
    """Success indicator phi of Sec. 5 per image."""
    xhat, x = np.atleast_2d(_c(xhat)), np.atleast_2d(_c(x))
    return np.array([lib().orc_success(_p(_c(xhat[q])), _p(_c(x[q])), x.shape[1], thr)
                     for q in range(x.shape[0])])


def dct_matrix(n):
    C = np.empty((n, n))
    lib().orc_dct_matrix(n, _p(C))
    return C


def spectral_norm(phi, iters=300):
    phi = _c(phi)
    return lib().orc_spectral_norm(_p(phi), phi.shape[0], phi.shape[1], iters)


def ista_dct(phi, y, n1, n2, stages=12, iters=300, decay=0.3):
    """Classical reference: ISTA in the 2-D DCT basis with continuation and debias."""
    phi, y = _c(phi), _c(y)
    M = phi.shape[0]
    s = np.empty(n1 * n2)
    x = np.empty(n1 * n2)
    ns = lib().orc_ista_dct(_p(phi), _p(y), M, n1, n2, stages, iters, decay, _p(s), _p(x))
    return x, s.reshape(n1, n2), ns


def ista_dct_batch(phi, Y, n1, n2, stages=12, iters=300, decay=0.3):
    """ista_dct on every row of Y [B][M] (same steps and sums per image; the passes
    over Phi are shared).  Returns X [B][N], S [B][n1][n2], support sizes [B]."""
    phi, Y = _c(phi), _c(np.atleast_2d(Y))
    B, M = Y.shape
    N = n1 * n2
    S = np.empty((B, N))
    X = np.empty((B, N))
    ns = np.zeros(B, dtype=np.int32)
    lib().orc_ista_dct_batch(_p(phi), _p(Y), B, M, n1, n2, stages, iters, decay, _p(S), _p(X),
                             ns.ctypes.data_as(ctypes.c_void_p))
    return X, S.reshape(B, n1, n2), ns
