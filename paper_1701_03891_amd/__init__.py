"""DeepInverse recovery path on one MI355X (gfx950), behind the libdsi C ABI.

Mousavi & Baraniuk, "Learning to Invert: Signal Recovery via Deep
Convolutional Networks" (arXiv 1701.03891): measurements y = Phi x (Sec. 1)
go through a fixed fully connected layer Phi^T (the signal proxy, Sec. 4) and
a stack of 2-D convolutions with ReLU (Eq. 1; 1 -> 64 -> 32 -> 1 channels,
11 x 11 filters in Sec. 5) to the estimate xhat.

This package is a thin torch-facing layer over ``libdsi.so``: torch supplies
device memory and streams, every step of the path runs in the library's HIP
kernels.  There is no CPU path.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

from . import _lib
from ._lib import (DSI_BF16, DSI_F32, DSI_F64, DSI_FP8_E4M3, PREC, Adam, DsiError, NetDesc, Params)

__all__ = ["Context", "Net", "NetParams", "AdamState", "DsiError", "PAPER_C", "PAPER_K", "PREC",
           "DSI_F32", "DSI_BF16", "DSI_FP8_E4M3", "DSI_F64"]

PAPER_C = (1, 64, 32, 1)
PAPER_K = (11, 11, 11)


def _torch():
    import torch
    return torch


def _ptr(t):
    """Device pointer of a contiguous CUDA/HIP tensor (None passes NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libdsi takes device tensors")
    if not t.is_contiguous():
        raise ValueError("libdsi takes contiguous tensors")
    return ctypes.c_void_p(t.data_ptr())


def _f32(t, name):
    torch = _torch()
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32, got {t.dtype}")
    return t


def _stream(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


@dataclass
class NetParams:
    """Omega (Sec. 4) as float32 device tensors: w_fc [N][M], w[l] [Cout][Cin][k][k], b[l]."""

    w_fc: object
    w: list = field(default_factory=list)
    b: list = field(default_factory=list)

    def to_c(self) -> Params:
        p = Params()
        p.w_fc = _ptr(_f32(self.w_fc, "w_fc")).value
        for l, (w, b) in enumerate(zip(self.w, self.b)):
            p.w[l] = _ptr(_f32(w, f"w[{l}]")).value
            p.b[l] = _ptr(_f32(b, f"b[{l}]")).value
        return p

    @staticmethod
    def grads_like(params: "NetParams", with_fc: bool = False) -> "NetParams":
        torch = _torch()
        return NetParams(torch.zeros_like(params.w_fc) if with_fc else None,
                         [torch.zeros_like(w) for w in params.w], [torch.zeros_like(b) for b in params.b])

    def grads_to_c(self) -> Params:
        p = Params()
        if self.w_fc is not None:
            p.w_fc = _ptr(_f32(self.w_fc, "gw_fc")).value
        for l, (w, b) in enumerate(zip(self.w, self.b)):
            p.w[l] = _ptr(_f32(w, f"gw[{l}]")).value
            p.b[l] = _ptr(_f32(b, f"gb[{l}]")).value
        return p


@dataclass
class AdamState:
    m_w: list
    v_w: list
    m_b: list
    v_b: list
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    c: Adam | None = None

    m_fc: object = None
    v_fc: object = None

    @staticmethod
    def zeros_like(params: NetParams, beta1=0.9, beta2=0.999, eps=1e-8, with_fc=False) -> "AdamState":
        torch = _torch()
        z = lambda ts: [torch.zeros_like(t) for t in ts]  # noqa: E731
        s = AdamState(z(params.w), z(params.w), z(params.b), z(params.b), beta1, beta2, eps)
        c = Adam()
        if with_fc:
            s.m_fc, s.v_fc = torch.zeros_like(params.w_fc), torch.zeros_like(params.w_fc)
            c.m_fc, c.v_fc = s.m_fc.data_ptr(), s.v_fc.data_ptr()
        for l in range(len(params.w)):
            c.m_w[l] = s.m_w[l].data_ptr()
            c.v_w[l] = s.v_w[l].data_ptr()
            c.m_b[l] = s.m_b[l].data_ptr()
            c.v_b[l] = s.v_b[l].data_ptr()
        c.beta1, c.beta2, c.eps, c.step = beta1, beta2, eps, 0
        s.c = c
        return s

    @property
    def step(self) -> int:
        return int(self.c.step)


def make_desc(n1, n2, M, C=PAPER_C, k=PAPER_K, bias_per_pixel=True, relu_last=False,
              fc_trainable=False) -> NetDesc:
    d = NetDesc()
    d.fc_trainable = int(fc_trainable)
    d.n1, d.n2, d.M, d.L = n1, n2, M, len(k)
    for q, c in enumerate(C):
        d.C[q] = c
    for q, kk in enumerate(k):
        d.k[q] = kk
    d.bias_per_pixel, d.relu_last = int(bias_per_pixel), int(relu_last)
    return d


class Context:
    """A libdsi context on one HIP device (owns the workspace)."""

    def __init__(self, device: int = 0):
        self.device = device
        self.h = _lib.dsi_create(device)

    def close(self):
        if self.h:
            _lib.dsi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_workspace(self, buf):
        """Use the device tensor buf (uint8, contiguous) as the context's workspace (None:
        back to a library-owned one).  The caller keeps buf alive while it is in use."""
        if buf is None:
            _lib.dsi_set_workspace(self.h, None, 0)
            self._ws_ref = None
            return
        _lib.dsi_set_workspace(self.h, _ptr(buf), buf.numel() * buf.element_size())
        self._ws_ref = buf

    def set_recompute_budget(self, nbytes: int):
        """Workspace bytes one chunk of recompute-mode training may use (0: whole batch)."""
        _lib.dsi_set_recompute_budget(self.h, int(nbytes))

    def measure(self, phi, x, y=None):
        """y = Phi x (Sec. 1). phi [M][N], x [B][N] float32 device tensors."""
        torch = _torch()
        M, N = phi.shape
        B = x.shape[0]
        if x.shape[1] != N:
            raise ValueError("x and phi disagree on N")
        if y is None:
            y = torch.empty((B, M), dtype=torch.float32, device=x.device)
        _lib.dsi_measure(self.h, _ptr(_f32(phi, "phi")), _ptr(_f32(x, "x")), _ptr(y), B, M, N,
                         _stream(self.device))
        return y

    def measure_noisy(self, phi, x, e, snr_db, y=None):
        """y = Phi x + s e with per-vector SNR snr_db (Sec. 5, Table 3). e [B][M] is the noise draw."""
        torch = _torch()
        M, N = phi.shape
        B = x.shape[0]
        if y is None:
            y = torch.empty((B, M), dtype=torch.float32, device=x.device)
        _lib.dsi_measure_noisy(self.h, _ptr(_f32(phi, "phi")), _ptr(_f32(x, "x")), _ptr(_f32(e, "e")), snr_db,
                               _ptr(y), B, M, N, _stream(self.device))
        return y

    def prepare(self, n1, n2, M, params: NetParams, prec="bf16", C=PAPER_C, k=PAPER_K,
                bias_per_pixel=True, relu_last=False, fc_trainable=False) -> "Net":
        desc = make_desc(n1, n2, M, C, k, bias_per_pixel, relu_last, fc_trainable)
        p = PREC[prec] if isinstance(prec, str) else int(prec)
        h = _lib.dsi_net_prepare(self.h, desc, params.to_c(), p, _stream(self.device))
        return Net(self, h, desc, p)

    def metrics(self, xhat, x):
        """Per-image FP64 [sse, PSNR, rel. error, success] (Sec. 5) computed on the device."""
        torch = _torch()
        B, N = xhat.shape[0], xhat[0].numel()
        out = torch.empty((B, 4), dtype=torch.float64, device=xhat.device)
        _lib.dsi_metrics(self.h, _ptr(_f32(xhat, "xhat")), _ptr(_f32(x, "x")), B, N, _ptr(out),
                         _stream(self.device))
        return out


class Net:
    """A prepared network: packed weights in one precision."""

    def __init__(self, ctx: Context, h, desc: NetDesc, prec: int):
        self.ctx, self.h, self.desc, self.prec = ctx, h, desc, prec
        self.n1, self.n2, self.M = desc.n1, desc.n2, desc.M
        self.N = desc.n1 * desc.n2

    def free(self):
        if self.h:
            _lib.dsi_net_free(self.ctx.h, self.h)
            self.h = None

    def update(self, params: NetParams):
        _lib.dsi_net_update(self.ctx.h, self.h, params.to_c(), _stream(self.ctx.device))

    def set_act_scales(self, scales):
        _lib.dsi_net_set_act_scales(self.h, list(scales))

    def calibrate(self, y):
        """FP8 nets: static activation scales from a calibration batch y [B][M]."""
        _lib.dsi_net_calibrate(self.ctx.h, self.h, _ptr(_f32(y, "y")), y.shape[0], _stream(self.ctx.device))

    def scales(self):
        """{W_fc, W2, s_y, s_x~, s_a1, s_a2} scales (1 except for FP8 nets)."""
        return _lib.dsi_net_get_scales(self.h, 6)

    def reserve(self, B, train=False):
        _lib.dsi_reserve(self.ctx.h, self.h, B, train)

    def workspace_size(self, B, train=False) -> int:
        return _lib.dsi_workspace_size(self.h, B, train)

    def recover(self, y, xhat=None):
        """xhat = M(y, Omega) (Sec. 4). y [B][M] -> xhat [B][n1][n2]."""
        torch = _torch()
        B = y.shape[0]
        if y.shape[1] != self.M:
            raise ValueError(f"y has {y.shape[1]} measurements, net expects {self.M}")
        if xhat is None:
            xhat = torch.empty((B, self.n1, self.n2), dtype=torch.float32, device=y.device)
        _lib.dsi_recover(self.ctx.h, self.h, _ptr(_f32(y, "y")), _ptr(xhat), B, _stream(self.ctx.device))
        return xhat

    def saved_bytes(self, B, recompute=False) -> int:
        """Bytes of the state forward_train keeps for a batch of B images."""
        return _lib.dsi_workspace_size(self.h, B, 2 if recompute else 1)

    def forward_train(self, y, recompute=False):
        """xhat and the state the backward pass needs: every activation, or (recompute)
        only the proxy and the output, the hidden layers being recomputed by backward."""
        torch = _torch()
        B = y.shape[0]
        nbytes = self.saved_bytes(B, recompute)
        saved = torch.empty(nbytes, dtype=torch.uint8, device=y.device)
        xhat = torch.empty((B, self.n1, self.n2), dtype=torch.float32, device=y.device)
        _lib.dsi_forward_train(self.ctx.h, self.h, _ptr(_f32(y, "y")), _ptr(xhat), B, _ptr(saved), nbytes,
                               int(recompute), _stream(self.ctx.device))
        return xhat, saved

    def saved_activation(self, saved, B, layer):
        """Activation `layer` (0 = proxy, L = xhat) of a forward_train state, as float32 [B][C][n1][n2]."""
        torch = _torch()
        C = self.desc.C[layer]
        out = torch.empty((B, C, self.n1, self.n2), dtype=torch.float32, device=saved.device)
        _lib.dsi_saved_activation(self.ctx.h, self.h, _ptr(saved), saved.numel(), B, layer, _ptr(out),
                                  _stream(self.ctx.device))
        return out

    def backward(self, gxhat, saved, params_like: NetParams, want_gy=False, recompute=False):
        torch = _torch()
        B = gxhat.shape[0]
        g = NetParams.grads_like(params_like, with_fc=bool(self.desc.fc_trainable))
        gy = torch.empty((B, self.M), dtype=torch.float32, device=gxhat.device) if want_gy else None
        _lib.dsi_backward(self.ctx.h, self.h, _ptr(_f32(gxhat.contiguous(), "gxhat")), _ptr(saved),
                          saved.numel(), int(recompute), B, g.grads_to_c(), _ptr(gy), _stream(self.ctx.device))
        return g, gy

    def loss_grad(self, y, x, params_like: NetParams, want_gy=False):
        torch = _torch()
        B = y.shape[0]
        g = NetParams.grads_like(params_like, with_fc=bool(self.desc.fc_trainable))
        gy = torch.empty((B, self.M), dtype=torch.float32, device=y.device) if want_gy else None
        loss = torch.empty((), dtype=torch.float64, device=y.device)
        _lib.dsi_loss_grad(self.ctx.h, self.h, _ptr(_f32(y, "y")), _ptr(_f32(x, "x")), B, g.grads_to_c(),
                           _ptr(gy), _ptr(loss), _stream(self.ctx.device))
        return loss, g, gy

    def train_step(self, params: NetParams, opt: AdamState, y, x, lr=1e-3):
        torch = _torch()
        B = y.shape[0]
        loss = torch.empty((), dtype=torch.float64, device=y.device)
        _lib.dsi_train_step(self.ctx.h, self.h, params.to_c(), opt.c, _ptr(_f32(y, "y")), _ptr(_f32(x, "x")),
                            B, float(lr), _ptr(loss), _stream(self.ctx.device))
        return loss
