"""torch.autograd over the library's training calls.

Sec. 4 learns Omega by minimising L(Omega) = (1/l) sum_i ||M(y_i, Omega) - x_i||^2
with backpropagation.  DeepInverseFn puts the network's forward pass
(dsi_forward_train) and its hand-written backward kernels (dsi_backward) under
torch's autograd, so any loss written in torch differentiates through them;
DeepInverse is an nn.Module that owns the FP32 master parameters and keeps the
library's packed copy in step with them.

Recompute: dsi_forward_train can keep only the proxy and the output and let
dsi_backward recompute the hidden activations (chunk by chunk when the
context has a recompute budget).  DeepInverse selects it when the state that
keeps every activation would exceed `saved_budget_bytes` (by default a quarter
of the device memory free at the call), or as forced by `recompute`.
"""
from __future__ import annotations

import torch

from . import PAPER_C, PAPER_K, Context, NetParams


class _Handle:
    """What the autograd function needs besides tensors: the prepared network, the
    parameter layout its gradients come back in, and the recompute flag."""

    def __init__(self, net, params_like: NetParams, recompute: bool):
        self.net, self.params_like, self.recompute = net, params_like, recompute


class DeepInverseFn(torch.autograd.Function):
    """xhat = M(y, Omega) with gradients from the library's backward kernels.

    apply(y, handle, w_fc, w[0], b[0], ..., w[L-1], b[L-1]); the parameter tensors
    are passed so autograd routes their gradients; their values are the ones the
    network was last packed from (DeepInverse re-packs after they change)."""

    @staticmethod
    def forward(ctx, y, handle: _Handle, *params):
        xhat, saved = handle.net.forward_train(y.contiguous(), recompute=handle.recompute)
        ctx.handle, ctx.state = handle, saved
        return xhat

    @staticmethod
    def backward(ctx, gxhat):
        h = ctx.handle
        want_gy = bool(ctx.needs_input_grad[0])
        g, gy = h.net.backward(gxhat.contiguous(), ctx.state, h.params_like, want_gy=want_gy,
                               recompute=h.recompute)
        ctx.state = None
        out = [gy, None, g.w_fc if ctx.needs_input_grad[2] else None]
        for l in range(len(g.w)):
            out.append(g.w[l] if ctx.needs_input_grad[3 + 2 * l] else None)
            out.append(g.b[l] if ctx.needs_input_grad[4 + 2 * l] else None)
        return tuple(out)


class DeepInverse(torch.nn.Module):
    """The recovery network of Sec. 4 as a module: FC layer W_fc [N][M] (fixed at
    Phi^T unless fc_trainable), conv weights w[l] [Cout][Cin][k][k] and biases b[l]
    ([Cout][n1][n2] per pixel, or [Cout]), FP32 master parameters on the device;
    arithmetic in `prec` (f32, bf16, f64 for training; fp8 recovers only)."""

    def __init__(self, n1, n2, M, w_fc, w, b, prec="bf16", C=PAPER_C, k=PAPER_K, bias_per_pixel=True,
                 relu_last=False, fc_trainable=False, device=0, context: Context | None = None,
                 recompute: bool | None = None, saved_budget_bytes: int | None = None):
        super().__init__()
        dev = torch.device("cuda", device)
        p = lambda t, rg=True: torch.nn.Parameter(torch.as_tensor(t, dtype=torch.float32, device=dev).contiguous(),  # noqa: E731
                                                   requires_grad=rg)
        self.w_fc = p(w_fc, bool(fc_trainable))
        self.w = torch.nn.ParameterList([p(t) for t in w])
        self.b = torch.nn.ParameterList([p(t) for t in b])
        self.ctx = context if context is not None else Context(device)
        self._own_ctx = context is None
        self.n1, self.n2, self.M = n1, n2, M
        self.net = self.ctx.prepare(n1, n2, M, self._params(), prec=prec, C=C, k=k,
                                    bias_per_pixel=bias_per_pixel, relu_last=relu_last,
                                    fc_trainable=fc_trainable)
        self._versions = self._param_versions()
        self.recompute = recompute
        self.saved_budget_bytes = saved_budget_bytes
        self.last_recompute: bool | None = None

    def _params(self) -> NetParams:
        return NetParams(self.w_fc.data, [t.data for t in self.w], [t.data for t in self.b])

    def _param_versions(self):
        return tuple(t._version for t in [self.w_fc, *self.w, *self.b])

    def sync(self):
        """Re-pack the network if any master parameter changed since the last packing."""
        v = self._param_versions()
        if v != self._versions:
            self.net.update(self._params())
            self._versions = v

    def _use_recompute(self, B) -> bool:
        if self.recompute is not None:
            return bool(self.recompute)
        budget = self.saved_budget_bytes
        if budget is None:
            budget = torch.cuda.mem_get_info(self.w_fc.device)[0] // 4
        return self.net.saved_bytes(B, recompute=False) > budget

    def forward(self, y):
        self.sync()
        params = [self.w_fc, *[t for pair in zip(self.w, self.b) for t in pair]]
        if not torch.is_grad_enabled() or not (y.requires_grad or any(t.requires_grad for t in params)):
            return self.net.recover(y.contiguous())
        rc = self._use_recompute(y.shape[0])
        self.last_recompute = rc
        return DeepInverseFn.apply(y, _Handle(self.net, self._params(), rc), *params)

    def close(self):
        if self.net is not None:
            self.net.free()
            self.net = None
        if self._own_ctx and self.ctx is not None:
            self.ctx.close()
            self.ctx = None
