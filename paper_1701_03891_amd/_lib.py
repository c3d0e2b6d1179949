"""ctypes binding of libdsi (include/dsi.h): argument marshalling only.

Every function here has the C name and forwards to the library; no step of
the recovery path runs in Python.  Loading fails loudly when libdsi.so is
missing: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libdsi.so")

MAX_LAYERS = 8

# dsi_status
DSI_OK, DSI_E_NULL, DSI_E_SHAPE, DSI_E_DTYPE, DSI_E_ALIGN, DSI_E_NOMEM, DSI_E_HIP, DSI_E_STATE = range(8)
STATUS_NAMES = ["DSI_OK", "DSI_E_NULL", "DSI_E_SHAPE", "DSI_E_DTYPE", "DSI_E_ALIGN", "DSI_E_NOMEM",
                "DSI_E_HIP", "DSI_E_STATE"]
# dsi_prec
DSI_F32, DSI_BF16, DSI_FP8_E4M3, DSI_F64 = 0, 1, 2, 3
PREC = {"f32": DSI_F32, "fp32": DSI_F32, "bf16": DSI_BF16, "fp8": DSI_FP8_E4M3, "f64": DSI_F64,
        "fp64": DSI_F64}

EXPORTS = ["dsi_create", "dsi_destroy", "dsi_last_error", "dsi_version", "dsi_measure",
           "dsi_net_prepare", "dsi_net_update", "dsi_net_set_act_scales", "dsi_net_free",
           "dsi_net_info", "dsi_workspace_size", "dsi_reserve", "dsi_recover",
           "dsi_forward_train", "dsi_backward", "dsi_loss_grad", "dsi_train_step", "dsi_metrics",
           "dsi_set_stage_timing", "dsi_stage_times", "dsi_saved_activation", "dsi_net_calibrate",
           "dsi_net_get_scales", "dsi_measure_noisy", "dsi_recover_noalloc",
           "dsi_set_recompute_budget", "dsi_set_workspace", "dsi_stage_times_each",
           "dsi_set_stage_timing_mask"]

NOALLOC_SCRATCH_BYTES = 64 << 20     # DSI_NOALLOC_SCRATCH_BYTES


class DsiError(RuntimeError):
    def __init__(self, status: int, fn: str, msg: str):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{fn} -> {name}: {msg}")


class NetDesc(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int), ("n2", ctypes.c_int), ("M", ctypes.c_int), ("L", ctypes.c_int),
                ("C", ctypes.c_int * (MAX_LAYERS + 1)), ("k", ctypes.c_int * MAX_LAYERS),
                ("bias_per_pixel", ctypes.c_int), ("relu_last", ctypes.c_int),
                ("fc_trainable", ctypes.c_int)]


class Params(ctypes.Structure):
    _fields_ = [("w_fc", ctypes.c_void_p), ("w", ctypes.c_void_p * MAX_LAYERS),
                ("b", ctypes.c_void_p * MAX_LAYERS)]


class Adam(ctypes.Structure):
    _fields_ = [("m_w", ctypes.c_void_p * MAX_LAYERS), ("v_w", ctypes.c_void_p * MAX_LAYERS),
                ("m_b", ctypes.c_void_p * MAX_LAYERS), ("v_b", ctypes.c_void_p * MAX_LAYERS),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("step", ctypes.c_long), ("m_fc", ctypes.c_void_p), ("v_fc", ctypes.c_void_p)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libdsi.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO_PATH):
        raise RuntimeError(f"libdsi.so not found at {SO_PATH}: build it with "
                           "`python -m paper_1701_03891_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(SO_PATH)
    P, i, z = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    st = ctypes.c_int
    sig = {
        "dsi_create": (st, [ctypes.POINTER(P), i]),
        "dsi_destroy": (st, [P]),
        "dsi_last_error": (ctypes.c_char_p, []),
        "dsi_version": (ctypes.c_char_p, []),
        "dsi_measure": (st, [P, P, P, P, i, i, i, P]),
        "dsi_measure_noisy": (st, [P, P, P, P, ctypes.c_double, P, i, i, i, P]),
        "dsi_net_prepare": (st, [P, ctypes.POINTER(NetDesc), ctypes.POINTER(Params), i, ctypes.POINTER(P), P]),
        "dsi_net_update": (st, [P, P, ctypes.POINTER(Params), P]),
        "dsi_net_set_act_scales": (st, [P, ctypes.POINTER(ctypes.c_float), i]),
        "dsi_net_free": (st, [P, P]),
        "dsi_net_info": (st, [P, ctypes.POINTER(NetDesc), ctypes.POINTER(ctypes.c_int)]),
        "dsi_workspace_size": (st, [P, i, i, ctypes.POINTER(z)]),
        "dsi_reserve": (st, [P, P, i, i]),
        "dsi_recover": (st, [P, P, P, P, i, P]),
        "dsi_recover_noalloc": (st, [P, P, P, P, i, P]),
        "dsi_forward_train": (st, [P, P, P, P, i, P, z, i, P]),
        "dsi_backward": (st, [P, P, P, P, z, i, i, ctypes.POINTER(Params), P, P]),
        "dsi_set_recompute_budget": (st, [P, z]),
        "dsi_set_workspace": (st, [P, P, z]),
        "dsi_loss_grad": (st, [P, P, P, P, i, ctypes.POINTER(Params), P, P, P]),
        "dsi_train_step": (st, [P, P, ctypes.POINTER(Params), ctypes.POINTER(Adam), P, P, i,
                                ctypes.c_float, P, P]),
        "dsi_metrics": (st, [P, P, P, i, i, P, P]),
        "dsi_set_stage_timing": (st, [P, i]),
        "dsi_saved_activation": (st, [P, P, P, z, i, i, P, P]),
        "dsi_net_calibrate": (st, [P, P, P, i, P]),
        "dsi_net_get_scales": (st, [P, ctypes.POINTER(ctypes.c_float), i]),
        "dsi_stage_times": (st, [P, ctypes.POINTER(ctypes.c_double), i, ctypes.POINTER(ctypes.c_int)]),
        "dsi_stage_times_each": (st, [P, ctypes.POINTER(ctypes.c_double), i, i, ctypes.POINTER(ctypes.c_int)]),
        "dsi_set_stage_timing_mask": (st, [P, ctypes.c_uint]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(status: int, fn: str) -> None:
    if status != DSI_OK:
        raise DsiError(status, fn, lib().dsi_last_error().decode())


def call(name: str, *args) -> None:
    """Call dsi_<name>(*args) and raise DsiError on a non-OK status."""
    check(getattr(lib(), name)(*args), name)


# Same-name wrappers (raise on error).
def dsi_create(device: int = 0) -> int:
    h = ctypes.c_void_p()
    call("dsi_create", ctypes.byref(h), device)
    return h.value


def dsi_destroy(ctx):
    call("dsi_destroy", ctx)


def dsi_last_error() -> str:
    return lib().dsi_last_error().decode()


def dsi_version() -> str:
    return lib().dsi_version().decode()


def dsi_measure(ctx, phi, x, y, B, M, N, stream):
    call("dsi_measure", ctx, phi, x, y, B, M, N, stream)


def dsi_net_prepare(ctx, desc: NetDesc, params: Params, prec: int, stream) -> int:
    h = ctypes.c_void_p()
    call("dsi_net_prepare", ctx, ctypes.byref(desc), ctypes.byref(params), prec, ctypes.byref(h), stream)
    return h.value


def dsi_net_update(ctx, net, params: Params, stream):
    call("dsi_net_update", ctx, net, ctypes.byref(params), stream)


def dsi_net_set_act_scales(net, scales):
    arr = (ctypes.c_float * len(scales))(*scales)
    call("dsi_net_set_act_scales", net, arr, len(scales))


def dsi_net_free(ctx, net):
    call("dsi_net_free", ctx, net)


def dsi_workspace_size(net, B, train) -> int:
    z = ctypes.c_size_t()
    call("dsi_workspace_size", net, B, int(train), ctypes.byref(z))
    return z.value


def dsi_reserve(ctx, net, B, train):
    call("dsi_reserve", ctx, net, B, int(train))


def dsi_recover(ctx, net, y, xhat, B, stream):
    call("dsi_recover", ctx, net, y, xhat, B, stream)


def dsi_recover_noalloc(ctx, net, y, xhat, B, stream):
    call("dsi_recover_noalloc", ctx, net, y, xhat, B, stream)


def dsi_forward_train(ctx, net, y, xhat, B, saved, saved_bytes, recompute, stream):
    call("dsi_forward_train", ctx, net, y, xhat, B, saved, saved_bytes, int(recompute), stream)


def dsi_backward(ctx, net, gxhat, saved, saved_bytes, recompute, B, grads: Params, gy, stream):
    call("dsi_backward", ctx, net, gxhat, saved, saved_bytes, int(recompute), B, ctypes.byref(grads), gy, stream)


def dsi_set_workspace(ctx, ws, nbytes):
    call("dsi_set_workspace", ctx, ws, int(nbytes))


def dsi_set_recompute_budget(ctx, nbytes):
    call("dsi_set_recompute_budget", ctx, int(nbytes))


def dsi_loss_grad(ctx, net, y, x, B, grads: Params, gy, loss_dev, stream):
    call("dsi_loss_grad", ctx, net, y, x, B, ctypes.byref(grads), gy, loss_dev, stream)


def dsi_train_step(ctx, net, params: Params, opt: Adam, y, x, B, lr, loss_dev, stream):
    call("dsi_train_step", ctx, net, ctypes.byref(params), ctypes.byref(opt), y, x, B, lr, loss_dev, stream)


def dsi_metrics(ctx, xhat, x, B, N, out, stream):
    call("dsi_metrics", ctx, xhat, x, B, N, out, stream)


def dsi_set_stage_timing(ctx, enable):
    call("dsi_set_stage_timing", ctx, int(enable))


def dsi_stage_times(ctx, nstages=4):
    arr = (ctypes.c_double * nstages)()
    n = ctypes.c_int()
    call("dsi_stage_times", ctx, arr, nstages, ctypes.byref(n))
    return list(arr), n.value


def dsi_set_stage_timing_mask(ctx, stages):
    call("dsi_set_stage_timing_mask", ctx, int(stages))


def dsi_stage_times_each(ctx, nstages, max_passes):
    """(rows, calls): rows[p] = the p-th timed pass's nstages stage times followed by the time
    from its first event to the next pass's first event."""
    w = nstages + 1
    arr = (ctypes.c_double * (w * max_passes))()
    n = ctypes.c_int()
    call("dsi_stage_times_each", ctx, arr, nstages, max_passes, ctypes.byref(n))
    return [list(arr[p * w:(p + 1) * w]) for p in range(min(n.value, max_passes))], n.value


def dsi_saved_activation(ctx, net, saved, saved_bytes, B, layer, out, stream):
    call("dsi_saved_activation", ctx, net, saved, saved_bytes, B, layer, out, stream)


def dsi_net_calibrate(ctx, net, y, B, stream):
    call("dsi_net_calibrate", ctx, net, y, B, stream)


def dsi_net_get_scales(net, n=6):
    arr = (ctypes.c_float * n)()
    call("dsi_net_get_scales", net, arr, n)
    return list(arr)


def dsi_measure_noisy(ctx, phi, x, e, snr_db, y, B, M, N, stream):
    call("dsi_measure_noisy", ctx, phi, x, e, float(snr_db), y, B, M, N, stream)
