"""Python binding of the warm-start network C ABI (include/ot_net.h).

Same rules as otdyn: the functions carry the C names and marshal arguments
only; the network's forward pass, gradients and optimiser run in the HIP
kernels of libotdyn.so.  Device pointers are torch CUDA tensors or integers.
"""
from __future__ import annotations

import ctypes
from ctypes import POINTER, byref, c_char_p, c_double, c_float, c_int, c_size_t, c_void_p

from . import otdyn
from .otdyn import OtDynError, _ptr, ot_dyn_desc


class ot_net_desc(ctypes.Structure):
    _fields_ = [
        ("H", c_int), ("W", c_int), ("in_ch", c_int), ("out_ch", c_int),
        ("base", c_int), ("levels", c_int), ("max_batch", c_int),
        ("beta1", c_double), ("beta2", c_double), ("eps", c_double),
    ]


EXPORTS = [
    "ot_net_default_desc", "ot_net_param_count", "ot_net_workspace_size", "ot_net_create",
    "ot_net_set_params", "ot_net_get_params", "ot_net_forward", "ot_net_grad",
    "ot_net_train_step", "ot_net_destroy", "ot_net_last_error",
    "ot_warm_inputs", "ot_warm_targets", "ot_warm_state", "ot_warm_restrict",
    "ot_warm_prolong",
]

_done = False


def lib() -> ctypes.CDLL:
    global _done
    L = otdyn.lib()
    if _done:
        return L
    P = c_void_p
    LL = ctypes.c_longlong
    D = POINTER(ot_net_desc)
    L.ot_net_default_desc.argtypes = [c_int, c_int, c_int, c_int, c_int, D]
    L.ot_net_param_count.argtypes = [D, POINTER(LL)]
    L.ot_net_workspace_size.argtypes = [D, POINTER(c_size_t)]
    L.ot_net_create.argtypes = [D, P, P, c_size_t, POINTER(c_void_p)]
    L.ot_net_set_params.argtypes = [P, P]
    L.ot_net_get_params.argtypes = [P, P]
    L.ot_net_forward.argtypes = [P, c_int, P, P]
    L.ot_net_grad.argtypes = [P, c_int, P, P, P, P, POINTER(c_double)]
    L.ot_net_train_step.argtypes = [P, c_int, P, P, P, c_float, POINTER(c_double)]
    L.ot_net_destroy.argtypes = [P]
    L.ot_net_last_error.argtypes = [P]
    L.ot_net_last_error.restype = c_char_p
    DD = POINTER(ot_dyn_desc)
    L.ot_warm_inputs.argtypes = [DD, c_int, P, P, P, P, P]
    L.ot_warm_targets.argtypes = [DD, c_int, P, P, P, LL, P, P, P, LL, P, P, P]
    L.ot_warm_state.argtypes = [DD, c_int, P, P, P, P, P, LL, P, P, P, LL, P]
    L.ot_warm_restrict.argtypes = [DD, c_int, P, P, P]
    L.ot_warm_prolong.argtypes = [DD, DD, c_int, P, LL, P, P, P, LL, P, LL, P, P, P, LL, P]
    for name in EXPORTS:
        if name != "ot_net_last_error":
            getattr(L, name).restype = c_int
    _done = True
    return L


def _check(status: int, net=None) -> int:
    if status < 0:
        msg = otdyn.lib().ot_dyn_status_str(status).decode()
        if net:
            detail = lib().ot_net_last_error(net).decode()
            if detail:
                msg += f" ({detail})"
        raise OtDynError(status, msg)
    return status


def ot_net_default_desc(H, W, in_ch, out_ch, max_batch) -> ot_net_desc:
    d = ot_net_desc()
    _check(lib().ot_net_default_desc(H, W, in_ch, out_ch, max_batch, byref(d)))
    return d


def ot_net_param_count(d: ot_net_desc) -> int:
    n = ctypes.c_longlong()
    _check(lib().ot_net_param_count(byref(d), byref(n)))
    return n.value


def ot_net_workspace_size(d: ot_net_desc) -> int:
    n = c_size_t()
    _check(lib().ot_net_workspace_size(byref(d), byref(n)))
    return n.value


def ot_net_create(d: ot_net_desc, stream, ws, ws_bytes: int) -> int:
    out = c_void_p()
    _check(lib().ot_net_create(byref(d), c_void_p(stream), _ptr(ws), ws_bytes, byref(out)))
    return out.value


def ot_net_set_params(net, params) -> int:
    return _check(lib().ot_net_set_params(net, _ptr(params)), net)


def ot_net_get_params(net, params) -> int:
    return _check(lib().ot_net_get_params(net, _ptr(params)), net)


def ot_net_forward(net, batch, x, y) -> int:
    return _check(lib().ot_net_forward(net, batch, _ptr(x), _ptr(y)), net)


def ot_net_grad(net, batch, x, t, cw, grad=None, want_loss=True):
    loss = c_double()
    _check(lib().ot_net_grad(net, batch, _ptr(x), _ptr(t), _ptr(cw),
                             _ptr(grad) if grad is not None else None,
                             byref(loss) if want_loss else None), net)
    return loss.value if want_loss else None


def ot_net_train_step(net, batch, x, t, cw, lr: float, want_loss=True):
    loss = c_double()
    _check(lib().ot_net_train_step(net, batch, _ptr(x), _ptr(t), _ptr(cw), lr,
                                   byref(loss) if want_loss else None), net)
    return loss.value if want_loss else None


def ot_net_destroy(net) -> int:
    return _check(lib().ot_net_destroy(net))


def ot_warm_inputs(d: ot_dyn_desc, batch, f0, f1, base, x, stream) -> int:
    return _check(lib().ot_warm_inputs(byref(d), batch, _ptr(f0), _ptr(f1), _ptr(base), _ptr(x),
                                       c_void_p(stream)))


def ot_warm_targets(d: ot_dyn_desc, batch, f0, f1, F, sF, Mx, My, Mc, sM, base, t,
                    stream) -> int:
    return _check(lib().ot_warm_targets(byref(d), batch, _ptr(f0), _ptr(f1), _ptr(F), sF,
                                        _ptr(Mx), _ptr(My), _ptr(Mc), sM, _ptr(base), _ptr(t),
                                        c_void_p(stream)))


def ot_warm_state(d: ot_dyn_desc, batch, f0, f1, y, base, F, sF, Mx, My, Mc, sM, stream) -> int:
    return _check(lib().ot_warm_state(byref(d), batch, _ptr(f0), _ptr(f1), _ptr(y), _ptr(base),
                                      _ptr(F), sF, _ptr(Mx), _ptr(My), _ptr(Mc), sM,
                                      c_void_p(stream)))


def ot_warm_restrict(d: ot_dyn_desc, batch, f, fc, stream) -> int:
    return _check(lib().ot_warm_restrict(byref(d), batch, _ptr(f), _ptr(fc), c_void_p(stream)))


def ot_warm_prolong(dc: ot_dyn_desc, df: ot_dyn_desc, batch, Fc, sFc, Mxc, Myc, Mcc, sMc,
                    F, sF, Mx, My, Mc, sM, stream) -> int:
    return _check(lib().ot_warm_prolong(byref(dc), byref(df), batch, _ptr(Fc), sFc, _ptr(Mxc),
                                        _ptr(Myc), _ptr(Mcc), sMc, _ptr(F), sF, _ptr(Mx),
                                        _ptr(My), _ptr(Mc), sM, c_void_p(stream)))


def warm_channels(C: int, P: int) -> int:
    """Output channels of the warm-start network for C colours, P steps."""
    return C * (P - 1) + 3 * C * P


class Net:
    """Owns the workspace of one network (torch for device memory only)."""

    def __init__(self, desc: ot_net_desc, device="cuda"):
        import torch
        self.desc = desc
        self.device = torch.device(device)
        self.nparams = ot_net_param_count(desc)
        self.ws_bytes = ot_net_workspace_size(desc)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        self.ws_ptr = (self.ws.data_ptr() + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        self.net = ot_net_create(desc, self.stream.cuda_stream, self.ws_ptr, self.ws_bytes)

    def set_params(self, flat):
        import torch
        flat = torch.as_tensor(flat, dtype=torch.float32).to(self.device).contiguous()
        assert flat.numel() == self.nparams
        self._p = flat
        ot_net_set_params(self.net, flat)

    def get_params(self):
        import torch
        out = torch.empty(self.nparams, dtype=torch.float32, device=self.device)
        ot_net_get_params(self.net, out)
        return out

    def forward(self, x, batch=None):
        import torch
        nb = x.shape[0] if batch is None else batch
        d = self.desc
        y = torch.empty((nb, d.H, d.W, d.out_ch), dtype=torch.float32, device=self.device)
        ot_net_forward(self.net, nb, x, y)
        return y

    def grad(self, x, t, cw):
        import torch
        g = torch.empty(self.nparams, dtype=torch.float32, device=self.device)
        loss = ot_net_grad(self.net, x.shape[0], x, t, cw, g)
        return loss, g

    def train_step(self, x, t, cw, lr, want_loss=True):
        return ot_net_train_step(self.net, x.shape[0], x, t, cw, lr, want_loss)

    def close(self):
        if getattr(self, "net", None):
            ot_net_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
