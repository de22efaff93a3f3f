"""Python binding of the ot_dyn C ABI (include/ot_dyn.h).

The functions below carry the C names and only marshal arguments: every step
of the solver runs in the HIP kernels of libotdyn.so.  Device pointers may be
given as torch CUDA tensors (their data_ptr is passed) or as integers.
PyTorch is used for device memory and streams only.

There is no CPU fallback: importing works without a GPU, but any call needs
the built library and raises if it is missing.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
# OT_DYN_LIB selects another build of the library (the host-sanitized one
# of build.py); by default the in-tree libotdyn.so
LIB_PATH = os.environ.get("OT_DYN_LIB") or os.path.join(HERE, "libotdyn.so")

OT_OK = 0
OT_NOT_CONVERGED = 1
OT_ERR_PARAM = -1
OT_ERR_SHAPE = -2
OT_ERR_INPUT = -3
OT_ERR_MASS = -4
OT_ERR_HIP = -5
OT_ERR_NONFINITE = -6
OT_ERR_STATE = -7

OT_BC_NEUMANN = 0
OT_BC_PERIODIC = 1

OT_PHASE_DIV = 0
OT_PHASE_XFORM_X = 1
OT_PHASE_XFORM_Y = 2
OT_PHASE_TC = 3
OT_PHASE_REFINE = 4
OT_PHASE_UPDATE = 5
OT_PHASE_COUNT = 6
PHASE_NAMES = ["div", "xform_x", "xform_y", "tc", "refine", "update"]

OT_INIT_COLD = 0
OT_INIT_PRIMAL = 1
OT_INIT_PRIMAL_DUAL = 2
OT_INIT_FALLBACK = 4

OT_REFINE_OFF = 0
OT_REFINE_ALWAYS = 1
OT_REFINE_ADAPTIVE = 2
OT_REFINE_CARRY = 3

OT_PROX_NEWTON = 0
OT_PROX_CLOSED = 1
OT_PROX_CLOSED_RAW = 2


class ot_dyn_desc(ctypes.Structure):
    _fields_ = [
        ("X", c_int), ("Y", c_int), ("C", c_int), ("P", c_int),
        ("bc", c_int * 3),
        ("extent", c_double * 3),
        ("tau", c_double), ("sigma", c_double), ("theta", c_double),
        ("check_every", c_int),
        ("tol_res", c_double), ("tol_div", c_double), ("tol_mass", c_double),
        ("refine", c_int),
        ("batch", c_int),
        ("adapt", c_int),
        ("prox", c_int),
        ("carry_refine", c_int),
    ]


class ot_dyn_report(ctypes.Structure):
    _fields_ = [
        ("iterations", c_int), ("converged", c_int), ("total_iterations", c_int),
        ("worst_problem", c_int),
        ("r_prim", c_double), ("r_dual", c_double), ("r_div", c_double),
        ("cost", c_double), ("e_mass", c_double),
        ("mass0", c_double), ("mass1", c_double), ("ms", c_double),
        ("fallback", c_int),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class OtDynError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ot_dyn status {status}: {msg}")
        self.status = status


_lib = None

EXPORTS = [
    "ot_dyn_default_desc", "ot_dyn_workspace_size", "ot_dyn_create",
    "ot_dyn_set_boundary", "ot_dyn_init", "ot_dyn_step", "ot_dyn_solve",
    "ot_dyn_residuals", "ot_dyn_destroy", "ot_dyn_status_str", "ot_dyn_last_error",
    "ot_dyn_profile", "ot_dyn_profile_read", "ot_dyn_get_dual", "ot_dyn_set_dual",
    "ot_dyn_get_dual_bar",
    "ot_dyn_batch_workspace_size", "ot_dyn_batch_create", "ot_dyn_batch_offsets",
    "ot_dyn_batch_set_boundary", "ot_dyn_batch_autotune", "ot_dyn_batch_solve",
    "ot_dyn_batch_problem", "ot_dyn_batch_get_state", "ot_dyn_batch_set_state",
    "ot_dyn_batch_get_dual", "ot_dyn_batch_set_dual",
    "ot_dyn_batch_tuning", "ot_dyn_batch_destroy", "ot_dyn_batch_last_error",
    "ot_dyn_prox_eval", "ot_dyn_solve_static",
]


def lib() -> ctypes.CDLL:
    """Load libotdyn.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
            "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    L.ot_dyn_default_desc.argtypes = [POINTER(ot_dyn_desc), c_int, c_int, c_int, c_int]
    L.ot_dyn_workspace_size.argtypes = [POINTER(ot_dyn_desc), POINTER(c_size_t)]
    L.ot_dyn_create.argtypes = [POINTER(ot_dyn_desc), P, P, c_size_t, POINTER(c_void_p)]
    L.ot_dyn_set_boundary.argtypes = [P, P, P]
    L.ot_dyn_init.argtypes = [P, c_int, P, P, P, P]
    L.ot_dyn_step.argtypes = [P, P, P, P, P, c_int]
    L.ot_dyn_solve.argtypes = [P, P, P, P, P, c_int, POINTER(ot_dyn_report)]
    L.ot_dyn_residuals.argtypes = [P, P, P, P, P, POINTER(ot_dyn_report)]
    L.ot_dyn_destroy.argtypes = [P]
    L.ot_dyn_profile.argtypes = [P, c_int]
    L.ot_dyn_profile_read.argtypes = [P, POINTER(c_double), POINTER(ctypes.c_longlong), c_int]
    LL = ctypes.c_longlong
    L.ot_dyn_batch_workspace_size.argtypes = [POINTER(ot_dyn_desc), c_int, POINTER(c_int),
                                              POINTER(c_size_t)]
    L.ot_dyn_batch_create.argtypes = [POINTER(ot_dyn_desc), c_int, POINTER(c_int), P, P,
                                      c_size_t, POINTER(c_void_p)]
    L.ot_dyn_batch_offsets.argtypes = [P, POINTER(LL), POINTER(LL), POINTER(LL)]
    L.ot_dyn_batch_set_boundary.argtypes = [P, P, P]
    L.ot_dyn_batch_autotune.argtypes = [P, c_int]
    L.ot_dyn_batch_solve.argtypes = [P, c_int, c_int, POINTER(ot_dyn_report)]
    L.ot_dyn_batch_problem.argtypes = [P, c_int, POINTER(ot_dyn_report)]
    L.ot_dyn_batch_get_state.argtypes = [P, P, P]
    L.ot_dyn_batch_set_state.argtypes = [P, P, P, c_int]
    L.ot_dyn_batch_get_dual.argtypes = [P, P]
    L.ot_dyn_batch_set_dual.argtypes = [P, P]
    L.ot_dyn_get_dual.argtypes = [P, P]
    L.ot_dyn_set_dual.argtypes = [P, P]
    L.ot_dyn_get_dual_bar.argtypes = [P, P]
    L.ot_dyn_batch_tuning.argtypes = [P, c_int, POINTER(c_int), POINTER(c_int)]
    L.ot_dyn_batch_destroy.argtypes = [P]
    L.ot_dyn_batch_last_error.argtypes = [P]
    L.ot_dyn_batch_last_error.restype = c_char_p
    L.ot_dyn_prox_eval.argtypes = [c_int, LL, P, P, ctypes.c_float, P, P, P]
    L.ot_dyn_solve_static.argtypes = [POINTER(ot_dyn_desc), P, P, P, P, P, P, P, c_int,
                                      POINTER(ot_dyn_report)]
    L.ot_dyn_status_str.argtypes = [c_int]
    L.ot_dyn_status_str.restype = c_char_p
    L.ot_dyn_last_error.argtypes = [P]
    L.ot_dyn_last_error.restype = c_char_p
    for name in EXPORTS:
        if name not in ("ot_dyn_status_str", "ot_dyn_last_error", "ot_dyn_batch_last_error"):
            getattr(L, name).restype = c_int
    _lib = L
    return L


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def _check(status: int, plan=None) -> int:
    if status < 0:
        L = lib()
        msg = L.ot_dyn_status_str(status).decode()
        if plan:
            extra = L.ot_dyn_last_error(plan).decode()
            if extra:
                msg += f" ({extra})"
        raise OtDynError(status, msg)
    return status


# ---- the C entry points ---------------------------------------------------

def ot_dyn_default_desc(X: int, Y: int, C: int, P: int) -> ot_dyn_desc:
    d = ot_dyn_desc()
    _check(lib().ot_dyn_default_desc(byref(d), X, Y, C, P))
    return d


def ot_dyn_workspace_size(d: ot_dyn_desc) -> int:
    n = c_size_t(0)
    _check(lib().ot_dyn_workspace_size(byref(d), byref(n)))
    return int(n.value)


def ot_dyn_create(d: ot_dyn_desc, stream, workspace, ws_bytes: int) -> int:
    out = c_void_p(0)
    _check(lib().ot_dyn_create(byref(d), _ptr(stream), _ptr(workspace), ws_bytes, byref(out)))
    return out.value


def ot_dyn_set_boundary(plan: int, f0, f1) -> int:
    return _check(lib().ot_dyn_set_boundary(plan, _ptr(f0), _ptr(f1)), plan)


def ot_dyn_init(plan: int, mode: int, F, Mx, My, Mc) -> int:
    return _check(lib().ot_dyn_init(plan, mode, _ptr(F), _ptr(Mx), _ptr(My), _ptr(Mc)), plan)


def ot_dyn_step(plan: int, F, Mx, My, Mc, iters: int) -> int:
    return _check(lib().ot_dyn_step(plan, _ptr(F), _ptr(Mx), _ptr(My), _ptr(Mc), iters), plan)


def ot_dyn_solve(plan: int, F, Mx, My, Mc, max_iters: int):
    rep = ot_dyn_report()
    st = _check(lib().ot_dyn_solve(plan, _ptr(F), _ptr(Mx), _ptr(My), _ptr(Mc), max_iters,
                                   byref(rep)), plan)
    return st, rep


def ot_dyn_residuals(plan: int, F, Mx, My, Mc):
    rep = ot_dyn_report()
    st = _check(lib().ot_dyn_residuals(plan, _ptr(F), _ptr(Mx), _ptr(My), _ptr(Mc),
                                       byref(rep)), plan)
    return st, rep


def ot_dyn_get_dual(plan: int, b) -> int:
    """Copy the dual b of the plan into b [batch][4][P][C][Y][X] (device)."""
    return _check(lib().ot_dyn_get_dual(plan, _ptr(b)), plan)


def ot_dyn_set_dual(plan: int, b) -> int:
    """Set the dual b (and b_bar = b) from b [batch][4][P][C][Y][X] (device)."""
    return _check(lib().ot_dyn_set_dual(plan, _ptr(b)), plan)


def ot_dyn_get_dual_bar(plan: int, b_bar) -> int:
    """Copy the extrapolated dual b_bar into b_bar [batch][4][P][C][Y][X] (device)."""
    return _check(lib().ot_dyn_get_dual_bar(plan, _ptr(b_bar)), plan)


def ot_dyn_profile(plan: int, mask: int) -> int:
    return _check(lib().ot_dyn_profile(plan, mask), plan)


def ot_dyn_profile_read(plan: int):
    """{phase name: (milliseconds, launches)} accumulated since ot_dyn_profile."""
    ms = (c_double * OT_PHASE_COUNT)()
    n = (ctypes.c_longlong * OT_PHASE_COUNT)()
    _check(lib().ot_dyn_profile_read(plan, ms, n, OT_PHASE_COUNT), plan)
    return {PHASE_NAMES[i]: (ms[i], n[i]) for i in range(OT_PHASE_COUNT)}


def ot_dyn_destroy(plan: int) -> int:
    return _check(lib().ot_dyn_destroy(plan))


def _checkb(status: int, bt) -> int:
    if status < 0:
        L = lib()
        msg = L.ot_dyn_status_str(status).decode()
        extra = L.ot_dyn_batch_last_error(bt).decode() if bt else ""
        raise OtDynError(status, msg + (f" ({extra})" if extra else ""))
    return status


def ot_dyn_batch_last_error(bt: int) -> str:
    return lib().ot_dyn_batch_last_error(bt).decode()


def _dims_array(dims):
    flat = [int(v) for d in dims for v in d]
    return (c_int * len(flat))(*flat), len(dims)


def ot_dyn_batch_workspace_size(base: ot_dyn_desc, dims) -> int:
    arr, n = _dims_array(dims)
    out = c_size_t(0)
    _check(lib().ot_dyn_batch_workspace_size(byref(base), n, arr, byref(out)))
    return int(out.value)


def ot_dyn_batch_create(base: ot_dyn_desc, dims, stream, workspace, ws_bytes: int) -> int:
    arr, n = _dims_array(dims)
    out = c_void_p(0)
    _check(lib().ot_dyn_batch_create(byref(base), n, arr, _ptr(stream), _ptr(workspace),
                                     ws_bytes, byref(out)))
    return out.value


def ot_dyn_batch_offsets(bt: int, count: int):
    LL = ctypes.c_longlong
    a, b, c = (LL * (count + 1))(), (LL * (count + 1))(), (LL * (count + 1))()
    _checkb(lib().ot_dyn_batch_offsets(bt, a, b, c), bt)
    return list(a), list(b), list(c)


def ot_dyn_batch_set_boundary(bt: int, f0, f1) -> int:
    return _checkb(lib().ot_dyn_batch_set_boundary(bt, _ptr(f0), _ptr(f1)), bt)


def ot_dyn_batch_autotune(bt: int, trials: int) -> int:
    return _checkb(lib().ot_dyn_batch_autotune(bt, trials), bt)


def ot_dyn_batch_solve(bt: int, max_iters: int, chunk: int):
    rep = ot_dyn_report()
    st = _checkb(lib().ot_dyn_batch_solve(bt, max_iters, chunk, byref(rep)), bt)
    return st, rep


def ot_dyn_batch_problem(bt: int, i: int) -> ot_dyn_report:
    rep = ot_dyn_report()
    _checkb(lib().ot_dyn_batch_problem(bt, i, byref(rep)), bt)
    return rep


def ot_dyn_batch_get_state(bt: int, F, M) -> int:
    return _checkb(lib().ot_dyn_batch_get_state(bt, _ptr(F), _ptr(M)), bt)


def ot_dyn_batch_set_state(bt: int, F, M, mode: int) -> int:
    return _checkb(lib().ot_dyn_batch_set_state(bt, _ptr(F), _ptr(M), mode), bt)


def ot_dyn_batch_get_dual(bt: int, Bd) -> int:
    return _checkb(lib().ot_dyn_batch_get_dual(bt, _ptr(Bd)), bt)


def ot_dyn_batch_set_dual(bt: int, Bd) -> int:
    return _checkb(lib().ot_dyn_batch_set_dual(bt, _ptr(Bd)), bt)


def ot_dyn_prox_eval(kind: int, am, af, sigma: float, u, v, stream=None) -> int:
    """Device prox of J / sigma on n nodes: am, u [3, n] and af, v [n]
    float32 device tensors (see include/ot_dyn.h)."""
    n = af.numel()
    return _check(lib().ot_dyn_prox_eval(kind, n, _ptr(am), _ptr(af), float(sigma), _ptr(u),
                                         _ptr(v), stream))


OT_DYN_STATIC_BYTES = 32 << 20


def ot_dyn_solve_static(d: ot_dyn_desc, stream, f0, f1, F, Mx, My, Mc, max_iters: int):
    """Cold-start certified solve over the library's own device workspace (no
    device allocation; problems whose workspace fits OT_DYN_STATIC_BYTES)."""
    rep = ot_dyn_report()
    st = _check(lib().ot_dyn_solve_static(byref(d), _ptr(stream), _ptr(f0), _ptr(f1), _ptr(F),
                                          _ptr(Mx), _ptr(My), _ptr(Mc), max_iters, byref(rep)))
    return st, rep


def ot_dyn_batch_tuning(bt: int, i: int):
    a, b = c_int(0), c_int(0)
    _check(lib().ot_dyn_batch_tuning(bt, i, byref(a), byref(b)))
    return a.value, b.value


def ot_dyn_batch_destroy(bt: int) -> int:
    return _check(lib().ot_dyn_batch_destroy(bt))


def ot_dyn_status_str(status: int) -> str:
    return lib().ot_dyn_status_str(status).decode()


def ot_dyn_last_error(plan: int) -> str:
    return lib().ot_dyn_last_error(plan).decode()


# ---- device buffers for one plan (torch for memory and streams only) -------

class Problem:
    """Owns the device buffers of one plan: F, Mx, My, Mc and the workspace.

    Shapes follow the C layout: F [B, P+1, C, Y, X], M* [B, P, C, Y, X].
    """

    def __init__(self, desc: ot_dyn_desc, device="cuda", stream=None):
        import torch
        self.desc = desc
        self.device = torch.device(device)
        B, P, C, Y, X = desc.batch, desc.P, desc.C, desc.Y, desc.X
        f32 = dict(dtype=torch.float32, device=self.device)
        self.F = torch.zeros((B, P + 1, C, Y, X), **f32)
        self.Mx = torch.zeros((B, P, C, Y, X), **f32)
        self.My = torch.zeros((B, P, C, Y, X), **f32)
        self.Mc = torch.zeros((B, P, C, Y, X), **f32)
        self.ws_bytes = ot_dyn_workspace_size(desc)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.plan = ot_dyn_create(desc, self.stream.cuda_stream, self.ws_ptr, self.ws_bytes)

    def state(self):
        return (self.F, self.Mx, self.My, self.Mc)

    def set_boundary(self, f0, f1):
        import torch
        B, C, Y, X = self.desc.batch, self.desc.C, self.desc.Y, self.desc.X
        f0 = torch.as_tensor(f0, dtype=torch.float32).reshape(B, C, Y, X).to(self.device).contiguous()
        f1 = torch.as_tensor(f1, dtype=torch.float32).reshape(B, C, Y, X).to(self.device).contiguous()
        self._f0, self._f1 = f0, f1
        torch.cuda.current_stream(self.device).synchronize()
        return ot_dyn_set_boundary(self.plan, f0, f1)

    def init(self, mode: int = OT_INIT_COLD):
        return ot_dyn_init(self.plan, mode, *self.state())

    def get_dual(self):
        """The dual iterate as a device tensor [B, 4, P, C, Y, X] (a copy)."""
        import torch
        d = self.desc
        b = torch.empty((d.batch, 4, d.P, d.C, d.Y, d.X), dtype=torch.float32, device=self.device)
        ot_dyn_get_dual(self.plan, b)
        return b

    def set_dual(self, b):
        return ot_dyn_set_dual(self.plan, b)

    def get_dual_bar(self):
        """The extrapolated dual b_bar as a device tensor [B, 4, P, C, Y, X] (a copy)."""
        import torch
        d = self.desc
        b = torch.empty((d.batch, 4, d.P, d.C, d.Y, d.X), dtype=torch.float32, device=self.device)
        ot_dyn_get_dual_bar(self.plan, b)
        return b

    def step(self, iters: int):
        return ot_dyn_step(self.plan, *self.state(), iters)

    def solve(self, max_iters: int):
        return ot_dyn_solve(self.plan, *self.state(), max_iters)

    def residuals(self):
        return ot_dyn_residuals(self.plan, *self.state())

    def close(self):
        if getattr(self, "plan", None):
            ot_dyn_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Device buffers of a batch of uneven problems (packed layout of the C
    API): dims is a list of (X, Y, C, P); f0 / f1 are lists of arrays of
    shape (C, Y, X)."""

    def __init__(self, base: ot_dyn_desc, dims, device="cuda"):
        import torch
        self.base = base
        self.dims = [tuple(int(v) for v in d) for d in dims]
        self.count = len(self.dims)
        self.device = torch.device(device)
        self.ws_bytes = ot_dyn_batch_workspace_size(base, self.dims)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        self.ws_ptr = (self.ws.data_ptr() + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        self.bt = ot_dyn_batch_create(base, self.dims, self.stream.cuda_stream, self.ws_ptr,
                                      self.ws_bytes)
        self.off_h, self.off_F, self.off_M = ot_dyn_batch_offsets(self.bt, self.count)

    def set_boundary(self, f0s, f1s):
        import numpy as np
        import torch
        h0 = np.concatenate([np.asarray(a, np.float32).ravel() for a in f0s])
        h1 = np.concatenate([np.asarray(a, np.float32).ravel() for a in f1s])
        self._h0 = torch.from_numpy(h0).to(self.device)
        self._h1 = torch.from_numpy(h1).to(self.device)
        torch.cuda.synchronize(self.device)
        return ot_dyn_batch_set_boundary(self.bt, self._h0, self._h1)

    def set_boundary_packed(self, h0, h1):
        """Boundary densities already packed in device memory (kept alive)."""
        import torch
        self._h0, self._h1 = h0, h1
        torch.cuda.synchronize(self.device)
        return ot_dyn_batch_set_boundary(self.bt, h0, h1)

    def autotune(self, trials: int = 10):
        return ot_dyn_batch_autotune(self.bt, trials)

    def solve(self, max_iters: int, chunk: int = 100):
        return ot_dyn_batch_solve(self.bt, max_iters, chunk)

    def problem(self, i: int) -> ot_dyn_report:
        return ot_dyn_batch_problem(self.bt, i)

    def state(self, i: int):
        """(F, Mx, My, Mc) of problem i as host numpy arrays of the C layout."""
        import torch
        if not hasattr(self, "_F"):
            self._F = torch.empty(self.off_F[-1], dtype=torch.float32, device=self.device)
            self._M = torch.empty(self.off_M[-1], dtype=torch.float32, device=self.device)
        ot_dyn_batch_get_state(self.bt, self._F, self._M)
        X, Y, C, P = self.dims[i]
        F = self._F[self.off_F[i]:self.off_F[i + 1]].reshape(P + 1, C, Y, X)
        M = self._M[self.off_M[i]:self.off_M[i + 1]].reshape(3, P, C, Y, X)
        return (F.cpu().numpy(), M[0].cpu().numpy(), M[1].cpu().numpy(), M[2].cpu().numpy())

    def packed_state(self):
        """Packed (F, M) device tensors of the whole batch (a copy)."""
        import torch
        F = torch.empty(self.off_F[-1], dtype=torch.float32, device=self.device)
        M = torch.empty(self.off_M[-1], dtype=torch.float32, device=self.device)
        ot_dyn_batch_get_state(self.bt, F, M)
        return F, M

    def packed_dual(self):
        """Packed duals of the whole batch (a copy, device)."""
        import torch
        Bd = torch.empty(self.off_M[-1] // 3 * 4, dtype=torch.float32, device=self.device)
        ot_dyn_batch_get_dual(self.bt, Bd)
        return Bd

    def set_dual(self, Bd):
        """Replace the starting dual of the next solve (after set_state)."""
        import torch
        torch.cuda.current_stream(self.device).synchronize()
        return ot_dyn_batch_set_dual(self.bt, Bd)

    def set_state(self, F, M, mode: int = OT_INIT_PRIMAL_DUAL):
        """Start the next solve from the packed state (F, M) (device)."""
        import torch
        torch.cuda.current_stream(self.device).synchronize()
        return ot_dyn_batch_set_state(self.bt, F, M, mode)

    def close(self):
        if getattr(self, "bt", None):
            ot_dyn_batch_destroy(self.bt)
            self.bt = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
