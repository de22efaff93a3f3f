"""Python binding of the hue image pipeline C ABI (include/ot_hue.h).

Same rules as otdyn: the functions carry the C names and marshal arguments
only; hues, histograms, the strict order and the frames are computed by the
HIP kernels of libotdyn.so.  Device pointers are torch CUDA tensors or
integers.
"""
from __future__ import annotations

import ctypes
from ctypes import POINTER, byref, c_int, c_void_p

from . import otdyn
from .otdyn import OtDynError, _ptr

EXPORTS = ["ot_hue_workspace_size", "ot_hue_create", "ot_hue_destroy", "ot_hue_set_source", "ot_hue_histogram",
           "ot_hue_render", "ot_hue_plan", "ot_hue_apply", "ot_hue_plan_info",
           "ot_hue_rgb_to_hsv", "ot_hue_hsv_to_rgb"]

_done = False


def lib() -> ctypes.CDLL:
    global _done
    L = otdyn.lib()
    if _done:
        return L
    P = c_void_p
    LL = ctypes.c_longlong
    L.ot_hue_workspace_size.argtypes = [LL, c_int, c_int, POINTER(ctypes.c_size_t)]
    L.ot_hue_create.argtypes = [LL, c_int, c_int, P, P, ctypes.c_size_t, POINTER(c_void_p)]
    L.ot_hue_destroy.argtypes = [P]
    L.ot_hue_destroy.restype = None
    L.ot_hue_set_source.argtypes = [P, P]
    L.ot_hue_histogram.argtypes = [P, P, P]
    L.ot_hue_render.argtypes = [P, P, c_int, P, P]
    L.ot_hue_plan.argtypes = [P, P, c_int]
    L.ot_hue_apply.argtypes = [P, P, P]
    L.ot_hue_plan_info.argtypes = [P, c_int, P, POINTER(LL)]
    L.ot_hue_rgb_to_hsv.argtypes = [P, LL, P, P]
    L.ot_hue_hsv_to_rgb.argtypes = [P, LL, P, P]
    for name in EXPORTS:
        if name != "ot_hue_destroy":
            getattr(L, name).restype = c_int
    _done = True
    return L


def _check(status: int) -> int:
    if status < 0:
        raise OtDynError(status, otdyn.lib().ot_dyn_status_str(status).decode())
    return status


def ot_hue_workspace_size(npix: int, nbins: int, max_frames: int = 1) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().ot_hue_workspace_size(npix, nbins, max_frames, byref(n)))
    return int(n.value)


def ot_hue_create(npix: int, nbins: int, max_frames: int, stream, workspace, ws_bytes: int) -> int:
    h = c_void_p()
    _check(lib().ot_hue_create(npix, nbins, max_frames, _ptr(stream), _ptr(workspace), ws_bytes,
                               byref(h)))
    return h.value


def ot_hue_destroy(h: int) -> None:
    lib().ot_hue_destroy(h)


def ot_hue_set_source(h: int, rgb) -> int:
    return _check(lib().ot_hue_set_source(h, _ptr(rgb)))


def ot_hue_histogram(h: int, counts=None, density=None) -> int:
    return _check(lib().ot_hue_histogram(h, _ptr(counts), _ptr(density)))


def ot_hue_render(h: int, targets, frames: int, rgb_out, bins_out=None) -> int:
    return _check(lib().ot_hue_render(h, _ptr(targets), frames, _ptr(rgb_out), _ptr(bins_out)))


def ot_hue_plan(h: int, targets, frames: int = 1) -> int:
    return _check(lib().ot_hue_plan(h, _ptr(targets), frames))


def ot_hue_apply(h: int, rgb_out, bins_out=None) -> int:
    return _check(lib().ot_hue_apply(h, _ptr(rgb_out), _ptr(bins_out)))


def ot_hue_plan_info(h: int, frame: int = 0, counts=None):
    """(status, shift) of one frame of the last plan; counts: a host int32
    array (numpy) or None."""
    s = ctypes.c_longlong()
    cp = counts.ctypes.data if counts is not None else 0
    st = _check(lib().ot_hue_plan_info(h, frame, cp, byref(s)))
    return st, s.value


def ot_hue_rgb_to_hsv(rgb, npix: int, hsv, stream=None) -> int:
    return _check(lib().ot_hue_rgb_to_hsv(_ptr(rgb), npix, _ptr(hsv), _ptr(stream)))


def ot_hue_hsv_to_rgb(hsv, npix: int, rgb, stream=None) -> int:
    return _check(lib().ot_hue_hsv_to_rgb(_ptr(hsv), npix, _ptr(rgb), _ptr(stream)))


class HueRenderer:
    """Owns one ot_hue object, its device workspace (torch memory) and the
    source image tensor it reads.  A call with more frames than the workspace
    plans for makes a renderer with room for them (and prepares the source
    again)."""

    def __init__(self, npix: int, nbins: int, device="cuda:0", max_frames: int = 64):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.npix, self.nbins = npix, nbins
        self.stream = torch.cuda.current_stream(self.device)
        self.h = None
        self.src = None
        self._make(max_frames)

    def _make(self, max_frames: int):
        t = self.torch
        if self.h:
            ot_hue_destroy(self.h)
            self.h = None
        self.max_frames = max_frames
        n = ot_hue_workspace_size(self.npix, self.nbins, max_frames)
        self.ws = t.empty(n + 256, dtype=t.uint8, device=self.device)
        ptr = (self.ws.data_ptr() + 255) // 256 * 256
        self.h = ot_hue_create(self.npix, self.nbins, max_frames, self.stream.cuda_stream, ptr, n)
        if self.src is not None:
            ot_hue_set_source(self.h, self.src)

    def set_source(self, rgb):
        """rgb: uint8 tensor on the device with npix * 3 elements."""
        t = self.torch
        assert rgb.dtype == t.uint8 and rgb.is_cuda and rgb.numel() == 3 * self.npix
        self.src = rgb.contiguous()
        ot_hue_set_source(self.h, self.src)

    def reserve(self, frames: int):
        """Room for calls of `frames` frames."""
        if frames > self.max_frames:
            self._make(frames)

    def histogram(self):
        t = self.torch
        c = t.empty(self.nbins, dtype=t.int32, device=self.device)
        d = t.empty(self.nbins, dtype=t.float32, device=self.device)
        ot_hue_histogram(self.h, c, d)
        return c, d

    def render(self, target, with_bins: bool = False):
        """The frame for a device float density on the bins: uint8 (npix, 3)
        and, with with_bins, each pixel's output bin (int32)."""
        assert target.numel() == self.nbins, "target must have nbins entries"
        out, bins = self.render_frames(target.reshape(1, -1), True)
        return (out[0], bins[0]) if with_bins else out[0]

    def render_frames(self, targets, with_bins: bool = False):
        """Frames for device float densities [frames, nbins]: uint8
        (frames, npix, 3) and, with with_bins, the output bins (frames, npix)."""
        t = self.torch
        assert targets.dtype == t.float32 and targets.is_cuda
        assert targets.dim() == 2 and targets.shape[1] == self.nbins and targets.shape[0] >= 1, \
            "targets must be [frames, nbins]"
        F = targets.shape[0]
        self.reserve(F)
        out = t.empty(F, self.npix, 3, dtype=t.uint8, device=self.device)
        bins = t.empty(F, self.npix, dtype=t.int32, device=self.device) if with_bins else None
        ot_hue_render(self.h, targets.contiguous(), F, out, bins)
        return (out, bins) if with_bins else out

    def plan_info(self, frame: int = 0):
        import numpy as np
        c = np.empty(self.nbins, dtype=np.int32)
        _, s = ot_hue_plan_info(self.h, frame, c)
        return c, s

    def close(self):
        if self.h:
            ot_hue_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
