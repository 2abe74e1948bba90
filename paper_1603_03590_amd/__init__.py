"""Dense Inverse Search optical flow (Kroeger et al., ECCV 2016) on AMD MI355X.

Every step of the method runs in the HIP kernels of ``libdis.so``; this
module marshals torch tensors (device memory and the current HIP stream) into
the C entry points of include/dis.h.  There is no CPU fallback: without the
built library or a GPU these functions raise.
"""
from __future__ import annotations

import numpy as np

from . import _lib
from ._lib import (DisError, DisLibraryMissing, dis_params, DIS_FLAG_KEEP_FOR_BACKWARD, DIS_FLAG_NO_GRAPH,
                   DIS_FLAG_PIXEL_CENTRE, DIS_FLAG_RAW_RESIDUAL, DIS_FLAG_IO_F64, DIS_FLAG_STEREO,
                   DIS_FLAG_FB_CONSISTENCY, DIS_FLAG_COLOUR)

__all__ = ["DIS", "params", "compute_flow", "dis_flow", "DisError", "DisLibraryMissing", "dis_params",
           "DIS_FLAG_KEEP_FOR_BACKWARD", "DIS_FLAG_NO_GRAPH", "DIS_FLAG_PIXEL_CENTRE",
           "DIS_FLAG_RAW_RESIDUAL", "DIS_FLAG_IO_F64", "DIS_FLAG_STEREO", "DIS_FLAG_FB_CONSISTENCY", "DIS_FLAG_COLOUR"]

PRESETS = {"op1": 1, "op2": 2, "op3": 3, "op4": 4, "c1": 101, "c2a": 102, "c2b": 103, "c3": 104,
           "c5": 105, "c4": 106}


def params(preset=2, **overrides) -> dis_params:
    """Parameter block from a preset (int or name in PRESETS) plus overrides."""
    if isinstance(preset, str):
        preset = PRESETS[preset]
    p = _lib.dis_default_params(int(preset))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, int(v) if isinstance(v, bool) else v)
    return p


def _torch():
    import torch
    return torch


class DIS:
    """A handle: all device scratch for frames up to max_w x max_h and up to
    ``max_batch`` pairs, bound to a HIP stream (default: torch's current)."""

    def __init__(self, p: dis_params, max_w: int, max_h: int, max_batch: int = 1, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("DIS needs a visible GPU")
        self.p = p
        self.max_w, self.max_h = max_w, max_h
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.handle = _lib.dis_create(p, max_w, max_h, max_batch, self.stream.cuda_stream)
        self.dtype = torch.float64 if (p.flags & DIS_FLAG_IO_F64) else torch.float32

    def close(self):
        if getattr(self, "handle", None):
            _lib.dis_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _frame(self, I):
        colour = bool(int(self.p.flags) & _lib.DIS_FLAG_COLOUR)
        dims = 3 if colour else 2
        if I.dtype != self.dtype or I.device.type != "cuda" or I.dim() != dims:
            kind = "[3, H, W]" if colour else "[H, W]"
            raise ValueError(f"frames must be {kind} {self.dtype} tensors on the GPU")
        if I.stride(-1) != 1:
            raise ValueError("frames must have unit column stride")
        if colour and (I.shape[0] != 3 or I.stride(0) != I.shape[1] * I.stride(1)):
            raise ValueError("colour frames must hold 3 planes, channel stride = height x row pitch")
        return I

    def flow(self, I0, I1, out=None):
        """Dense flow [2, H, W] from I0 to I1 (device tensors, same shape)."""
        torch = _torch()
        I0 = self._frame(I0)
        I1 = self._frame(I1)
        if I0.shape != I1.shape or I0.stride() != I1.stride():
            raise ValueError("frames must have the same shape and strides")
        h, w = I0.shape[-2:]
        cur = self._enter(I0.device)
        if out is None:
            out = torch.empty((2, h, w), dtype=self.dtype, device=I0.device)
        _lib.dis_compute_flow(self.handle, I0.data_ptr(), I1.data_ptr(), w, h, I0.stride(-2), out.data_ptr())
        self._leave(cur)
        self._generation = getattr(self, "_generation", 0) + 1
        self._last_frames = (I0, I1)     # dis_autotune reads them again
        return out

    def _enter(self, device):
        """The caller's current stream, after making the handle's stream wait
        for the work queued on it (the frames' producers)."""
        torch = _torch()
        cur = torch.cuda.current_stream(device)
        if cur != self.stream:
            self.stream.wait_stream(cur)
        return cur

    def _leave(self, cur):
        """Order the caller's stream after the handle's work, so that results
        (and freeing the inputs) follow the kernels that use them."""
        if cur != self.stream:
            cur.wait_stream(self.stream)

    def flow_batched(self, I0s, I1s, outs=None):
        """Flows of many pairs (lists of device tensors), one launch per level."""
        torch = _torch()
        I0s = [self._frame(a) for a in I0s]
        I1s = [self._frame(b) for b in I1s]
        cur = self._enter(I0s[0].device) if I0s else None
        if outs is None:
            outs = [torch.empty((2,) + a.shape, dtype=self.dtype, device=a.device) for a in I0s]
        _lib.dis_compute_flow_batched(self.handle, [a.data_ptr() for a in I0s], [b.data_ptr() for b in I1s],
                                      [a.shape[1] for a in I0s], [a.shape[0] for a in I0s],
                                      [a.stride(0) for a in I0s], [o.data_ptr() for o in outs])
        if cur is not None:
            self._leave(cur)
        self._generation = getattr(self, "_generation", 0) + 1
        self._last_frames = (list(I0s), list(I1s))     # dis_autotune reads them again
        return outs

    def backward(self, grad_flow, shape=None):
        """dL/dI0, dL/dI1 ([H, W], dense) for the most recent ``flow`` call on
        this handle, from dL/dflow [2, H, W]; the handle needs
        DIS_FLAG_KEEP_FOR_BACKWARD.  Runs on the handle's stream."""
        torch = _torch()
        if grad_flow.dtype != self.dtype or grad_flow.device.type != "cuda" or grad_flow.dim() != 3:
            raise ValueError(f"grad_flow must be a [2, H, W] {self.dtype} tensor on the GPU")
        shape = tuple(shape) if shape is not None else tuple(grad_flow.shape[1:])
        if tuple(grad_flow.shape) != (2,) + shape:
            raise ValueError(f"grad_flow has shape {tuple(grad_flow.shape)}, expected {(2,) + shape}")
        gf = grad_flow.contiguous()
        cur = self._enter(grad_flow.device)
        g0 = torch.empty(shape, dtype=self.dtype, device=grad_flow.device)
        g1 = torch.empty(shape, dtype=self.dtype, device=grad_flow.device)
        _lib.dis_flow_backward(self.handle, gf.data_ptr(), g0.data_ptr(), g1.data_ptr())
        self._leave(cur)
        self._keep = gf      # alive until the next call on this handle
        return g0, g1

    def set_tunables(self, lanes_per_patch=None, refine_tile=0, launch_mode=0):
        _lib.dis_set_tunables(self.handle, lanes_per_patch, refine_tile, launch_mode)

    def tunables(self) -> dict:
        return _lib.dis_get_tunables(self.handle)

    def autotune(self, cache_path=None):
        """Time the result-invariant launch choices on a replay of the last
        flow call (its frames, kept alive by this object; the flow it
        returned is not written) and keep the fastest."""
        _lib.dis_autotune(self.handle, cache_path)

    def debug_level(self, s: int, what: int):
        """Intermediate of the last forward at scale s as a float64 numpy array."""
        if what == _lib.DIS_DBG_WAIT_ERRORS:
            n = np.zeros(1, np.int32)
            _lib.dis_debug_level(self.handle, s, what, n.ctypes.data, n.nbytes)
            return int(n[0])
        info = np.zeros(6, np.int32)
        _lib.dis_debug_level(self.handle, s, _lib.DIS_DBG_INFO, info.ctypes.data, info.nbytes)
        W, H, N = int(info[0]), int(info[1]), int(info[2])
        if what == _lib.DIS_DBG_INFO:
            return info
        shape = {_lib.DIS_DBG_J0: (H, W), _lib.DIS_DBG_J1: (H, W), _lib.DIS_DBG_UINIT: (N, 2),
                 _lib.DIS_DBG_UPATCH: (N, 2), _lib.DIS_DBG_UDENSE: (2, H, W),
                 _lib.DIS_DBG_UREFINED: (2, H, W), _lib.DIS_DBG_GRAD_J0: (H, W), _lib.DIS_DBG_GRAD_J1: (H, W),
                 _lib.DIS_DBG_GRAD_U: (2, H, W), _lib.DIS_DBG_GRAD_PATCH: (N, 4),
                 _lib.DIS_DBG_UREFINED_BWD: (2, H, W)}[what]
        out = np.zeros(shape, np.float64)
        _lib.dis_debug_level(self.handle, s, what, out.ctypes.data, out.nbytes)
        return out


def dis_flow(I0, I1, dis: DIS):
    """Flow of (I0, I1) through ``dis`` as a differentiable torch op: the
    backward pass runs the hand-written adjoint (dis_flow_backward).  The
    handle must keep forward state (DIS_FLAG_KEEP_FOR_BACKWARD), and the
    backward of a result must run before the handle's next forward call."""
    from .autograd import DISFlow
    return DISFlow.apply(I0, I1, dis)


def compute_flow(I0, I1, p: dis_params | None = None):
    """One-shot flow of a pair of device frames."""
    p = p if p is not None else params(2)
    h, w = I0.shape
    d = DIS(p, w, h)
    try:
        out = d.flow(I0, I1)
        d.stream.synchronize()
        return out
    finally:
        d.close()
