"""ctypes binding of ``libdis.so`` (declared in include/dis.h).

Each function here has the name of the C entry point it calls and only
marshals arguments: pointers are passed as integers (``tensor.data_ptr()``)
and streams as ``torch.cuda.Stream.cuda_stream`` handles.  A missing library
raises ``DisLibraryMissing``; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_size_t, c_uint32, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdis.so")

DIS_OK = 0
DIS_EINVAL = -1
DIS_ESIZE = -2
DIS_EHIP = -3
DIS_ESTATE = -4
DIS_ENOMEM = -5

DIS_FLAG_KEEP_FOR_BACKWARD = 0x1
DIS_FLAG_NO_GRAPH = 0x2
DIS_FLAG_PIXEL_CENTRE = 0x4
DIS_FLAG_RAW_RESIDUAL = 0x8
DIS_FLAG_IO_F64 = 0x10
DIS_FLAG_STEREO = 0x20
DIS_FLAG_FB_CONSISTENCY = 0x40
DIS_FLAG_COLOUR = 0x80

DIS_NORM_L2 = 0
DIS_NORM_L1 = 1
DIS_NORM_HUBER = 2

DIS_DBG_J0 = 0
DIS_DBG_J1 = 1
DIS_DBG_UINIT = 2
DIS_DBG_UPATCH = 3
DIS_DBG_UDENSE = 4
DIS_DBG_UREFINED = 5
DIS_DBG_INFO = 6
DIS_DBG_WAIT_ERRORS = 7
DIS_DBG_GRAD_J0 = 8
DIS_DBG_GRAD_J1 = 9
DIS_DBG_GRAD_U = 10
DIS_DBG_GRAD_PATCH = 11
DIS_DBG_UREFINED_BWD = 12

# every symbol include/dis.h declares
EXPORTS = (
    "dis_default_params", "dis_create", "dis_compute_flow", "dis_compute_flow_batched",
    "dis_flow_backward", "dis_autotune", "dis_last_error", "dis_set_stream",
    "dis_debug_level", "dis_destroy", "dis_profile_enable", "dis_profile_read", "dis_set_tunables",
    "dis_get_tunables", "dis_compute_flow_noalloc",
)


class DisLibraryMissing(RuntimeError):
    pass


class DisError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"DIS error {code}: {msg}")
        self.code = code


class dis_params(ctypes.Structure):
    _fields_ = [
        ("patch_size", c_int32),
        ("overlap", c_double),
        ("coarsest_scale", c_int32),
        ("finest_scale", c_int32),
        ("gn_iters", c_int32),
        ("var_outer", c_int32),
        ("var_inner", c_int32),
        ("w_intensity", c_double),
        ("w_gradient", c_double),
        ("w_smooth", c_double),
        ("sor_omega", c_double),
        ("refine", c_int32),
        ("flags", c_uint32),
        ("norm", c_int32),
        ("huber_b", c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class dis_kernel_stat(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 32),
        ("launches", c_int32),
        ("total_ms", c_double),
        ("bytes", c_double),
        ("flops", c_double),
    ]


_lib = None


def load(path: str = LIB_PATH):
    """Load the library once and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise DisLibraryMissing(f"{path} not found: build it with `python -m paper_1603_03590_amd.build`")
    lib = ctypes.CDLL(path)
    H = c_void_p
    lib.dis_default_params.argtypes = [c_int, POINTER(dis_params)]
    lib.dis_create.argtypes = [POINTER(dis_params), c_int, c_int, c_int, c_void_p, POINTER(c_void_p)]
    lib.dis_compute_flow.argtypes = [H, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p]
    lib.dis_compute_flow_batched.argtypes = [H, c_int, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_int),
                                             POINTER(c_int), POINTER(c_int), POINTER(c_void_p)]
    lib.dis_flow_backward.argtypes = [H, c_void_p, c_void_p, c_void_p]
    lib.dis_autotune.argtypes = [H, c_char_p]
    lib.dis_last_error.argtypes = [H]
    lib.dis_last_error.restype = c_char_p
    lib.dis_set_stream.argtypes = [H, c_void_p]
    lib.dis_debug_level.argtypes = [H, c_int, c_int, c_void_p, c_size_t]
    lib.dis_profile_enable.argtypes = [H, c_int]
    lib.dis_profile_read.argtypes = [H, POINTER(dis_kernel_stat), c_int, POINTER(c_int)]
    lib.dis_set_tunables.argtypes = [H, POINTER(c_int), c_int, c_int]
    lib.dis_get_tunables.argtypes = [H, POINTER(c_int), POINTER(c_int), POINTER(c_int)]
    lib.dis_compute_flow_noalloc.argtypes = [POINTER(dis_params), c_void_p, c_void_p, c_int, c_int, c_int, c_void_p,
                                             c_void_p]
    lib.dis_destroy.argtypes = [H]
    lib.dis_destroy.restype = None
    for name in EXPORTS:
        if name not in ("dis_last_error", "dis_destroy"):
            getattr(lib, name).restype = c_int
    _lib = lib
    return lib


def _check(code, handle=None):
    if code != DIS_OK:
        msg = load().dis_last_error(handle)
        raise DisError(code, msg.decode() if msg else "")


def dis_default_params(preset: int) -> dis_params:
    p = dis_params()
    _check(load().dis_default_params(preset, ctypes.byref(p)))
    return p


def dis_create(params: dis_params, max_w: int, max_h: int, max_batch: int = 1, stream: int = 0) -> int:
    h = c_void_p()
    _check(load().dis_create(ctypes.byref(params), max_w, max_h, max_batch, c_void_p(stream), ctypes.byref(h)))
    return h.value


def dis_compute_flow(handle: int, I0: int, I1: int, w: int, h: int, pitch: int, flow: int) -> None:
    _check(load().dis_compute_flow(c_void_p(handle), c_void_p(I0), c_void_p(I1), w, h, pitch, c_void_p(flow)),
           c_void_p(handle))


def dis_compute_flow_batched(handle: int, I0s, I1s, ws, hs, pitches, flows) -> None:
    n = len(I0s)
    arr = lambda T, xs: (T * n)(*xs)
    _check(load().dis_compute_flow_batched(
        c_void_p(handle), n, arr(c_void_p, I0s), arr(c_void_p, I1s), arr(c_int, ws), arr(c_int, hs),
        arr(c_int, pitches), arr(c_void_p, flows)), c_void_p(handle))


def dis_flow_backward(handle: int, grad_flow: int, grad_I0: int, grad_I1: int) -> None:
    _check(load().dis_flow_backward(c_void_p(handle), c_void_p(grad_flow), c_void_p(grad_I0), c_void_p(grad_I1)),
           c_void_p(handle))


def dis_autotune(handle: int, cache_path: str | None = None) -> None:
    _check(load().dis_autotune(c_void_p(handle), cache_path.encode() if cache_path else None), c_void_p(handle))


def dis_last_error(handle: int | None = None) -> str:
    msg = load().dis_last_error(c_void_p(handle) if handle else None)
    return msg.decode() if msg else ""


def dis_set_stream(handle: int, stream: int) -> None:
    _check(load().dis_set_stream(c_void_p(handle), c_void_p(stream)), c_void_p(handle))


def dis_debug_level(handle: int, s: int, what: int, dst: int, nbytes: int) -> None:
    _check(load().dis_debug_level(c_void_p(handle), s, what, c_void_p(dst), nbytes), c_void_p(handle))


def dis_destroy(handle: int) -> None:
    load().dis_destroy(c_void_p(handle))


def dis_profile_enable(handle: int, on: bool) -> None:
    _check(load().dis_profile_enable(c_void_p(handle), 1 if on else 0), c_void_p(handle))


def dis_profile_read(handle: int, max_kernels: int = 32):
    """[{name, launches, total_ms, bytes, flops}] accumulated since the last read."""
    arr = (dis_kernel_stat * max_kernels)()
    n = c_int()
    _check(load().dis_profile_read(c_void_p(handle), arr, max_kernels, ctypes.byref(n)), c_void_p(handle))
    return [dict(name=arr[i].name.decode(), launches=arr[i].launches, total_ms=arr[i].total_ms,
                 bytes=arr[i].bytes, flops=arr[i].flops) for i in range(min(n.value, max_kernels))]


def dis_get_tunables(handle: int) -> dict:
    """{lanes_per_patch: [16 ints], refine_tile, launch_mode} in force on the handle."""
    arr = (c_int * 16)()
    tile = c_int()
    mode = c_int()
    _check(load().dis_get_tunables(c_void_p(handle), arr, ctypes.byref(tile), ctypes.byref(mode)), c_void_p(handle))
    return {"lanes_per_patch": list(arr), "refine_tile": tile.value, "launch_mode": mode.value}


def dis_set_tunables(handle: int, lanes_per_patch=None, refine_tile: int = 0, launch_mode: int = 0) -> None:
    """lanes_per_patch: None or 16 ints (per scale, 0 = automatic)."""
    arr = None
    if lanes_per_patch is not None:
        vals = list(lanes_per_patch) + [0] * (16 - len(lanes_per_patch))
        arr = (c_int * 16)(*vals[:16])
    _check(load().dis_set_tunables(c_void_p(handle), arr, refine_tile, launch_mode), c_void_p(handle))


def dis_compute_flow_noalloc(params: dis_params, I0: int, I1: int, w: int, h: int, pitch: int, flow: int,
                             stream: int = 0) -> None:
    _check(load().dis_compute_flow_noalloc(ctypes.byref(params), c_void_p(I0), c_void_p(I1), w, h, pitch,
                                           c_void_p(flow), c_void_p(stream)))
