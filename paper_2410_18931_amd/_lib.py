"""ctypes binding of libwsr.so (the C-ABI declared in include/wsr.h).

Argument marshalling only: every step of the rendering path runs in the HIP
kernels of the library.  Loading fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# WSR_LIB may point at another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("WSR_LIB", os.path.join(_PKG, "libwsr.so"))

WSR_OK, WSR_ERR_INVALID, WSR_ERR_WORKSPACE, WSR_ERR_CAPACITY, WSR_ERR_HIP = range(5)
WEIGHT_KINDS = {"dir": 0, "exp": 1, "lc": 2}
OPACITY_MODES = {"logit": 0, "sh": 1}
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
MAX_VIEWS = 256
ABI_VERSION = 6

EXPORTED = ("wsr_abi_version", "wsr_status_string", "wsr_workspace_bytes", "wsr_pair_bytes", "wsr_project", "wsr_bin",
            "wsr_render_fwd", "wsr_render_bwd", "wsr_raster_bwd", "wsr_project_bwd", "wsr_project_bwd_adam",
            "wsr_pair_count", "wsr_check", "wsr_loss_workspace_bytes", "wsr_loss", "wsr_loss_noalloc", "wsr_adam",
            "wsr_sort_tiles", "wsr_render_sorted")


class WsrScene(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("storage", C.c_int32),
                ("opacity_mode", C.c_int32), ("reserved_", C.c_int32),
                ("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("sh", C.c_void_p), ("opacity_logit", C.c_void_p), ("lc_v", C.c_void_p)]


class WsrCamera(C.Structure):
    _fields_ = [("viewmat", C.c_float * 12), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class WsrParams(C.Structure):
    _fields_ = [("weight_kind", C.c_int32), ("tile", C.c_int32), ("tau", C.c_float),
                ("dilation", C.c_float), ("near_z", C.c_float), ("opacity_offset", C.c_float),
                ("flags", C.c_int32), ("alpha_cut", C.c_float), ("batch", C.c_int32)]


FLAG_UNNORMALISED = 1
FLAG_OIT = 2
FLAG_PERSISTENT = 4
WSR_ERR_TILE_LIST = 5
WSR_ERR_STATIC = 6
LOSS_STATIC_BYTES = 72 << 20
SORT_MAX = 16384


class WsrBlend(C.Structure):
    _fields_ = [("alpha_max", C.c_float), ("alpha_min", C.c_float), ("t_min", C.c_float),
                ("reserved_", C.c_int32)]


class WsrGrads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("sh", C.c_void_p), ("opacity_logit", C.c_void_p), ("lc_v", C.c_void_p),
                ("globals", C.c_void_p)]


class WsrAdamParams(C.Structure):
    _fields_ = [("lr_means", C.c_float), ("lr_log_scales", C.c_float), ("lr_quats", C.c_float),
                ("lr_sh0", C.c_float), ("lr_shN", C.c_float), ("lr_opacity_logit", C.c_float),
                ("lr_lc_v", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("step", C.c_int32), ("reserved_", C.c_int32)]


class WsrError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn} failed: {status_string(status)} (status {status})")
        self.status = status


_lib = None


def load():
    """Load libwsr.so (built by ``paper_2410_18931_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2410_18931_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
    lib.wsr_abi_version.restype = I32
    lib.wsr_status_string.restype = C.c_char_p
    lib.wsr_status_string.argtypes = [I32]
    lib.wsr_workspace_bytes.restype = I64
    lib.wsr_workspace_bytes.argtypes = [I64, P, I32, I32]
    lib.wsr_pair_bytes.restype = I64
    lib.wsr_project.restype = I32
    lib.wsr_project.argtypes = [P, P, I32, P, P, P, I64, P, P]
    lib.wsr_bin.restype = I32
    lib.wsr_bin.argtypes = [P, I32, P, I64, P, I64, P, I64, P]
    lib.wsr_render_fwd.restype = I32
    lib.wsr_render_fwd.argtypes = [P, I32, P, I64, P, P, I64, P, I64, P, P, P, P]
    lib.wsr_render_bwd.restype = I32
    lib.wsr_render_bwd.argtypes = [P, P, I32, P, P, P, I64, P, I64, P, P, P, P, P, P]
    lib.wsr_raster_bwd.restype = I32
    lib.wsr_raster_bwd.argtypes = [P, I32, P, I64, P, P, I64, P, I64, P, P, P, P]
    lib.wsr_project_bwd.restype = I32
    lib.wsr_project_bwd.argtypes = [P, P, I32, P, P, P, I64, P, I64, P, P, P]
    lib.wsr_project_bwd_adam.restype = I32
    lib.wsr_project_bwd_adam.argtypes = [P, P, I32, P, P, P, I64, P, I64, P, P, P, P, P, P]
    lib.wsr_pair_count.restype = I32
    lib.wsr_pair_count.argtypes = [P, I64, C.POINTER(C.c_int64), P]
    lib.wsr_check.restype = I32
    lib.wsr_check.argtypes = [P, I64, P]
    F = C.c_float
    lib.wsr_loss_workspace_bytes.restype = I64
    lib.wsr_loss_workspace_bytes.argtypes = [P, I32]
    lib.wsr_loss.restype = I32
    lib.wsr_loss.argtypes = [P, I32, P, P, F, P, I64, P, P, P]
    lib.wsr_loss_noalloc.restype = I32
    lib.wsr_loss_noalloc.argtypes = [P, I32, P, P, F, P, P, P]
    lib.wsr_adam.restype = I32
    lib.wsr_adam.argtypes = [P, P, P, P, I64, I32, F, F, F, F, P]
    lib.wsr_sort_tiles.restype = I32
    lib.wsr_sort_tiles.argtypes = [P, I32, P, I64, P, I64, P, I64, P]
    lib.wsr_render_sorted.restype = I32
    lib.wsr_render_sorted.argtypes = [P, I32, P, I64, P, P, P, I64, P, I64, P, P, P]
    if lib.wsr_abi_version() != ABI_VERSION:
        raise RuntimeError("libwsr.so ABI version mismatch; rebuild the library")
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().wsr_status_string(int(status)).decode()


def check(fn: str, status: int) -> None:
    if status != WSR_OK:
        raise WsrError(fn, status)


def make_cameras(cams) -> "C.Array":
    arr = (WsrCamera * len(cams))()
    for k, c in enumerate(cams):
        vm = [float(x) for x in __import__("numpy").asarray(c["viewmat"], dtype="float64").reshape(12)]
        arr[k].viewmat = (C.c_float * 12)(*vm)
        arr[k].fx, arr[k].fy = float(c["fx"]), float(c["fy"])
        arr[k].cx, arr[k].cy = float(c["cx"]), float(c["cy"])
        arr[k].width, arr[k].height = int(c["width"]), int(c["height"])
    return arr


def make_params(settings, flags: int = 0) -> WsrParams:
    if getattr(settings, "oit", False):
        flags |= FLAG_OIT
    if getattr(settings, "persistent", False):
        flags |= FLAG_PERSISTENT
    return WsrParams(WEIGHT_KINDS[settings.weight_kind], int(settings.tile), float(settings.tau),
                     float(settings.dilation), float(settings.near), float(settings.opacity_offset), int(flags),
                     float(getattr(settings, "alpha_cut", 0.0)), int(getattr(settings, "batch", 0)))
