"""FP64 CPU reference for weighted sum rendering.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports this.

Thin ctypes wrapper around ``wsr_oracle.c`` (plain C, double precision,
OpenMP).  Inputs are the float32 scene arrays of ``wsr_synth`` (upcast to
float64 here); outputs are float64 numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wsr_oracle.c")
# WSR_ORACLE_LIB loads another build of the same source (the mutation tests
# load copies with a planted mistake)
_LIB = os.environ.get("WSR_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
PROJ_STRIDE = 25
WEIGHT_KINDS = {"dir": 0, "exp": 1, "lc": 2}
OPACITY_MODES = {"logit": 0, "sh": 1}


def build(force: bool = True, src: str | None = None, out: str | None = None) -> str:
    """Compile the checker (gcc, -O2, OpenMP) into oracle/liboracle.so, or
    the source `src` into `out`."""
    src = src or _SRC
    out = out or _LIB
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wno-unknown-pragmas", "-o", tmp, src, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


class _Scene(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("opacity_mode", C.c_int32),
                ("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("sh", C.c_void_p), ("opacity_logit", C.c_void_p), ("lc_v", C.c_void_p)]


class _Camera(C.Structure):
    _fields_ = [("viewmat", C.c_double * 12), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("width", C.c_int32),
                ("height", C.c_int32), ("pad_", C.c_int32 * 2)]


class _Params(C.Structure):
    _fields_ = [("weight_kind", C.c_int32), ("pad_", C.c_int32), ("sigma", C.c_double),
                ("beta", C.c_double), ("w_bg", C.c_double), ("bg", C.c_double * 3),
                ("tau", C.c_double), ("dilation", C.c_double), ("near_z", C.c_double),
                ("opacity_offset", C.c_double), ("alpha_cut", C.c_double), ("oit", C.c_int32),
                ("pad2_", C.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        lib.ora_project.argtypes = [P, P, P, P]
        lib.ora_render.argtypes = [P, P, P, C.c_int64, C.c_int64, C.c_int64, C.c_int64,
                                   C.c_int32, C.c_double, C.c_double, P, P, P, P, P, P, P]
        lib.ora_render_bwd.argtypes = [P, P, P, C.c_int64, C.c_int64, C.c_int64, C.c_int64,
                                       P, P, P, P, P, P, P, P, P]
        D = C.c_double
        lib.ora_render_sorted.argtypes = [P, P, P, C.c_int64, C.c_int64, C.c_int64, C.c_int64, D, D, D, D, D,
                                          P, P, P]
        lib.ora_sh_basis.argtypes = [P, C.c_int64, C.c_int32, P]
        lib.ora_quat_to_rot.argtypes = [P, C.c_int64, P]
        lib.ora_num_threads.restype = C.c_int32
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class _Packed:
    """Keeps the float64 copies alive while the C structs point at them."""

    def __init__(self, scene, cam, settings):
        self.arrs = {k: _f64(v) for k, v in scene.items()}
        sh = self.arrs["sh"]
        k = sh.shape[0]
        deg = int(round(k ** 0.5)) - 1
        if (deg + 1) ** 2 != k or deg > 3:
            raise ValueError("SH coefficient count must be 1, 4, 9 or 16")
        n = self.arrs["means"].shape[1]
        self.n = n
        self.K = k
        self.scene = _Scene(n, deg, OPACITY_MODES[settings.opacity_mode],
                            _ptr(self.arrs["means"]), _ptr(self.arrs["log_scales"]),
                            _ptr(self.arrs["quats"]), _ptr(self.arrs["sh"]),
                            _ptr(self.arrs["opacity_logit"]), _ptr(self.arrs["lc_v"]))
        vm = np.asarray(cam["viewmat"], dtype=np.float64).reshape(12)
        self.cam = _Camera((C.c_double * 12)(*vm), cam["fx"], cam["fy"], cam["cx"], cam["cy"],
                           int(cam["width"]), int(cam["height"]), (C.c_int32 * 2)(0, 0))
        self.params = _Params(WEIGHT_KINDS[settings.weight_kind], 0, settings.sigma, settings.beta,
                              settings.w_bg, (C.c_double * 3)(*settings.bg), settings.tau,
                              settings.dilation, settings.near, settings.opacity_offset,
                              getattr(settings, "alpha_cut", 0.0), int(bool(getattr(settings, "oit", False))), 0)


def num_threads() -> int:
    return int(_load().ora_num_threads())


def project(scene, cam, settings) -> dict:
    """Per-Gaussian projected quantities of one view (Sec. 3, Eqs. 3-5; Sec.
    4.2-4.3 for the weights and opacity)."""
    pk = _Packed(scene, cam, settings)
    out = np.zeros((pk.n, PROJ_STRIDE), dtype=np.float64)
    _load().ora_project(C.byref(pk.scene), C.byref(pk.cam), C.byref(pk.params), _ptr(out))
    return {
        "visible": out[:, 0] > 0.5, "mu": out[:, 1:3], "cov2d": out[:, 3:6],
        "conic": out[:, 6:9], "rgb": out[:, 9:12], "u": out[:, 12], "w": out[:, 13],
        "depth": out[:, 14], "t": out[:, 15:18], "dir": out[:, 18:21], "rgb_raw": out[:, 21:24],
        "cut": out[:, 24],
    }


def _window(cam, crop):
    if crop is None:
        return 0, 0, int(cam["width"]), int(cam["height"])
    x0, y0, x1, y1 = (int(v) for v in crop)
    return x0, y0, x1, y1


def render(scene, cam, settings, crop=None, mode: str = "strict", eta: float = 1e-6, pos_h: float = 0.0) -> dict:
    """Weighted sum rendering of one view (Sec. 4.2, Eq. 7) over the pixel
    window ``crop = (x0, y0, x1, y1)`` (whole image by default).  ``amb`` /
    ``amb_c`` report the pairs within ``eta`` (relative to the magnitude of
    the terms of q) of the support cutoff, widened by the effect of a centre
    rounded to float32 relative to a point within ``pos_h`` pixels;
    ``abs_den`` is |w_B| + sum |a|."""
    pk = _Packed(scene, cam, settings)
    x0, y0, x1, y1 = _window(cam, crop)
    h, w = max(y1 - y0, 0), max(x1 - x0, 0)
    Cimg = np.zeros((h, w, 3))
    num = np.zeros((h, w, 3))
    den = np.zeros((h, w))
    amb = np.zeros((h, w))
    ambc = np.zeros((h, w))
    absden = np.zeros((h, w))
    cnt = np.zeros((h, w), dtype=np.int64)
    _load().ora_render(C.byref(pk.scene), C.byref(pk.cam), C.byref(pk.params), x0, y0, x1, y1,
                       {"strict": 0, "aabb": 1}[mode], float(eta), float(pos_h), _ptr(Cimg), _ptr(num),
                       _ptr(den), _ptr(amb), _ptr(ambc), _ptr(absden), _ptr(cnt))
    return {"C": Cimg, "num": num, "den": den, "amb": amb, "amb_c": ambc, "abs_den": absden, "count": cnt}


def render_sorted(scene, cam, settings, crop=None, alpha_max: float = 0.99, alpha_min: float = 0.0,
                  t_min: float = 0.0, eta: float = 1e-6, pos_h: float = 0.0) -> dict:
    """Sorted alpha blending (Eq. 6) of the same splats, front to back by
    camera depth, alpha = min(alpha_max, u exp(-q/2)) with u the opacity (no
    depth weight), layers below alpha_min skipped, composition stopped once
    the transmittance falls below t_min, background c_B behind.  Returns the
    colour, the final transmittance and the per-pixel sum of alpha over
    layers within the window of ``render`` of the support cutoff."""
    pk = _Packed(scene, cam, settings)
    x0, y0, x1, y1 = _window(cam, crop)
    h, w = max(y1 - y0, 0), max(x1 - x0, 0)
    out = {"C": np.zeros((h, w, 3)), "T": np.zeros((h, w)), "amb": np.zeros((h, w))}
    _load().ora_render_sorted(C.byref(pk.scene), C.byref(pk.cam), C.byref(pk.params), x0, y0, x1, y1,
                              float(alpha_max), float(alpha_min), float(t_min), float(eta), float(pos_h),
                              _ptr(out["C"]),
                              _ptr(out["T"]), _ptr(out["amb"]))
    return out


def render_bwd(scene, cam, settings, dL_dC, crop=None) -> dict:
    """Gradient of L with respect to every scene input and the global
    parameters, given dL/dC over the window (chain rule through Eqs. 3-11)."""
    pk = _Packed(scene, cam, settings)
    x0, y0, x1, y1 = _window(cam, crop)
    g = _f64(dL_dC)
    assert g.shape == (max(y1 - y0, 0), max(x1 - x0, 0), 3)
    n, K = pk.n, pk.K
    out = {
        "means": np.zeros((3, n)), "log_scales": np.zeros((3, n)), "quats": np.zeros((4, n)),
        "sh": np.zeros((K, n, 4)), "opacity_logit": np.zeros(n), "lc_v": np.zeros(n),
        "globals": np.zeros(6), "grad2d": np.zeros((n, 9)),
    }
    _load().ora_render_bwd(C.byref(pk.scene), C.byref(pk.cam), C.byref(pk.params), x0, y0, x1, y1,
                           _ptr(g), _ptr(out["means"]), _ptr(out["log_scales"]), _ptr(out["quats"]),
                           _ptr(out["sh"]), _ptr(out["opacity_logit"]), _ptr(out["lc_v"]),
                           _ptr(out["globals"]), _ptr(out["grad2d"]))
    return out


def render_bwd_views(scene, cams, settings, grads, crops=None) -> dict:
    """Sum of the per-view gradients (the loss is a sum over views)."""
    total = None
    for v, cam in enumerate(cams):
        r = render_bwd(scene, cam, settings, grads[v], None if crops is None else crops[v])
        r.pop("grad2d")
        if total is None:
            total = r
        else:
            for k in total:
                total[k] += r[k]
    return total


def sh_basis(dirs, degree: int = 3) -> np.ndarray:
    """Real SH basis values [m][16] at unit directions [m][3]."""
    d = _f64(dirs).reshape(-1, 3)
    out = np.zeros((d.shape[0], 16))
    _load().ora_sh_basis(_ptr(d), d.shape[0], int(degree), _ptr(out))
    return out


def quat_to_rot(quats) -> np.ndarray:
    """Rotation matrices [m][3][3] of quaternions [m][4] in (w, x, y, z) order."""
    q = _f64(quats).reshape(-1, 4)
    out = np.zeros((q.shape[0], 3, 3))
    _load().ora_quat_to_rot(_ptr(q), q.shape[0], _ptr(out))
    return out
