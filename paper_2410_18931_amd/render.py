"""Torch-facing API of the WSR rasterizer.

PyTorch supplies device memory and the stream; every step of the rendering
path (projection, binning, forward and backward raster, projection backward)
runs in the HIP kernels of libwsr.so, reached through the C-ABI.

    ctx = WSRContext(n, cameras, settings)
    rgb, den = render(scene_tensors, globals_, ctx)     # differentiable
    loss(rgb).backward()

``scene_tensors`` holds device tensors in the planar layouts of ``wsr.h``:
means [3][N], log_scales [3][N], quats [4][N], sh [K][N][4] (float32, float16
or bfloat16 — one dtype for all four), opacity_logit [N] and lc_v [N]
(float32).  ``globals_`` is a float32 device tensor [6] = (sigma, beta, w_B,
c_B rgb).  Images of all views are concatenated: ``rgb`` is [P][3] and
``den`` [P] with P the total pixel count; ``ctx.views(rgb)`` splits them.
"""
from __future__ import annotations

import ctypes as C
import math

import torch

from . import _lib

_STORAGE_OF = {torch.float32: "f32", torch.float16: "f16", torch.bfloat16: "bf16"}


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def globals_tensor(settings, device="cuda") -> torch.Tensor:
    return torch.tensor([settings.sigma, settings.beta, settings.w_bg, *settings.bg],
                        dtype=torch.float32, device=device)


def scene_to_device(scene: dict, device="cuda", storage: str = "f32") -> dict:
    """numpy scene (wsr_synth layout) -> device tensors; ``storage`` picks the
    dtype of means, log-scales, quaternions and SH."""
    dt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[storage]
    out = {}
    for k, v in scene.items():
        t = torch.from_numpy(v).to(device)
        out[k] = t.to(dt) if k in ("means", "log_scales", "quats", "sh") else t.to(torch.float32)
        out[k] = out[k].contiguous()
    return out


class WSRContext:
    """Device workspace and id list for one (Gaussian count, cameras, settings)
    configuration.  One forward/backward pair may be in flight per context."""

    def __init__(self, n: int, cams: list, settings, device="cuda", capacity: int | None = None):
        self.lib = _lib.load()
        self.n = int(n)
        self.cams = list(cams)
        self.settings = settings
        self.device = torch.device(device)
        self.cams_c = _lib.make_cameras(self.cams)
        self.params = _lib.make_params(settings)
        self.nv = len(self.cams)
        if self.nv < 1 or self.nv > _lib.MAX_VIEWS:
            raise ValueError("between 1 and 256 views are supported")
        nbytes = self.lib.wsr_workspace_bytes(self.n, self.cams_c, self.nv, int(settings.tile))
        if nbytes < 0:
            raise ValueError("invalid configuration (Gaussian count, camera sizes or tile)")
        self.ws_bytes = int(nbytes)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.pix_counts = [int(c["width"]) * int(c["height"]) for c in self.cams]
        self.total_pixels = sum(self.pix_counts)
        if capacity is None:
            capacity = max(1 << 16, 4 * self.total_pixels)
        self.pair_bytes = int(self.lib.wsr_pair_bytes())
        self._alloc_pairs(int(capacity))
        self.generation = 0      # bumps on every projection
        self.last_pairs = None

    # ---------------------------------------------------------------- helpers
    def _alloc_pairs(self, capacity: int) -> None:
        """Per-pair buffer (id lists + backward scratch), 256-byte aligned."""
        self.capacity = int(capacity)
        self.pairs = torch.empty(max(self.capacity, 1) * self.pair_bytes, dtype=torch.uint8, device=self.device)

    def views(self, img: torch.Tensor) -> list:
        """Split a concatenated per-pixel tensor into per-view [H][W][...] tensors."""
        out, o = [], 0
        for c, p in zip(self.cams, self.pix_counts):
            out.append(img[o:o + p].reshape(int(c["height"]), int(c["width"]), *img.shape[1:]))
            o += p
        return out

    def scene_struct(self, scene: dict) -> _lib.WsrScene:
        means = scene["means"]
        if means.dim() != 2 or means.shape[0] != 3 or means.shape[1] != self.n:
            raise ValueError("means must be [3][n] for this context")
        storage = _STORAGE_OF[means.dtype]
        for k in ("log_scales", "quats", "sh"):
            if scene[k].dtype != means.dtype or not scene[k].is_contiguous():
                raise ValueError(f"{k} must be contiguous and share the dtype of means")
        K = scene["sh"].shape[0]
        deg = int(round(math.sqrt(K))) - 1
        if (deg + 1) ** 2 != K or scene["sh"].shape[1:] != (self.n, 4):
            raise ValueError("sh must be [K][n][4] with K in {1, 4, 9, 16}")
        return _lib.WsrScene(self.n, deg, _lib.STORAGE[storage], _lib.OPACITY_MODES[self.settings.opacity_mode], 0,
                             means.data_ptr(), scene["log_scales"].data_ptr(), scene["quats"].data_ptr(),
                             scene["sh"].data_ptr(), scene["opacity_logit"].data_ptr(),
                             scene["lc_v"].data_ptr())

    # ---------------------------------------------------------------- steps
    def project(self, scene: dict, globals_: torch.Tensor, out_proj: torch.Tensor | None = None):
        sc = self.scene_struct(scene)
        st = self.lib.wsr_project(C.byref(sc), self.cams_c, self.nv, C.byref(self.params), _ptr(globals_),
                                  _ptr(self.ws), self.ws_bytes, _ptr(out_proj), _stream())
        _lib.check("wsr_project", st)
        self.generation += 1

    def bin(self, grow: bool = True):
        """Bin splats into tiles.  With ``grow`` the pair count is read back
        (one stream sync) and the id list is enlarged and the binning redone
        if it overflowed; without it, an overflow is only recorded in the
        workspace flag (see ``check``)."""
        st = self.lib.wsr_bin(self.cams_c, self.nv, C.byref(self.params), self.n, _ptr(self.ws), self.ws_bytes,
                              _ptr(self.pairs), self.capacity, _stream())
        _lib.check("wsr_bin", st)
        if grow:
            total = self.pair_count()
            self.last_pairs = total
            if total > self.capacity:
                self._alloc_pairs(int(total * 1.25) + 1024)
                st = self.lib.wsr_bin(self.cams_c, self.nv, C.byref(self.params), self.n, _ptr(self.ws),
                                      self.ws_bytes, _ptr(self.pairs), self.capacity, _stream())
                _lib.check("wsr_bin", st)

    def pair_count(self) -> int:
        out = C.c_int64(0)
        _lib.check("wsr_pair_count", self.lib.wsr_pair_count(_ptr(self.ws), self.ws_bytes, C.byref(out), _stream()))
        return int(out.value)

    def check(self) -> None:
        _lib.check("wsr_check", self.lib.wsr_check(_ptr(self.ws), self.ws_bytes, _stream()))

    def render_fwd(self, globals_: torch.Tensor, count: bool = False, out=None, unnormalised: bool = False):
        if out is None:
            rgb = torch.empty((self.total_pixels, 3), dtype=torch.float32, device=self.device)
            den = torch.empty((self.total_pixels,), dtype=torch.float32, device=self.device)
        else:
            rgb, den = out
        cnt = torch.empty((self.total_pixels,), dtype=torch.int32, device=self.device) if count else None
        params = _lib.make_params(self.settings, _lib.FLAG_UNNORMALISED) if unnormalised else self.params
        st = self.lib.wsr_render_fwd(self.cams_c, self.nv, C.byref(params), self.n, _ptr(globals_),
                                     _ptr(self.ws), self.ws_bytes, _ptr(self.pairs), self.capacity,
                                     _ptr(rgb), _ptr(den), _ptr(cnt), _stream())
        _lib.check("wsr_render_fwd", st)
        return (rgb, den, cnt) if count else (rgb, den)

    def render_sorted(self, globals_: torch.Tensor, alpha_max: float = 0.99, alpha_min: float = 0.0,
                      t_min: float = 0.0, out=None):
        """Sorted alpha blending of the binned splats (Eq. 6, the baseline
        without the method): sort every tile list by depth, then composite
        front to back.  The context's settings must use the DIR weight.
        Returns (rgb [P][3], final transmittance [P])."""
        if self.settings.weight_kind != "dir":
            raise ValueError("sorted blending needs weight_kind='dir' (the amplitude must be the opacity)")
        if out is None:
            rgb = torch.empty((self.total_pixels, 3), dtype=torch.float32, device=self.device)
            T = torch.empty((self.total_pixels,), dtype=torch.float32, device=self.device)
        else:
            rgb, T = out
        st = self.lib.wsr_sort_tiles(self.cams_c, self.nv, C.byref(self.params), self.n, _ptr(self.ws),
                                     self.ws_bytes, _ptr(self.pairs), self.capacity, _stream())
        _lib.check("wsr_sort_tiles", st)
        blend = _lib.WsrBlend(float(alpha_max), float(alpha_min), float(t_min), 0)
        st = self.lib.wsr_render_sorted(self.cams_c, self.nv, C.byref(self.params), self.n, _ptr(globals_),
                                        C.byref(blend), _ptr(self.ws), self.ws_bytes, _ptr(self.pairs),
                                        self.capacity, _ptr(rgb), _ptr(T), _stream())
        _lib.check("wsr_render_sorted", st)
        return rgb, T

    def alloc_grads(self, scene: dict) -> dict:
        dev = self.device
        K = scene["sh"].shape[0]
        return {
            "means": torch.empty((3, self.n), dtype=torch.float32, device=dev),
            "log_scales": torch.empty((3, self.n), dtype=torch.float32, device=dev),
            "quats": torch.empty((4, self.n), dtype=torch.float32, device=dev),
            "sh": torch.empty((K, self.n, 4), dtype=torch.float32, device=dev),
            "opacity_logit": torch.empty((self.n,), dtype=torch.float32, device=dev),
            "lc_v": torch.empty((self.n,), dtype=torch.float32, device=dev),
            "globals": torch.empty((6,), dtype=torch.float32, device=dev),
        }

    @staticmethod
    def grads_struct(g: dict) -> _lib.WsrGrads:
        """A wsr_grads struct over the tensors of a gradient-shaped dict (see
        alloc_grads); also the layout of Adam's moments."""
        return _lib.WsrGrads(g["means"].data_ptr(), g["log_scales"].data_ptr(), g["quats"].data_ptr(),
                             g["sh"].data_ptr(), g["opacity_logit"].data_ptr(), g["lc_v"].data_ptr(),
                             g["globals"].data_ptr())

    def render_bwd(self, scene: dict, globals_: torch.Tensor, dL_drgb: torch.Tensor, rgb: torch.Tensor,
                   den: torch.Tensor, grads: dict | None = None, grad2d: torch.Tensor | None = None) -> dict:
        sc = self.scene_struct(scene)
        g = self.alloc_grads(scene) if grads is None else grads
        gs = self.grads_struct(g)
        dL = dL_drgb.contiguous()
        st = self.lib.wsr_render_bwd(C.byref(sc), self.cams_c, self.nv, C.byref(self.params), _ptr(globals_),
                                     _ptr(self.ws), self.ws_bytes, _ptr(self.pairs), self.capacity, _ptr(dL),
                                     _ptr(rgb), _ptr(den), C.byref(gs), _ptr(grad2d), _stream())
        _lib.check("wsr_render_bwd", st)
        return g

    def raster_bwd(self, globals_: torch.Tensor, dL_drgb: torch.Tensor, rgb: torch.Tensor, den: torch.Tensor):
        """wsr_raster_bwd: the per-pair partial 2D gradients (first half of
        render_bwd)."""
        dL = dL_drgb.contiguous()
        st = self.lib.wsr_raster_bwd(self.cams_c, self.nv, C.byref(self.params), self.n, _ptr(globals_),
                                     _ptr(self.ws), self.ws_bytes, _ptr(self.pairs), self.capacity, _ptr(dL),
                                     _ptr(rgb), _ptr(den), _stream())
        _lib.check("wsr_raster_bwd", st)

    def project_bwd(self, scene: dict, globals_: torch.Tensor, grads: dict) -> dict:
        """wsr_project_bwd after raster_bwd: the scene gradients into
        ``grads`` (second half of render_bwd)."""
        sc = self.scene_struct(scene)
        gs = self.grads_struct(grads)
        st = self.lib.wsr_project_bwd(C.byref(sc), self.cams_c, self.nv, C.byref(self.params), _ptr(globals_),
                                      _ptr(self.ws), self.ws_bytes, _ptr(self.pairs), self.capacity, C.byref(gs),
                                      None, _stream())
        _lib.check("wsr_project_bwd", st)
        return grads

    def project_bwd_adam(self, scene: dict, globals_: torch.Tensor, m: dict, v: dict, adam: _lib.WsrAdamParams,
                         grad_globals: torch.Tensor) -> None:
        """wsr_project_bwd_adam after raster_bwd: one Adam step of the
        scene's per-Gaussian float32 tensors in place, moments ``m`` and
        ``v`` shaped like alloc_grads; the global parameters' gradient goes
        to ``grad_globals`` [6]."""
        sc = self.scene_struct(scene)
        ms, vs = self.grads_struct(m), self.grads_struct(v)
        st = self.lib.wsr_project_bwd_adam(C.byref(sc), self.cams_c, self.nv, C.byref(self.params), _ptr(globals_),
                                           _ptr(self.ws), self.ws_bytes, _ptr(self.pairs), self.capacity,
                                           C.byref(ms), C.byref(vs), C.byref(adam), _ptr(grad_globals), None,
                                           _stream())
        _lib.check("wsr_project_bwd_adam", st)

    def forward(self, scene: dict, globals_: torch.Tensor, grow: bool = True, count: bool = False):
        self.project(scene, globals_)
        self.bin(grow=grow)
        return self.render_fwd(globals_, count=count)


_SCENE_KEYS = ("means", "log_scales", "quats", "sh", "opacity_logit", "lc_v")


class _WSRFunction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, ctx: WSRContext, globals_, means, log_scales, quats, sh, opacity_logit, lc_v):
        scene = dict(zip(_SCENE_KEYS, (means, log_scales, quats, sh, opacity_logit, lc_v)))
        rgb, den = ctx.forward(scene, globals_)
        fctx.ctx = ctx
        fctx.generation = ctx.generation
        fctx.save_for_backward(globals_, means, log_scales, quats, sh, opacity_logit, lc_v, rgb, den)
        fctx.mark_non_differentiable(den)
        return rgb, den

    @staticmethod
    def backward(fctx, g_rgb, g_den):
        ctx: WSRContext = fctx.ctx
        globals_, means, log_scales, quats, sh, opacity_logit, lc_v, rgb, den = fctx.saved_tensors
        scene = dict(zip(_SCENE_KEYS, (means, log_scales, quats, sh, opacity_logit, lc_v)))
        if ctx.generation != fctx.generation:
            # the workspace was reused by a later forward: rebuild this one's
            # projection and tile lists (nothing per pair is stored anyway)
            ctx.project(scene, globals_)
            ctx.bin(grow=True)
            fctx.generation = ctx.generation
        if g_rgb is None:
            g_rgb = torch.zeros_like(rgb)
        g = ctx.render_bwd(scene, globals_, g_rgb, rgb, den)
        out = [None, g["globals"]]
        for k, src in zip(_SCENE_KEYS, (means, log_scales, quats, sh, opacity_logit, lc_v)):
            out.append(g[k].to(src.dtype))
        return tuple(out)


def render(scene: dict, globals_: torch.Tensor, ctx: WSRContext):
    """Differentiable weighted sum rendering of every view of ``ctx``.
    Returns (rgb [P][3], den [P]) concatenated over views."""
    return _WSRFunction.apply(ctx, globals_, *(scene[k] for k in _SCENE_KEYS))
