"""Training step of the WSR renderer (Sec. 5, implementation details): render
every view, the l1 + 0.2 D-SSIM loss against target images, the backward, and
an Adam update of every attribute and of the global parameters (sigma, beta,
w_B, c_B).  Every stage runs in libwsr.so through the C-ABI; this module
only holds the tensors and calls the entry points in order.

    step = TrainStep(ctx, scene, globals_, targets)
    for it in range(iters):
        loss = step.step()          # DEVICE scalar, no host synchronisation

The learning rates default to those 3D Gaussian Splatting uses for its
attributes (positions 1.6e-4 times the scene extent, log-scales 5e-3,
rotations 1e-3, opacity 5e-2, SH degree 0 2.5e-3 and higher degrees 1/20 of
it); the paper does not state rates for its own parameters, so sigma, beta,
w_B, c_B and the LC weights use 1e-3 (a choice of this implementation).
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from .render import WSRContext


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Loss:
    """l1 + lambda D-SSIM loss of concatenated images against targets."""

    def __init__(self, cams: list, lam: float = 0.2, device="cuda"):
        self.lib = _lib.load()
        self.cams_c = _lib.make_cameras(cams)
        self.nv = len(cams)
        self.lam = float(lam)
        nbytes = self.lib.wsr_loss_workspace_bytes(self.cams_c, self.nv)
        if nbytes < 0:
            raise ValueError("invalid cameras for the loss")
        self.ws = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        self.value = torch.empty((1,), dtype=torch.float32, device=device)

    def __call__(self, img: torch.Tensor, target: torch.Tensor, dL: torch.Tensor | None = None):
        if dL is None:
            dL = torch.empty_like(img)
        st = self.lib.wsr_loss(self.cams_c, self.nv, _ptr(img), _ptr(target), C.c_float(self.lam), _ptr(self.ws),
                               self.ws.numel(), _ptr(self.value), _ptr(dL), _stream())
        _lib.check("wsr_loss", st)
        return self.value, dL


def loss_noalloc(cams_c, n_views: int, img: torch.Tensor, target: torch.Tensor, lam: float, loss: torch.Tensor,
                 dL: torch.Tensor) -> None:
    """wsr_loss_noalloc: the loss and its gradient into the caller's ``loss``
    [1] and ``dL`` [P][3], with the library's static workspace (nothing is
    allocated)."""
    lib = _lib.load()
    st = lib.wsr_loss_noalloc(cams_c, int(n_views), _ptr(img), _ptr(target), C.c_float(lam), _ptr(loss), _ptr(dL),
                              _stream())
    _lib.check("wsr_loss_noalloc", st)


def adam_(param: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int, lr: float,
          beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15) -> None:
    """In-place Adam update of a contiguous float32 device tensor."""
    for t in (param, grad, m, v):
        if t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError("adam_ needs contiguous float32 tensors")
    lib = _lib.load()
    st = lib.wsr_adam(_ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(), int(step), C.c_float(lr),
                      C.c_float(beta1), C.c_float(beta2), C.c_float(eps), _stream())
    _lib.check("wsr_adam", st)


def default_lrs(extent: float = 1.0) -> dict:
    return {"means": 1.6e-4 * extent, "log_scales": 5e-3, "quats": 1e-3, "opacity_logit": 5e-2,
            "sh0": 2.5e-3, "shN": 2.5e-3 / 20.0, "lc_v": 1e-3, "globals": 1e-3}


class TrainStep:
    """One optimisation step over all views of ``ctx``: forward, loss,
    backward, Adam.  ``scene`` holds float32 device tensors that are updated
    in place; ``targets`` is the concatenated [P][3] target image.

    With ``fused`` (the default) the per-Gaussian parameters take their Adam
    step inside the projection backward (wsr_project_bwd_adam), and only the
    six global parameters go through wsr_adam; otherwise the backward writes
    every gradient and wsr_adam updates each parameter group.  Both give the
    same bits."""

    BETA1, BETA2, EPS = 0.9, 0.999, 1e-15

    def __init__(self, ctx: WSRContext, scene: dict, globals_: torch.Tensor, targets: torch.Tensor,
                 lrs: dict | None = None, lam: float = 0.2, grow: bool = True, fused: bool = True):
        for k in ("means", "log_scales", "quats", "sh"):
            if scene[k].dtype != torch.float32:
                raise ValueError("training needs float32 attribute storage")
        self.ctx, self.scene, self.globals_, self.targets = ctx, scene, globals_, targets
        self.lrs = dict(default_lrs(), **(lrs or {}))
        self.loss = Loss(ctx.cams, lam, device=ctx.device)
        self.grads = ctx.alloc_grads(scene)
        # Adam's moments, laid out like the gradients
        self.m = {k: torch.zeros_like(t) for k, t in self.grads.items()}
        self.v = {k: torch.zeros_like(t) for k, t in self.grads.items()}
        self.grow = grow
        self.fused = fused
        self.it = 0
        self._groups = []   # (param view, grad view, lr key, m view, v view)
        for key, p, field, sl in (("means", scene["means"], "means", None),
                                  ("log_scales", scene["log_scales"], "log_scales", None),
                                  ("quats", scene["quats"], "quats", None),
                                  ("opacity_logit", scene["opacity_logit"], "opacity_logit", None),
                                  ("lc_v", scene["lc_v"], "lc_v", None),
                                  ("sh0", scene["sh"][0], "sh", 0),
                                  ("shN", scene["sh"][1:], "sh", slice(1, None)),
                                  ("globals", globals_, "globals", None)):
            if p.numel() == 0:
                continue
            pick = (lambda t: t) if sl is None else (lambda t, sl=sl: t[sl])
            self._groups.append((p, pick(self.grads[field]), key, pick(self.m[field]), pick(self.v[field])))
        self.dL = torch.empty((ctx.total_pixels, 3), dtype=torch.float32, device=ctx.device)

    def adam_params(self, step: int) -> _lib.WsrAdamParams:
        lr = self.lrs
        return _lib.WsrAdamParams(lr["means"], lr["log_scales"], lr["quats"], lr["sh0"], lr["shN"],
                                  lr["opacity_logit"], lr["lc_v"], self.BETA1, self.BETA2, self.EPS, int(step), 0)

    def step(self) -> torch.Tensor:
        ctx = self.ctx
        ctx.project(self.scene, self.globals_)
        ctx.bin(grow=self.grow)
        rgb, den = ctx.render_fwd(self.globals_)
        value, _ = self.loss(rgb, self.targets, self.dL)
        self.it += 1
        if self.fused:
            ctx.raster_bwd(self.globals_, self.dL, rgb, den)
            ctx.project_bwd_adam(self.scene, self.globals_, self.m, self.v, self.adam_params(self.it),
                                 self.grads["globals"])
            adam_(self.globals_, self.grads["globals"], self.m["globals"], self.v["globals"], self.it,
                  self.lrs["globals"], self.BETA1, self.BETA2, self.EPS)
        else:
            ctx.render_bwd(self.scene, self.globals_, self.dL, rgb, den, grads=self.grads)
            for p, g, key, m, v in self._groups:
                adam_(p, g, m, v, self.it, self.lrs[key], self.BETA1, self.BETA2, self.EPS)
        return value
