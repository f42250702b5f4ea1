"""Helpers for the GPU parity tests: run the HIP path through the C-ABI
binding and compare with the FP64 checker."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
import wsr_synth as ws
from paper_2410_18931_amd import WSRContext, globals_tensor, scene_to_device

IMG_TOL = 1e-4      # max-abs on [0, 1] colours
GRAD_TOL = 1e-3     # per tensor: max |g_gpu - g_ref| <= GRAD_TOL * max |g_ref|
AMB_ETA = 1e-6      # pairs with |q - tau| <= AMB_ETA * (A dx^2 + 2|B dx dy| + C dy^2) may flip in float32
ILL_COND = 10.0     # (|w_B| + sum|a|) / |den| above this: ill-conditioned pixel, counted not gated


def amb_kw(settings) -> dict:
    """The checker's ambiguity window for the kernels' arithmetic: the
    rounding of q (AMB_ETA of the magnitude of its terms) plus that of the
    splat centre, which the kernels form in float32 relative to the tile's
    centre, so within half a tile of every pixel centre they evaluate."""
    return {"eta": AMB_ETA, "pos_h": settings.tile / 2}


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_forward(scene, cams, settings, storage="f32", count=False, capacity=None):
    ctx = WSRContext(scene["means"].shape[1], cams, settings, capacity=capacity)
    dev = scene_to_device(scene, storage=storage)
    g = globals_tensor(settings)
    out = ctx.forward(dev, g, count=count)
    torch.cuda.synchronize()
    ctx.check()
    return ctx, dev, g, out


def to_views(ctx, t):
    return [v.detach().cpu().numpy() for v in ctx.views(t)]


def compare_image(C_gpu, ref, tol=IMG_TOL, label="", max_amb_frac=0.02):
    """Max-abs comparison that accounts for pairs whose support decision is
    within float32 rounding of the cutoff (the reference reports, per pixel,
    the sum over such pairs of |a| * max|rgb - C|): those pixels may differ by
    up to 2 * that sum / |den| more.  Pixels whose denominator cancels
    ((|w_B| + sum|a|) / |den| > ILL_COND) are counted, not gated.  At most
    max_amb_frac of the pixels may hold such a pair (a wider window would
    hide errors).  Returns a dict of statistics."""
    C_ref, den = ref["C"], ref["den"]
    err = np.abs(C_gpu.astype(np.float64) - C_ref).max(axis=-1)
    zero = den == 0
    cond = np.where(zero, 1.0, ref["abs_den"] / np.where(zero, 1.0, np.abs(den)))
    ill = cond > ILL_COND
    amb = ref["amb_c"] > 0
    bound = tol + 2.0 * ref["amb_c"] / np.where(zero, 1.0, np.abs(den))
    clean = ~amb & ~ill
    ok = ~ill
    st = {
        "max_err_clean": float(err[clean].max()) if clean.any() else 0.0,
        "max_err_all": float(err[ok].max()) if ok.any() else 0.0,
        "ambiguous_px": int(amb.sum()), "ill_px": int(ill.sum()), "px": int(err.size),
        "over_bound": int((err[ok] > bound[ok]).sum()),
    }
    log(f"[image {label}] {st}")
    assert st["max_err_clean"] <= tol, st
    assert st["over_bound"] == 0, st
    assert st["ill_px"] <= max(2, 0.001 * err.size), st
    assert st["ambiguous_px"] <= max(20, max_amb_frac * err.size), st
    return st


def compare_grads(g_gpu: dict, g_ref: dict, keys, tol=GRAD_TOL, label=""):
    for k in keys:
        a = np.asarray(g_gpu[k], dtype=np.float64)
        b = np.asarray(g_ref[k], dtype=np.float64)
        assert a.shape == b.shape, (k, a.shape, b.shape)
        scale = np.abs(b).max()
        e = np.abs(a - b).ravel()
        err = e.max() if e.size else 0.0
        # per-element statistics: error of each element relative to the
        # tensor's max |ref|, and relative to its own |ref| where that is at
        # least 1e-2 of the max (smaller elements cancel)
        rel = e / max(scale, 1e-30)
        big = np.abs(b).ravel() >= 1e-2 * scale
        own = e[big] / np.abs(b).ravel()[big] if big.any() else np.zeros(1)
        log(f"[grad {label}] {k}: max|ref|={scale:.4g} max|err|={err:.4g} rel={err / max(scale, 1e-30):.3g} "
            f"p50/p99 of err/max|ref| {np.percentile(rel, 50):.2g}/{np.percentile(rel, 99):.2g}, "
            f"p50/p99/max of err/|ref| (|ref| >= 1e-2 max) {np.percentile(own, 50):.2g}/"
            f"{np.percentile(own, 99):.2g}/{own.max():.2g}")
        if scale == 0.0:
            assert err <= 1e-6, (k, err)
        else:
            assert err <= tol * scale, (k, err, scale)


def unambiguous(ref) -> np.ndarray:
    """[H][W][1] mask, 0 on the pixels where the reference reports a pair
    within float32 rounding of the support cutoff.  There either support
    decision is correct, and a flipped pair changes the gradients of that
    pixel's Gaussians by up to its whole term; an upstream gradient of zero
    there takes those pixels out of the comparison on both sides."""
    return (ref["amb_c"] == 0)[..., None].astype(np.float32)


def seeded_normal_like(t: torch.Tensor, seed: int) -> torch.Tensor:
    """Standard normal values of ``t``'s shape from a seeded numpy generator
    (the same numbers on every run, whatever ran before), on ``t``'s device."""
    r = np.random.default_rng([int(seed), 4321]).standard_normal(tuple(t.shape)).astype(np.float32)
    return torch.from_numpy(r).to(t.device)


def grads_to_numpy(g: dict) -> dict:
    return {k: v.detach().cpu().numpy() for k, v in g.items()}


def densest_crop(count_img: np.ndarray, size=64) -> tuple:
    """(x0, y0, x1, y1) of the size x size window with the most pairs."""
    H, W = count_img.shape
    c = np.cumsum(np.cumsum(np.pad(count_img.astype(np.int64), ((1, 0), (1, 0))), 0), 1)
    s = c[size:, size:] - c[:-size, size:] - c[size:, :-size] + c[:-size, :-size]
    y, x = np.unravel_index(np.argmax(s), s.shape)
    return int(x), int(y), int(x) + size, int(y) + size
