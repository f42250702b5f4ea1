"""Small hand-built scenes for the reference-checker pins (CPU only)."""
from __future__ import annotations

import math

import numpy as np

import wsr_synth as ws

SQRT_PI = math.sqrt(math.pi)


def scene_from(means, log_scales=None, quats=None, sh=None, logit=None, lc_v=None,
               dtype=np.float64) -> dict:
    means = np.asarray(means, dtype=np.float64).reshape(-1, 3).T
    n = means.shape[1]
    if log_scales is None:
        log_scales = np.full((3, n), -2.0)
    log_scales = np.asarray(log_scales, dtype=np.float64)
    if log_scales.ndim == 1:
        log_scales = np.repeat(log_scales[None, :], 3, axis=0)
    if quats is None:
        quats = np.zeros((4, n))
        quats[0] = 1.0
    if sh is None:
        sh = np.zeros((1, n, 4))
    if logit is None:
        logit = np.zeros(n)
    if lc_v is None:
        lc_v = np.ones(n)
    return {
        "means": np.ascontiguousarray(means, dtype=dtype),
        "log_scales": np.ascontiguousarray(log_scales, dtype=dtype),
        "quats": np.ascontiguousarray(quats, dtype=dtype),
        "sh": np.ascontiguousarray(sh, dtype=dtype),
        "opacity_logit": np.ascontiguousarray(logit, dtype=dtype),
        "lc_v": np.ascontiguousarray(lc_v, dtype=dtype),
    }


def dc_for_colour(rgb) -> np.ndarray:
    """DC coefficients whose degree-0 colour (basis value 1/(2 sqrt(pi)), plus
    the 0.5 offset) is ``rgb``."""
    return (np.asarray(rgb, dtype=np.float64) - 0.5) * 2.0 * SQRT_PI


def empty_like(scene: dict) -> dict:
    out = {}
    for k, v in scene.items():
        if k == "sh":
            out[k] = np.zeros((v.shape[0], 0, 4), dtype=v.dtype)
        elif v.ndim == 2:
            out[k] = np.zeros((v.shape[0], 0), dtype=v.dtype)
        else:
            out[k] = np.zeros(0, dtype=v.dtype)
    return out


def subset(scene: dict, keep: np.ndarray) -> dict:
    idx = np.nonzero(keep)[0]
    return ws.permute(scene, idx)
