"""Seeded synthetic scenes and cameras for the weighted-sum-rendering path.

This module is shared by the tests, the benchmark and the reference checker.
It only draws random numbers and builds look-at cameras; it contains none of
the rendering arithmetic (no projection, no spherical harmonics, no blending).

Layout of a scene (all float32 numpy arrays, planar structure-of-arrays):

    means        [3][N]       Gaussian centres, world space
    log_scales   [3][N]       per-axis log standard deviations
    quats        [4][N]       rotation quaternions, component order (w, x, y, z)
    sh           [K][N][4]    SH coefficients, RGBA interleaved per coefficient,
                              K = (degree+1)^2; the A slot holds the opacity SH
    opacity_logit [N]         logit of the maximum opacity (logit opacity mode)
    lc_v         [N]          per-Gaussian linear-correction weights

A camera is a dict with ``viewmat`` (3x4 float64, world -> camera, +z forward,
+y down), ``fx, fy, cx, cy`` (pixels) and ``width, height``.

The workloads follow the paper's problem statement (3D Gaussians with SH
colour, view-dependent opacity, depth weights) at the sizes of the benchmark
configurations; the real-scene datasets the paper evaluates on are not
available, so these seeded scenes stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Half-range of the DC coefficient draw.  Under an orthonormal real SH basis the
# degree-0 basis value is 1/(2*sqrt(pi)), so a coefficient uniform on
# [-sqrt(pi), sqrt(pi)] plus the 0.5 offset gives a DC colour uniform on [0, 1].
DC_HALF_RANGE = math.sqrt(math.pi)

CONFIG_IDS = {"c1": 1, "c2": 2, "c3": 3, "c4": 4, "headline": 6, "tiny": 7}


def _rng(seed: int, config: str) -> np.random.Generator:
    return np.random.default_rng([int(seed), CONFIG_IDS.get(config, 99)])


def look_at_camera(position, width: int, height: int, fov_y_deg: float = 60.0,
                   target=(0.0, 0.0, 0.0)) -> dict:
    """Pinhole camera at ``position`` looking at ``target`` (+z forward, +y down)."""
    c = np.asarray(position, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - c
    f /= np.linalg.norm(f)
    up = np.array([0.0, -1.0, 0.0])
    if abs(float(np.dot(up, f))) > 0.999:
        up = np.array([0.0, 0.0, 1.0])
    r = np.cross(up, f)
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    rot = np.stack([r, d, f])  # rows: camera x (right), y (down), z (forward)
    trans = -rot @ c
    fy = 0.5 * height / math.tan(math.radians(fov_y_deg) * 0.5)
    # the renderer's camera is float32: hand out exactly representable values
    # so that every consumer sees the same camera
    f32 = lambda x: float(np.float32(x))  # noqa: E731
    return {
        "viewmat": np.concatenate([rot, trans[:, None]], axis=1).astype(np.float32).astype(np.float64),
        "fx": f32(fy), "fy": f32(fy), "cx": f32(0.5 * width), "cy": f32(0.5 * height),
        "width": int(width), "height": int(height),
    }


@dataclass
class Settings:
    """Renderer settings (the paper's weight variants and the readings of the
    points it leaves open).  ``sigma``/``beta`` initial values follow Sec. 4.4."""
    weight_kind: str = "exp"          # "dir" | "exp" | "lc"
    opacity_mode: str = "logit"       # "logit" | "sh"
    sigma: float = 0.1
    beta: float = 0.8
    w_bg: float = 1.0
    bg: tuple = (0.25, 0.5, 0.75)
    tau: float = 9.0                  # support cutoff on the Mahalanobis form q
    dilation: float = 0.3             # added to the 2D covariance diagonal (px^2)
    near: float = 0.2
    opacity_offset: float = 0.5
    tile: int = 16
    alpha_cut: float = 0.0            # opacity early-out threshold (0: off)
    oit: bool = False                 # weighted-blended OIT (Eq. 2) instead of Eq. 7
    batch: int = 0                    # raster records staged per LDS batch (0: the renderer's default)
    persistent: bool = False          # raster stages as persistent grids

    def copy(self, **kw) -> "Settings":
        d = dict(self.__dict__)
        d.update(kw)
        return Settings(**d)


def _quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q.astype(np.float32)


def _sh(rng, n, degree, hi_std, vd_opacity):
    k = (degree + 1) ** 2
    sh = np.zeros((k, n, 4), dtype=np.float32)
    sh[0, :, :] = rng.uniform(-DC_HALF_RANGE, DC_HALF_RANGE, size=(n, 4))
    if k > 1:
        sh[1:, :, :] = rng.normal(0.0, hi_std, size=(k - 1, n, 4))
    if not vd_opacity:
        sh[:, :, 3] = 0.0
    return sh


def make_scene(config: str, seed: int = 0, n: int | None = None) -> tuple[dict, list, Settings]:
    """Return (scene, cameras, settings) for one of the benchmark workloads.

    c1        4,096 Gaussians, 128x128, SH degree 0, logit opacity, EXP weight
    c2        200k Gaussians, 1280x720, SH degree 3, SH opacity, LC weight
    c3        1.2M Gaussians in 32 blobs, 1920x1080, otherwise as c2
    headline  the c3 generator at 1M Gaussians, one 1920x1080 view
    c4        the c3 generator at 1M Gaussians, 16 cameras of uneven size
    tiny      a few Gaussians on a 16x16 image (gradient checks)
    """
    rng = _rng(seed, config)
    if config == "c1":
        n = 4096 if n is None else n
        means = rng.normal(0.0, 1.0, size=(3, n))
        log_s = rng.normal(-3.0, 0.5, size=(3, n))
        quats = _quats(rng, n)
        logit = rng.normal(0.0, 1.0, size=n)
        sh = _sh(rng, n, 0, 0.0, False)
        lc_v = np.full(n, 0.1)
        settings = Settings(weight_kind="exp", opacity_mode="logit", sigma=0.1, beta=0.8)
        cams = [look_at_camera((0.0, 0.0, -4.0), 128, 128)]
    elif config in ("c2", "c3", "headline", "c4"):
        if config == "c2":
            n = 200_000 if n is None else n
            means = rng.normal(0.0, 2.0, size=(3, n))
        else:
            n = (1_200_000 if config == "c3" else 1_000_000) if n is None else n
            centres = rng.normal(0.0, 2.0, size=(32, 3))
            stds = rng.uniform(0.2, 0.6, size=32)
            blob = rng.integers(0, 32, size=n)
            means = (centres[blob] + rng.standard_normal((n, 3)) * stds[blob, None]).T
        log_s = rng.normal(-4.0, 0.7, size=(3, n))
        quats = _quats(rng, n)
        sh = _sh(rng, n, 3, 0.1, True)
        logit = np.zeros(n)
        lc_v = rng.uniform(0.5, 1.5, size=n)
        settings = Settings(weight_kind="lc", opacity_mode="sh", sigma=10.0, beta=0.8)
        if config == "c2":
            cams = [look_at_camera((0.0, 0.0, -4.0), 1280, 720)]
        elif config in ("c3", "headline"):
            cams = [look_at_camera((0.0, 0.0, -4.0), 1920, 1080)]
        else:
            cams = []
            for _ in range(16):
                w = int(rng.integers(640, 1921))
                h = int(round(9 * w / 16))
                u = rng.standard_normal(3)
                u /= np.linalg.norm(u)
                r = rng.uniform(4.0, 6.0)
                cams.append(look_at_camera(u * r, w, h))
    elif config == "tiny":
        n = 6 if n is None else n
        means = rng.normal(0.0, 0.3, size=(3, n))
        log_s = rng.normal(-1.6, 0.3, size=(3, n))
        quats = rng.standard_normal((4, n)).astype(np.float32)  # deliberately unnormalised
        sh = _sh(rng, n, 3, 0.2, True)
        logit = rng.normal(0.0, 1.0, size=n)
        lc_v = rng.uniform(0.5, 1.5, size=n)
        settings = Settings(weight_kind="exp", opacity_mode="sh", tau=1.0e4)
        cams = [look_at_camera((0.3, -0.2, -3.0), 16, 16)]
    else:
        raise ValueError(f"unknown config {config!r}")
    scene = {
        "means": np.ascontiguousarray(means, dtype=np.float32),
        "log_scales": np.ascontiguousarray(log_s, dtype=np.float32),
        "quats": np.ascontiguousarray(quats, dtype=np.float32),
        "sh": np.ascontiguousarray(sh, dtype=np.float32),
        "opacity_logit": np.ascontiguousarray(logit, dtype=np.float32),
        "lc_v": np.ascontiguousarray(lc_v, dtype=np.float32),
    }
    return scene, cams, settings


def sh_degree(scene: dict) -> int:
    k = scene["sh"].shape[0]
    d = int(round(math.sqrt(k))) - 1
    assert (d + 1) ** 2 == k, "SH coefficient count must be a square"
    return d


def upstream_grad(cams: list, seed: int = 0) -> list:
    """Seeded upstream gradient dL/dC ~ N(0, 1), one [H][W][3] array per view."""
    rng = np.random.default_rng([int(seed), 1234])
    return [rng.standard_normal((c["height"], c["width"], 3)).astype(np.float32) for c in cams]


def permute(scene: dict, perm: np.ndarray) -> dict:
    """Reorder the Gaussians of a scene (for order-independence checks)."""
    out = {}
    for k, v in scene.items():
        if k == "sh":
            out[k] = np.ascontiguousarray(v[:, perm, :])
        elif v.ndim == 2:
            out[k] = np.ascontiguousarray(v[:, perm])
        else:
            out[k] = np.ascontiguousarray(v[perm])
    return out


def quantise(scene: dict, dtype: str) -> dict:
    """Round means, log-scales, quaternions and SH to fp16/bf16 (round to
    nearest even) and return the dequantised float32 arrays alongside the raw
    16-bit words: {"f32": scene_dequantised, "bits": {name: uint16 array}}."""
    out = dict(scene)
    bits = {}
    for k in ("means", "log_scales", "quats", "sh"):
        x = np.ascontiguousarray(scene[k], dtype=np.float32)
        if dtype == "f16":
            h = x.astype(np.float16)
            bits[k] = h.view(np.uint16)
            out[k] = h.astype(np.float32)
        elif dtype == "bf16":
            u = x.view(np.uint32).astype(np.uint64)
            rounding = 0x7FFF + ((u >> 16) & 1)
            b = ((u + rounding) >> 16).astype(np.uint16)
            bits[k] = b
            out[k] = (b.astype(np.uint32) << 16).view(np.float32)
        else:
            raise ValueError(dtype)
    return {"f32": out, "bits": bits}
