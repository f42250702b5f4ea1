"""Launch autotuner for the WSR path.

For a scene and a camera set it captures one forward + backward step per
candidate launch configuration as a HIP graph, times replays with HIP events
and keeps the fastest.  The candidates are every tile size (8, 16, 32), every
raster batch the tile size is built for (splat records staged in LDS per
batch: 64 for tile 8; 64, 128, 256 for tile 16; 128, 256 for tile 32) and both
raster launch forms (one workgroup per work item, or a persistent grid).
Results are cached in a JSON file keyed by the problem's shape class:
Gaussian count (rounded to 2 significant digits), number of views, total
pixels (rounded likewise), attribute storage type, SH degree, weight and
opacity modes.
"""
from __future__ import annotations

import json
import math
import os

import torch

from .graph import GraphStep
from .render import WSRContext

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "wsr_autotune.json")
TILES = (8, 16, 32)
BATCHES = {8: (64,), 16: (64, 128, 256), 32: (128, 256)}


def candidates(tiles=TILES, persistent=(False, True)) -> list:
    """(tile, batch, persistent) launch configurations to time."""
    return [(t, b, p) for t in tiles for b in BATCHES[t] for p in persistent]


def config_name(tile: int, batch: int, persistent: bool) -> str:
    return f"{tile}/{batch}/{'persistent' if persistent else 'grid'}"


def _round2(x: int) -> int:
    if x <= 0:
        return 0
    p = 10 ** max(int(math.floor(math.log10(x))) - 1, 0)
    return int(round(x / p) * p)


def shape_key(scene: dict, cams: list, settings) -> str:
    n = scene["means"].shape[1]
    pixels = sum(int(c["width"]) * int(c["height"]) for c in cams)
    dtype = str(scene["means"].dtype).replace("torch.", "")
    deg = int(round(math.sqrt(scene["sh"].shape[0]))) - 1
    return (f"n{_round2(n)}-v{len(cams)}-px{_round2(pixels)}-{dtype}-deg{deg}-"
            f"{settings.weight_kind}-{settings.opacity_mode}")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def autotune(scene: dict, cams: list, settings, globals_: torch.Tensor, dL: torch.Tensor | None = None,
             tiles=TILES, persistent=(False, True), reps: int = 10, cache: str | None = DEFAULT_CACHE,
             force: bool = False) -> dict:
    """Return {"tile", "batch", "persistent": the fastest configuration,
    "ms": {"tile/batch/grid|persistent": ms per fwd+bwd step}, "key": ...}.
    ``scene`` holds device tensors (see ``render.scene_to_device``)."""
    key = shape_key(scene, cams, settings)
    if cache and not force:
        hit = _load(cache).get(key)
        if hit is not None:
            return dict(hit, key=key, cached=True)
    n = scene["means"].shape[1]
    times = {}
    for t, b, p in candidates(tiles, persistent):
        st = settings.copy(tile=t, batch=b, persistent=p)
        ctx = WSRContext(n, cams, st)
        step = GraphStep(ctx, scene, globals_, dL)
        step.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            step.replay()
        e1.record()
        torch.cuda.synchronize()
        step.check()
        times[(t, b, p)] = e0.elapsed_time(e1) / reps
        del step, ctx
    t, b, p = min(times, key=times.get)
    res = {"tile": int(t), "batch": int(b), "persistent": bool(p),
           "ms": {config_name(*k): round(v, 4) for k, v in times.items()}}
    if cache:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        data = _load(cache)
        data[key] = res
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return dict(res, key=key, cached=False)
