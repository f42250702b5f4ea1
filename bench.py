"""Benchmark: weighted-sum-rendering forward + backward on one MI355X.

One step = one pass of the whole path over one synthetic frame: projection
(+ SH colour/opacity + depth weights), binning, raster forward, raster
backward and projection backward, for 1,000,000 Gaussians (32-blob mixture,
SH degree 3 with view-dependent opacity, linear-correction weights) seen by
one 1920x1080 camera.  Inputs are resident in HBM before timing starts.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--tile 16]
                    [--storage f32|f16|bf16] [--no-cpu-baseline]
                    [--config c4 --graph --autotune --per-view --errors]

Prints one JSON line.  Per-kernel durations come from HIP events recorded on
the stream the kernels run on.
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd frames/s and Gaussian-pixel evals/s at 1M splats 1080p; % HBM peak"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
# algorithmic FP32 work per in-support (pixel, Gaussian) pair: Eq. 7, and
# weighted-blended OIT (Eq. 2), which adds the coverage product
FWD_FLOPS_PER_PAIR = 20
BWD_FLOPS_PER_PAIR = 48
FWD_FLOPS_PER_PAIR_OIT = 23
BWD_FLOPS_PER_PAIR_OIT = 56


def flops_per_pair(kernel: str, oit: bool) -> int:
    if kernel == "raster_fwd":
        return FWD_FLOPS_PER_PAIR_OIT if oit else FWD_FLOPS_PER_PAIR
    return BWD_FLOPS_PER_PAIR_OIT if oit else BWD_FLOPS_PER_PAIR


# HBM traffic of the dominant kernel, from `rocprofv3 --pmc FETCH_SIZE` and
# `--pmc WRITE_SIZE` runs of this benchmark (KiB per dispatch), each scaled by
# what the same counter reads for a plain device copy of known size
# (`--calibrate-copy`).  Valid only for the kernel sources (the raster kernels
# and the constants they are built with) and the workload it was measured on.
TRAFFIC = [
    {"kernel": "raster_bwd", "source": ["raster.hip", "wsr_internal.h"], "source_sha": "6a40cfa509c8bfb9",
     "workload": {"config": "headline", "tile": 16, "storage": "f32", "oit": False, "alpha_cut": 0.0},
     "fetch_kib": 554230.3, "write_kib": 535894.2,
     "fetch_factor": 262157.8 / 524288.0, "write_factor": 524288.0 / 524288.0},
    {"kernel": "raster_bwd", "source": ["raster.hip", "wsr_internal.h"], "source_sha": "6a40cfa509c8bfb9",
     "workload": {"config": "headline", "tile": 16, "storage": "f32", "oit": True, "alpha_cut": 0.0},
     "fetch_kib": 511316.7, "write_kib": 736161.0,
     "fetch_factor": 262157.8 / 524288.0, "write_factor": 524288.0 / 524288.0},
    {"kernel": "raster_bwd", "source": ["raster.hip", "wsr_internal.h"], "source_sha": "6a40cfa509c8bfb9",
     "workload": {"config": "headline", "tile": 16, "storage": "f32", "oit": False, "alpha_cut": 1.0 / 255.0},
     "fetch_kib": 507989.0, "write_kib": 492707.4,
     "fetch_factor": 262157.8 / 524288.0, "write_factor": 524288.0 / 524288.0},
]


def _source_sha(names) -> str:
    """sha256 prefix of the named kernel sources (one name or a list, hashed in order)."""
    h = hashlib.sha256()
    for name in ([names] if isinstance(names, str) else names):
        with open(os.path.join(ROOT, "paper_2410_18931_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_bytes(kernel: str, args) -> float | None:
    for t in TRAFFIC:
        if t["kernel"] != kernel or t["source_sha"] != _source_sha(t["source"]):
            continue
        if any(getattr(args, k) != v for k, v in t["workload"].items()):
            continue
        return t["fetch_kib"] * 1024 / t["fetch_factor"] + t["write_kib"] * 1024 / t["write_factor"]
    return None


def calibrate_copy(mb: int, reps: int = 5) -> None:
    """A plain device copy of `mb` MiB, for scaling the HBM byte counters."""
    import torch
    n = mb * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "reps": reps}))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--config", default="headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="time budget of the CPU baseline sample")
    ap.add_argument("--graph", action="store_true", help="time replays of the whole step captured as one HIP graph")
    ap.add_argument("--batch", type=int, default=0, help="raster records staged per LDS batch (0: default)")
    ap.add_argument("--persistent", action="store_true", help="raster stages as persistent grids")
    ap.add_argument("--autotune", action="store_true",
                    help="pick tile, batch and launch form with the autotuner first (overrides --tile/--batch)")
    ap.add_argument("--per-view", action="store_true",
                    help="also time the plain FP32 path view by view (one fwd+bwd step per view, eager)")
    ap.add_argument("--errors", action="store_true",
                    help="also report image and gradient errors against the FP64 checker on the densest "
                         "64x64 crops of two views (and against the FP32 source with 16-bit storage)")
    ap.add_argument("--oit", action="store_true", help="weighted-blended OIT (Eq. 2) instead of Eq. 7")
    ap.add_argument("--alpha-cut", type=float, default=0.0,
                    help="opacity early-out threshold (0: off); the line then also reports the image error "
                         "against the exact renderer")
    ap.add_argument("--mode", default="render", choices=["render", "train", "sorted"],
                    help="render: forward + backward of the renderer (the headline metric); train: whole "
                         "training steps (forward, l1 + 0.2 D-SSIM loss, backward, Adam); sorted: forward "
                         "only, weighted sum against sorted alpha blending of the same splats")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this size (for scaling HBM byte counters)")
    return ap.parse_args()


def algorithmic_bytes(n: int, pixels: int, storage: str, binned: int, nv: int = 1) -> dict:
    """HBM bytes the method must move per step (SH degree 3 RGBA, LC weights).
    Attributes: means 3, log-scales 3, quaternion 4, SH 16x4 values + v_i."""
    vals = 3 + 3 + 4 + 64
    attr = n * (vals * (4 if storage == "f32" else 2) + 4)
    grads = n * (vals + 1) * 4
    return {
        "project": attr + n * nv * 56,                       # attributes in, 2D record + rect out
        "bin": n * nv * 16 + binned * 4,                     # rects read twice, ids written
        "raster_fwd": n * nv * 48 + pixels * 16,             # 2D records in, colour + denominator out
        "raster_bwd": n * nv * (48 + 36) + pixels * 28,      # 2D records, dL/dC, C, D in; 2D gradients out
        "project_bwd": attr + n * nv * 36 + grads,           # attributes + 2D grads in, grads out
        "step": 2 * attr + grads + pixels * 44,
    }


def cpu_baseline(scene, cams, settings, seconds: float) -> dict:
    """The FP64 reference checker as it stands, on a bounded sample of the
    same frame: full-width strips of 4 rows, visited in a seeded random order,
    forward + backward, until `seconds` have passed (at least one strip);
    frames/s = sampled fraction of the frame / time."""
    import oracle
    cam = cams[0]
    H, W = int(cam["height"]), int(cam["width"])
    h = 4
    order = np.random.default_rng(0).permutation(np.arange(0, H - h + 1, h))
    rng = np.random.default_rng(1)
    done = 0
    t0 = time.perf_counter()
    for y in order:
        crop = (0, int(y), W, int(y) + h)
        oracle.render(scene, cam, settings, crop=crop)
        oracle.render_bwd(scene, cam, settings, rng.standard_normal((h, W, 3)), crop=crop)
        done += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    frac = done * h / H
    return {"value": frac / dt, "unit": "frames/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"FP64 C checker (strict all-pairs mode), forward+backward on {done} full-width strips of "
                      f"{h} rows ({done * h} of {H} rows, seeded random positions) of the same frame, "
                      f"{dt:.1f} s; frames/s = sampled fraction / time"}


def per_view_fp32(scene, cams, settings, args) -> dict:
    """The plain path the batched line is compared with: FP32 attribute
    storage, tile 16, default batch, one fwd+bwd step per view (each view its
    own projection, binning, raster and backward), eager launches; the time
    of one pass over all views."""
    import torch

    from paper_2410_18931_amd import WSRContext, globals_tensor, scene_to_device
    st = settings.copy(tile=16, batch=0, persistent=False)
    n = scene["means"].shape[1]
    dev = scene_to_device(scene, storage="f32")
    g = globals_tensor(st)
    steps = []
    for cam in cams:
        ctx = WSRContext(n, [cam], st)
        ctx.forward(dev, g)
        ctx._alloc_pairs(int(ctx.last_pairs * 1.1) + 1024)
        rgb = torch.empty((ctx.total_pixels, 3), device="cuda")
        den = torch.empty((ctx.total_pixels,), device="cuda")
        dL = torch.randn((ctx.total_pixels, 3), generator=torch.Generator(device="cuda").manual_seed(1),
                         device="cuda")
        grads = ctx.alloc_grads(dev)
        steps.append((ctx, rgb, den, dL, grads))

    def one_pass():
        for ctx, rgb, den, dL, grads in steps:
            ctx.project(dev, g)
            ctx.bin(grow=False)
            ctx.render_fwd(g, out=(rgb, den))
            ctx.render_bwd(dev, g, dL, rgb, den, grads=grads)

    for _ in range(max(1, args.warmup)):
        one_pass()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(1, args.steps // 4)
    e0.record()
    for _ in range(reps):
        one_pass()
    e1.record()
    torch.cuda.synchronize()
    for ctx, *_ in steps:
        ctx.check()
    ms = e0.elapsed_time(e1) / reps
    return {"ms_per_pass": round(ms, 4), "views": len(cams), "views_per_s": round(len(cams) * 1e3 / ms, 2),
            "what": "FP32 storage, tile 16, one eager fwd+bwd step per view"}


def checker_errors(scene, cams, settings, storage: str, ctx, dev, g) -> dict:
    """Image and gradient errors of this line's configuration against the FP64
    checker, on the densest 64x64 crop of two views: images (max-abs over the
    pixels whose support decisions are not within float32 rounding of a
    cutoff, and the count of those), gradients through both crops (max |err|
    relative to the tensor's max |ref|).  With 16-bit storage, against the
    checker on the dequantised inputs (the kernels' arithmetic) and on the
    FP32 source (the storage rounding included)."""
    import torch

    import oracle
    import wsr_synth as ws
    rgb, den, cnt = ctx.forward(dev, g, count=True)
    views = [0, len(cams) // 2] if len(cams) > 1 else [0]
    imgs, counts = ctx.views(rgb), ctx.views(cnt)
    src = {"dequantised": ws.quantise(scene, storage)["f32"], "fp32_source": scene} if storage != "f32" else \
        {"fp32_source": scene}
    crops, dLs = {}, []
    rng = np.random.default_rng(17)
    for v, cam in enumerate(cams):
        r = np.zeros((cam["height"], cam["width"], 3), np.float32)
        if v in views:
            c = counts[v].cpu().numpy()
            H, W = c.shape
            s = 64
            cs = np.cumsum(np.cumsum(np.pad(c.astype(np.int64), ((1, 0), (1, 0))), 0), 1)
            tot = cs[s:, s:] - cs[:-s, s:] - cs[s:, :-s] + cs[:-s, :-s]
            y, x = np.unravel_index(np.argmax(tot), tot.shape)
            crops[v] = (int(x), int(y), int(x) + s, int(y) + s)
            amb = oracle.render(src.get("dequantised", scene), cam, settings, crop=crops[v], eta=1e-6,
                                pos_h=settings.tile / 2)["amb_c"] > 0
            r[y:y + s, x:x + s] = rng.standard_normal((s, s, 3)) * (~amb)[..., None]
        dLs.append(r)
    dL = torch.cat([torch.from_numpy(r.reshape(-1, 3)) for r in dLs]).cuda()
    gg = {k: v.detach().cpu().numpy() for k, v in ctx.render_bwd(dev, g, dL, rgb, den).items()}
    keys = ["means", "log_scales", "quats", "sh"] + (["lc_v"] if settings.weight_kind == "lc" else []) + \
        (["opacity_logit"] if settings.opacity_mode == "logit" else [])
    out = {"crops": {str(v): crops[v] for v in views}}
    for name, sc in src.items():
        print(f"# checker errors: {name}", file=sys.stderr, flush=True)
        img_err, amb_px = 0.0, 0
        for v in views:
            x0, y0, x1, y1 = crops[v]
            ref = oracle.render(sc, cams[v], settings, crop=crops[v], eta=1e-6, pos_h=settings.tile / 2)
            e = np.abs(imgs[v][y0:y1, x0:x1].cpu().numpy().astype(np.float64) - ref["C"]).max(axis=-1)
            clean = ref["amb_c"] == 0
            img_err = max(img_err, float(e[clean].max()))
            amb_px += int((~clean).sum())
        gref = oracle.render_bwd_views(sc, [cams[v] for v in views], settings,
                                       [dLs[v][crops[v][1]:crops[v][3], crops[v][0]:crops[v][2]] for v in views],
                                       [crops[v] for v in views])
        rel = {k: float(np.abs(gg[k] - gref[k]).max() / max(np.abs(gref[k]).max(), 1e-30)) for k in keys}
        out[name] = {"image_max_abs": img_err, "ambiguous_px": amb_px, "grad_rel_to_max": rel,
                     "grad_rel_to_max_worst": max(rel.values())}
    return out


def bench_train(args) -> None:
    """Whole training steps on the workload: forward, loss, backward and Adam
    over every attribute and the global parameters, with the id list sized
    once up front (no per-step host synchronisation)."""
    import torch

    import wsr_synth as ws
    from paper_2410_18931_amd import WSRContext, globals_tensor, scene_to_device
    from paper_2410_18931_amd.train import Loss, TrainStep, adam_

    scene, cams, st = ws.make_scene(args.config)
    st = st.copy(tile=args.tile)
    n = scene["means"].shape[1]
    g = globals_tensor(st)
    ctx = WSRContext(n, cams, st)
    # target images: the same scene with its degree-0 colour shifted, so the
    # loss and every gradient are non-trivial
    tgt = {k: v.copy() for k, v in scene.items()}
    tgt["sh"][0, :, :3] += 0.1
    targets = ctx.forward(scene_to_device(tgt), g)[0].clone()
    ctx._alloc_pairs(int(ctx.last_pairs * 1.3) + 1024)
    dev = scene_to_device(scene)
    trainer = TrainStep(ctx, dev, g.clone(), targets, grow=False)
    for _ in range(args.warmup):
        trainer.step()
    torch.cuda.synchronize()
    ctx.check()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        loss = trainer.step()
    e1.record()
    torch.cuda.synchronize()
    ctx.check()
    ms = e0.elapsed_time(e1) / args.steps
    # the loss and the optimiser on their own (same tensors, same sizes)
    lossf = Loss(cams)
    rgb, _ = ctx.render_fwd(trainer.globals_)
    dL = torch.empty_like(rgb)
    e0.record()
    for _ in range(args.steps):
        lossf(rgb, targets, dL)
    e1.record()
    torch.cuda.synchronize()
    loss_ms = e0.elapsed_time(e1) / args.steps
    # the projection backward with the fused update (the step's own call),
    # and for comparison the plain projection backward followed by Adam on
    # every group (zero learning rates: the scene stays as it is)
    frozen = trainer.adam_params(1000)
    for f in ("lr_means", "lr_log_scales", "lr_quats", "lr_sh0", "lr_shN", "lr_opacity_logit", "lr_lc_v"):
        setattr(frozen, f, 0.0)
    e0.record()
    for _ in range(args.steps):
        ctx.project_bwd_adam(trainer.scene, trainer.globals_, trainer.m, trainer.v, frozen,
                             trainer.grads["globals"])
    e1.record()
    torch.cuda.synchronize()
    fused_ms = e0.elapsed_time(e1) / args.steps
    e0.record()
    for _ in range(args.steps):
        ctx.project_bwd(trainer.scene, trainer.globals_, trainer.grads)
    e1.record()
    torch.cuda.synchronize()
    pbwd_ms = e0.elapsed_time(e1) / args.steps
    e0.record()
    for k in range(args.steps):
        for p_, g_, key, m_, v_ in trainer._groups:
            adam_(p_, g_, m_, v_, 1000 + k, 0.0)
    e1.record()
    torch.cuda.synchronize()
    adam_ms = e0.elapsed_time(e1) / args.steps
    ctx.check()
    out = {
        "metric": "training steps/s (forward, l1 + 0.2 D-SSIM loss, backward, Adam over all attributes) "
                  "at 1M splats 1080p",
        "value": round(1e3 / ms, 3), "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.config}: {n:,} Gaussians, {ctx.nv} view(s), {ctx.total_pixels:,} px, "
                               f"tile {args.tile}, f32, training", "gaussians": n, "views": ctx.nv,
                   "pixels": ctx.total_pixels, "tile": args.tile},
        "stages_ms": {"loss": round(loss_ms, 4), "project_bwd_adam": round(fused_ms, 4)},
        "unfused_ms": {"project_bwd": round(pbwd_ms, 4), "adam_all_groups": round(adam_ms, 4)},
        "final_loss": float(loss.item()),
    }
    # the stage the training step adds to the render step, against HBM: the
    # per-pair partial sums (36 B read per pair, 36 B per (view, Gaussian)
    # written and read back) and, per per-Gaussian parameter, p, m, v read and
    # written (24 B); the raster kernels are those of the render benchmark
    n_params = sum(p_.numel() for p_, _, key, *_ in trainer._groups if key != "globals")
    pairs = ctx.pair_count()
    nbytes = 36.0 * pairs + 72.0 * n * ctx.nv + 24.0 * n_params
    gbs = nbytes / (fused_ms * 1e-3) / 1e9
    out["roofline"] = {"kernel": "projection backward with the fused Adam step (pair sums, chain, update)",
                       "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None, "algorithmic_bytes": nbytes,
                       "parameters": n_params, "launch_ms": round(fused_ms, 4)}
    print(json.dumps(out), flush=True)


def bench_sorted(args) -> None:
    """Forward only: the weighted sum (projection, binning, Eq. 7) against
    sorted alpha blending of the same splats (projection with the DIR
    weight, binning, per-tile depth sort, Eq. 6 front to back), exactly and
    with the usual 3DGS skip / early-stop settings."""
    import torch

    import wsr_synth as ws
    from paper_2410_18931_amd import WSRContext, globals_tensor, scene_to_device

    scene, cams, st = ws.make_scene(args.config)
    st = st.copy(tile=args.tile)
    n = scene["means"].shape[1]
    dev = scene_to_device(scene)
    g = globals_tensor(st)

    def timed(fn, reps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    wsr = WSRContext(n, cams, st)
    wsr.forward(dev, g)
    wsr._alloc_pairs(int(wsr.last_pairs * 1.1) + 1024)
    rgb = torch.empty((wsr.total_pixels, 3), device="cuda")
    den = torch.empty((wsr.total_pixels,), device="cuda")

    def wsr_fwd():
        wsr.project(dev, g)
        wsr.bin(grow=False)
        wsr.render_fwd(g, out=(rgb, den))

    ms_wsr = timed(wsr_fwd, args.steps)
    wsr.check()
    # the weighted-sum raster alone (the dominant kernel of its forward), for
    # the roofline: in-support pairs counted once, untimed
    _, _, cnt = wsr.render_fwd(g, count=True)
    pairs = int(cnt.sum().item())
    ms_raster = timed(lambda: wsr.render_fwd(g, out=(rgb, den)), args.steps)
    sd = WSRContext(n, cams, st.copy(weight_kind="dir"))
    sd.forward(dev, g)
    sd._alloc_pairs(int(sd.last_pairs * 1.1) + 1024)
    T = torch.empty((sd.total_pixels,), device="cuda")
    out = {}
    for name, blend in (("exact", {}), ("3dgs", {"alpha_min": 1.0 / 255.0, "t_min": 1e-4})):
        def sorted_fwd(blend=blend):
            sd.project(dev, g)
            sd.bin(grow=False)
            sd.render_sorted(g, out=(rgb, T), **blend)
        out[name] = timed(sorted_fwd, args.steps)
        sd.check()
    # the depth sort on its own (sorting sorted lists costs the same: bitonic)
    import ctypes as C
    from paper_2410_18931_amd import _lib
    sp = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    ms_sort = timed(lambda: _lib.check("wsr_sort_tiles", sd.lib.wsr_sort_tiles(
        sd.cams_c, sd.nv, C.byref(sd.params), n, C.c_void_p(sd.ws.data_ptr()), sd.ws_bytes,
        C.c_void_p(sd.pairs.data_ptr()), sd.capacity, sp)), args.steps)
    res = {
        "metric": "forward frames/s at 1M splats 1080p: weighted sum (Eq. 7) against sorted alpha blending "
                  "(Eq. 6, per-tile depth sort) of the same splats",
        "value": round(1e3 / ms_wsr, 3), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_wsr, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.config}: {n:,} Gaussians, {wsr.nv} view(s), tile {args.tile}, forward only",
                   "gaussians": n, "pixels": wsr.total_pixels, "tile": args.tile},
        "sorted_exact_ms": round(out["exact"], 4), "sorted_3dgs_ms": round(out["3dgs"], 4),
        "sort_ms": round(ms_sort, 4),
        "speedup_vs_sorted_exact": round(out["exact"] / ms_wsr, 3),
        "speedup_vs_sorted_3dgs": round(out["3dgs"] / ms_wsr, 3),
    }
    achieved = pairs * FWD_FLOPS_PER_PAIR / (ms_raster * 1e-3) / 1e12
    res["roofline"] = {"kernel": "raster_fwd (raster_fwd_kernel)", "bound": "alu", "achieved": round(achieved, 3),
                       "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": None,
                       "flops_per_pair": FWD_FLOPS_PER_PAIR, "launch_ms": round(ms_raster, 4),
                       "in_support_pairs": pairs}
    print(json.dumps(res), flush=True)


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this weighted-sum path is a single-GPU build; sharding "
              "Gaussians over GPUs (one all-reduce of the unnormalised sums) is designed, not implemented",
              file=sys.stderr)
        sys.exit(2)
    if args.mode == "train":
        bench_train(args)
        return
    if args.mode == "sorted":
        bench_sorted(args)
        return

    import torch

    import wsr_synth as ws
    from paper_2410_18931_amd import WSRContext, _lib, globals_tensor, scene_to_device

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    scene, cams, st = ws.make_scene(args.config)
    st = st.copy(tile=args.tile, alpha_cut=args.alpha_cut, oit=args.oit, batch=args.batch,
                 persistent=args.persistent)
    n = scene["means"].shape[1]
    dev = scene_to_device(scene, storage=args.storage)
    g = globals_tensor(st)
    tuned = None
    if args.autotune:
        import tempfile
        from paper_2410_18931_amd.autotune import autotune
        with tempfile.TemporaryDirectory() as tmp:
            tuned = autotune(dev, cams, st, g, reps=5, cache=os.path.join(tmp, "tune.json"))
        st = st.copy(tile=tuned["tile"], batch=tuned["batch"], persistent=tuned["persistent"])
        args.tile = tuned["tile"]
        print(f"# autotune: {tuned}", file=sys.stderr, flush=True)
    ctx = WSRContext(n, cams, st)
    P = ctx.total_pixels
    rgb = torch.empty((P, 3), dtype=torch.float32, device="cuda")
    den = torch.empty((P,), dtype=torch.float32, device="cuda")
    dL = torch.randn((P, 3), generator=torch.Generator(device="cuda").manual_seed(0), device="cuda")
    grads = ctx.alloc_grads(dev)
    sc = ctx.scene_struct(dev)
    gs = _lib.WsrGrads(*(grads[k].data_ptr() for k in ("means", "log_scales", "quats", "sh", "opacity_logit",
                                                       "lc_v", "globals")))
    lib = ctx.lib
    stream = torch.cuda.current_stream()
    sp = C.c_void_p(stream.cuda_stream)
    ptr = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
    wsp = ptr(ctx.ws)

    # size the id list once (untimed), and count the in-support pairs
    ctx.project(dev, g)
    ctx.bin(grow=True)
    _, _, cnt = ctx.render_fwd(g, count=True)
    pairs = int(cnt.sum().item())
    binned = ctx.last_pairs

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        _lib.check("wsr_project", lib.wsr_project(C.byref(sc), ctx.cams_c, ctx.nv, C.byref(ctx.params), ptr(g),
                                                  wsp, ctx.ws_bytes, None, sp))
        if ev:
            ev[1].record(stream)
        _lib.check("wsr_bin", lib.wsr_bin(ctx.cams_c, ctx.nv, C.byref(ctx.params), n, wsp, ctx.ws_bytes,
                                          ptr(ctx.pairs), ctx.capacity, sp))
        if ev:
            ev[2].record(stream)
        _lib.check("wsr_render_fwd", lib.wsr_render_fwd(ctx.cams_c, ctx.nv, C.byref(ctx.params), n, ptr(g), wsp,
                                                        ctx.ws_bytes, ptr(ctx.pairs), ctx.capacity, ptr(rgb),
                                                        ptr(den), None, sp))
        if ev:
            ev[3].record(stream)
        _lib.check("wsr_raster_bwd", lib.wsr_raster_bwd(ctx.cams_c, ctx.nv, C.byref(ctx.params), n, ptr(g), wsp,
                                                        ctx.ws_bytes, ptr(ctx.pairs), ctx.capacity, ptr(dL),
                                                        ptr(rgb), ptr(den), sp))
        if ev:
            ev[4].record(stream)
        _lib.check("wsr_project_bwd", lib.wsr_project_bwd(C.byref(sc), ctx.cams_c, ctx.nv, C.byref(ctx.params),
                                                          ptr(g), wsp, ctx.ws_bytes, ptr(ctx.pairs), ctx.capacity,
                                                          C.byref(gs), None, sp))
        if ev:
            ev[5].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.check()
    print(f"# warmup done: {n} Gaussians, {P} px, {binned} binned pairs, {pairs} in-support pairs", file=sys.stderr,
          flush=True)

    graph_ms = None
    if args.graph:
        from paper_2410_18931_amd.graph import GraphStep
        gstep = GraphStep(ctx, dev, g, dL)
        for _ in range(args.warmup):
            gstep.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            gstep.replay()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - t0) * 1e3 / args.steps
        gstep.check()

    events = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.check()  # the id list did not overflow during timing

    names = ["project", "bin", "raster_fwd", "raster_bwd", "project_bwd"]
    stage_ms = {nm: float(np.mean([ev[j].elapsed_time(ev[j + 1]) for ev in events])) for j, nm in enumerate(names)}
    ms = (t1 - t0) * 1e3 / args.steps
    eager_ms = ms
    if graph_ms is not None:
        ms = graph_ms
    fps = 1e3 / ms * ctx.nv      # views rendered (fwd+bwd) per second
    ab = algorithmic_bytes(n, P, args.storage, binned)
    dominant = max(("raster_fwd", "raster_bwd"), key=lambda s: stage_ms[s])
    fpp = flops_per_pair(dominant, args.oit)
    flops = pairs * fpp
    achieved = flops / (stage_ms[dominant] * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": round(fps, 3), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if args.storage == "f32" else f"{args.storage}-storage/f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {n:,} Gaussians, " + (
                       f"one {cams[0]['width']}x{cams[0]['height']} view" if ctx.nv == 1 else
                       f"{ctx.nv} views of uneven size, {P:,} px in total") +
                       f", tile {args.tile}" + (f", batch {st.batch}" if st.batch else "") +
                       (", persistent raster grids" if st.persistent else "") +
                       f", {args.storage} attribute storage" +
                       (f", opacity early-out at {args.alpha_cut:g}" if args.alpha_cut > 0 else "") +
                       (", weighted-blended OIT (Eq. 2)" if args.oit else "") +
                       (", whole step replayed as one HIP graph" if args.graph else ""),
                   "gaussians": n, "views": ctx.nv, "pixels": P, "tile": args.tile, "storage": args.storage,
                   "graph": bool(args.graph), "batch": st.batch, "persistent": bool(st.persistent)},
        "equivalent_1080p_frames_per_s": round(P / (ms * 1e-3) / 2073600.0, 3),
        "eager_ms_per_step": round(eager_ms, 4),
        "gaussian_pixel_evals_per_s": pairs / (ms * 1e-3),
        "in_support_pairs": pairs, "binned_tile_pairs": binned,
        "hbm_frac_step": ab["step"] / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "stages_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "roofline": {"kernel": f"{dominant} (raster_{'fwd' if dominant == 'raster_fwd' else 'bwd'}_kernel)",
                     "bound": "alu", "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                     "traffic": traffic_bytes(dominant, args),
                     "flops_per_pair": fpp,
                     "launch_ms": round(stage_ms[dominant], 4), "algorithmic_bytes": ab[dominant]},
        "stage_hbm_gbs": {k: round(ab[k] / (stage_ms[k] * 1e-3) / 1e9, 1) for k in names},
    }
    if tuned is not None:
        out["autotune"] = {"tile": tuned["tile"], "batch": tuned["batch"], "persistent": tuned["persistent"],
                           "ms": tuned["ms"]}
    if args.per_view:
        out["per_view_fp32"] = per_view_fp32(scene, cams, st, args)
        out["per_view_fp32"]["speedup_of_this_line"] = round(out["per_view_fp32"]["ms_per_pass"] / ms, 3)
    if args.errors:
        out["errors_vs_checker"] = checker_errors(scene, cams, st, args.storage, ctx, dev, g)
    if args.alpha_cut > 0:
        exact = WSRContext(n, cams, st.copy(alpha_cut=0.0))
        rgb_exact, _ = exact.forward(dev, g)
        rgb_cut, _ = ctx.forward(dev, g)
        diff = (rgb_cut - rgb_exact).abs()
        out["early_out"] = {"alpha_cut": args.alpha_cut, "binned_pairs_exact": exact.last_pairs,
                            "image_err_vs_exact": {"max": diff.max().item(), "mean": diff.mean().item()}}
    if not args.no_cpu_baseline:
        print("# cpu baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(scene, cams, st, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
