"""GPU tests of the sorted alpha-blending baseline (Eq. 6): per-tile depth
sort and front-to-back composition through the C-ABI, against the FP64
reference, exactly (no skip, no early stop) and with the usual 3D Gaussian
Splatting settings; and the per-tile sort limit."""
import numpy as np
import pytest
import torch

import oracle
import wsr_synth as ws
from paper_2410_18931_amd import WSRContext, _lib, globals_tensor, scene_to_device
from tests.gpu_helpers import amb_kw, IMG_TOL, densest_crop, log, to_views

pytestmark = pytest.mark.gpu


def _sorted_gpu(sc, cams, st, **blend):
    ctx = WSRContext(sc["means"].shape[1], cams, st)
    dev = scene_to_device(sc)
    g = globals_tensor(st)
    ctx.project(dev, g)
    ctx.bin(grow=True)
    rgb, T = ctx.render_sorted(g, **blend)
    torch.cuda.synchronize()
    ctx.check()
    return ctx, rgb, T


def _compare(C_gpu, T_gpu, ref, label):
    """Max-abs error; a layer whose support decision is within float32
    rounding of the cutoff (alpha summed in ``amb``) may flip and move the
    pixel by up to twice its alpha."""
    err = np.abs(C_gpu.astype(np.float64) - ref["C"]).max(axis=-1)
    terr = np.abs(T_gpu.astype(np.float64) - ref["T"])
    bound = IMG_TOL + 2.0 * ref["amb"]
    clean = ref["amb"] == 0
    log(f"{label}: max err clean {err[clean].max() if clean.any() else 0:.3g}, all {err.max():.3g}, "
        f"ambiguous px {int((~clean).sum())} of {err.size}, T err {terr[clean].max() if clean.any() else 0:.3g}")
    assert (err <= bound).all()
    assert (terr[clean] <= IMG_TOL).all()


@pytest.mark.parametrize("blend", [{}, {"alpha_min": 1.0 / 255.0, "t_min": 1e-4}])
def test_c1_sorted_full_frame(blend):
    sc, cams, st = ws.make_scene("c1")
    st = st.copy(weight_kind="dir")
    log(f"case: c1 sorted {blend}")
    ctx, rgb, T = _sorted_gpu(sc, cams, st, **blend)
    ref = oracle.render_sorted(sc, cams[0], st, **amb_kw(st), **blend)
    _compare(to_views(ctx, rgb)[0], to_views(ctx, T)[0], ref, "c1")


def test_c2_sorted_densest_crop():
    sc, cams, st = ws.make_scene("c2")
    st = st.copy(weight_kind="dir")
    log("case: c2 sorted densest crop")
    ctx0 = WSRContext(sc["means"].shape[1], cams, st)
    dev = scene_to_device(sc)
    g = globals_tensor(st)
    _, _, cnt = ctx0.forward(dev, g, count=True)
    x0, y0, x1, y1 = densest_crop(to_views(ctx0, cnt)[0])
    del ctx0
    ctx, rgb, T = _sorted_gpu(sc, cams, st)
    ref = oracle.render_sorted(sc, cams[0], st, crop=(x0, y0, x1, y1), **amb_kw(st))
    _compare(to_views(ctx, rgb)[0][y0:y1, x0:x1], to_views(ctx, T)[0][y0:y1, x0:x1], ref, "c2 crop")


@pytest.mark.parametrize("blend", [{}, {"alpha_min": 1.0 / 255.0, "t_min": 1e-4}])
def test_headline_sorted_densest_crop(blend):
    """1 M Gaussians, one 1080p view, as the benchmark compares them: the
    densest tile lists (up to about 8,000 splats) sorted and composited."""
    sc, cams, st = ws.make_scene("headline")
    st = st.copy(weight_kind="dir")
    log(f"case: headline sorted densest crop {blend}")
    ctx0 = WSRContext(sc["means"].shape[1], cams, st)
    dev = scene_to_device(sc)
    g = globals_tensor(st)
    _, _, cnt = ctx0.forward(dev, g, count=True)
    x0, y0, x1, y1 = densest_crop(to_views(ctx0, cnt)[0])
    del ctx0
    ctx, rgb, T = _sorted_gpu(sc, cams, st, **blend)
    ref = oracle.render_sorted(sc, cams[0], st, crop=(x0, y0, x1, y1), **amb_kw(st), **blend)
    _compare(to_views(ctx, rgb)[0][y0:y1, x0:x1], to_views(ctx, T)[0][y0:y1, x0:x1], ref, "headline crop")


def test_sorted_multi_view_uneven_sizes():
    sc, _, st = ws.make_scene("c1", n=2000)
    st = st.copy(weight_kind="dir", tile=8)
    cams = [ws.look_at_camera((0.0, 0.0, -4.0), 70, 45), ws.look_at_camera((3.0, 0.0, -3.0), 33, 81)]
    log("case: sorted two views")
    ctx, rgb, T = _sorted_gpu(sc, cams, st)
    for v, cam in enumerate(cams):
        ref = oracle.render_sorted(sc, cam, st, **amb_kw(st))
        _compare(to_views(ctx, rgb)[v], to_views(ctx, T)[v], ref, f"view {v}")


def test_c3_sorted_densest_crop_or_limit_reported():
    """The densest configuration (1.2 M Gaussians in 32 blobs, 1080p): every
    tile list either fits the per-tile sort, and the densest crop matches the
    reference, or the limit is reported by wsr_check (never a silently
    unsorted image)."""
    sc, cams, st = ws.make_scene("c3")
    st = st.copy(weight_kind="dir")
    log("case: c3 sorted densest crop")
    ctx0 = WSRContext(sc["means"].shape[1], cams, st)
    dev = scene_to_device(sc)
    g = globals_tensor(st)
    _, _, cnt = ctx0.forward(dev, g, count=True)
    x0, y0, x1, y1 = densest_crop(to_views(ctx0, cnt)[0])
    del ctx0
    ctx = WSRContext(sc["means"].shape[1], cams, st)
    ctx.project(dev, g)
    ctx.bin(grow=True)
    rgb, T = ctx.render_sorted(g)
    try:
        ctx.check()
    except _lib.WsrError as e:
        assert e.status == _lib.WSR_ERR_TILE_LIST
        log(f"c3: a tile list is longer than {_lib.SORT_MAX}: reported")
        return
    ref = oracle.render_sorted(sc, cams[0], st, crop=(x0, y0, x1, y1), **amb_kw(st))
    _compare(to_views(ctx, rgb)[0][y0:y1, x0:x1], to_views(ctx, T)[0][y0:y1, x0:x1], ref, "c3 crop")


def test_tile_list_longer_than_the_sort_limit_is_reported():
    """More small splats than the per-tile sort takes, all at one point, land
    in the same tiles: wsr_check reports the limit."""
    rng = np.random.default_rng(5)
    n = _lib.SORT_MAX + 800
    sc, cams, st = ws.make_scene("c1", n=n)
    sc["means"] = (rng.normal(0, 1e-3, (3, n))).astype(sc["means"].dtype)
    sc["log_scales"] = np.full((3, n), -4.0, dtype=sc["log_scales"].dtype)
    st = st.copy(weight_kind="dir")
    log("case: sort limit")
    ctx = WSRContext(n, cams, st)
    dev = scene_to_device(sc)
    g = globals_tensor(st)
    ctx.project(dev, g)
    ctx.bin(grow=True)
    assert ctx.last_pairs > _lib.SORT_MAX
    ctx.render_sorted(g)
    with pytest.raises(_lib.WsrError) as e:
        ctx.check()
    assert e.value.status == _lib.WSR_ERR_TILE_LIST
    # binning again clears the flag
    ctx.bin(grow=True)
    ctx.check()


def test_backward_after_the_sort_culls_on_its_own():
    """The forward stores each wave's culling masks by list position, and the
    backward reuses them; the per-tile sort moves the entries, so a backward
    that follows it (with the image of a forward on the binned lists) must
    cull again -- the sort clears the masks' flag.  Against the backward on
    the binned lists: only the float summation order may differ."""
    sc, cams, st = ws.make_scene("c1", seed=7)
    st = st.copy(weight_kind="dir")
    log("case: c1, DIR weight, Eq. 7 backward after the sort with the binned lists' forward")
    ctx = WSRContext(sc["means"].shape[1], cams, st)
    dev = scene_to_device(sc)
    g = globals_tensor(st)
    ctx.project(dev, g)
    ctx.bin(grow=True)
    rgb0, den0 = ctx.render_fwd(g)
    dL = torch.from_numpy(ws.upstream_grad(cams, seed=5)[0].reshape(-1, 3)).cuda()
    g0 = {k: v.clone() for k, v in ctx.render_bwd(dev, g, dL, rgb0, den0).items()}
    ctx.render_sorted(g)  # sorts the lists in place; no Eq. 7 forward after it
    g1 = ctx.render_bwd(dev, g, dL, rgb0, den0)
    torch.cuda.synchronize()
    ctx.check()
    for k in g0:
        ref = g0[k].abs().max().item()
        err = (g1[k] - g0[k]).abs().max().item()
        log(f"  {k}: max |after sort - binned| = {err:.3g} of max {ref:.3g}")
        assert err <= 1e-4 * max(ref, 1e-30), k


def test_sorted_lists_still_serve_the_weighted_sum_backward():
    """The per-tile sort reorders the list entries in place; every entry must
    keep its pair's Gaussian-major slot, so that Eq. 7's forward and backward
    run on the sorted lists exactly as on the binned ones.  Eq. 7 is a
    commutative sum (Sec. 4.2): only the float summation order changes."""
    sc, cams, st = ws.make_scene("c1", seed=7)
    st = st.copy(weight_kind="dir")
    log("case: c1, DIR weight, Eq. 7 backward before and after the depth sort")
    ctx = WSRContext(sc["means"].shape[1], cams, st)
    dev = scene_to_device(sc)
    g = globals_tensor(st)
    ctx.project(dev, g)
    ctx.bin(grow=True)
    rgb0, den0 = ctx.render_fwd(g)
    dL = torch.from_numpy(ws.upstream_grad(cams, seed=5)[0].reshape(-1, 3)).cuda()
    g0 = {k: v.clone() for k, v in ctx.render_bwd(dev, g, dL, rgb0, den0).items()}
    ctx.render_sorted(g)
    rgb1, den1 = ctx.render_fwd(g)
    g1 = ctx.render_bwd(dev, g, dL, rgb1, den1)
    torch.cuda.synchronize()
    ctx.check()
    assert (rgb1 - rgb0).abs().max().item() <= 1e-5
    assert ((den1 - den0).abs() / den0.abs()).max().item() <= 1e-5
    for k in g0:
        ref = g0[k].abs().max().item()
        err = (g1[k] - g0[k]).abs().max().item()
        log(f"  {k}: max |sorted - binned| = {err:.3g} of max {ref:.3g}")
        assert err <= 1e-4 * max(ref, 1e-30), k
