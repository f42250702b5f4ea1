"""GPU tests of the opacity early-out (App. D): forward and backward with
alpha_cut > 0 through the C-ABI against the FP64 reference that applies the
same rule, the rule's effect on the work (fewer binned pairs), and its image
error against the exact renderer (reported)."""
import numpy as np
import pytest
import torch

import oracle
import wsr_synth as ws
from tests.gpu_helpers import (amb_kw, compare_grads, compare_image, densest_crop, gpu_forward, grads_to_numpy,
                               log, to_views, unambiguous)
from tests.test_gpu_parity import _check_globals, _grad_keys, _oracle_globals

pytestmark = pytest.mark.gpu

CUT = float(np.float32(1.0 / 255.0))   # as the library holds it (wsr_params.alpha_cut is float32)


@pytest.fixture(scope="module")
def c2():
    return ws.make_scene("c2")


def test_c2_early_out_image(c2):
    sc, cams, st = c2
    log("case: c2 early-out image")
    st_cut = st.copy(alpha_cut=CUT)
    ctx, dev, g, (rgb, den) = gpu_forward(sc, cams, st_cut)
    ref = oracle.render(sc, cams[0], st_cut, mode="aabb", **amb_kw(st_cut))
    compare_image(to_views(ctx, rgb)[0], ref, label="c2 early-out")
    ctx0, _, _, (rgb0, _) = gpu_forward(sc, cams, st)
    log(f"early-out: {ctx.last_pairs} binned pairs vs {ctx0.last_pairs} exact; image max-abs vs exact "
        f"{(rgb - rgb0).abs().max().item():.3g}, mean {(rgb - rgb0).abs().mean().item():.3g}")
    assert ctx.last_pairs < ctx0.last_pairs


def test_c2_early_out_gradients_on_crop(c2):
    sc, cams, st = c2
    log("case: c2 early-out gradients on a crop")
    st_cut = st.copy(alpha_cut=CUT)
    ctx, dev, g, (rgb, den, cnt) = gpu_forward(sc, cams, st_cut, count=True)
    x0, y0, x1, y1 = crop = densest_crop(to_views(ctx, cnt)[0])
    r = np.zeros((720, 1280, 3), np.float32)
    r[y0:y1, x0:x1] = np.random.default_rng(6).standard_normal((y1 - y0, x1 - x0, 3))
    dL = torch.from_numpy(r.reshape(-1, 3)).cuda()
    gg = grads_to_numpy(ctx.render_bwd(dev, g, dL, rgb, den))
    gref = oracle.render_bwd(sc, cams[0], st_cut, r[y0:y1, x0:x1], crop=crop)
    compare_grads(gg, gref, _grad_keys(st_cut, 16), label="c2 early-out crop")
    _check_globals(gg["globals"], _oracle_globals(st_cut, gref["globals"]), "c2 early-out crop")


def test_headline_early_out_densest_crop():
    """1 M Gaussians, one 1080p view, as the benchmark runs the early-out:
    the densest crop's image, and every Gaussian's gradient through it (with
    an upstream gradient of zero on pixels whose support decision is within
    float32 rounding of a cutoff)."""
    sc, cams, st = ws.make_scene("headline")
    st_cut = st.copy(alpha_cut=CUT)
    log("case: headline early-out densest crop")
    ctx, dev, g, (rgb, den, cnt) = gpu_forward(sc, cams, st_cut, count=True)
    x0, y0, x1, y1 = crop = densest_crop(to_views(ctx, cnt)[0])
    ref = oracle.render(sc, cams[0], st_cut, crop=crop, mode="aabb", **amb_kw(st_cut))
    compare_image(to_views(ctx, rgb)[0][y0:y1, x0:x1], ref, label="headline early-out crop")
    r = np.zeros((1080, 1920, 3), np.float32)
    r[y0:y1, x0:x1] = np.random.default_rng(9).standard_normal((y1 - y0, x1 - x0, 3)) * unambiguous(ref)
    gg = grads_to_numpy(ctx.render_bwd(dev, g, torch.from_numpy(r.reshape(-1, 3)).cuda(), rgb, den))
    gref = oracle.render_bwd(sc, cams[0], st_cut, r[y0:y1, x0:x1], crop=crop)
    compare_grads(gg, gref, _grad_keys(st_cut, 16), label="headline early-out crop")
    _check_globals(gg["globals"], _oracle_globals(st_cut, gref["globals"]), "headline early-out crop")


def test_c1_early_out_culls_faint_gaussians():
    """A high threshold removes every Gaussian whose opacity is below it: the
    image equals the exact render of the remaining Gaussians with the same
    threshold."""
    sc, cams, st = ws.make_scene("c1")
    st_cut = st.copy(alpha_cut=0.5)
    log("case: c1 high threshold")
    ctx, dev, g, (rgb, den) = gpu_forward(sc, cams, st_cut)
    ref = oracle.render(sc, cams[0], st_cut, **amb_kw(st_cut))
    compare_image(to_views(ctx, rgb)[0], ref, label="c1 alpha_cut 0.5")
