"""GPU tests of weighted-blended OIT (Eq. 2) through the C-ABI against the
FP64 reference: images (including split tiles at 1080p, whose coverage
products are merged through their logarithms) and gradients."""
import numpy as np
import pytest
import torch

import oracle
import wsr_synth as ws
from tests.gpu_helpers import (amb_kw, compare_grads, compare_image, densest_crop, gpu_forward, grads_to_numpy,
                               log, to_views, unambiguous)
from tests.test_gpu_parity import _check_globals, _grad_keys, _oracle_globals

pytestmark = pytest.mark.gpu


def test_c1_oit_image_and_gradients():
    sc, cams, st = ws.make_scene("c1")
    st = st.copy(oit=True)
    log("case: c1 OIT")
    ctx, dev, g, (rgb, den) = gpu_forward(sc, cams, st)
    ref = oracle.render(sc, cams[0], st, **amb_kw(st))
    compare_image(to_views(ctx, rgb)[0], ref, label="c1 OIT")
    r = np.random.default_rng(3).standard_normal((128, 128, 3)).astype(np.float32)
    gg = grads_to_numpy(ctx.render_bwd(dev, g, torch.from_numpy(r.reshape(-1, 3)).cuda(), rgb, den))
    gref = oracle.render_bwd(sc, cams[0], st, r)
    compare_grads(gg, gref, _grad_keys(st, 1), label="c1 OIT")
    ref_g = _oracle_globals(st, gref["globals"])
    _check_globals(gg["globals"], ref_g, "c1 OIT")
    assert gg["globals"][2] == 0.0


def test_c2_oit_gradients_on_crop():
    sc, cams, st = ws.make_scene("c2")
    st = st.copy(oit=True)
    log("case: c2 OIT gradients on a crop")
    ctx, dev, g, (rgb, den, cnt) = gpu_forward(sc, cams, st, count=True)
    x0, y0, x1, y1 = crop = densest_crop(to_views(ctx, cnt)[0])
    ref = oracle.render(sc, cams[0], st, crop=crop, **amb_kw(st))
    compare_image(to_views(ctx, rgb)[0][y0:y1, x0:x1], ref, label="c2 OIT crop")
    r = np.zeros((720, 1280, 3), np.float32)
    r[y0:y1, x0:x1] = np.random.default_rng(8).standard_normal((y1 - y0, x1 - x0, 3))
    gg = grads_to_numpy(ctx.render_bwd(dev, g, torch.from_numpy(r.reshape(-1, 3)).cuda(), rgb, den))
    gref = oracle.render_bwd(sc, cams[0], st, r[y0:y1, x0:x1], crop=crop)
    compare_grads(gg, gref, _grad_keys(st, 16), label="c2 OIT crop")
    _check_globals(gg["globals"], _oracle_globals(st, gref["globals"]), "c2 OIT crop")


def test_headline_oit_split_tiles():
    """At 1M Gaussians / 1080p the densest tiles are split over several work
    items; their coverage products are combined as summed logarithms."""
    sc, cams, st = ws.make_scene("headline")
    st = st.copy(oit=True)
    log("case: headline OIT")
    ctx, dev, g, (rgb, den, cnt) = gpu_forward(sc, cams, st, count=True)
    C = to_views(ctx, rgb)[0]
    counts = to_views(ctx, cnt)[0]
    crop = densest_crop(counts)
    tiles_pairs = ctx.last_pairs
    log(f"headline OIT: binned pairs {tiles_pairs}, densest crop {crop}")
    refs = []
    for c in (crop, (928, 508, 992, 572)):
        x0, y0, x1, y1 = c
        refs.append(oracle.render(sc, cams[0], st, crop=c, **amb_kw(st)))
        compare_image(C[y0:y1, x0:x1], refs[-1], label=f"headline OIT {c}")
    # gradients through the densest crop
    x0, y0, x1, y1 = crop
    r = np.zeros((1080, 1920, 3), np.float32)
    r[y0:y1, x0:x1] = np.random.default_rng(12).standard_normal((y1 - y0, x1 - x0, 3)) * unambiguous(refs[0])
    gg = grads_to_numpy(ctx.render_bwd(dev, g, torch.from_numpy(r.reshape(-1, 3)).cuda(), rgb, den))
    gref = oracle.render_bwd(sc, cams[0], st, r[y0:y1, x0:x1], crop=crop)
    compare_grads(gg, gref, _grad_keys(st, 16), label="headline OIT crop")
    _check_globals(gg["globals"], _oracle_globals(st, gref["globals"]), "headline OIT crop")
