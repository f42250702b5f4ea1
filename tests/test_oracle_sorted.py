"""Pins of the sorted alpha-blending reference (Eq. 6, the baseline renderer
the method removes the sort from).  The per-layer opacity is taken from the
weighted-sum reference (with the DIR weight and w_B = 1 its denominator is
1 + u exp(-q/2)), so the compositing is checked against an independently
computed amplitude: one layer, two layers in both depth orders, input-order
invariance, the alpha clamp, the alpha skip and the early stop."""
import numpy as np

import oracle
import wsr_synth as ws
from tests.oracle_helpers import SQRT_PI, dc_for_colour, scene_from

CAM = ws.look_at_camera((0.0, 0.0, -4.0), 32, 32)
ST = ws.Settings(weight_kind="dir", opacity_mode="logit", w_bg=1.0, bg=(0.2, 0.4, 0.6))
BG = np.array(ST.bg)


def _scene(points, colours, logits, log_s=-2.0):
    sh = np.zeros((1, len(points), 4))
    sh[0, :, :3] = dc_for_colour(colours)
    return scene_from(points, log_scales=np.full(len(points), log_s), sh=sh, logit=np.asarray(logits, float))


def _alpha_and_colour(points, colours, logits, k, alpha_max=0.99):
    """Layer k alone: alpha from the weighted-sum reference, colour from the
    projection."""
    sc = _scene([points[k]], [colours[k]], [logits[k]])
    a = oracle.render(sc, CAM, ST)["den"] - 1.0
    rgb = oracle.project(sc, CAM, ST)["rgb"][0]
    return np.minimum(a, alpha_max)[..., None], rgb


def test_single_layer_over_background():
    pts, cols, lg = [(0.1, -0.05, 0.0)], [(0.9, 0.3, 0.1)], [1.2]
    a, c = _alpha_and_colour(pts, cols, lg, 0)
    out = oracle.render_sorted(_scene(pts, cols, lg), CAM, ST)
    assert np.abs(out["C"] - (c * a + (1 - a) * BG)).max() < 1e-13
    assert np.abs(out["T"] - (1 - a[..., 0])).max() < 1e-13
    assert a.max() > 0.3


def test_ambiguity_report_of_a_single_layer():
    """The report sums the alpha of layers whose support decision is within
    rounding of the cutoff: with one layer, every reported pixel inside the
    support carries exactly that layer's alpha, 1 - T; pixels far from the
    cutoff carry nothing."""
    pts, cols, lg = [(0.1, -0.05, 0.0)], [(0.9, 0.3, 0.1)], [1.2]
    out = oracle.render_sorted(_scene(pts, cols, lg, log_s=-1.0), CAM, ST, eta=0.05)
    m = (out["amb"] > 0) & (out["T"] < 1.0)
    assert m.sum() > 5
    np.testing.assert_allclose(out["amb"][m], 1.0 - out["T"][m], rtol=1e-12)
    centre = out["T"] == out["T"].min()
    assert (out["amb"][centre] == 0).all()


def test_two_layers_in_depth_order():
    cols, lg = [(0.9, 0.1, 0.1), (0.1, 0.8, 0.2)], [0.5, 2.0]
    for z_front in (-0.5, 0.5):           # swap which Gaussian is nearer the camera (at z = -4)
        pts = [(0.0, 0.0, z_front), (0.05, 0.0, -z_front)]
        a0, c0 = _alpha_and_colour(pts, cols, lg, 0)
        a1, c1 = _alpha_and_colour(pts, cols, lg, 1)
        (af, cf), (ab, cb) = ((a0, c0), (a1, c1)) if z_front < 0 else ((a1, c1), (a0, c0))
        expect = cf * af + cb * ab * (1 - af) + (1 - af) * (1 - ab) * BG
        out = oracle.render_sorted(_scene(pts, cols, lg), CAM, ST)
        assert np.abs(out["C"] - expect).max() < 1e-13
    # the order matters: the two depth orders give different images
    o1 = oracle.render_sorted(_scene([(0, 0, -0.5), (0.05, 0, 0.5)], cols, lg), CAM, ST)["C"]
    o2 = oracle.render_sorted(_scene([(0, 0, 0.5), (0.05, 0, -0.5)], cols, lg), CAM, ST)["C"]
    assert np.abs(o1 - o2).max() > 0.05


def test_input_order_does_not_matter():
    sc, _, st = ws.make_scene("c1", n=300)
    st = st.copy(weight_kind="dir")
    cam = ws.look_at_camera((0.0, 0.0, -4.0), 40, 36)
    a = oracle.render_sorted(sc, cam, st)["C"]
    perm = np.random.default_rng(3).permutation(300)
    b = oracle.render_sorted(ws.permute(sc, perm), cam, st)["C"]
    assert np.abs(a - b).max() < 1e-12


def test_alpha_clamp_with_opacity_above_one():
    """SH opacity is not clamped (Eq. 11): u = 1.5 at the centre gives
    alpha = 0.99, the clamp."""
    sh = np.zeros((1, 1, 4))
    sh[0, 0, :3] = dc_for_colour((0.7, 0.7, 0.7))
    sh[0, 0, 3] = (1.5 - 0.5) * 2.0 * SQRT_PI
    sc = scene_from([(0.0, 0.0, 0.0)], log_scales=np.full(1, -1.0), sh=sh)
    st = ST.copy(opacity_mode="sh")
    out = oracle.render_sorted(sc, CAM, st)
    centre = out["C"][16, 16]
    assert np.allclose(centre, 0.99 * 0.7 + 0.01 * BG, rtol=0, atol=1e-12)
    assert abs(out["T"][16, 16] - 0.01) < 1e-12


def test_alpha_skip_and_early_stop():
    cols = [(0.9, 0.2, 0.1), (0.2, 0.9, 0.1), (0.1, 0.2, 0.9)]
    pts = [(0.0, 0.0, -0.3), (0.0, 0.0, 0.0), (0.0, 0.0, 0.3)]
    lg = [3.0, 3.0, 3.0]
    full = oracle.render_sorted(_scene(pts, cols, lg), CAM, ST)
    # early stop: after the layer that takes T below t_min nothing is added
    stop = oracle.render_sorted(_scene(pts, cols, lg), CAM, ST, t_min=0.5)
    two = oracle.render_sorted(_scene(pts[:2], cols[:2], lg[:2]), CAM, ST)
    one = oracle.render_sorted(_scene(pts[:1], cols[:1], lg[:1]), CAM, ST)
    T1 = one["T"]
    # where the first layer alone leaves T < 0.5 the result is that layer's
    # colour plus T times the background, else two layers were composited
    # (the second always takes this stack below 0.5 where the first does not)
    sel = T1 < 0.5
    assert sel.any()
    assert np.abs(stop["C"][sel] - one["C"][sel]).max() < 1e-13
    sel2 = ~sel & (two["T"] < 0.5)
    assert sel2.any()
    assert np.abs(stop["C"][sel2] - two["C"][sel2]).max() < 1e-13
    # alpha skip: a faint layer below alpha_min contributes nothing
    faint = _scene(pts[:2], cols[:2], [3.0, -6.0])
    a_faint, _ = _alpha_and_colour(pts[:2], cols[:2], [3.0, -6.0], 1)
    assert a_faint.max() < 0.003
    skip = oracle.render_sorted(faint, CAM, ST, alpha_min=1.0 / 255.0)
    assert np.abs(skip["C"] - one["C"]).max() < 1e-13
    assert np.abs(full["C"] - one["C"]).max() > 0.01
