"""Pins of the opacity early-out (App. D proposes, without specifying it, to
stop evaluating Gaussians of low opacity): a pair contributes only while
u exp(-q/2) >= alpha_cut.  Checked against a brute-force numpy sum of
Eq. 7 with that rule, against removing the Gaussians that can never pass it,
and the backward against central differences away from the cutoffs."""
import numpy as np

import oracle
import wsr_synth as ws

CUT = 0.08


def _brute(sc, cam, st, cut):
    """Eq. 7 summed pair by pair in numpy from the projected quantities, with
    the early-out rule applied to every pair."""
    p = oracle.project(sc, cam, st.copy(alpha_cut=0.0))
    H, W = cam["height"], cam["width"]
    ys, xs = np.mgrid[0:H, 0:W]
    pcx, pcy = xs + 0.5, ys + 0.5
    num = np.zeros((H, W, 3)) + np.array(st.bg) * st.w_bg
    den = np.full((H, W), st.w_bg)
    for i in np.nonzero(p["visible"])[0]:
        A, B, Cc = p["conic"][i]
        dx, dy = pcx - p["mu"][i, 0], pcy - p["mu"][i, 1]
        q = A * dx * dx + 2 * B * dx * dy + Cc * dy * dy
        G = np.exp(-0.5 * q)
        keep = (q <= st.tau) & (p["u"][i] * G >= cut)
        a = np.where(keep, p["u"][i] * p["w"][i] * G, 0.0)
        num += a[..., None] * p["rgb"][i]
        den += a
    return num / den[..., None]


def test_early_out_matches_a_brute_force_pair_sum():
    sc, _, st = ws.make_scene("c1", n=60)
    cam = ws.look_at_camera((0.0, 0.0, -4.0), 28, 22)
    st = st.copy(tau=1e4)                       # the opacity rule alone decides the support
    got = oracle.render(sc, cam, st.copy(alpha_cut=CUT))["C"]
    assert np.abs(got - _brute(sc, cam, st, CUT)).max() < 1e-12
    # and it changes the image
    assert np.abs(got - oracle.render(sc, cam, st)["C"]).max() > 1e-3


def test_gaussians_below_the_cut_drop_out():
    sc, _, st = ws.make_scene("c1", n=300)
    cam = ws.look_at_camera((0.0, 0.0, -4.0), 40, 40)
    u = oracle.project(sc, cam, st)["u"]
    keep = u > 0.4
    assert 0 < keep.sum() < 300
    full = oracle.render(sc, cam, st.copy(alpha_cut=0.4))["C"]
    part = oracle.render(ws.permute(sc, np.nonzero(keep)[0]), cam, st.copy(alpha_cut=0.4))["C"]
    assert np.abs(full - part).max() < 1e-13
    p = oracle.project(sc, cam, st.copy(alpha_cut=0.4))
    assert not p["visible"][~keep].any()
    # the cutoff: 2 ln(u / alpha_cut), capped at tau
    vis = p["visible"]
    assert np.allclose(p["cut"][vis], np.minimum(st.tau, 2 * np.log(u[vis] / 0.4)), rtol=1e-14)


def test_early_out_backward_matches_central_differences():
    sc, cams, st = ws.make_scene("tiny", seed=4, n=5)
    sc = {k: v.astype(np.float64) for k, v in sc.items()}
    cam = cams[0]
    st = st.copy(weight_kind="exp", opacity_mode="logit", tau=1e4, alpha_cut=0.02)
    # no pixel centre lies near a cutoff, so small steps do not cross one
    p = oracle.project(sc, cam, st)
    ys, xs = np.mgrid[0:cam["height"], 0:cam["width"]]
    for i in np.nonzero(p["visible"])[0]:
        A, B, Cc = p["conic"][i]
        dx, dy = xs + 0.5 - p["mu"][i, 0], ys + 0.5 - p["mu"][i, 1]
        q = A * dx * dx + 2 * B * dx * dy + Cc * dy * dy
        assert np.abs(q - p["cut"][i]).min() > 1e-3
    r = np.random.default_rng(2).standard_normal((cam["height"], cam["width"], 3))
    g = oracle.render_bwd(sc, cam, st, r)
    h = 1e-6
    checked = 0
    for name in ("means", "log_scales", "sh", "opacity_logit"):
        flat = sc[name].reshape(-1)
        for j in range(flat.size):
            if name == "sh" and j % 4 == 3:
                continue
            old = flat[j]
            flat[j] = old + h
            lp = float(np.sum(oracle.render(sc, cam, st)["C"] * r))
            flat[j] = old - h
            lm = float(np.sum(oracle.render(sc, cam, st)["C"] * r))
            flat[j] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name].reshape(-1)[j]) <= 1e-6 * max(1.0, abs(fd)), (name, j)
            checked += abs(fd) > 1e-4
    assert checked > 10
