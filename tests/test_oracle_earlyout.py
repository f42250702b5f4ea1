"""Pins of the opacity early-out (App. D proposes, without specifying it, to
stop evaluating Gaussians of low opacity): a pair contributes only while
u exp(-q/2) >= alpha_cut.  Checked against a brute-force numpy sum of
Eq. 7 with that rule, against removing the Gaussians that can never pass it,
and the backward against central differences away from the cutoffs."""
import numpy as np

import oracle
import wsr_synth as ws
from tests.oracle_helpers import scene_from

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


def test_a_support_flip_from_the_float32_early_out_cutoff_is_reported():
    """The renderer evaluates an early-out cutoff 2 ln(u / alpha_cut) in double
    precision, rounds it to float32 once and multiplies it by a float32
    constant (the scale q carries too).  A Gaussian is chosen (over float32
    logits) whose two roundings move the cutoff by more than half of the
    report's window 2^-23 |cut|; a pixel whose exact q lies between the exact
    and the rounded cutoff, whose decision therefore flips, must be reported
    (with eta = 0 and no centre term, only the cutoff term covers it), and a
    pixel at 1.5 windows from the cutoff must not be.  So the window is
    neither a quarter as wide nor ten times as wide."""
    f32 = np.float32
    k32 = f32(0.72134752044448170)                # log2(e) / 2 as the renderer holds it
    alpha = float(f32(0.05))
    st = ws.Settings(weight_kind="dir", opacity_mode="logit", tau=9.0, alpha_cut=alpha)
    cam = ws.look_at_camera((0.0, 0.0, -4.0), 32, 32)
    px, py = 19, 16

    def cutoffs(logit):
        u = 1.0 / (1.0 + np.exp(-float(logit)))
        cut = 2.0 * np.log(u / alpha)
        eff = float(f32(f32(cut) * k32)) / float(k32)   # what the renderer compares q with
        return cut, eff

    chosen = None
    for logit in f32(np.linspace(-1.5, 3.0, 40001)):
        cut, eff = cutoffs(logit)
        if 0.5 < cut < st.tau and abs(eff - cut) > 0.55 * 2.0 ** -23 * cut:
            chosen = logit
            break
    assert chosen is not None
    cut, eff = cutoffs(chosen)
    win = 2.0 ** -23 * cut

    def scene(ls):
        return scene_from([(0.0, 0.0, 0.0)], log_scales=np.full(1, ls), logit=np.array([chosen]))

    def q_at(ls):
        p = oracle.project(scene(ls), cam, st)
        assert abs(p["cut"][0] - cut) <= 1e-12 * cut
        (A, B, C), (mux, muy) = p["conic"][0], p["mu"][0]
        dx, dy = px + 0.5 - mux, py + 0.5 - muy
        return A * dx * dx + 2 * B * dx * dy + C * dy * dy

    def log_scale_for(target):
        a, b = -4.0, 0.5                          # q falls as the splat grows
        for _ in range(200):
            m = 0.5 * (a + b)
            if q_at(m) > target:
                a = m
            else:
                b = m
        return 0.5 * (a + b)

    flip = log_scale_for(0.5 * (cut + eff))
    q = q_at(flip)
    assert (q <= cut) != (q <= eff)               # the rounded cutoff flips the decision
    assert abs(q - cut) <= win
    far = log_scale_for(cut + 1.5 * win * np.sign(eff - cut))
    assert abs(q_at(far) - cut) > win
    assert oracle.render(scene(flip), cam, st, eta=0.0, pos_h=0.0)["amb"][py, px] > 0
    assert oracle.render(scene(far), cam, st, eta=0.0, pos_h=0.0)["amb"][py, px] == 0
