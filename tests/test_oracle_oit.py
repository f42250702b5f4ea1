"""Pins of the weighted-blended OIT reference (Eq. 2, with c_0 = c_B, the
depth weights of Eqs. 8-10 and alpha_i = u_i exp(-q/2) clamped to [0, 1]):
a brute-force numpy evaluation of Eq. 2, a single layer against the sorted
alpha-blending reference (one layer: both are alpha blending), input-order
invariance, and the backward against central differences."""
import numpy as np
import pytest

import oracle
import wsr_synth as ws
from tests.oracle_helpers import dc_for_colour, scene_from
from tests.test_oracle_grad import FD_H, _tiny


def _brute(sc, cam, st, clamp=True):
    p = oracle.project(sc, cam, st.copy(oit=False))
    H, W = cam["height"], cam["width"]
    ys, xs = np.mgrid[0:H, 0:W]
    num = np.zeros((H, W, 3))
    den = np.zeros((H, W))
    cov = np.ones((H, W))
    for i in np.nonzero(p["visible"])[0]:
        A, B, Cc = p["conic"][i]
        dx, dy = xs + 0.5 - p["mu"][i, 0], ys + 0.5 - p["mu"][i, 1]
        q = A * dx * dx + 2 * B * dx * dy + Cc * dy * dy
        G = np.where(q <= st.tau, np.exp(-0.5 * q), 0.0)
        a = p["u"][i] * p["w"][i] * G
        num += a[..., None] * p["rgb"][i]
        den += a
        cov *= 1.0 - (np.clip(p["u"][i] * G, 0.0, 1.0) if clamp else p["u"][i] * G)
    avg = np.where(den[..., None] != 0, num / np.where(den == 0, 1, den)[..., None], 0.0)
    return cov[..., None] * np.array(st.bg) + (1 - cov[..., None]) * avg


@pytest.mark.parametrize("kind,mode", [("exp", "logit"), ("lc", "sh")])
def test_oit_matches_a_brute_force_evaluation(kind, mode):
    sc, _, st = ws.make_scene("c2" if mode == "sh" else "c1", n=80)
    cam = ws.look_at_camera((0.0, 0.0, -4.0), 30, 26)
    st = st.copy(weight_kind=kind, opacity_mode=mode, tau=1e4, oit=True)
    got = oracle.render(sc, cam, st)["C"]
    assert np.abs(got - _brute(sc, cam, st)).max() < 1e-12
    # it differs from Eq. 7
    assert np.abs(got - oracle.render(sc, cam, st.copy(oit=False))["C"]).max() > 1e-3


def test_opacities_outside_the_unit_interval_are_clamped_in_the_coverage():
    """With the unclamped SH opacity of Sec. 4.3, u can leave [0, 1]; Eq. 2's
    layer opacity alpha = u exp(-q/2) is clamped to [0, 1] in the coverage
    product (the weighted average keeps the raw amplitude)."""
    sc, _, st = ws.make_scene("c2", n=80)
    sc = {k: v.astype(np.float64) for k, v in sc.items()}
    rng = np.random.default_rng(17)
    u_target = np.where(rng.random(80) < 0.6, rng.uniform(1.2, 1.8, 80), rng.uniform(0.2, 0.9, 80))
    u_target[rng.random(80) < 0.1] = -0.2
    sc["sh"][0, :, 3] = dc_for_colour(u_target)     # same basis and offset as the colour
    sc["sh"][1:, :, 3] = 0.0
    cam = ws.look_at_camera((0.0, 0.0, -4.0), 30, 26)
    st = st.copy(weight_kind="lc", opacity_mode="sh", tau=1e4, oit=True)
    u = oracle.project(sc, cam, st)["u"]
    assert (u > 1.0).sum() > 20 and (u < 0.0).any()
    got = oracle.render(sc, cam, st)["C"]
    assert np.abs(got - _brute(sc, cam, st)).max() < 1e-12
    # the box-restricted mode takes the same decisions
    assert np.abs(oracle.render(sc, cam, st, mode="aabb")["C"] - got).max() < 1e-12
    # the clamp matters here: without it the image differs
    assert np.abs(got - _brute(sc, cam, st, clamp=False)).max() > 1e-3


def test_single_layer_is_alpha_blending():
    """With one Gaussian the weighted average is its colour and Eq. 2 is
    alpha blending over the background, as the sorted reference computes."""
    cam = ws.look_at_camera((0.0, 0.0, -4.0), 32, 32)
    sh = np.zeros((1, 1, 4))
    sh[0, 0, :3] = dc_for_colour((0.9, 0.2, 0.4))
    sc = scene_from([(0.05, -0.02, 0.0)], log_scales=np.full(1, -1.5), sh=sh, logit=np.array([0.7]))
    st = ws.Settings(weight_kind="exp", opacity_mode="logit", bg=(0.1, 0.6, 0.3))
    oit = oracle.render(sc, cam, st.copy(oit=True))["C"]
    srt = oracle.render_sorted(sc, cam, st.copy(weight_kind="dir"), alpha_max=1.0)["C"]
    assert np.abs(oit - srt).max() < 1e-13


def test_oit_is_order_independent():
    sc, _, st = ws.make_scene("c1", n=400)
    cam = ws.look_at_camera((0.0, 0.0, -4.0), 40, 30)
    st = st.copy(oit=True)
    a = oracle.render(sc, cam, st)["C"]
    perm = np.random.default_rng(9).permutation(400)
    b = oracle.render(ws.permute(sc, perm), cam, st)["C"]
    assert np.abs(a - b).max() < 1e-12


@pytest.mark.parametrize("kind,mode,degree", [("exp", "logit", 1), ("lc", "sh", 2), ("dir", "sh", 3)])
def test_oit_backward_matches_central_differences(kind, mode, degree):
    sc, cam, st = _tiny(kind, mode, degree, seed=31 + degree)
    st = st.copy(oit=True)
    r = np.random.default_rng(13).standard_normal((cam["height"], cam["width"], 3))
    g = oracle.render_bwd(sc, cam, st, r)

    def loss(s, stt):
        return float(np.sum(oracle.render(s, cam, stt)["C"] * r))

    scale, errs = 0.0, []
    for name in ("means", "log_scales", "quats", "sh", "opacity_logit", "lc_v"):
        if (name == "opacity_logit" and mode != "logit") or (name == "lc_v" and kind != "lc"):
            continue
        flat = sc[name].reshape(-1)
        for j in range(flat.size):
            if name == "sh" and mode == "logit" and j % 4 == 3:
                continue
            old = flat[j]
            flat[j] = old + FD_H
            lp = loss(sc, st)
            flat[j] = old - FD_H
            lm = loss(sc, st)
            flat[j] = old
            fd = (lp - lm) / (2 * FD_H)
            errs.append((name, j, fd, g[name].reshape(-1)[j]))
            scale = max(scale, abs(fd))
    for c in range(3):
        bp, bm = list(st.bg), list(st.bg)
        bp[c] += FD_H
        bm[c] -= FD_H
        fd = (loss(sc, st.copy(bg=tuple(bp))) - loss(sc, st.copy(bg=tuple(bm)))) / (2 * FD_H)
        errs.append(("bg", c, fd, g["globals"][3 + c]))
    if kind == "exp":
        for idx, field in ((0, "sigma"), (1, "beta")):
            v = getattr(st, field)
            fd = (loss(sc, st.copy(**{field: v + FD_H})) - loss(sc, st.copy(**{field: v - FD_H}))) / (2 * FD_H)
            errs.append((field, 0, fd, g["globals"][idx]))
    bad = [e for e in errs if abs(e[2] - e[3]) > 1e-6 * max(1.0, scale)]
    assert not bad, bad[:10]
    assert sum(1 for e in errs if abs(e[2]) > 1e-3) > 20
    assert g["globals"][2] == 0.0          # w_B does not enter Eq. 2
