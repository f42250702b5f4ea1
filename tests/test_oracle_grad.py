"""The reference checker's analytic backward, pinned by FP64 central finite
differences of its own forward on tiny scenes, and by identities that follow
from Eq. 7 (homogeneity, colour shift, quaternion scale invariance)."""
import math

import numpy as np
import pytest

import oracle
import wsr_synth as ws
from tests.oracle_helpers import dc_for_colour, scene_from

FD_H = 1e-6


def _loss(scene, cam, st, r, crop=None):
    return float(np.sum(oracle.render(scene, cam, st, crop=crop)["C"] * r))


def _tiny(kind, mode, degree, seed=0, n=6, clamp_case=False):
    sc, cams, st = ws.make_scene("tiny", seed=seed, n=n)
    sc = {k: v.astype(np.float64) for k, v in sc.items()}
    sc["sh"] = sc["sh"][: (degree + 1) ** 2].copy()
    cam = cams[0]
    if clamp_case:
        # one Gaussian far outside the lateral clamp (|tx/tz| ~ 1 > 0.75) but
        # large enough to reach the image
        W, T = cam["viewmat"][:, :3], cam["viewmat"][:, 3]
        t = np.array([3.2, 0.3, 3.2])
        sc["means"][:, 0] = W.T @ (t - T)
        sc["log_scales"][:, 0] = 0.0
    st = st.copy(weight_kind=kind, opacity_mode=mode, sigma={"dir": 0.1, "exp": 0.15, "lc": 6.0}[kind],
                 beta=0.9, w_bg=0.8, bg=(0.25, 0.5, 0.75), tau=1e4)
    return sc, cam, st


CASES = [
    ("dir", "logit", 0), ("exp", "logit", 1), ("lc", "logit", 2),
    ("dir", "sh", 3), ("exp", "sh", 3), ("lc", "sh", 3), ("exp", "sh", 2),
]


@pytest.mark.parametrize("kind,mode,degree", CASES)
def test_backward_matches_central_differences(kind, mode, degree):
    sc, cam, st = _tiny(kind, mode, degree, seed=hash((kind, mode, degree)) % 1000)
    r = np.random.default_rng(11).standard_normal((cam["height"], cam["width"], 3))
    g = oracle.render_bwd(sc, cam, st, r)
    scale = 0.0
    errs = []
    for name in ("means", "log_scales", "quats", "sh", "opacity_logit", "lc_v"):
        if name == "opacity_logit" and mode != "logit":
            continue
        if name == "lc_v" and kind != "lc":
            continue
        arr = sc[name]
        flat = arr.reshape(-1)
        for j in range(flat.size):
            if name == "sh" and mode == "logit" and j % 4 == 3:
                continue
            old = flat[j]
            flat[j] = old + FD_H
            lp = _loss(sc, cam, st, r)
            flat[j] = old - FD_H
            lm = _loss(sc, cam, st, r)
            flat[j] = old
            fd = (lp - lm) / (2 * FD_H)
            an = g[name].reshape(-1)[j]
            errs.append((name, j, fd, an))
            scale = max(scale, abs(fd))
    for idx, field in enumerate(("sigma", "beta", "w_bg")):
        if field == "sigma" and kind == "dir":
            continue
        if field == "beta" and kind != "exp":
            continue
        v = getattr(st, field)
        fd = (_loss(sc, cam, st.copy(**{field: v + FD_H}), r) -
              _loss(sc, cam, st.copy(**{field: v - FD_H}), r)) / (2 * FD_H)
        errs.append((field, 0, fd, g["globals"][idx]))
    for c in range(3):
        bp = list(st.bg)
        bm = list(st.bg)
        bp[c] += FD_H
        bm[c] -= FD_H
        fd = (_loss(sc, cam, st.copy(bg=tuple(bp)), r) - _loss(sc, cam, st.copy(bg=tuple(bm)), r)) / (2 * FD_H)
        errs.append(("bg", c, fd, g["globals"][3 + c]))
    bad = [(nm, j, fd, an) for nm, j, fd, an in errs if abs(fd - an) > 1e-6 * max(1.0, scale)]
    assert not bad, bad[:10]
    # the check is not vacuous
    assert sum(1 for e in errs if abs(e[2]) > 1e-3) > 20


def test_backward_through_jacobian_clamp():
    sc, cam, st = _tiny("exp", "sh", 1, seed=3, clamp_case=True)
    p = oracle.project(sc, cam, st)
    assert abs(p["t"][0, 0] / p["t"][0, 2]) > 1.3 * 0.5 * cam["width"] / cam["fx"]
    r = np.random.default_rng(12).standard_normal((cam["height"], cam["width"], 3))
    g = oracle.render_bwd(sc, cam, st, r)
    for name in ("means", "log_scales", "quats"):
        for j in range(3):
            arr = sc[name]
            old = arr[j, 0]
            arr[j, 0] = old + FD_H
            lp = _loss(sc, cam, st, r)
            arr[j, 0] = old - FD_H
            lm = _loss(sc, cam, st, r)
            arr[j, 0] = old
            fd = (lp - lm) / (2 * FD_H)
            assert abs(fd - g[name][j, 0]) <= 1e-6 * max(1.0, abs(fd)), (name, j, fd, g[name][j, 0])


def test_backward_with_support_cutoff_and_crop():
    """tau = 9 and a crop: the gradient of the crop loss matches differences of
    the crop render (perturbations small enough not to move pixels across the
    cutoff)."""
    sc, cams, st = ws.make_scene("c1", n=300)
    sc = {k: v.astype(np.float64) for k, v in sc.items()}
    cam = cams[0]
    crop = (40, 40, 72, 72)
    r = np.random.default_rng(13).standard_normal((32, 32, 3))
    g = oracle.render_bwd(sc, cam, st, r, crop=crop)
    rng = np.random.default_rng(14)
    checked = 0
    for name in ("means", "log_scales", "opacity_logit"):
        arr = sc[name].reshape(-1)
        nz = np.nonzero(np.abs(g[name].reshape(-1)) > 1e-4)[0]
        for j in rng.choice(nz, size=min(15, nz.size), replace=False):
            h = 1e-7
            old = arr[j]
            arr[j] = old + h
            lp = _loss(sc, cam, st, r, crop)
            arr[j] = old - h
            lm = _loss(sc, cam, st, r, crop)
            arr[j] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[j]
            assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (name, j, fd, an)
            checked += 1
    assert checked > 20


def test_euler_identity_lc_weights_and_background():
    """C is invariant under v_i -> k v_i, w_B -> k w_B, so
    sum_i v_i dL/dv_i + w_B dL/dw_B = 0."""
    sc, cam, st = _tiny("lc", "sh", 2, seed=5, n=10)
    r = np.random.default_rng(15).standard_normal((cam["height"], cam["width"], 3))
    g = oracle.render_bwd(sc, cam, st, r)
    lhs = float(np.dot(sc["lc_v"], g["lc_v"]) + st.w_bg * g["globals"][2])
    assert abs(lhs) < 1e-12 * max(1.0, np.abs(g["lc_v"]).max())
    assert np.abs(g["lc_v"]).max() > 1e-3


def test_euler_identity_amplitudes_in_2d_gradients():
    """Same homogeneity at the per-Gaussian amplitude a_i = u_i w_i:
    sum_i a_i dL/da_i + w_B dL/dw_B = 0."""
    sc, cam, st = _tiny("exp", "sh", 3, seed=6, n=10)
    r = np.random.default_rng(16).standard_normal((cam["height"], cam["width"], 3))
    g = oracle.render_bwd(sc, cam, st, r)
    p = oracle.project(sc, cam, st)
    a = p["u"] * p["w"] * p["visible"]
    lhs = float(np.dot(a, g["grad2d"][:, 8]) + st.w_bg * g["globals"][2])
    assert abs(lhs) < 1e-12 * max(1.0, np.abs(g["grad2d"][:, 8]).max())


def test_colour_shift_identity_in_2d_gradients():
    """rgb_i -> rgb_i + k and c_B -> c_B + k shifts C by k, so per channel
    sum_i dL/drgb_i + dL/dc_B = sum over pixels of dL/dC."""
    sc, cam, st = _tiny("lc", "logit", 1, seed=7, n=10)
    r = np.random.default_rng(17).standard_normal((cam["height"], cam["width"], 3))
    g = oracle.render_bwd(sc, cam, st, r)
    lhs = g["grad2d"][:, 5:8].sum(axis=0) + g["globals"][3:6]
    np.testing.assert_allclose(lhs, r.reshape(-1, 3).sum(axis=0), atol=1e-10)


def test_quaternion_scale_invariance():
    sc, cam, st = _tiny("exp", "sh", 3, seed=8, n=10)
    r = np.random.default_rng(18).standard_normal((cam["height"], cam["width"], 3))
    g = oracle.render_bwd(sc, cam, st, r)
    dots = np.einsum("kn,kn->n", sc["quats"], g["quats"])
    assert np.abs(dots).max() < 1e-12 * max(1.0, np.abs(g["quats"]).max())
    assert np.abs(g["quats"]).max() > 1e-3


def test_background_only_pixels_route_gradient_to_background_colour():
    """w_B = 0 and no coverage: C = c_B, so dL/dc_B = sum of dL/dC there."""
    cam = ws.look_at_camera((0.0, 0.0, -4.0), 8, 8)
    sc = scene_from([[0.0, 0.0, -10.0]])  # behind the camera
    st = ws.Settings(w_bg=0.0)
    r = np.random.default_rng(19).standard_normal((8, 8, 3))
    g = oracle.render_bwd(sc, cam, st, r)
    np.testing.assert_allclose(g["globals"][3:6], r.reshape(-1, 3).sum(0), atol=1e-12)
    assert g["globals"][2] == 0.0
