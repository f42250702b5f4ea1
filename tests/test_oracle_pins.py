"""Pins of the FP64 reference checker against things other than itself:
library routines (scipy), numerical Jacobians, closed forms, the outcomes the
paper states for its Fig. 3 example, and invariants of Eq. 7."""
import json
import math
import os

import numpy as np
import pytest
import scipy.special as sps
from scipy.spatial.transform import Rotation

import oracle
import wsr_synth as ws
from tests.oracle_helpers import dc_for_colour, empty_like, scene_from, subset

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _real_sh_scipy(l, m, dirs):
    """Real orthonormal SH built from scipy's complex SH (which carry the
    Condon-Shortley phase): m>0 -> sqrt2 (-1)^m Re Y_l^m, m<0 -> sqrt2 (-1)^m Im Y_l^|m|."""
    theta = np.arccos(np.clip(dirs[:, 2], -1, 1))
    phi = np.arctan2(dirs[:, 1], dirs[:, 0])
    if m == 0:
        return sps.sph_harm_y(l, 0, theta, phi).real
    y = sps.sph_harm_y(l, abs(m), theta, phi)
    return math.sqrt(2.0) * (-1) ** m * (y.real if m > 0 else y.imag)


def _unit(rng, m):
    d = rng.standard_normal((m, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


# --------------------------------------------------------------------------
# Spherical harmonics (Sec. 3, Eq. 4; Sec. 4.3, Eq. 11)
# --------------------------------------------------------------------------

def test_sh_basis_matches_scipy_real_sh():
    d = _unit(np.random.default_rng(1), 200)
    Y = oracle.sh_basis(d, 3)
    for l in range(4):
        for m in range(-l, l + 1):
            k = l * l + l + m
            np.testing.assert_allclose(Y[:, k], _real_sh_scipy(l, m, d), rtol=0, atol=1e-13)


def test_sh_basis_orthonormal_by_quadrature():
    x, wq = np.polynomial.legendre.leggauss(12)
    phi = np.arange(24) * (2 * np.pi / 24)
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=-1).reshape(-1, 3)
    w = (wq[:, None] * np.full(phi.shape, 2 * np.pi / 24)[None, :]).reshape(-1)
    Y = oracle.sh_basis(d, 3)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_basis_parity():
    d = _unit(np.random.default_rng(2), 50)
    Yp, Ym = oracle.sh_basis(d, 3), oracle.sh_basis(-d, 3)
    for l in range(4):
        ks = slice(l * l, (l + 1) * (l + 1))
        np.testing.assert_allclose(Ym[:, ks], (-1) ** l * Yp[:, ks], atol=1e-14)


def test_sh_degree_truncation():
    d = _unit(np.random.default_rng(3), 10)
    Y3 = oracle.sh_basis(d, 3)
    for deg in range(3):
        Yd = oracle.sh_basis(d, deg)
        K = (deg + 1) ** 2
        np.testing.assert_array_equal(Yd[:, :K], Y3[:, :K])
        assert np.all(Yd[:, K:] == 0)


# --------------------------------------------------------------------------
# Rotation and EWA projection (Sec. 3, Eqs. 3 and 5)
# --------------------------------------------------------------------------

def test_quaternion_rotation_matches_scipy():
    q = np.random.default_rng(4).standard_normal((100, 4)) * 3.0  # unnormalised
    R = oracle.quat_to_rot(q)
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()  # scipy: scalar last
    np.testing.assert_allclose(R, ref, atol=1e-13)


def _pinhole(cam, t):
    return np.array([cam["fx"] * t[0] / t[2] + cam["cx"], cam["fy"] * t[1] / t[2] + cam["cy"]])


def test_projection_matches_numerical_jacobian():
    """Sigma2D = J W Sigma3D W^T J^T + dilation with J the Jacobian of the
    pinhole map, obtained here by central differences; Sigma3D built from
    scipy's rotation."""
    rng = np.random.default_rng(5)
    cam = ws.look_at_camera((1.0, -0.5, -4.0), 320, 200)
    st = ws.Settings(weight_kind="dir", opacity_mode="logit", dilation=0.3)
    n = 40
    means = rng.normal(0, 0.8, size=(n, 3))
    quats = rng.standard_normal((4, n))
    log_s = rng.normal(-2.5, 0.5, size=(3, n))
    sc = scene_from(means, log_s, quats)
    p = oracle.project(sc, cam, st)
    W = cam["viewmat"][:, :3]
    T = cam["viewmat"][:, 3]
    lim = 1.3 * 0.5 * np.array([cam["width"] / cam["fx"], cam["height"] / cam["fy"]])
    checked = 0
    for i in range(n):
        t = W @ means[i] + T
        if t[2] <= st.near or np.any(np.abs(t[:2] / t[2]) >= lim):
            continue
        Rm = Rotation.from_quat(quats[[1, 2, 3, 0], i]).as_matrix()
        S3 = Rm @ np.diag(np.exp(2 * log_s[:, i])) @ Rm.T
        h = 1e-6
        Jn = np.zeros((2, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            Jn[:, k] = (_pinhole(cam, t + e) - _pinhole(cam, t - e)) / (2 * h)
        S2 = Jn @ W @ S3 @ W.T @ Jn.T + 0.3 * np.eye(2)
        got = p["cov2d"][i]
        np.testing.assert_allclose([got[0], got[1], got[2]], [S2[0, 0], S2[0, 1], S2[1, 1]],
                                   rtol=1e-7, atol=1e-9)
        np.testing.assert_allclose(p["mu"][i], _pinhole(cam, t), rtol=1e-13)
        con = np.linalg.inv(np.array([[got[0], got[1]], [got[1], got[2]]]))
        np.testing.assert_allclose(p["conic"][i], [con[0, 0], con[0, 1], con[1, 1]], rtol=1e-10)
        np.testing.assert_allclose(p["depth"][i], t[2], rtol=1e-14)
        checked += 1
    assert checked > 20


def test_isotropic_gaussian_closed_form_image():
    """A single isotropic Gaussian on the optical axis at depth d projects to
    Sigma2D = (f s / d)^2 I + dilation I, and the rendered image is
    (c_B w_B + rgb a G) / (w_B + a G) with G = exp(-r^2 / (2 var)) where q <= tau."""
    cam = ws.look_at_camera((0.0, 0.0, -4.0), 64, 48)
    s = 0.05
    rgb = np.array([0.9, 0.3, 0.1])
    sh = dc_for_colour(np.append(rgb, 0.5))[None, None, :]
    q = Rotation.random(random_state=7).as_quat()[[3, 0, 1, 2]][:, None]  # rotation irrelevant
    sc = scene_from([[0.0, 0.0, 0.0]], np.full(3, math.log(s)), q, sh, logit=[0.3])
    st = ws.Settings(weight_kind="exp", opacity_mode="logit", sigma=0.1, beta=0.8, w_bg=0.7,
                     bg=(0.2, 0.4, 0.6), tau=9.0, dilation=0.3)
    r = oracle.render(sc, cam, st)
    var = (cam["fx"] * s / 4.0) ** 2 + 0.3
    u = 1 / (1 + math.exp(-0.3))
    w = math.exp(-0.1 * 4.0 ** 0.8)
    ys, xs = np.mgrid[0:48, 0:64]
    r2 = (xs + 0.5 - 32.0) ** 2 + (ys + 0.5 - 24.0) ** 2
    G = np.where(r2 / var <= 9.0, np.exp(-r2 / (2 * var)), 0.0)
    a = u * w * G
    bg = np.array(st.bg)
    ref = (bg * 0.7 + a[..., None] * rgb) / (0.7 + a[..., None])
    np.testing.assert_allclose(r["C"], ref, atol=1e-12)
    p = oracle.project(sc, cam, st)
    np.testing.assert_allclose(p["cov2d"][0], [var, 0.0, var], atol=1e-12)


def test_view_direction_points_from_camera_to_gaussian():
    """Only the l=1, m=1 coefficient (basis proportional to x) is set on red:
    the colour shift is positive exactly for Gaussians with p_x > camera_x."""
    cpos = np.array([0.5, 0.2, -4.0])
    cam = ws.look_at_camera(cpos, 64, 64)
    means = np.array([[1.5, 0.2, 0.0], [-0.5, 0.2, 0.0]])
    sh = np.zeros((4, 2, 4))
    sh[3, :, 0] = 1.0
    sc = scene_from(means, sh=sh)
    p = oracle.project(sc, cam, ws.Settings(opacity_mode="logit"))
    d = (means - cpos) / np.linalg.norm(means - cpos, axis=1, keepdims=True)
    # the camera is float32 (its centre is exact only to ~1e-7)
    np.testing.assert_allclose(p["dir"], d, atol=1e-6)
    k1 = math.sqrt(3 / (4 * math.pi))
    np.testing.assert_allclose(p["rgb_raw"][:, 0], 0.5 + k1 * p["dir"][:, 0], atol=1e-14)


def test_near_plane_and_degenerate_culling():
    cam = ws.look_at_camera((0.0, 0.0, -4.0), 32, 32)
    # depth 4.1 -> visible, depth 0.1 (< near) -> culled, behind camera -> culled
    sc = scene_from([[0.0, 0.0, 0.1], [0.0, 0.0, -3.9], [0.0, 0.0, -6.0]])
    sc["quats"][:, 0] = [1.0, 0, 0, 0]
    p = oracle.project(sc, cam, ws.Settings())
    assert list(p["visible"]) == [True, False, False]
    # a zero quaternion has no rotation: culled
    sc2 = scene_from([[0.0, 0.0, 0.0]], quats=np.zeros((4, 1)))
    assert not oracle.project(sc2, cam, ws.Settings())["visible"][0]


# --------------------------------------------------------------------------
# Weights (Sec. 4.2, Eqs. 8-10; Fig. 3) and the initial constants (Sec. 4.4)
# --------------------------------------------------------------------------

def test_settings_defaults_match_paper_constants():
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    st = ws.Settings()
    assert st.sigma == g["exp_sigma_init"] and st.beta == g["exp_beta_init"]
    _, _, st2 = ws.make_scene("c2", n=10)
    assert st2.weight_kind == "lc" and st2.sigma == g["lc_sigma_init"]


def _fig3(kind, sigma=0.1, beta=0.8):
    """Red Gaussian at depth 3 in front of a blue one at depth 5, both with
    opacity 1 and the same on-screen footprint."""
    g = json.load(open(os.path.join(GOLDEN, "fig3_two_gaussians.json")))
    cam = ws.look_at_camera((0.0, 0.0, -4.0), 32, 32)
    sh = np.zeros((1, 2, 4))
    sh[0, 0, :3] = dc_for_colour(g["red"])
    sh[0, 1, :3] = dc_for_colour(g["blue"])
    s_red = 0.05
    ls = np.log(np.array([s_red, s_red * 5.0 / 3.0]))
    sc = scene_from([[0, 0, -1.0], [0, 0, 1.0]], np.repeat(ls[None, :], 3, 0), sh=sh)
    st = ws.Settings(weight_kind=kind, opacity_mode="sh", opacity_offset=1.0, w_bg=0.0,
                     sigma=sigma, beta=beta, tau=9.0)
    return g, oracle.render(sc, cam, st, crop=(15, 15, 17, 17))["C"]


def test_fig3_dir_gives_even_mix():
    g, C = _fig3("dir")
    np.testing.assert_allclose(C.reshape(-1, 3), np.tile(g["dir_expected"], (4, 1)), atol=1e-9)


def test_fig3_exp_leans_to_the_nearer_gaussian():
    g, C = _fig3("exp", sigma=0.1, beta=0.8)
    C = C.reshape(-1, 3)
    wr, wb = math.exp(-0.1 * 3 ** 0.8), math.exp(-0.1 * 5 ** 0.8)
    assert np.all(C[:, 0] > C[:, 2]) and np.all(C[:, 2] > 0)
    np.testing.assert_allclose(C[:, 0], wr / (wr + wb), atol=1e-9)


def test_fig3_lc_can_remove_the_far_gaussian():
    g, C = _fig3("lc", sigma=4.0)  # blue at depth 5 > sigma -> weight exactly 0
    np.testing.assert_allclose(C.reshape(-1, 3), np.tile(g["lc_far_expected"], (4, 1)), atol=1e-12)


def test_exp_beta1_keeps_weight_ratios_under_z_motion():
    """Sec. C (moving the camera along z): EXP with beta = 1 keeps the weight
    ratio of two Gaussians; LC does not."""
    sc = scene_from([[0.1, 0.0, -1.0], [-0.2, 0.1, 1.5]], lc_v=[1.0, 1.0])
    ratios = {"exp": [], "lc": []}
    for dz in (0.0, 0.7, 1.5):
        cam = ws.look_at_camera((0.0, 0.0, -4.0 - dz), 32, 32)
        for kind, st in (("exp", ws.Settings(weight_kind="exp", sigma=0.3, beta=1.0)),
                         ("lc", ws.Settings(weight_kind="lc", sigma=10.0))):
            w = oracle.project(sc, cam, st)["w"]
            ratios[kind].append(w[0] / w[1])
    np.testing.assert_allclose(ratios["exp"], ratios["exp"][0], rtol=1e-12)
    assert abs(ratios["lc"][2] - ratios["lc"][0]) > 1e-3


# --------------------------------------------------------------------------
# Weighted sum (Sec. 4.2, Eq. 7) invariants
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c1():
    return ws.make_scene("c1")


def test_permutation_invariance(c1):
    sc, cams, st = c1
    perm = np.random.default_rng(8).permutation(sc["means"].shape[1])
    a = oracle.render(sc, cams[0], st)["C"]
    b = oracle.render(ws.permute(sc, perm), cams[0], st)["C"]
    np.testing.assert_allclose(a, b, atol=1e-12)


def test_empty_and_all_culled_scenes_render_background(c1):
    sc, cams, st = c1
    bg = np.array(st.bg)
    r = oracle.render(empty_like(sc), cams[0], st)
    assert np.all(r["C"] == bg) and np.all(r["den"] == st.w_bg)
    behind = dict(sc)
    behind["means"] = sc["means"].copy()
    behind["means"][2] = -10.0  # every centre behind the camera at z = -4
    r = oracle.render(behind, cams[0], st)
    assert np.all(r["C"] == bg)
    # w_B = 0 and nothing covers a pixel: den == 0 -> background colour
    r = oracle.render(empty_like(sc), cams[0], st.copy(w_bg=0.0))
    assert np.all(r["C"] == bg) and np.all(r["den"] == 0.0)


def test_uniform_colour_renders_that_colour(c1):
    sc, cams, st = c1
    c = np.array([0.3, 0.6, 0.2])
    u = dict(sc)
    u["sh"] = np.zeros_like(sc["sh"], dtype=np.float64)
    u["sh"][0, :, :3] = dc_for_colour(c)
    r = oracle.render(u, cams[0], st.copy(w_bg=0.0))
    cov = r["den"] != 0
    assert cov.mean() > 0.3
    np.testing.assert_allclose(r["C"][cov], np.broadcast_to(c, r["C"][cov].shape), atol=1e-12)
    r = oracle.render(u, cams[0], st.copy(bg=tuple(c)))
    np.testing.assert_allclose(r["C"], np.broadcast_to(c, r["C"].shape), atol=1e-12)


def test_homogeneity_in_amplitudes(c1):
    """Scaling every LC weight v_i and w_B by k leaves C unchanged."""
    sc, cams, st = c1
    st = st.copy(weight_kind="lc", sigma=10.0)
    a = oracle.render(sc, cams[0], st)["C"]
    s2 = dict(sc)
    s2["lc_v"] = sc["lc_v"].astype(np.float64) * 3.7
    b = oracle.render(s2, cams[0], st.copy(w_bg=st.w_bg * 3.7))["C"]
    np.testing.assert_allclose(a, b, atol=1e-12)


def test_colour_shift_equivariance(c1):
    """rgb_i -> rgb_i + k for every Gaussian and c_B -> c_B + k gives C -> C + k."""
    sc, cams, st = c1
    k = 0.125
    s2 = dict(sc)
    s2["sh"] = sc["sh"].astype(np.float64).copy()
    s2["sh"][0, :, :3] += k * 2.0 * math.sqrt(math.pi)
    a = oracle.render(sc, cams[0], st)["C"]
    b = oracle.render(s2, cams[0], st.copy(bg=tuple(np.array(st.bg) + k)))["C"]
    np.testing.assert_allclose(b, a + k, atol=1e-12)


def test_strict_and_aabb_modes_agree(c1):
    sc, cams, st = c1
    a = oracle.render(sc, cams[0], st, mode="strict")
    b = oracle.render(sc, cams[0], st, mode="aabb")
    np.testing.assert_allclose(a["C"], b["C"], atol=1e-12)
    assert np.array_equal(a["count"], b["count"])
    sc2, cams2, st2 = ws.make_scene("c2", n=20000)
    crop = (600, 320, 664, 384)
    a = oracle.render(sc2, cams2[0], st2, crop=crop, mode="strict")
    b = oracle.render(sc2, cams2[0], st2, crop=crop, mode="aabb")
    np.testing.assert_allclose(a["C"], b["C"], atol=1e-12)
    assert np.array_equal(a["count"], b["count"])
    for k in ("den", "abs_den"):
        np.testing.assert_allclose(a[k], b[k], rtol=1e-12, atol=1e-12)


def test_ambiguity_report_weighs_each_pair_by_its_colour_distance():
    """With one Gaussian, every reported pixel holds exactly that pair, so
    amb_c / amb is the largest channel distance between its colour and the
    rendered colour there (the most the pair's flip can move the pixel, per
    unit of |a|)."""
    cam = ws.look_at_camera((0.0, 0.0, -4.0), 40, 40)
    sh = np.zeros((1, 1, 4))
    sh[0, 0, :3] = dc_for_colour((0.9, 0.1, 0.6))
    sc = scene_from([(0.03, -0.02, 0.0)], log_scales=np.full(1, -1.2), sh=sh, logit=np.array([1.2]))
    st = ws.Settings(weight_kind="exp", opacity_mode="logit", bg=(0.2, 0.7, 0.4))
    r = oracle.render(sc, cam, st, eta=0.05)
    m = r["amb"] > 0
    assert m.sum() > 10
    rgb = oracle.project(sc, cam, st)["rgb"][0]
    want = np.abs(rgb[None, :] - r["C"][m]).max(axis=-1)
    np.testing.assert_allclose(r["amb_c"][m] / r["amb"][m], want, rtol=1e-12)
    assert (r["amb_c"][~m] == 0).all()


def test_a_support_flip_from_the_float32_centre_is_reported():
    """The renderer forms a splat's centre relative to its tile's centre in
    float32 (the integer part exact, the fraction rounded once).  A pair is
    built whose exact q lies just above tau while q from that rounded centre
    lies below it (the rest of the arithmetic exact): the report's centre
    term (pos_h = half a tile) must flag the pixel, and without it (pos_h = 0,
    eta = 0) nothing is flagged.  The shift is two thirds of the reported
    window here, so a window a quarter as wide would miss it."""
    T, px, py, x = 16, 50, 31, -0.56
    cam = ws.look_at_camera((0.0, 0.0, -4.0), 64, 64)
    st = ws.Settings(weight_kind="exp", opacity_mode="logit", bg=(0.2, 0.7, 0.4), tau=9.0)
    f32 = np.float32

    def scene(ls):
        return scene_from([(x, 0.013, 0.0)], log_scales=np.full(1, ls), logit=np.array([1.0]))

    def q_exact_and_rounded(ls):
        p = oracle.project(scene(ls), cam, st)
        (A, B, C), (mux, muy) = p["conic"][0], p["mu"][0]

        def offset(mu, pix):                      # pixel centre minus the float32 centre
            o, tc = np.floor(mu), (pix // T) * T + T / 2
            return (pix + 0.5 - tc) - float(f32(f32(o - tc) + f32(mu - o)))

        q = lambda dx, dy: A * dx * dx + 2 * B * dx * dy + C * dy * dy  # noqa: E731
        return q(px + 0.5 - mux, py + 0.5 - muy), q(offset(mux, px), offset(muy, py))

    # bisect the log-scale so that the exact q sits halfway across the shift
    a, b = -3.0, 0.5
    g = lambda ls: sum(q_exact_and_rounded(ls)) / 2 - st.tau  # noqa: E731
    ga = g(a)
    for _ in range(80):
        m = 0.5 * (a + b)
        if (g(m) > 0) == (ga > 0):
            a, ga = m, g(m)
        else:
            b = m
    ls = 0.5 * (a + b)
    q, qr = q_exact_and_rounded(ls)
    assert (q <= st.tau) != (qr <= st.tau)            # the rounded centre flips the decision
    assert abs(qr - q) > 5e-7
    with_term = oracle.render(scene(ls), cam, st, eta=0.0, pos_h=T / 2)
    without = oracle.render(scene(ls), cam, st, eta=0.0, pos_h=0.0)
    assert with_term["amb"][py, px] > 0
    assert without["amb"][py, px] == 0


def test_denominator_magnitude_counts_negative_amplitudes():
    """abs_den = |w_B| + sum |a| (the conditioning report of Eq. 7's
    denominator), against a brute-force sum, in both evaluation modes, on a
    scene whose unclamped SH opacities (Sec. 4.3) make some amplitudes
    negative."""
    sc, _, st = ws.make_scene("c2", n=60)
    sc = {k: v.astype(np.float64) for k, v in sc.items()}
    rng = np.random.default_rng(23)
    sc["sh"][0, :, 3] = dc_for_colour(np.where(rng.random(60) < 0.3, -0.4, 0.7))
    sc["sh"][1:, :, 3] = 0.0
    cam = ws.look_at_camera((0.0, 0.0, -4.0), 24, 20)
    st = st.copy(tau=1e4)
    p = oracle.project(sc, cam, st)
    assert (p["u"][p["visible"]] < 0).sum() > 5
    ys, xs = np.mgrid[0:cam["height"], 0:cam["width"]]
    want = np.full((cam["height"], cam["width"]), abs(st.w_bg))
    for i in np.nonzero(p["visible"])[0]:
        A, B, Cc = p["conic"][i]
        dx, dy = xs + 0.5 - p["mu"][i, 0], ys + 0.5 - p["mu"][i, 1]
        q = A * dx * dx + 2 * B * dx * dy + Cc * dy * dy
        want += np.where(q <= st.tau, np.abs(p["u"][i] * p["w"][i] * np.exp(-0.5 * q)), 0.0)
    for mode in ("strict", "aabb"):
        got = oracle.render(sc, cam, st, mode=mode)["abs_den"]
        np.testing.assert_allclose(got, want, rtol=1e-12)


def test_ambiguity_window_widens_only_the_report(c1):
    """The centre-rounding term of the ambiguity report (pos_h) only widens
    the set of pairs reported near the cutoff; the image is unchanged, and
    pos_h = 0 gives the plain window."""
    sc, cams, st = c1
    a = oracle.render(sc, cams[0], st, eta=1e-6)
    b = oracle.render(sc, cams[0], st, eta=1e-6, pos_h=0.0)
    c = oracle.render(sc, cams[0], st, eta=1e-6, pos_h=8.0)
    assert np.array_equal(a["amb"], b["amb"]) and np.array_equal(a["C"], c["C"])
    assert (c["amb"] >= a["amb"]).all() and (c["amb_c"] >= a["amb_c"]).all()
    assert (oracle.render(sc, cams[0], st, eta=1e-6, pos_h=1e5)["amb"] > a["amb"]).any()
    s0 = oracle.render_sorted(sc, cams[0], st.copy(weight_kind="dir"), eta=1e-6)
    s1 = oracle.render_sorted(sc, cams[0], st.copy(weight_kind="dir"), eta=1e-6, pos_h=8.0)
    assert np.array_equal(s0["C"], s1["C"]) and (s1["amb"] >= s0["amb"]).all()


def test_crop_is_window_of_full_image(c1):
    sc, cams, st = c1
    full = oracle.render(sc, cams[0], st)["C"]
    part = oracle.render(sc, cams[0], st, crop=(37, 5, 101, 60))["C"]
    np.testing.assert_allclose(part, full[5:60, 37:101], atol=1e-12)


def test_lc_zero_weight_gaussians_drop_out(c1):
    sc, cams, st = c1
    st = st.copy(weight_kind="lc", sigma=4.0)
    p = oracle.project(sc, cams[0], st)
    far = p["depth"] >= 4.0
    assert 0.2 < far.mean() < 0.8
    a = oracle.render(sc, cams[0], st)["C"]
    b = oracle.render(subset(sc, ~far), cams[0], st)["C"]
    np.testing.assert_allclose(a, b, atol=1e-12)


def test_unconstrained_opacity_allows_negative_and_large_u():
    """Sec. 4.2 / 4.3: u is not clamped; a negative-u Gaussian subtracts."""
    cam = ws.look_at_camera((0.0, 0.0, -4.0), 16, 16)
    sh = np.zeros((1, 2, 4))
    sh[0, :, :3] = dc_for_colour([1.0, 0.0, 0.0])
    sh[0, 1, 3] = -3.0 * 2 * math.sqrt(math.pi)  # u = -3 + offset
    sc = scene_from([[0, 0, 0], [0, 0, 0.5]], np.full((3, 2), -2.0), sh=sh)
    st = ws.Settings(weight_kind="dir", opacity_mode="sh", opacity_offset=0.5)
    p = oracle.project(sc, cam, st)
    np.testing.assert_allclose(p["u"], [0.5, -2.5], atol=1e-12)
    r = oracle.render(sc, cam, st)
    assert np.any(r["den"] < 0)


def test_jacobian_clamp_beyond_the_field_of_view():
    """Reading of the 3DGS pre-processing the paper keeps: beyond 1.3x the half
    field of view (per axis) the Jacobian is that of the pinhole map at the
    point moved laterally onto the limit, depth unchanged."""
    rng = np.random.default_rng(21)
    cam = ws.look_at_camera((0.0, 0.0, -4.0), 320, 200)
    W, T = cam["viewmat"][:, :3], cam["viewmat"][:, 3]
    lim = 1.3 * 0.5 * np.array([cam["width"] / cam["fx"], cam["height"] / cam["fy"]])
    cases = [(2.0, 0.1), (-1.5, 0.2), (0.1, 1.4), (0.3, -1.2), (1.8, -1.9), (0.5, 0.3)]
    means, ts = [], []
    for rx, ry in cases:
        tz = 3.0 + rng.uniform()
        t = np.array([rx * tz, ry * tz, tz])
        ts.append(t)
        means.append(W.T @ (t - T))
    quats = rng.standard_normal((4, len(cases)))
    log_s = rng.normal(-2.0, 0.3, size=(3, len(cases)))
    p = oracle.project(scene_from(means, log_s, quats), cam, ws.Settings(dilation=0.3))
    for i, t in enumerate(ts):
        tc = t.copy()
        tc[:2] = np.clip(t[:2] / t[2], -lim, lim) * t[2]
        Rm = Rotation.from_quat(quats[[1, 2, 3, 0], i]).as_matrix()
        S3 = Rm @ np.diag(np.exp(2 * log_s[:, i])) @ Rm.T
        Jn = np.zeros((2, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = 1e-6
            Jn[:, k] = (_pinhole(cam, tc + e) - _pinhole(cam, tc - e)) / 2e-6
        S2 = Jn @ W @ S3 @ W.T @ Jn.T + 0.3 * np.eye(2)
        np.testing.assert_allclose(p["cov2d"][i], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-7, atol=1e-9)
        np.testing.assert_allclose(p["mu"][i], _pinhole(cam, t), rtol=1e-13)  # centre never clamped
