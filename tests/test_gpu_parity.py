"""GPU parity: the HIP path (through the C-ABI) against the FP64 checker on
the same seeded inputs.  Images within 1e-4 max-abs (plus the documented
allowance for pairs within float rounding of the support cutoff), gradients
within 1e-3 of each tensor's max-abs."""
import numpy as np
import pytest
import torch

import oracle
import wsr_synth as ws
from paper_2410_18931_amd import WSRContext, globals_tensor, render, scene_to_device
from tests.gpu_helpers import (amb_kw, compare_grads, compare_image, densest_crop, gpu_forward, unambiguous,
                               grads_to_numpy, log, seeded_normal_like, to_views)
from tests.oracle_helpers import empty_like

pytestmark = pytest.mark.gpu

SCENE_KEYS = ("means", "log_scales", "quats", "sh", "opacity_logit", "lc_v")


def _grad_keys(settings, K):
    keys = ["means", "log_scales", "quats", "sh"]
    if settings.opacity_mode == "logit":
        keys.append("opacity_logit")
    if settings.weight_kind == "lc":
        keys.append("lc_v")
    return keys


def _oracle_globals(settings, gref):
    out = gref.copy()
    if settings.weight_kind == "dir":
        out[0] = 0.0
    if settings.weight_kind != "exp":
        out[1] = 0.0
    return out


def _check_globals(g_gpu, g_ref, label):
    a, b = np.asarray(g_gpu, np.float64), np.asarray(g_ref, np.float64)
    log(f"[globals {label}] gpu={a} ref={b}")
    np.testing.assert_allclose(a, b, rtol=1e-3, atol=1e-3 * max(1.0, np.abs(b).max()))


# ---------------------------------------------------------------- c1 (small)

@pytest.fixture(scope="module")
def c1():
    return ws.make_scene("c1")


def test_c1_projection_stage(c1):
    sc, cams, st = c1
    log("case: c1 projection stage")
    ctx = WSRContext(sc["means"].shape[1], cams, st)
    dev = scene_to_device(sc)
    g = globals_tensor(st)
    proj = torch.zeros((1, ctx.n, 16), dtype=torch.float32, device="cuda")
    ctx.project(dev, g, out_proj=proj)
    torch.cuda.synchronize()
    p = proj[0].cpu().numpy().astype(np.float64)
    ref = oracle.project(sc, cams[0], st)
    vis = ref["visible"]
    assert np.array_equal(p[:, 0] > 0.5, vis)
    np.testing.assert_allclose(p[vis, 1:3], ref["mu"][vis], atol=2e-4)
    np.testing.assert_allclose(p[vis, 3:6], ref["conic"][vis], rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(p[vis, 6:9], ref["rgb"][vis], atol=2e-6)
    np.testing.assert_allclose(p[vis, 9], ref["u"][vis], atol=2e-6)
    np.testing.assert_allclose(p[vis, 10], ref["w"][vis], rtol=2e-6)
    np.testing.assert_allclose(p[:, 11], ref["depth"], rtol=1e-6)


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_c1_image_and_counts(c1, tile):
    sc, cams, st = c1
    st = st.copy(tile=tile)
    log(f"case: c1 image tile={tile}")
    ctx, dev, g, (rgb, den, cnt) = gpu_forward(sc, cams, st, count=True)
    ref = oracle.render(sc, cams[0], st, **amb_kw(st))
    C = to_views(ctx, rgb)[0]
    compare_image(C, ref, label=f"c1 t{tile}")
    D = to_views(ctx, den)[0]
    np.testing.assert_allclose(D, ref["den"], rtol=1e-5, atol=1e-5)
    n_gpu = to_views(ctx, cnt)[0]
    differ = n_gpu != ref["count"]
    assert np.all(ref["amb"][differ] > 0), "count differs away from the cutoff"
    assert ctx.last_pairs > 0


def test_c1_tile_size_invariance(c1):
    """Tiles 8, 16 and 32 evaluate the same expression per pair; only the
    float32 rounding of the tile-relative centre differs, so the images agree
    to 1e-6 except where a pair lies within that rounding of the cutoff (the
    checker's ambiguity report for the largest tile bounds those pixels)."""
    sc, cams, st = c1
    imgs = []
    for tile in (8, 16, 32):
        log(f"case: c1 tile invariance tile={tile}")
        ctx, dev, g, (rgb, den) = gpu_forward(sc, cams, st.copy(tile=tile))
        imgs.append(rgb.cpu().numpy().reshape(cams[0]["height"], cams[0]["width"], 3))
    ref = oracle.render(sc, cams[0], st, **amb_kw(st.copy(tile=32)))
    den = np.abs(ref["den"])
    bound = 1e-6 + 4.0 * ref["amb_c"] / np.where(den == 0, 1.0, den)
    for other in (imgs[1], imgs[2]):
        diff = np.abs(imgs[0] - other).max(axis=-1)
        log(f"tile invariance: max diff {diff.max():.3g}, ambiguous px {int((ref['amb_c'] > 0).sum())}")
        assert (diff <= bound).all()
        assert diff[ref["amb_c"] == 0].max() <= 1e-6


def test_c1_gradients(c1):
    sc, cams, st = c1
    log("case: c1 gradients")
    ctx, dev, g, (rgb, den) = gpu_forward(sc, cams, st)
    r = ws.upstream_grad(cams, seed=3)
    dL = torch.from_numpy(r[0].reshape(-1, 3)).cuda()
    grad2d = torch.zeros((1, ctx.n, 9), dtype=torch.float32, device="cuda")
    gg = grads_to_numpy(ctx.render_bwd(dev, g, dL, rgb, den, grad2d=grad2d))
    gref = oracle.render_bwd(sc, cams[0], st, r[0])
    compare_grads(gg, gref, _grad_keys(st, 1), label="c1")
    compare_grads({"grad2d": grad2d[0].cpu().numpy()}, {"grad2d": gref["grad2d"]}, ["grad2d"], label="c1 2d")
    _check_globals(gg["globals"], _oracle_globals(st, gref["globals"]), "c1")


def _small_c2(deg: int, n: int = 20000, width: int = 320, height: int = 180):
    """The c2 generator at n Gaussians with its SH cut to degree ``deg``,
    seen by one width x height camera at distance 4."""
    sc, _, st = ws.make_scene("c2", n=n)
    sc = dict(sc)
    sc["sh"] = np.ascontiguousarray(sc["sh"][: (deg + 1) ** 2])
    return sc, [ws.look_at_camera((0.0, 0.0, -4.0), width, height)], st


@pytest.mark.parametrize("weight,deg,opacity", [
    ("dir", 0, "logit"), ("dir", 1, "logit"), ("dir", 3, "sh"),
    ("exp", 1, "sh"), ("exp", 2, "logit"), ("lc", 1, "logit"), ("lc", 2, "sh"),
])
def test_weight_kinds_and_sh_degrees(weight, deg, opacity):
    """Each depth weight of Sec. 4.2 (Eq. 8 DIR, Eq. 9 EXP, Eq. 10 LC) with
    SH colour of degrees 0-3 (Eq. 4) and either opacity (sigmoid of a logit,
    or the unclamped SH opacity of Eq. 11): the full image and every
    gradient, globals included (DIR has no sigma or beta, so their gradients
    are zero), against the checker."""
    if deg == 0:
        sc, cams, st = ws.make_scene("c1")
    else:
        sc, cams, st = _small_c2(deg)
    st = st.copy(weight_kind=weight, opacity_mode=opacity,
                 sigma={"dir": 0.1, "exp": 0.1, "lc": 10.0}[weight], beta=0.8)
    log(f"case: weight {weight}, SH degree {deg}, opacity {opacity}")
    ctx, dev, g, (rgb, den) = gpu_forward(sc, cams, st)
    ref = oracle.render(sc, cams[0], st, mode="aabb", **amb_kw(st))
    compare_image(to_views(ctx, rgb)[0], ref, label=f"{weight} deg {deg} {opacity}")
    r = ws.upstream_grad(cams, seed=40 + deg)[0] * unambiguous(ref)
    grad2d = torch.zeros((1, ctx.n, 9), dtype=torch.float32, device="cuda")
    gg = grads_to_numpy(ctx.render_bwd(dev, g, torch.from_numpy(r.reshape(-1, 3)).cuda(), rgb, den,
                                       grad2d=grad2d))
    gref = oracle.render_bwd(sc, cams[0], st, r)
    compare_grads(gg, gref, _grad_keys(st, (deg + 1) ** 2), label=f"{weight} deg {deg} {opacity}")
    compare_grads({"grad2d": grad2d[0].cpu().numpy()}, {"grad2d": gref["grad2d"]}, ["grad2d"],
                  label=f"{weight} deg {deg} {opacity} 2d")
    _check_globals(gg["globals"], _oracle_globals(st, gref["globals"]), f"{weight} deg {deg}")
    if weight == "dir":
        assert gg["globals"][0] == 0.0 and gg["globals"][1] == 0.0


@pytest.mark.parametrize("oit", [False, True])
def test_every_pair_slot_is_written_by_the_backward(c1, oit):
    """The raster backward stores every binned pair's partial sums, zeros
    included, and the per-Gaussian sums read only those slots: with the
    partial-gradient regions of the pair buffer filled with NaN beforehand,
    the gradients still match the reference."""
    sc, cams, st = c1
    st = st.copy(oit=oit)
    log(f"case: c1 pair slots over a NaN-filled buffer, oit={oit}")
    ctx = WSRContext(sc["means"].shape[1], cams, st)
    dev = scene_to_device(sc)
    g = globals_tensor(st)
    ctx.project(dev, g)
    ctx.bin(grow=True)
    # pair buffer layout: [capacity][36 B] partials, [capacity] dL/du, [capacity] (id, slot) list entries,
    # [capacity][4 B] culling masks
    assert ctx.pair_bytes == 52
    ctx.pairs[: 36 * ctx.capacity].fill_(0xFF)                     # every partial slot NaN
    ctx.pairs[36 * ctx.capacity: 40 * ctx.capacity].fill_(0xFF)    # and every dL/du slot
    ctx.bin(grow=False)
    rgb, den = ctx.render_fwd(g)
    r = ws.upstream_grad(cams, seed=3)
    gg = grads_to_numpy(ctx.render_bwd(dev, g, torch.from_numpy(r[0].reshape(-1, 3)).cuda(), rgb, den))
    torch.cuda.synchronize()
    ctx.check()
    for k, v in gg.items():
        assert np.isfinite(v).all(), k
    gref = oracle.render_bwd(sc, cams[0], st, r[0])
    compare_grads(gg, gref, _grad_keys(st, 1), label="c1 NaN-filled pair buffer")


def test_autograd_function_matches_direct_backward(c1):
    sc, cams, st = c1
    log("case: autograd wrapper")
    ctx = WSRContext(sc["means"].shape[1], cams, st)
    dev = scene_to_device(sc)
    leaves = {k: v.clone().requires_grad_(True) for k, v in dev.items()}
    g = globals_tensor(st).requires_grad_(True)
    rgb, den = render(leaves, g, ctx)
    r = torch.from_numpy(ws.upstream_grad(cams, seed=4)[0].reshape(-1, 3)).cuda()
    (rgb * r).sum().backward()
    direct = ctx.render_bwd(dev, g.detach(), r, rgb.detach(), den)
    # the same binning and upstream gradient: the same sums in the same order
    for k in ("means", "log_scales", "quats", "sh", "opacity_logit"):
        assert torch.equal(leaves[k].grad, direct[k]), k
    assert torch.equal(g.grad, direct["globals"])


# ---------------------------------------------------------------- c2 (720p)

@pytest.fixture(scope="module")
def c2():
    return ws.make_scene("c2")


def test_c2_image_full_frame(c2):
    sc, cams, st = c2
    log("case: c2 full-frame image")
    ctx, dev, g, (rgb, den) = gpu_forward(sc, cams, st)
    ref = oracle.render(sc, cams[0], st, mode="aabb", **amb_kw(st))
    compare_image(to_views(ctx, rgb)[0], ref, label="c2")


def test_c2_gradients_on_crop(c2):
    sc, cams, st = c2
    log("case: c2 gradients on a crop")
    ctx, dev, g, (rgb, den, cnt) = gpu_forward(sc, cams, st, count=True)
    crop = densest_crop(to_views(ctx, cnt)[0])
    x0, y0, x1, y1 = crop
    r = np.zeros((720, 1280, 3), np.float32)
    r[y0:y1, x0:x1] = np.random.default_rng(5).standard_normal((y1 - y0, x1 - x0, 3))
    dL = torch.from_numpy(r.reshape(-1, 3)).cuda()
    gg = grads_to_numpy(ctx.render_bwd(dev, g, dL, rgb, den))
    gref = oracle.render_bwd(sc, cams[0], st, r[y0:y1, x0:x1], crop=crop)
    compare_grads(gg, gref, _grad_keys(st, 16), label="c2 crop")
    _check_globals(gg["globals"], _oracle_globals(st, gref["globals"]), "c2 crop")


def test_c2_reduced_precision_storage(c2):
    sc, cams, st = c2
    for dt in ("f16", "bf16"):
        log(f"case: c2 storage {dt}")
        q = ws.quantise(sc, dt)
        ctx, dev, g, (rgb, den) = gpu_forward(sc, cams, st, storage=dt)
        crop = (600, 320, 664, 384)
        ref = oracle.render(q["f32"], cams[0], st, crop=crop, **amb_kw(st))
        C = to_views(ctx, rgb)[0][320:384, 600:664]
        compare_image(C, ref, label=f"c2 {dt} vs dequantised")
        src = oracle.render(sc, cams[0], st, crop=crop)
        log(f"[c2 {dt}] end-to-end max-abs vs fp32 source: {np.abs(C - src['C']).max():.3g}")


def test_gpu_permutation_invariance(c2):
    sc, cams, st = c2
    log("case: permutation invariance")
    perm = np.random.default_rng(9).permutation(sc["means"].shape[1])
    _, _, _, (a, _) = gpu_forward(sc, cams, st)
    _, _, _, (b, _) = gpu_forward(ws.permute(sc, perm), cams, st)
    assert (a - b).abs().max().item() <= 2e-6


# ---------------------------------------------------------------- c3 and the 1M / 1080p configuration

@pytest.mark.parametrize("config", ["c3", "headline"])
def test_1080p_crops(config):
    sc, cams, st = ws.make_scene(config)
    log(f"case: {config} n={sc['means'].shape[1]} 1080p")
    ctx, dev, g, (rgb, den, cnt) = gpu_forward(sc, cams, st, count=True)
    C = to_views(ctx, rgb)[0]
    counts = to_views(ctx, cnt)[0]
    log(f"[{config}] pairs in support {int(counts.sum())}, binned pairs {ctx.last_pairs}")
    crops = [densest_crop(counts), (0, 0, 64, 64), (1856, 1016, 1920, 1080), (928, 508, 992, 572)]
    refs = []
    for crop in crops:
        x0, y0, x1, y1 = crop
        refs.append(oracle.render(sc, cams[0], st, crop=crop, **amb_kw(st)))
        compare_image(C[y0:y1, x0:x1], refs[-1], label=f"{config} {crop}")
    # gradients through the densest crop, in the launch configuration the
    # benchmark times (every Gaussian of the frame is in the backward)
    x0, y0, x1, y1 = crops[0]
    r = np.zeros((1080, 1920, 3), np.float32)
    r[y0:y1, x0:x1] = np.random.default_rng(6).standard_normal((y1 - y0, x1 - x0, 3)) * unambiguous(refs[0])
    gg = grads_to_numpy(ctx.render_bwd(dev, g, torch.from_numpy(r.reshape(-1, 3)).cuda(), rgb, den))
    gref = oracle.render_bwd(sc, cams[0], st, r[y0:y1, x0:x1], crop=crops[0])
    compare_grads(gg, gref, _grad_keys(st, 16), label=f"{config} crop")


# ---------------------------------------------------------------- several views

def test_multi_view_uneven_sizes():
    sc, _, st = ws.make_scene("c3", n=40000)
    rng = np.random.default_rng(3)
    cams = []
    for k in range(4):
        w = int(rng.integers(96, 257))
        u = rng.standard_normal(3)
        cams.append(ws.look_at_camera(u / np.linalg.norm(u) * rng.uniform(4, 6), w, int(round(9 * w / 16))))
    log("case: multi-view " + str([(c["width"], c["height"]) for c in cams]))
    ctx, dev, g, (rgb, den) = gpu_forward(sc, cams, st)
    imgs = to_views(ctx, rgb)
    rs = ws.upstream_grad(cams, seed=8)
    for v, cam in enumerate(cams):
        compare_image(imgs[v], oracle.render(sc, cam, st, mode="aabb", **amb_kw(st)), label=f"view {v}")
    dL = torch.cat([torch.from_numpy(r.reshape(-1, 3)) for r in rs]).cuda()
    gg = grads_to_numpy(ctx.render_bwd(dev, g, dL, rgb, den))
    gref = oracle.render_bwd_views(sc, cams, st, rs)
    compare_grads(gg, gref, _grad_keys(st, 16), label="multi-view")


def test_c4_sixteen_uneven_views_at_full_size():
    """The 16-view batch of the benchmark (1 M Gaussians, views from 697x392
    to 1902x1070, 14.5 Mpx in one launch sequence): densest crops of four
    views, and every Gaussian's gradient through the densest crops of two
    views (per-view gradients add up; pixels with a pair within rounding of
    the cutoff carry no upstream gradient)."""
    sc, cams, st = ws.make_scene("c4")
    log(f"case: c4 {len(cams)} views, {sum(c['width'] * c['height'] for c in cams)} px")
    ctx, dev, g, (rgb, den, cnt) = gpu_forward(sc, cams, st, count=True)
    imgs, counts = to_views(ctx, rgb), to_views(ctx, cnt)
    refs = {}
    for v in (0, 2, 9, 15):
        crop = densest_crop(counts[v])
        x0, y0, x1, y1 = crop
        refs[v] = (crop, oracle.render(sc, cams[v], st, crop=crop, mode="aabb", **amb_kw(st)))
        compare_image(imgs[v][y0:y1, x0:x1], refs[v][1], label=f"c4 view {v} {crop}")
    rng = np.random.default_rng(21)
    rs = [np.zeros((c["height"], c["width"], 3), np.float32) for c in cams]
    gsum = None
    for v in (2, 9):
        (x0, y0, x1, y1), ref = refs[v]
        rs[v][y0:y1, x0:x1] = rng.standard_normal((y1 - y0, x1 - x0, 3)) * unambiguous(ref)
        gv = oracle.render_bwd(sc, cams[v], st, rs[v][y0:y1, x0:x1], crop=refs[v][0])
        gsum = gv if gsum is None else {k: gsum[k] + gv[k] for k in gv if k != "grad2d"}
    dL = torch.cat([torch.from_numpy(r.reshape(-1, 3)) for r in rs]).cuda()
    gg = grads_to_numpy(ctx.render_bwd(dev, g, dL, rgb, den))
    compare_grads(gg, gsum, _grad_keys(st, 16), label="c4 two-view crops")
    _check_globals(gg["globals"], _oracle_globals(st, gsum["globals"]), "c4 two-view crops")


# ---------------------------------------------------------------- edge cases

def test_empty_scene_and_all_culled():
    sc, cams, st = ws.make_scene("c1", n=64)
    log("case: empty scene")
    e = empty_like(sc)
    ctx, dev, g, (rgb, den) = gpu_forward(e, cams, st)
    assert torch.all(rgb == torch.tensor(st.bg, device="cuda")).item()
    assert torch.all(den == st.w_bg).item()
    r = seeded_normal_like(rgb, 31)
    gg = ctx.render_bwd(dev, g, r, rgb, den)
    gb = gg["globals"].cpu().numpy()
    np.testing.assert_allclose(gb[3:6], r.sum(0).cpu().numpy() / st.w_bg * st.w_bg, rtol=1e-4)
    log("case: all behind the camera")
    b = dict(sc)
    b["means"] = sc["means"].copy()
    b["means"][2] = -10.0
    ctx, dev, g, (rgb, den) = gpu_forward(b, cams, st)
    assert torch.all(rgb == torch.tensor(st.bg, device="cuda")).item()
    gg = ctx.render_bwd(dev, g, seeded_normal_like(rgb, 32), rgb, den)
    assert gg["means"].abs().max().item() == 0.0


def test_zero_background_weight_and_uncovered_pixels():
    sc, cams, st = ws.make_scene("c1", n=200)
    st = st.copy(w_bg=0.0)
    log("case: w_B = 0")
    ctx, dev, g, (rgb, den) = gpu_forward(sc, cams, st)
    ref = oracle.render(sc, cams[0], st, **amb_kw(st))
    assert np.any(ref["den"] == 0)
    C = to_views(ctx, rgb)[0]
    compare_image(C, ref, label="w_B=0")
    r = ws.upstream_grad(cams, seed=2)[0]
    gg = grads_to_numpy(ctx.render_bwd(dev, g, torch.from_numpy(r.reshape(-1, 3)).cuda(), rgb, den))
    gref = oracle.render_bwd(sc, cams[0], st, r)
    compare_grads(gg, gref, _grad_keys(st, 1), label="w_B=0")
    _check_globals(gg["globals"], _oracle_globals(st, gref["globals"]), "w_B=0")


def test_ragged_image_and_single_gaussian():
    sc, _, st = ws.make_scene("c1", n=1)
    sc["means"][:] = 0.0
    sc["log_scales"][:] = -1.5
    for (w, h) in ((100, 37), (1, 1), (33, 65)):
        cams = [ws.look_at_camera((0.0, 0.0, -4.0), w, h)]
        for tile in (8, 16, 32):
            log(f"case: single Gaussian {w}x{h} tile {tile}")
            ctx, dev, g, (rgb, den) = gpu_forward(sc, cams, st.copy(tile=tile))
            compare_image(to_views(ctx, rgb)[0], oracle.render(sc, cams[0], st, **amb_kw(st)), label=f"{w}x{h}")


@pytest.mark.parametrize("count", [1, 5, 8, 9, 16, 17, 32, 33, 64, 65, 100])
def test_one_block_lists_of_every_length(count):
    """count small splats inside the first 8x8 pixel block of a 32x32 view:
    that wave's culled list has exactly count entries, so the backward's last
    chunk takes each of its shapes (8, 4, 2 lanes per splat for tails of at
    most 8, 16, 32 splats, one lane above) and 65 and 100 add a full chunk."""
    from tests.oracle_helpers import dc_for_colour, scene_from
    rng = np.random.default_rng(1000 + count)
    cam = ws.look_at_camera((0.0, 0.0, -4.0), 32, 32)
    V = np.asarray(cam["viewmat"])
    R, Tv = V[:, :3], V[:, 3]
    px = rng.uniform(2.5, 5.5, (count, 2))
    pc = np.stack([(px[:, 0] - cam["cx"]) * 4.0 / cam["fx"], (px[:, 1] - cam["cy"]) * 4.0 / cam["fy"],
                   np.full(count, 4.0)], axis=1)
    means = (pc - Tv) @ R  # world positions (R is a rotation)
    sh = np.zeros((1, count, 4))
    sh[0, :, :3] = dc_for_colour(rng.uniform(0.05, 0.95, (count, 3)))
    quats = rng.normal(size=(4, count))
    sc = scene_from(means, log_scales=rng.uniform(-4.3, -3.7, (3, count)), quats=quats, sh=sh,
                    logit=rng.normal(0.0, 1.0, count), dtype=np.float32)
    st = ws.Settings()
    cams = [cam]
    p = oracle.project(sc, cam, st)
    assert p["visible"].all()
    log(f"case: one-block lists, {count} splats")
    ctx, dev, g, (rgb, den, cnt) = gpu_forward(sc, cams, st, count=True)
    compare_image(to_views(ctx, rgb)[0], oracle.render(sc, cam, st, **amb_kw(st)), label=f"{count} splats")
    counts = to_views(ctx, cnt)[0]
    assert counts[8:].sum() == 0 and counts[:, 8:].sum() == 0  # every pair lies in the first block
    r = rng.standard_normal((32, 32, 3)).astype(np.float32)
    grad2d = torch.zeros((1, ctx.n, 9), dtype=torch.float32, device="cuda")
    gg = grads_to_numpy(ctx.render_bwd(dev, g, torch.from_numpy(r.reshape(-1, 3)).cuda(), rgb, den,
                                       grad2d=grad2d))
    gref = oracle.render_bwd(sc, cam, st, r)
    compare_grads(gg, gref, _grad_keys(st, 1), label=f"{count} splats")
    compare_grads({"grad2d": grad2d[0].cpu().numpy()}, {"grad2d": gref["grad2d"]}, ["grad2d"],
                  label=f"{count} splats 2d")
    _check_globals(gg["globals"], _oracle_globals(st, gref["globals"]), f"{count} splats")


def test_huge_and_degenerate_splats():
    sc, cams, st = ws.make_scene("c1", n=50)
    sc["log_scales"][:, 0] = 1.0          # covers the whole image
    sc["quats"][:, 1] = 0.0               # zero quaternion: culled
    sc["log_scales"][:, 2] = [-30.0, -30.0, -30.0]  # vanishing: only the dilation remains
    log("case: huge / degenerate splats")
    ctx, dev, g, (rgb, den) = gpu_forward(sc, cams, st)
    ref = oracle.render(sc, cams[0], st, **amb_kw(st))
    compare_image(to_views(ctx, rgb)[0], ref, label="huge+degenerate")
    r = ws.upstream_grad(cams, seed=1)[0]
    gg = grads_to_numpy(ctx.render_bwd(dev, g, torch.from_numpy(r.reshape(-1, 3)).cuda(), rgb, den))
    gref = oracle.render_bwd(sc, cams[0], st, r)
    compare_grads(gg, gref, _grad_keys(st, 1), label="huge+degenerate")


def test_capacity_overflow_is_reported_then_recovered():
    sc, cams, st = ws.make_scene("c1")
    log("case: id-list overflow")
    ctx = WSRContext(sc["means"].shape[1], cams, st, capacity=1000)
    dev = scene_to_device(sc)
    g = globals_tensor(st)
    ctx.project(dev, g)
    ctx.bin(grow=False)
    from paper_2410_18931_amd._lib import WSR_ERR_CAPACITY, WsrError
    with pytest.raises(WsrError) as ei:
        ctx.check()
    assert ei.value.status == WSR_ERR_CAPACITY
    rgb, den = ctx.render_fwd(g)     # incomplete but memory-safe
    torch.cuda.synchronize()
    ctx.bin(grow=True)
    ctx.check()
    rgb, den = ctx.render_fwd(g)
    compare_image(to_views(ctx, rgb)[0], oracle.render(sc, cams[0], st, **amb_kw(st)), label="after regrow")


# ---------------------------------------------------------------- graphs and autotuning

def _small_multiview():
    sc, _, st = ws.make_scene("c3", n=30000)
    rng = np.random.default_rng(11)
    cams = []
    for _ in range(3):
        w = int(rng.integers(96, 193))
        u = rng.standard_normal(3)
        cams.append(ws.look_at_camera(u / np.linalg.norm(u) * rng.uniform(4, 6), w, int(round(9 * w / 16))))
    return sc, cams, st


def test_graph_replays_match_eager():
    from paper_2410_18931_amd.graph import GraphStep
    sc, cams, st = _small_multiview()
    log("case: graph replay vs eager, views " + str([(c["width"], c["height"]) for c in cams]))
    dev = scene_to_device(sc)
    g = globals_tensor(st)
    ctx_e = WSRContext(sc["means"].shape[1], cams, st)
    rgb_e, den_e = ctx_e.forward(dev, g)
    dL = seeded_normal_like(rgb_e, 33)
    ge = ctx_e.render_bwd(dev, g, dL, rgb_e, den_e)
    ctx_g = WSRContext(sc["means"].shape[1], cams, st)
    step = GraphStep(ctx_g, dev, g, dL)
    for rep in range(3):
        step.replay()
        torch.cuda.synchronize()
        step.check()
        assert (step.rgb - rgb_e).abs().max().item() <= 1e-5, rep
        assert (step.den - den_e).abs().max().item() <= 1e-4 * den_e.abs().max().item(), rep
        for k in ("means", "log_scales", "quats", "sh", "lc_v"):
            d = (step.grads[k] - ge[k]).abs().max().item()
            assert d <= 1e-4 * ge[k].abs().max().item(), (rep, k, d)
        # eager work on the same device between replays
        ctx_e.forward(dev, g)
        torch.cuda.synchronize()


def test_autotune_picks_a_launch_configuration_and_caches(tmp_path):
    from paper_2410_18931_amd.autotune import BATCHES, autotune, candidates, config_name
    sc, cams, st = _small_multiview()
    log("case: autotune")
    dev = scene_to_device(sc)
    g = globals_tensor(st)
    cache = str(tmp_path / "tune.json")
    r1 = autotune(dev, cams, st, g, reps=3, cache=cache)
    log(f"autotune: {r1}")
    assert r1["tile"] in (8, 16, 32) and r1["batch"] in BATCHES[r1["tile"]] and not r1["cached"]
    assert set(r1["ms"]) == {config_name(*c) for c in candidates()} and len(r1["ms"]) == 12
    r2 = autotune(dev, cams, st, g, reps=3, cache=cache)
    assert r2["cached"] and (r2["tile"], r2["batch"], r2["persistent"]) == (r1["tile"], r1["batch"],
                                                                             r1["persistent"])


@pytest.mark.parametrize("tile,batch,persistent", [(16, 64, False), (16, 128, True), (16, 256, True),
                                                   (32, 128, False), (8, 64, True)])
def test_launch_configurations(tile, batch, persistent):
    """The raster batch size and the persistent launch only change how the
    work is scheduled (the uneven multi-view batch, every view's tiles in one
    launch).  The forward sums every pixel over its tile list in list order
    whatever the batch, and a work item computes the same sums whichever
    workgroup runs it, so the image equals the default launch's bit for bit,
    and so do the gradients when only the launch form changes.  Another batch
    size regroups the backward's chunks (a splat's pixels may then be summed
    by several lanes), so its gradients are held to the checker's at the
    gradient bar."""
    sc, cams, st = _small_multiview()
    st = st.copy(tile=tile)
    default_batch = 64 if tile == 8 else 256
    log(f"case: launch tile {tile} batch {batch} persistent {persistent}")
    dev = scene_to_device(sc)
    g = globals_tensor(st)
    rs = ws.upstream_grad(cams, seed=37)
    dL = torch.cat([torch.from_numpy(r.reshape(-1, 3)) for r in rs]).cuda()
    outs = []
    for s in (st, st.copy(batch=batch, persistent=persistent)):
        ctx = WSRContext(sc["means"].shape[1], cams, s)
        rgb, den = ctx.forward(dev, g)
        grads = ctx.render_bwd(dev, g, dL, rgb, den)
        torch.cuda.synchronize()
        ctx.check()
        outs.append((rgb, den, grads))
    (r1, d1, g1), (r2, d2, g2) = outs
    assert torch.equal(r1, r2) and torch.equal(d1, d2)
    if batch == default_batch:
        for k in g1:
            assert torch.equal(g1[k], g2[k]), k
    else:
        gref = oracle.render_bwd_views(sc, cams, st, rs)
        compare_grads(grads_to_numpy(g2), gref, _grad_keys(st, 16), label=f"batch {batch}")
        _check_globals(g2["globals"].cpu().numpy(), _oracle_globals(st, gref["globals"]), f"batch {batch}")


# ---------------------------------------------------------------- sharding proxy and reduced precision

@pytest.mark.parametrize("config,oit", [("c2", False), ("headline", False), ("headline", True)])
def test_full_step_is_bit_reproducible(config, oit):
    """The whole step -- projection, binning, forward, backward -- run twice
    on the same inputs in fresh workspaces gives bit-identical tile lists,
    images and gradients: the binning's scatter is stable (every tile list in
    Gaussian order), a split tile's partial sums are added in item order, and
    the backward forms every sum in a fixed order.  The 1 M / 1080p frame has
    tile lists longer than one work item, so the split path is exercised."""
    sc, cams, st = ws.make_scene(config)
    st = st.copy(oit=oit)
    log(f"case: bit reproducibility {config} oit={oit}")
    dev = scene_to_device(sc)
    g = globals_tensor(st)
    outs = []
    for rep in range(2):
        ctx = WSRContext(sc["means"].shape[1], cams, st)
        rgb, den = ctx.forward(dev, g)
        dL = seeded_normal_like(rgb, 35)
        grad2d = torch.zeros((1, ctx.n, 9), dtype=torch.float32, device="cuda")
        gr = ctx.render_bwd(dev, g, dL, rgb, den, grad2d=grad2d)
        torch.cuda.synchronize()
        ctx.check()
        # the list entries: (Gaussian id, Gaussian-major slot) per position
        ids = ctx.pairs[40 * ctx.capacity: 40 * ctx.capacity + 8 * ctx.last_pairs].clone()
        outs.append((ids, rgb, den, grad2d, gr))
        del ctx
    (i1, r1, d1, q1, g1), (i2, r2, d2, q2, g2) = outs
    assert torch.equal(i1, i2), "tile lists differ"
    assert torch.equal(r1, r2) and torch.equal(d1, d2), "images differ"
    assert torch.equal(q1, q2), "2D gradients differ"
    for k in g1:
        assert torch.equal(g1[k], g2[k]), k


def test_gaussian_shards_sum_to_the_full_render():
    """Eq. 7 is a sum over Gaussians: unnormalised renders of two disjoint
    shards add up to the full image, and each shard's backward (given the
    full C and D) gives the full-scene gradients of its Gaussians.

    The shard-summed image is checked against the checker's full render at
    the image bar, and against the GPU's own full render within the float32
    bound of re-ordered summation: both add the same per-pair terms (a
    pair's term depends only on its record and tile), so each sum of m terms
    is within gamma_m = m u / (1 - m u) of sum |term| of the exact value
    (u = 2^-24).  The shards' gradients are checked against the checker at
    the gradient bar on a crop (upstream gradient zero on the pixels with a
    pair within rounding of the cutoff)."""
    sc, cams, st = ws.make_scene("c2", n=60000)
    cam = cams[0]
    H, W = cam["height"], cam["width"]
    n = sc["means"].shape[1]
    perm = np.random.default_rng(12).permutation(n)
    shards = [np.sort(perm[: n // 2]), np.sort(perm[n // 2:])]
    log("case: shard sum")
    ctx, dev, g, (rgb, den, cnt) = gpu_forward(sc, cams, st, count=True)
    num = torch.zeros_like(rgb)
    dsum = torch.zeros_like(den)
    parts = []
    for idx in shards:
        s_sc = ws.permute(sc, idx)
        c_s = WSRContext(len(idx), cams, st)
        d_s = scene_to_device(s_sc)
        c_s.project(d_s, g)
        c_s.bin()
        N, D = c_s.render_fwd(g, unnormalised=True)
        num += N
        dsum += D
        parts.append((idx, c_s, d_s))
    wbg, bg = st.w_bg, torch.tensor(st.bg, device="cuda")
    C = ((bg * wbg + num) / (wbg + dsum)[:, None]).cpu().numpy().astype(np.float64).reshape(H, W, 3)
    ref = oracle.render(sc, cam, st, mode="aabb", **amb_kw(st))
    compare_image(C.astype(np.float32), ref, label="shard sum vs checker")
    # against the full GPU render: |dN| <= 2 gamma_m cmax sum|a| + rounding of
    # the final sums, |dD| <= 2 gamma_m sum|a| + ..., |dC| <= (|dN| + |C||dD|) / |D|
    u = 2.0 ** -24
    m = ref["count"].astype(np.float64) + 16.0   # pairs may flip within rounding of the cutoff
    gam = m * u / (1.0 - m * u)
    cmax = max(float(oracle.project(sc, cam, st)["rgb"].max()), float(max(st.bg)))
    s_abs = ref["abs_den"] - abs(wbg)
    Cf = rgb.cpu().numpy().astype(np.float64).reshape(H, W, 3)
    Df = np.abs(den.cpu().numpy().astype(np.float64).reshape(H, W))
    dN = 2 * gam * cmax * s_abs + 4 * u * (cmax * s_abs + abs(wbg) * max(st.bg))
    dD = 2 * gam * s_abs + 4 * u * ref["abs_den"]
    bound = (dN + np.abs(Cf).max(axis=-1) * dD) / np.where(Df == 0, 1.0, Df) + 8 * u * np.abs(Cf).max(axis=-1)
    diff = np.abs(C - Cf).max(axis=-1)
    log(f"[shard sum vs full render] max diff {diff.max():.3g}, smallest margin {(bound - diff).min():.3g}")
    assert (diff <= bound).all()
    dD_gpu = np.abs((wbg + dsum).cpu().numpy().astype(np.float64).reshape(H, W) - Df)
    assert (dD_gpu <= dD + 4 * u * Df).all()

    # backward: seeded upstream gradient on the densest crop
    crop = densest_crop(to_views(ctx, cnt)[0])
    x0, y0, x1, y1 = crop
    cref = oracle.render(sc, cam, st, crop=crop, **amb_kw(st))
    r = np.zeros((H, W, 3), np.float32)
    r[y0:y1, x0:x1] = np.random.default_rng(14).standard_normal((y1 - y0, x1 - x0, 3)) * unambiguous(cref)
    dL = torch.from_numpy(r.reshape(-1, 3)).cuda()
    gref = oracle.render_bwd(sc, cam, st, r[y0:y1, x0:x1], crop=crop)
    keys = _grad_keys(st, 16)
    full = grads_to_numpy(ctx.render_bwd(dev, g, dL, rgb, den))
    compare_grads(full, gref, keys, label="full scene")
    sig = 0.0
    for si, (idx, c_s, d_s) in enumerate(parts):
        gs = grads_to_numpy(c_s.render_bwd(d_s, g, dL, rgb, den))
        sref = {k: (gref[k][:, idx, :] if k == "sh" else gref[k][..., idx]) for k in keys}
        compare_grads(gs, sref, keys, label=f"shard {si}")
        # the background gradients are per-pixel terms summed per tile in a
        # fixed order: every shard forms them from the same dL/dC, C and D
        assert np.array_equal(gs["globals"][2:], full["globals"][2:])
        sig += float(gs["globals"][0])
    _check_globals(np.array([sig, 0.0, *full["globals"][2:]]), _oracle_globals(st, gref["globals"]), "shard sum")


@pytest.mark.parametrize("dt", ["f16", "bf16"])
def test_reduced_precision_batched_errors(dt):
    """16-bit storage of means, log-scales, quaternions and SH with float32
    arithmetic: against the checker on the dequantised inputs the kernels meet
    the float32 bars; against the float32 source the storage error is
    reported."""
    sc, _, st = ws.make_scene("c3", n=200000)
    rng = np.random.default_rng(13)
    cams = []
    for _ in range(4):
        w = int(rng.integers(320, 641))
        u = rng.standard_normal(3)
        cams.append(ws.look_at_camera(u / np.linalg.norm(u) * rng.uniform(4, 6), w, int(round(9 * w / 16))))
    q = ws.quantise(sc, dt)
    log(f"case: reduced precision {dt}")
    ctx, dev, g, (rgb, den, cnt) = gpu_forward(sc, cams, st, storage=dt, count=True)
    imgs, counts = to_views(ctx, rgb), to_views(ctx, cnt)
    rs = [np.zeros((c["height"], c["width"], 3), np.float32) for c in cams]
    crops = []
    worst_src = 0.0
    for v, cam in enumerate(cams):
        crop = densest_crop(counts[v], 48)
        crops.append(crop)
        x0, y0, x1, y1 = crop
        compare_image(imgs[v][y0:y1, x0:x1], oracle.render(q["f32"], cam, st, crop=crop, **amb_kw(st)),
                      label=f"{dt} view {v} vs dequantised")
        src = oracle.render(sc, cam, st, crop=crop)
        worst_src = max(worst_src, float(np.abs(imgs[v][y0:y1, x0:x1] - src["C"]).max()))
        rs[v][y0:y1, x0:x1] = rng.standard_normal((y1 - y0, x1 - x0, 3))
    log(f"[{dt}] image max-abs vs float32 source inputs: {worst_src:.3g}")
    dL = torch.cat([torch.from_numpy(r.reshape(-1, 3)) for r in rs]).cuda()
    gg = grads_to_numpy(ctx.render_bwd(dev, g, dL, rgb, den))
    gq = oracle.render_bwd_views(q["f32"], cams, st, [r[y0:y1, x0:x1] for r, (x0, y0, x1, y1) in zip(rs, crops)],
                                 crops)
    compare_grads(gg, gq, _grad_keys(st, 16), label=f"{dt} vs dequantised")
    gs = oracle.render_bwd_views(sc, cams, st, [r[y0:y1, x0:x1] for r, (x0, y0, x1, y1) in zip(rs, crops)], crops)
    for k in _grad_keys(st, 16):
        rel = np.abs(gg[k] - gs[k]).max() / max(np.abs(gs[k]).max(), 1e-30)
        log(f"[{dt}] grad {k} rel-to-max vs float32 source inputs: {rel:.3g}")


def test_culling_masks_follow_the_pair_buffer_room():
    """The raster backward takes the forward's per-wave culling masks from the
    pair buffer where it has room for them (a 64-bit word per wave and 64 list
    entries, plus one group per tile) and culls on its own otherwise.  A few
    Gaussians on a 1080p frame (8,160 tiles) need a large buffer for the
    masks: with the pair buffer sized to the pairs exactly there is no room,
    and the lists, image and gradients must equal those of a buffer with room
    bit for bit."""
    sc, _, st = ws.make_scene("c1", n=64)
    cams = [ws.look_at_camera((0.0, 0.0, -4.0), 1920, 1080)]
    log("case: culling masks with and without room, c1 n=64 at 1920x1080")
    dev = scene_to_device(sc)
    g = globals_tensor(st)
    big = WSRContext(64, cams, st)
    rgb_b, den_b = big.forward(dev, g)
    pairs = big.last_pairs
    tiles = ((1920 + st.tile - 1) // st.tile) * ((1080 + st.tile - 1) // st.tile)
    log(f"pairs {pairs}, tiles {tiles}, capacities {big.capacity} and {pairs}")
    assert 0 < pairs < 9 * tiles  # then a buffer of `pairs` entries has no room for the masks
    small = WSRContext(64, cams, st, capacity=pairs)
    rgb_s, den_s = small.forward(dev, g)
    dL = seeded_normal_like(rgb_b, 17)
    gb = big.render_bwd(dev, g, dL, rgb_b, den_b)
    gs = small.render_bwd(dev, g, dL, rgb_s, den_s)
    torch.cuda.synchronize()
    big.check()
    small.check()
    assert torch.equal(rgb_b, rgb_s) and torch.equal(den_b, den_s)
    for k in ("means", "log_scales", "quats", "sh", "opacity_logit", "globals"):
        assert torch.equal(gb[k], gs[k]), k
