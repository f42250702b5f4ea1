"""The seeded synthetic workloads hold the sizes, distributions and structure
their recipe states (the stand-in for the paper's captured scenes), and are
reproducible from their seed."""
import numpy as np
import pytest

import wsr_synth as ws


def test_same_seed_same_scene_other_seed_other_scene():
    a, ca, _ = ws.make_scene("c1", seed=3)
    b, cb, _ = ws.make_scene("c1", seed=3)
    c, _, _ = ws.make_scene("c1", seed=4)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    assert not np.array_equal(a["means"], c["means"])
    assert np.array_equal(np.asarray(ca[0]["viewmat"]), np.asarray(cb[0]["viewmat"]))


@pytest.mark.parametrize("config,n,size,degree", [("c1", 4096, (128, 128), 0), ("c2", 200_000, (1280, 720), 3)])
def test_small_configurations(config, n, size, degree):
    sc, cams, st = ws.make_scene(config)
    assert sc["means"].shape == (3, n)
    assert (cams[0]["width"], cams[0]["height"]) == size
    assert ws.sh_degree(sc) == degree
    ls = sc["log_scales"].astype(np.float64)
    mu, sd = (-3.0, 0.5) if config == "c1" else (-4.0, 0.7)
    assert abs(ls.mean() - mu) < 0.02 and abs(ls.std() - sd) < 0.02
    # degree-0 colour uniform on [0, 1]: DC coefficients on (-sqrt(pi), sqrt(pi))
    dc = sc["sh"][0, :, :3].astype(np.float64)
    assert dc.min() >= -np.sqrt(np.pi) and dc.max() <= np.sqrt(np.pi)
    assert abs(dc.mean()) < 0.05
    q = sc["quats"].astype(np.float64)
    assert np.allclose(np.linalg.norm(q, axis=0), 1.0, atol=1e-6)
    if config == "c2":
        assert st.weight_kind == "lc" and st.opacity_mode == "sh"
        v = sc["lc_v"].astype(np.float64)
        assert v.min() >= 0.5 and v.max() <= 1.5


def test_headline_and_batch_configurations():
    sc, cams, st = ws.make_scene("headline")
    assert sc["means"].shape == (3, 1_000_000)
    assert len(cams) == 1 and (cams[0]["width"], cams[0]["height"]) == (1920, 1080)
    assert ws.sh_degree(sc) == 3 and st.tile == 16 and st.tau == 9.0
    sc4, cams4, _ = ws.make_scene("c4")
    assert sc4["means"].shape == (3, 1_000_000) and len(cams4) == 16
    for c in cams4:
        assert 640 <= c["width"] <= 1920 and c["height"] == round(9 * c["width"] / 16)
    # cameras are float32-exact: the renderer and the reference see the same numbers
    for c in cams + cams4:
        for key in ("fx", "fy", "cx", "cy"):
            assert float(np.float32(c[key])) == c[key]
        vm = np.asarray(c["viewmat"], dtype=np.float64)
        assert np.array_equal(vm.astype(np.float32).astype(np.float64), vm)
