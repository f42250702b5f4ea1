"""The C-ABI library loads and exports every entry point include/wsr.h
declares; host-side argument checks reject bad input before any launch.
No compute calls (these run without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import wsr_synth as ws
from paper_2410_18931_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wsr.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(wsr_[a-z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    lib = _lib.load()
    names = _declared()
    assert len(names) >= 9
    for nm in names:
        assert hasattr(lib, nm), nm
    assert set(names) == set(_lib.EXPORTED)


def test_abi_version_and_status_strings():
    lib = _lib.load()
    assert lib.wsr_abi_version() == _lib.ABI_VERSION
    for s in range(5):
        assert _lib.status_string(s)
    assert "overflow" in _lib.status_string(_lib.WSR_ERR_CAPACITY)


def test_workspace_bytes_validation():
    lib = _lib.load()
    _, cams, st = ws.make_scene("c1", n=8)
    cc = _lib.make_cameras(cams)
    good = lib.wsr_workspace_bytes(8, cc, 1, 16)
    assert good > 0
    assert lib.wsr_workspace_bytes(8, cc, 1, 12) == -1          # tile must be 8/16/32
    assert lib.wsr_workspace_bytes(-1, cc, 1, 16) == -1
    assert lib.wsr_workspace_bytes(8, cc, 0, 16) == -1
    assert lib.wsr_workspace_bytes(8, cc, 300, 16) == -1         # > WSR_MAX_VIEWS
    assert lib.wsr_workspace_bytes(8, None, 1, 16) == -1
    big = dict(cams[0], width=40000)
    assert lib.wsr_workspace_bytes(8, _lib.make_cameras([big]), 1, 16) == -1
    # more Gaussians, more views and smaller tiles all need more space
    assert lib.wsr_workspace_bytes(80000, cc, 1, 16) > good
    assert lib.wsr_workspace_bytes(8, _lib.make_cameras(cams * 3), 3, 16) > good
    assert lib.wsr_workspace_bytes(8, cc, 1, 8) > lib.wsr_workspace_bytes(8, cc, 1, 32)


def test_entry_points_reject_bad_arguments_before_launch():
    lib = _lib.load()
    sc, cams, st = ws.make_scene("c1", n=8)
    cc = _lib.make_cameras(cams)
    p = _lib.make_params(st)
    bad_tile = _lib.make_params(st.copy(tile=12))
    dummy = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    scene = _lib.WsrScene(8, 0, 0, 0, 0, dummy, dummy, dummy, dummy, dummy, dummy)
    bad_deg = _lib.WsrScene(8, 4, 0, 0, 0, dummy, dummy, dummy, dummy, dummy, dummy)
    no_means = _lib.WsrScene(8, 0, 0, 0, 0, None, dummy, dummy, dummy, dummy, dummy)
    INV, WSP = _lib.WSR_ERR_INVALID, _lib.WSR_ERR_WORKSPACE
    assert lib.wsr_project(C.byref(bad_deg), cc, 1, C.byref(p), dummy, dummy, 1 << 30, None, None) == INV
    assert lib.wsr_project(C.byref(no_means), cc, 1, C.byref(p), dummy, dummy, 1 << 30, None, None) == INV
    assert lib.wsr_project(C.byref(scene), cc, 1, C.byref(bad_tile), dummy, dummy, 1 << 30, None, None) == INV
    assert lib.wsr_project(C.byref(scene), cc, 1, C.byref(p), None, dummy, 1 << 30, None, None) == INV
    assert lib.wsr_project(C.byref(scene), cc, 1, C.byref(p), dummy, dummy, 16, None, None) == WSP
    assert lib.wsr_bin(cc, 1, C.byref(p), 8, dummy, 16, dummy, 10, None) == WSP
    assert lib.wsr_bin(cc, 1, C.byref(p), 8, dummy, 1 << 30, None, 10, None) == INV
    assert lib.wsr_render_fwd(cc, 1, C.byref(p), 8, dummy, dummy, 1 << 30, dummy, 10, None, dummy, None,
                              None) == INV
    g = _lib.WsrGrads(dummy, dummy, dummy, dummy, dummy, dummy, None)
    assert lib.wsr_render_bwd(C.byref(scene), cc, 1, C.byref(p), dummy, dummy, 1 << 30, dummy, 10, dummy,
                              dummy, dummy, C.byref(g), None, None) == INV
    # raster batch sizes a tile size is not built for
    for tile, batch in ((16, 100), (8, 128), (32, 64), (16, 512)):
        bad_batch = _lib.make_params(st.copy(tile=tile, batch=batch))
        assert lib.wsr_bin(cc, 1, C.byref(bad_batch), 8, dummy, 1 << 30, dummy, 10, None) == INV
    assert lib.wsr_bin(cc, 1, C.byref(_lib.make_params(st.copy(tile=8, batch=64, persistent=True))), 8, dummy,
                       16, dummy, 10, None) == WSP     # a valid batch and flag pass the checks
    out = C.c_int64(0)
    assert lib.wsr_pair_count(None, 0, C.byref(out), None) == INV
    assert lib.wsr_check(None, 0, None) == INV


def test_lc_requires_weights_and_logit_mode_requires_logits():
    lib = _lib.load()
    _, cams, st = ws.make_scene("c1", n=8)
    cc = _lib.make_cameras(cams)
    dummy = C.c_void_p(0x1000)
    p_lc = _lib.make_params(st.copy(weight_kind="lc"))
    no_v = _lib.WsrScene(8, 0, 0, 0, 0, dummy, dummy, dummy, dummy, dummy, None)
    assert lib.wsr_project(C.byref(no_v), cc, 1, C.byref(p_lc), dummy, dummy, 1 << 30, None, None) == 1
    p = _lib.make_params(st)
    no_logit = _lib.WsrScene(8, 0, 0, 0, 0, dummy, dummy, dummy, dummy, None, dummy)
    assert lib.wsr_project(C.byref(no_logit), cc, 1, C.byref(p), dummy, dummy, 1 << 30, None, None) == 1


def test_loss_and_adam_reject_bad_arguments_before_launch():
    lib = _lib.load()
    _, cams, _ = ws.make_scene("c1", n=8)
    cc = _lib.make_cameras(cams)
    dummy = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    INV, WSP = _lib.WSR_ERR_INVALID, _lib.WSR_ERR_WORKSPACE
    need = lib.wsr_loss_workspace_bytes(cc, 1)
    # 9 float maps per pixel plus one FP64 share per (16x16 tile, channel)
    assert need >= 9 * 4 * 128 * 128 + 8 * 3 * 64
    assert lib.wsr_loss_workspace_bytes(cc, 0) == -1
    assert lib.wsr_loss_workspace_bytes(None, 1) == -1
    F = C.c_float
    assert lib.wsr_loss(cc, 1, dummy, dummy, F(0.2), dummy, need - 1, dummy, dummy, None) == WSP
    assert lib.wsr_loss(cc, 1, dummy, dummy, F(1.5), dummy, need, dummy, dummy, None) == INV
    assert lib.wsr_loss(cc, 1, None, dummy, F(0.2), dummy, need, dummy, dummy, None) == INV
    assert lib.wsr_loss(cc, 1, dummy, dummy, F(0.2), C.c_void_p(0x1004), need, dummy, dummy, None) == INV
    # the allocation-free variant: the same checks, and a request beyond its
    # static workspace refused before any device call
    assert lib.wsr_loss_noalloc(cc, 1, None, dummy, F(0.2), dummy, dummy, None) == INV
    assert lib.wsr_loss_noalloc(cc, 1, dummy, dummy, F(-0.1), dummy, dummy, None) == INV
    assert lib.wsr_loss_noalloc(cc, 0, dummy, dummy, F(0.2), dummy, dummy, None) == INV
    big = _lib.make_cameras([ws.look_at_camera((0.0, 0.0, -4.0), 1920, 1090)])
    assert lib.wsr_loss_workspace_bytes(big, 1) > _lib.LOSS_STATIC_BYTES
    assert lib.wsr_loss_noalloc(big, 1, dummy, dummy, F(0.2), dummy, dummy, None) == _lib.WSR_ERR_STATIC
    hd = _lib.make_cameras([ws.look_at_camera((0.0, 0.0, -4.0), 1920, 1080)])
    assert lib.wsr_loss_workspace_bytes(hd, 1) <= _lib.LOSS_STATIC_BYTES
    assert "static" in _lib.status_string(_lib.WSR_ERR_STATIC)
    assert lib.wsr_adam(dummy, dummy, dummy, dummy, 10, 0, F(0.1), F(0.9), F(0.999), F(1e-15), None) == INV
    assert lib.wsr_adam(dummy, dummy, dummy, dummy, 10, 1, F(0.1), F(1.0), F(0.999), F(1e-15), None) == INV
    assert lib.wsr_adam(None, dummy, dummy, dummy, 10, 1, F(0.1), F(0.9), F(0.999), F(1e-15), None) == INV
    assert lib.wsr_adam(None, None, None, None, 0, 1, F(0.1), F(0.9), F(0.999), F(1e-15), None) == _lib.WSR_OK


def test_sorted_entry_points_reject_bad_arguments_before_launch():
    lib = _lib.load()
    _, cams, st = ws.make_scene("c1", n=8)
    cc = _lib.make_cameras(cams)
    dummy = C.c_void_p(0x1000)
    INV = _lib.WSR_ERR_INVALID
    p_exp = _lib.make_params(st)                      # EXP weight: not allowed for sorted blending
    p_dir = _lib.make_params(st.copy(weight_kind="dir"))
    ok = _lib.WsrBlend(0.99, 0.0, 0.0, 0)
    assert lib.wsr_render_sorted(cc, 1, C.byref(p_exp), 8, dummy, C.byref(ok), dummy, 1 << 30, dummy, 10,
                                 dummy, dummy, None) == INV
    for bad in (_lib.WsrBlend(0.0, 0.0, 0.0, 0), _lib.WsrBlend(1.5, 0.0, 0.0, 0), _lib.WsrBlend(0.9, -1.0, 0.0, 0),
                _lib.WsrBlend(0.9, 0.0, -1.0, 0)):
        assert lib.wsr_render_sorted(cc, 1, C.byref(p_dir), 8, dummy, C.byref(bad), dummy, 1 << 30, dummy, 10,
                                     dummy, dummy, None) == INV
    assert lib.wsr_render_sorted(cc, 1, C.byref(p_dir), 8, dummy, C.byref(ok), dummy, 16, dummy, 10,
                                 dummy, dummy, None) == _lib.WSR_ERR_WORKSPACE
    assert lib.wsr_sort_tiles(cc, 1, C.byref(p_dir), 8, dummy, 1 << 30, C.c_void_p(0x1004), 10, None) == INV
    assert lib.wsr_sort_tiles(cc, 1, C.byref(p_dir), 8, dummy, 16, dummy, 10, None) == _lib.WSR_ERR_WORKSPACE
    assert "sort" in _lib.status_string(_lib.WSR_ERR_TILE_LIST)


def test_fused_adam_backward_rejects_bad_arguments_before_launch():
    lib = _lib.load()
    _, cams, st = ws.make_scene("c1", n=8)
    cc = _lib.make_cameras(cams)
    p = _lib.make_params(st)
    dummy = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    INV, WSP = _lib.WSR_ERR_INVALID, _lib.WSR_ERR_WORKSPACE
    f32 = _lib.WsrScene(8, 0, 0, 0, 0, dummy, dummy, dummy, dummy, dummy, dummy)
    bf16 = _lib.WsrScene(8, 0, 2, 0, 0, dummy, dummy, dummy, dummy, dummy, dummy)
    mom = _lib.WsrGrads(dummy, dummy, dummy, dummy, None, None, None)
    no_sh = _lib.WsrGrads(dummy, dummy, dummy, None, None, None, None)

    def adam(**kw):
        a = dict(lr_means=1e-4, lr_log_scales=5e-3, lr_quats=1e-3, lr_sh0=2.5e-3, lr_shN=1.25e-4,
                 lr_opacity_logit=5e-2, lr_lc_v=1e-3, beta1=0.9, beta2=0.999, eps=1e-15, step=1, reserved_=0)
        a.update(kw)
        return _lib.WsrAdamParams(**a)

    def call(scene, m, v, hp, ws_bytes=1 << 30, grad_globals=dummy):
        return lib.wsr_project_bwd_adam(C.byref(scene), cc, 1, C.byref(p), dummy, dummy, ws_bytes, dummy, 10,
                                        C.byref(m), C.byref(v), C.byref(hp), grad_globals, None, None)

    assert call(f32, mom, mom, adam(), ws_bytes=16) == WSP      # valid settings reach the workspace check
    assert call(bf16, mom, mom, adam(), ws_bytes=16) == INV     # the update needs FP32 storage
    assert call(f32, mom, no_sh, adam(), ws_bytes=16) == INV    # every per-Gaussian moment array
    assert call(f32, mom, mom, adam(step=0), ws_bytes=16) == INV
    assert call(f32, mom, mom, adam(beta1=1.0), ws_bytes=16) == INV
    assert call(f32, mom, mom, adam(beta2=-0.1), ws_bytes=16) == INV
    assert call(f32, mom, mom, adam(), ws_bytes=16, grad_globals=None) == INV
