"""The allocation-free loss entry point (wsr_loss_noalloc, static workspace)
against wsr_loss with a caller-allocated workspace, through the C-ABI: the
same kernels on the same inputs, so the loss and its image gradient must be
bit-identical.  Two calls in a row on one device, the second smaller than
the first (the static array still holds the first call's contents), then a
request larger than the static workspace, which is refused before any
launch."""
import ctypes as C

import numpy as np
import pytest
import torch

import wsr_synth as ws
from paper_2410_18931_amd import _lib
from paper_2410_18931_amd.train import Loss, loss_noalloc

pytestmark = pytest.mark.gpu


def _images(cams, seed):
    rng = np.random.default_rng(seed)
    P = sum(c["width"] * c["height"] for c in cams)
    img = torch.from_numpy(rng.uniform(0.0, 1.0, (P, 3)).astype(np.float32)).cuda()
    tgt = torch.from_numpy(rng.uniform(0.0, 1.0, (P, 3)).astype(np.float32)).cuda()
    return img, tgt


def _both(cams, seed, lam=0.2):
    img, tgt = _images(cams, seed)
    ref_loss, ref_dL = Loss(cams, lam)(img, tgt)
    loss = torch.full((1,), float("nan"), device="cuda")
    dL = torch.full_like(img, float("nan"))
    loss_noalloc(_lib.make_cameras(cams), len(cams), img, tgt, lam, loss, dL)
    torch.cuda.synchronize()
    return (ref_loss.clone(), ref_dL), (loss, dL)


def test_noalloc_loss_equals_workspace_loss_on_two_calls():
    # first call: the largest input the static workspace takes, one 1080p view
    big = [ws.look_at_camera((0.0, 0.0, -4.0), 1920, 1080)]
    print("case: noalloc loss 1920x1080", flush=True)
    (l0, g0), (l1, g1) = _both(big, seed=1)
    assert torch.isfinite(l1).all() and torch.isfinite(g1).all()
    assert torch.equal(l0, l1), (l0.item(), l1.item())
    assert torch.equal(g0, g1)
    # second call: smaller, ragged, several views
    small = [ws.look_at_camera((0.0, 0.0, -4.0), 317, 181), ws.look_at_camera((1.0, 0.0, -4.0), 64, 37),
             ws.look_at_camera((0.0, 2.0, -4.0), 200, 90)]
    print("case: noalloc loss three ragged views", flush=True)
    (l0, g0), (l1, g1) = _both(small, seed=2, lam=0.35)
    assert torch.equal(l0, l1), (l0.item(), l1.item())
    assert torch.equal(g0, g1)


def test_noalloc_loss_refuses_more_than_its_static_workspace():
    cams = [ws.look_at_camera((0.0, 0.0, -4.0), 1920, 1090)]
    cc = _lib.make_cameras(cams)
    lib = _lib.load()
    assert lib.wsr_loss_workspace_bytes(cc, 1) > _lib.LOSS_STATIC_BYTES
    img, tgt = _images(cams, 3)
    loss = torch.zeros((1,), device="cuda")
    dL = torch.zeros_like(img)
    st = lib.wsr_loss_noalloc(cc, 1, C.c_void_p(img.data_ptr()), C.c_void_p(tgt.data_ptr()), C.c_float(0.2),
                              C.c_void_p(loss.data_ptr()), C.c_void_p(dL.data_ptr()),
                              C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.WSR_ERR_STATIC
    torch.cuda.synchronize()
    assert loss.item() == 0.0 and dL.abs().max().item() == 0.0   # nothing ran
