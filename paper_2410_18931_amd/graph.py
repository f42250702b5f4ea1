"""One forward + backward step of the WSR path captured as a HIP graph.

Every kernel of the step (projection, binning, raster forward, raster
backward, projection backward) is enqueued through the C-ABI on the capture
stream, so a replay is a single graph launch with no host work.  Buffers are
static: inputs are read from, and outputs written to, the tensors held by the
step, so callers copy new data into ``step.scene`` / ``step.globals_`` /
``step.dL`` between replays.

The id-list capacity must be sized before capture (a replay cannot grow it);
``GraphStep`` does that with one eager, synchronising binning pass, and
``check()`` after a replay reports an overflow (then rebuild the step).
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from .render import WSRContext

_GRAD_KEYS = ("means", "log_scales", "quats", "sh", "opacity_logit", "lc_v", "globals")


class GraphStep:
    def __init__(self, ctx: WSRContext, scene: dict, globals_: torch.Tensor, dL: torch.Tensor | None = None,
                 backward: bool = True, headroom: float = 1.1):
        self.ctx = ctx
        self.scene = scene
        self.globals_ = globals_
        self.backward = backward
        P = ctx.total_pixels
        dev = ctx.device
        self.rgb = torch.empty((P, 3), dtype=torch.float32, device=dev)
        self.den = torch.empty((P,), dtype=torch.float32, device=dev)
        self.dL = dL if dL is not None else torch.zeros((P, 3), dtype=torch.float32, device=dev)
        self.grads = ctx.alloc_grads(scene) if backward else None
        # size the pair buffer eagerly (one synchronising pass), with headroom
        ctx.project(scene, globals_)
        ctx.bin(grow=True)
        need = int(ctx.last_pairs * headroom) + 1024
        if need > ctx.capacity:
            ctx._alloc_pairs(need)
        self._sc = ctx.scene_struct(scene)
        if backward:
            g = self.grads
            self._gs = _lib.WsrGrads(*(g[k].data_ptr() for k in _GRAD_KEYS))
        self.graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            self._enqueue()          # warm-up outside capture
        torch.cuda.current_stream(dev).wait_stream(side)
        torch.cuda.synchronize(dev)
        with torch.cuda.graph(self.graph):
            self._enqueue()

    def _enqueue(self):
        ctx, lib = self.ctx, self.ctx.lib
        sp = C.c_void_p(torch.cuda.current_stream(ctx.device).cuda_stream)
        p = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
        ws = p(ctx.ws)
        _lib.check("wsr_project", lib.wsr_project(C.byref(self._sc), ctx.cams_c, ctx.nv, C.byref(ctx.params),
                                                  p(self.globals_), ws, ctx.ws_bytes, None, sp))
        _lib.check("wsr_bin", lib.wsr_bin(ctx.cams_c, ctx.nv, C.byref(ctx.params), ctx.n, ws, ctx.ws_bytes,
                                          p(ctx.pairs), ctx.capacity, sp))
        _lib.check("wsr_render_fwd", lib.wsr_render_fwd(ctx.cams_c, ctx.nv, C.byref(ctx.params), ctx.n,
                                                        p(self.globals_), ws, ctx.ws_bytes, p(ctx.pairs),
                                                        ctx.capacity, p(self.rgb), p(self.den), None, sp))
        if self.backward:
            _lib.check("wsr_render_bwd", lib.wsr_render_bwd(C.byref(self._sc), ctx.cams_c, ctx.nv,
                                                            C.byref(ctx.params), p(self.globals_), ws, ctx.ws_bytes,
                                                            p(ctx.pairs), ctx.capacity, p(self.dL), p(self.rgb),
                                                            p(self.den), C.byref(self._gs), None, sp))

    def replay(self):
        self.graph.replay()

    def check(self):
        self.ctx.check()
