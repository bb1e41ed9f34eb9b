"""Renderer objects over the C ABI: workspaces, capacity management, the
autograd function and the batched multi-view renderer.

Everything here is bookkeeping around libgs.so: tensors are allocated once
and reused, each call enqueues the five hot-path entry points on torch's
current stream.  Key-buffer overflow (more tile instances than capacity) is
detected on the device; `Renderer.render` checks the flag once per call
(eager mode) and re-runs the binning with a larger capacity, while graph
replays (`CapturedRender`) never synchronise and check the flag afterwards
(`CapturedRender.overflowed`).
"""
from __future__ import annotations

import math

import torch

from . import binding as B


def _grow(n):
    return max(1 << 16, 1 << int(math.ceil(math.log2(max(1, int(n * 1.25))))))


class Frame:
    """Device outputs and saved state of one forward call."""

    def __init__(self):
        self.rgb = self.depth = self.alpha = self.t_final = self.n_contrib = None
        self.tiles_touched = self.rec = self.keys = self.vals = self.ranges = None
        self.num = self.overflow = self.order = self.ckpt = None


class Renderer:
    """Forward (and backward) renderer for a fixed image size.

    segments: list of gaussian dicts of device tensors (means [n,3],
    log_scales [n,3], quats [n,4], opacity [n], sh [n,K,3], sh_degree, or
    cov6 [n,6] instead of log_scales/quats); cams: [V,16] float32 device
    tensor; view_segs: per-view lists of segment indices."""

    # Segment checkpoints pay off while the (view, tile) lists alone leave
    # the GPU short of waves (four per list): up to this many lists.
    AUTO_CHECKPOINT_ITEMS = 2048

    def __init__(self, width, height, bg=(0.0, 0.0, 0.0), capacity=1 << 20, device="cuda", checkpoints=False,
                 **overrides):
        """checkpoints: True / False / "auto" -- the forward records segment
        checkpoints so that the backward differentiates long tile lists in
        parallel segments ("auto": when there are at most
        AUTO_CHECKPOINT_ITEMS (view, tile) lists)."""
        B.load()
        if checkpoints not in (True, False, "auto"):
            raise ValueError("checkpoints must be True, False or 'auto'")
        self.checkpoints = checkpoints
        self.W, self.H = int(width), int(height)
        self.params = B.make_params(self.W, self.H, bg=bg, **overrides)
        self.TX = (self.W + B.TILE - 1) // B.TILE
        self.TY = (self.H + B.TILE - 1) // B.TILE
        self.T = self.TX * self.TY
        self.device = torch.device(device)
        self.capacity = int(capacity)
        self._bufs = {}

    # -- buffers ------------------------------------------------------------
    def _buf(self, name, shape, dtype, zero=False):
        t = self._bufs.get(name)
        n = 1
        for s in shape:
            n *= int(s)
        if t is None or t.numel() < n or t.dtype != dtype:
            t = (torch.zeros if zero else torch.empty)(max(n, 1), dtype=dtype, device=self.device)
            self._bufs[name] = t
        return t[:n].view(*shape) if len(shape) else t[:1]

    def alloc_frame(self, n_inst, n_views, ckpt=False):
        f = Frame()
        f.tiles_touched = self._buf("tt", (n_inst,), torch.int32)
        f.rec = self._buf("rec", (n_inst, B.REC_FLOATS), torch.float32)
        f.keys = self._buf("keys", (self.capacity,), torch.int64)
        f.vals = self._buf("vals", (self.capacity,), torch.int32)
        f.ranges = self._buf("ranges", (n_views * self.T, 2), torch.int32)
        f.order = self._buf("order", (B.tile_order_words(n_views, self.params),), torch.int32)
        f.ckpt = self._buf("ckpt", (B.checkpoint_floats(self.capacity),), torch.float32) if ckpt else None
        f.num = self._buf("num", (1,), torch.int64)
        f.overflow = self._buf("ovf", (1,), torch.int32)
        ws = B.bin_sort_workspace(n_inst, self.capacity, n_views, self.params)
        f.sort_ws = self._buf("sort_ws", ((ws + 255) // 256 * 256,), torch.uint8)
        # zeroed once; gs_composite leaves its queue counters at zero
        f.comp_ws = self._buf("comp_ws", (B.composite_workspace(n_views, self.params),), torch.uint8, zero=True)
        hw = (n_views, self.H, self.W)
        f.rgb = self._buf("rgb", hw + (3,), torch.float32)
        f.depth = self._buf("depth", hw, torch.float32)
        f.alpha = self._buf("alpha", hw, torch.float32)
        f.t_final = self._buf("t_final", hw, torch.float32)
        f.n_contrib = self._buf("n_contrib", hw, torch.int32)
        return f

    # -- stages ---------------------------------------------------------------
    def project(self, segs, cams, view_segs, f):
        B.project(segs, cams, view_segs, self.params, f.tiles_touched, f.rec)

    def bin_sort(self, f, n_views):
        B.bin_sort(f.tiles_touched, f.rec, n_views, self.params, f.sort_ws, f.keys, f.vals, f.ranges, f.num,
                   f.overflow, order=f.order)

    def composite(self, f, n_views):
        B.composite(f.rec, f.vals, f.ranges, n_views, self.params, f.comp_ws, f.rgb, f.depth, f.alpha, f.t_final,
                    f.n_contrib, order=f.order, ckpt=f.ckpt)

    def enqueue(self, segs, cams, view_segs, f):
        """All forward stages, no host synchronisation."""
        n_views = len(view_segs)
        self.project(segs, cams, view_segs, f)
        self.bin_sort(f, n_views)
        self.composite(f, n_views)

    def render(self, segs, cams, view_segs=None, sync_check=True, checkpoints=None):
        """Eager forward.  Returns a Frame whose tensors are views of the
        renderer's buffers (valid until the next call).  checkpoints (default:
        the renderer's setting; True, False or "auto") records segment
        checkpoints for a faster backward."""
        if view_segs is None:
            view_segs = [list(range(len(segs)))] * int(cams.shape[0])
        mode = self.checkpoints if checkpoints is None else checkpoints
        n_views = len(view_segs)
        ckpt = (n_views * self.T <= self.AUTO_CHECKPOINT_ITEMS) if mode == "auto" else bool(mode)
        n_inst = B.instance_offsets(segs, view_segs)[-1]
        f = self.alloc_frame(n_inst, n_views, ckpt)
        self.project(segs, cams, view_segs, f)
        self.bin_sort(f, n_views)
        if sync_check and int(f.overflow.item()):
            self.capacity = min(_grow(int(f.num.item())), B.MAX_CAPACITY)
            f = self.alloc_frame(n_inst, n_views, ckpt)
            self.project(segs, cams, view_segs, f)
            self.bin_sort(f, n_views)
            if int(f.overflow.item()):
                raise RuntimeError("tile instances %d exceed the maximum capacity" % int(f.num.item()))
        self.composite(f, n_views)
        f.n_views = n_views
        f.n_inst = n_inst
        return f

    def backward(self, segs, cams, view_segs, f, d_rgb, d_depth, d_alpha):
        """Dense gradients (list of dicts per segment) for the frame f."""
        grads = []
        for g in segs:
            n = int(g["means"].shape[0])
            K = (int(g["sh_degree"]) + 1) ** 2
            d = {"means": torch.empty(n, 3, device=self.device), "opacity": torch.empty(n, device=self.device),
                 "sh": torch.empty(n, K, 3, device=self.device)}
            if g.get("cov6") is not None:
                d["cov6"] = torch.empty(n, 6, device=self.device)
            else:
                d["log_scales"] = torch.empty(n, 3, device=self.device)
                d["quats"] = torch.empty(n, 4, device=self.device)
            grads.append(d)
        ws = self._buf("bwd_ws", ((B.render_backward_workspace(f.n_inst) + 3) // 4,), torch.float32)
        B.render_backward(segs, cams, view_segs, self.params, f.tiles_touched, f.rec, f.vals, f.ranges, f.t_final,
                          f.n_contrib, d_rgb, d_depth, d_alpha, ws, grads, ckpt=f.ckpt, order=f.order)
        return grads


def _c(t):
    return None if t is None else t.contiguous()


class _RasterizeFn(torch.autograd.Function):
    """One gaussian set (scale/rotation parametrised), V views."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity, sh, cams, renderer, sh_degree):
        seg = {"means": means.contiguous(), "log_scales": log_scales.contiguous(), "quats": quats.contiguous(),
               "opacity": opacity.contiguous(), "sh": sh.contiguous(), "sh_degree": sh_degree}
        view_segs = [[0]] * int(cams.shape[0])
        f = renderer.render([seg], cams, view_segs, checkpoints="auto")
        ctx.renderer, ctx.seg, ctx.view_segs, ctx.frame = renderer, seg, view_segs, f
        ctx.save_for_backward(cams)
        return f.rgb.clone(), f.depth.clone(), f.alpha.clone()

    @staticmethod
    def backward(ctx, d_rgb, d_depth, d_alpha):
        (cams,) = ctx.saved_tensors
        g = ctx.renderer.backward([ctx.seg], cams, ctx.view_segs, ctx.frame, _c(d_rgb), _c(d_depth), _c(d_alpha))[0]
        return g["means"], g["log_scales"], g["quats"], g["opacity"], g["sh"], None, None, None


def rasterize(means, log_scales, quats, opacity, sh, cams, renderer, sh_degree=None):
    """Differentiable render of one gaussian set into V views: (rgb [V,H,W,3],
    depth [V,H,W], alpha [V,H,W]).  Gradients flow to means, log_scales,
    quats, opacity (activated) and sh.  The renderer's saved frame is reused
    by the backward, so call backward before the next render on it."""
    if sh_degree is None:
        sh_degree = int(round(math.sqrt(sh.shape[1]))) - 1
    return _RasterizeFn.apply(means, log_scales, quats, opacity, sh, cams, renderer, sh_degree)


def observation(rgb, depth, alpha, mesh_rgba=None, mesh_depth=None, out=None):
    """The sensor observation of rendered views: (rgba uint8 [V, H, W, 4],
    metric depth [V, H, W]), optionally resolved against a mesh pass by the
    nearer-fragment rule (gs_sensor_compose).  `out` reuses a previous
    (rgba, depth) pair of the same shape."""
    V, H, W = (int(x) for x in depth.shape)
    if out is None:
        out = (torch.empty((V, H, W, 4), dtype=torch.uint8, device=depth.device),
               torch.empty((V, H, W), dtype=torch.float32, device=depth.device))
    B.sensor_compose(_c(rgb), _c(depth), _c(alpha), out[0], out[1], _c(mesh_rgba), _c(mesh_depth))
    return out


def observation_two_pass(scene, avatars, out=None):
    """The paper's own way of adding avatars (Sec. 3.2): scene and avatars
    rasterized in separate passes, then each pixel keeps the nearer of the
    two fragments (the avatar pass wins ties), with the same 8-bit / metric
    depth hand-off.  `scene` and `avatars` are rendered frames of the same
    views (any objects with rgb, depth and alpha).  The union rendering --
    avatars as a second segment of one pass -- blends the two instead."""
    av = observation(avatars.rgb, avatars.depth, avatars.alpha)
    return observation(scene.rgb, scene.depth, scene.alpha, mesh_rgba=av[0], mesh_depth=av[1], out=out)


class CapturedRender:
    """A forward frame (optionally preceded by other launches, e.g. the
    skinning of avatar Gaussians, and followed by others, e.g. a loss
    adjoint and the backward) captured once into a HIP graph and replayed
    with no host work per frame.

    The captured kernels hold raw device pointers: to the renderer's
    buffers, to the frame's outputs and to the inputs (segments, cameras,
    and whatever `before` writes).  A graph does not keep those tensors
    alive, and `torch.cuda.graph` returns every unused cached block to the
    device when it starts a capture, so a buffer whose Python owner is
    dropped while its graph can still be replayed is unmapped memory the next
    replay writes to.  This object therefore holds references to everything
    the graph touches for as long as it lives; the renderer passed in is
    reserved for it (a later call that grows one of its buffers would leave
    the graph on the old one).

    The key capacity is sized by an eager render first (growing on
    overflow).  A replay cannot grow it: after replays, `overflowed()`
    synchronises and reports whether any frame needed more keys than the
    capacity (its image is then incomplete; capture again).

    after(frame), when given, is called after the forward's launches, in
    the capture and in its eager warm-up; what it returns (say, the
    gradient tensors of a backward) is kept as `self.after_out`, the
    tensors the replays write."""

    def __init__(self, renderer, segs, cams, view_segs=None, checkpoints=False, before=None, after=None):
        if view_segs is None:
            view_segs = [list(range(len(segs)))] * int(cams.shape[0])
        self.renderer = renderer
        self.segs = list(segs)
        self.cams = cams
        self.view_segs = [list(v) for v in view_segs]
        self.before = before
        self.after = after
        self.after_out = None
        if before is not None:
            before()
        self.frame = renderer.render(self.segs, cams, self.view_segs, checkpoints=checkpoints)
        self.n_views = len(self.view_segs)
        # warm-up launches on a side stream (the capture stream's allocator
        # state and the library's lazily loaded kernels), then the capture
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self._enqueue()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.after_out = self._enqueue()
        torch.cuda.synchronize()

    def _enqueue(self):
        if self.before is not None:
            self.before()
        self.renderer.enqueue(self.segs, self.cams, self.view_segs, self.frame)
        return self.after(self.frame) if self.after is not None else None

    def replay(self):
        """Enqueue one frame on torch's current stream; outputs in self.frame."""
        self.graph.replay()
        return self.frame

    def overflowed(self):
        torch.cuda.synchronize()
        return bool(int(self.frame.overflow.item()))
