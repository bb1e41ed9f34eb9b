"""HIP-graph capture of the forward frame (render.CapturedRender).

The graph's kernels hold raw device pointers to the renderer's buffers and
to the inputs; CapturedRender owns all of them.  Regression test for a graph
whose buffers had lost their owners: every name outside the capture is
dropped and the allocator's cache emptied before the replays, which must
still reproduce the eager frame bit for bit, with eager work in between."""
import gc
import sys

import numpy as np
import pytest

from paper_2604_12626_amd import synth

from parity import to_dev

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_captured_headline_frame_replays_bit_exact():
    import torch
    from paper_2604_12626_amd import binding, render
    assert torch.cuda.is_available()
    binding.load()
    dev = torch.device("cuda:0")
    cfg = synth.config(1)
    W, H = cfg["W"], cfg["H"]
    say("graph capture: room1M 640x480 headline frame")
    segs = [to_dev(cfg["segments"][0], dev)]
    cams = torch.from_numpy(cfg["cams"]).to(dev)
    eager = render.Renderer(W, H, capacity=1 << 22, device=dev)
    f = eager.render(segs, cams, [[0]])
    ref = [t.clone() for t in (f.rgb, f.depth, f.alpha, f.n_contrib)]
    cap = render.CapturedRender(render.Renderer(W, H, capacity=1 << 22, device=dev),
                                [to_dev(cfg["segments"][0], dev)], torch.from_numpy(cfg["cams"]).to(dev), [[0]])
    gc.collect()
    torch.cuda.empty_cache()
    for k in range(3):
        for t in (cap.frame.rgb, cap.frame.depth, cap.frame.alpha):
            t.fill_(-1.0)
        cap.frame.n_contrib.fill_(-1)
        out = cap.replay()
        torch.cuda.synchronize()
        for a, b in zip((out.rgb, out.depth, out.alpha, out.n_contrib), ref):
            assert torch.equal(a, b), k
        eager.render(segs, cams, [[0]])  # eager work between replays
        torch.cuda.synchronize()
        say("  replay %d equals the eager frame" % k)
    assert not cap.overflowed()
    assert np.isfinite(cap.frame.rgb.cpu().numpy()).all()


def _replays_equal_eager(cap, ref, n=3, between=None):
    import torch
    for k in range(n):
        for t in (cap.frame.rgb, cap.frame.depth, cap.frame.alpha):
            t.fill_(-1.0)
        out = cap.replay()
        torch.cuda.synchronize()
        for a, b in zip((out.rgb, out.depth, out.alpha, out.n_contrib), ref):
            assert torch.equal(a, b), k
        if between is not None:
            between()
            torch.cuda.synchronize()
    assert not cap.overflowed()


def test_captured_batched_frame_replays_bit_exact():
    """The batched frame (64 views at 256x256 of 8 scenes at 1/20 of their
    size: scene-major projection, onesweep binning past 4096 tiles, one
    persistent compositing launch) captured into one graph."""
    import torch
    from paper_2604_12626_amd import binding, render
    binding.load()
    dev = torch.device("cuda:0")
    cfg = synth.config(3, scale=0.05)
    W, H = cfg["W"], cfg["H"]
    say("graph capture: batched 64 views, 8 scenes")
    segs = [to_dev(g, dev) for g in cfg["segments"]]
    cams = torch.from_numpy(cfg["cams"]).to(dev)
    vs = cfg["view_segs"]
    eager = render.Renderer(W, H, capacity=1 << 22, device=dev)
    f = eager.render(segs, cams, vs)
    ref = [t.clone() for t in (f.rgb, f.depth, f.alpha, f.n_contrib)]
    cap = render.CapturedRender(render.Renderer(W, H, capacity=1 << 22, device=dev),
                                [to_dev(g, dev) for g in cfg["segments"]], torch.from_numpy(cfg["cams"]).to(dev), vs)
    gc.collect()
    torch.cuda.empty_cache()
    _replays_equal_eager(cap, ref, between=lambda: eager.render(segs, cams, vs))
    say("  3 replays equal the eager frame")


def test_captured_avatar_frame_with_skinning_replays_bit_exact():
    """Skinning of the avatar Gaussians and the union frame (room + posed
    avatars, 4 views) captured together: the graph re-poses the avatars from
    the current joint matrices on every replay."""
    import torch
    from paper_2604_12626_amd import binding as B, render
    B.load()
    dev = torch.device("cuda:0")
    cfg = synth.config(4, scale=0.05)
    W, H = cfg["W"], cfg["H"]
    say("graph capture: skinning + room/avatar frame, 4 views")
    room = to_dev(cfg["segments"][0], dev)
    av = to_dev(cfg["avatars"], dev)
    skin = torch.from_numpy(cfg["skin"]).to(dev)
    n = av["means"].shape[0]
    posed = {"means": torch.empty(n, 3, device=dev), "cov6": torch.empty(n, 6, device=dev),
             "opacity": av["opacity"], "sh": av["sh"], "sh_degree": 3}
    cams = torch.from_numpy(cfg["cams"][:4]).to(dev)
    vs = cfg["view_segs"][:4]

    def lbs():
        B.deform_lbs(av["means"], av["log_scales"], av["quats"], av["joint_idx"], av["weights"], av["avatar_of"],
                     skin, posed["means"], posed["cov6"])

    cap = render.CapturedRender(render.Renderer(W, H, capacity=1 << 22, device=dev), [room, posed], cams, vs,
                                before=lbs)
    eager = render.Renderer(W, H, capacity=1 << 22, device=dev)
    # a new pose: the replay must pick up the new joint matrices
    skin.copy_(torch.from_numpy(np.ascontiguousarray(cfg["skin"][::-1])).to(dev))
    lbs()
    f = eager.render([room, posed], cams, vs)
    ref = [t.clone() for t in (f.rgb, f.depth, f.alpha, f.n_contrib)]
    _replays_equal_eager(cap, ref, between=lambda: eager.render([room, posed], cams, vs))
    say("  3 replays after a pose change equal the eager frame")


def test_captured_forward_backward_step_replays():
    """The whole training step of the 500k-Gaussian view at 1/10 of its size
    -- forward with segment checkpoints, the L2 loss adjoint, the backward to
    every parameter -- captured into one graph: each replay reproduces the
    eager step's images bit for bit and its gradients up to the order of the
    FP64 accumulators' atomic additions (1e-6 of each block's largest)."""
    import torch
    from paper_2604_12626_amd import binding as B, render
    B.load()
    dev = torch.device("cuda:0")
    cfg = synth.config(2, scale=0.1)
    W, H = cfg["W"], cfg["H"]
    say("graph capture: forward + loss adjoint + backward, 256x256")
    segs = [to_dev(cfg["segments"][0], dev)]
    cams = torch.from_numpy(cfg["cams"]).to(dev)
    target = torch.rand(1, H, W, 3, device=dev)
    neg2_t = -2.0 * target
    d_rgb = torch.empty_like(target)
    eager = render.Renderer(W, H, capacity=1 << 20, device=dev, checkpoints="auto")
    fe = eager.render(segs, cams, [[0]])
    ge = eager.backward(segs, cams, [[0]], fe, 2.0 * (fe.rgb - target), None, None)[0]
    ref_img = [t.clone() for t in (fe.rgb, fe.depth, fe.alpha)]
    ref_g = {k: v.clone() for k, v in ge.items()}
    rc = render.Renderer(W, H, capacity=1 << 20, device=dev, checkpoints="auto")

    def after(f):
        torch.add(neg2_t, f.rgb, alpha=2.0, out=d_rgb)
        return rc.backward(segs, cams, [[0]], f, d_rgb, None, None)

    cap = render.CapturedRender(rc, segs, cams, [[0]], checkpoints="auto", after=after)
    gc.collect()
    torch.cuda.empty_cache()
    for k in range(3):
        for t in (cap.frame.rgb, cap.frame.depth, cap.frame.alpha):
            t.fill_(-1.0)
        for t in cap.after_out[0].values():
            t.fill_(float("nan"))
        cap.replay()
        torch.cuda.synchronize()
        for a, b in zip((cap.frame.rgb, cap.frame.depth, cap.frame.alpha), ref_img):
            assert torch.equal(a, b), k
        for name, ref in ref_g.items():
            got = cap.after_out[0][name]
            err = float((got - ref).abs().max() / ref.abs().max())
            assert err <= 1e-6, (k, name, err)
        eager.render(segs, cams, [[0]])  # eager work between replays
        torch.cuda.synchronize()
        say("  replay %d: images equal, gradients within 1e-6" % k)
    assert not cap.overflowed()
