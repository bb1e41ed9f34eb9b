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
