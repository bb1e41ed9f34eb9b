"""gs_composite_noalloc (through the C ABI) against gs_composite: the same
kernels with the workspace in the library's own per-GPU scratch, so the
images, transmittances and n_contrib must be bit-identical.  Two calls in a
row, the second with a smaller launch (fewer views, a smaller image), each
with the binning's work order and without it (the order is then built in
the scratch)."""
import sys

import numpy as np
import pytest

from paper_2604_12626_amd import synth

from parity import to_dev

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _frame(dev, W, H, n_views, seed):
    import torch
    from paper_2604_12626_amd import render
    rng = np.random.default_rng(seed)
    g = synth.gaussians_room(30000, rng, sh_degree=3)
    cams = torch.from_numpy(np.stack([synth.camera_room(rng, W, H) for _ in range(n_views)])).to(dev)
    r = render.Renderer(W, H, capacity=1 << 21, device=dev)
    f = r.render([to_dev(g, dev)], cams, [[0]] * n_views)
    torch.cuda.synchronize()
    return r, f


def test_composite_noalloc_equals_composite():
    import torch
    from paper_2604_12626_amd import binding as B
    assert torch.cuda.is_available()
    B.load()
    dev = torch.device("cuda:0")
    for W, H, V, seed in ((640, 480, 6, 1), (200, 120, 2, 2)):  # the second launch is smaller
        say("composite_noalloc vs composite: %d views at %dx%d" % (V, W, H))
        r, f = _frame(dev, W, H, V, seed)
        for order in (f.order, None):
            outs = []
            for fn in ("ws", "noalloc"):
                rgb = torch.full((V, H, W, 3), -1.0, device=dev)
                depth = torch.full((V, H, W), -1.0, device=dev)
                alpha = torch.full((V, H, W), -1.0, device=dev)
                tfin = torch.full((V, H, W), -1.0, device=dev)
                nc = torch.full((V, H, W), -1, dtype=torch.int32, device=dev)
                if fn == "ws":
                    B.composite(f.rec, f.vals, f.ranges, V, r.params, f.comp_ws, rgb, depth, alpha, tfin, nc,
                                order=order)
                else:
                    B.composite_noalloc(f.rec, f.vals, f.ranges, V, r.params, rgb, depth, alpha, tfin, nc,
                                        order=order)
                torch.cuda.synchronize()
                outs.append((rgb, depth, alpha, tfin, nc))
            for a, b in zip(*outs):
                assert torch.equal(a, b)
            assert float(outs[1][2].max().item()) > 0.5  # something was drawn
            say("  order %s: bit-identical" % ("from the binning" if order is not None else "built in the scratch"))
