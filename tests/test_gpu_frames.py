"""GPU parity of whole forward frames at the sizes the benchmark runs and on
the paths only those sizes reach, against the FP64 oracle (Sec. 2.2 / Sec.
3.2 of the paper: tile-based rasterization into colour and depth, avatars in
the same pass as the scene).

Protocol: P2 -- the oracle's binning of the GPU's FP32 records equals the
GPU's keys, values and ranges bit for bit; P3 -- the oracle composites those
records along those lists in FP64 and every pixel matches one of its
enumerated results within 1e-4; P3' -- the independent oracle render (its own
projection and lists) matches every pixel it does not flag, and flags under
1% of them."""
import sys

import numpy as np
import pytest

from paper_2604_12626_amd import synth

from parity import TOL_ALPHA, TOL_DEPTH_REL, TOL_RGB, frame_to_numpy, pixel_match, to_dev

pytestmark = pytest.mark.gpu

F32 = np.float32


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2604_12626_amd import binding
    binding.load()
    return torch.device("cuda:0")


def check_p2_p3(orc, f, n_views, W, H, label):
    """P2 bit-exact binning and P3 compositing of the GPU's records."""
    K = int(f.num.item())
    assert int(f.overflow.item()) == 0
    rec = f.rec.cpu().numpy()
    tt = f.tiles_touched.cpu().numpy().view(np.uint32)
    tt_o, keys_o, vals_o, ranges_o, K_o = orc.bin_records(rec, tt > 0, W, H, n_views)
    assert K == K_o and np.array_equal(tt, tt_o)
    assert np.array_equal(f.keys[:K].cpu().numpy().view(np.uint64), keys_o)
    assert np.array_equal(f.vals[:K].cpu().numpy().view(np.uint32), vals_o)
    assert np.array_equal(f.ranges.cpu().numpy().view(np.uint32), ranges_o)
    img_o, ncand, cands = orc.composite(rec, vals_o, ranges_o, n_views, orc.params(W, H))
    bad = 0
    for v in range(n_views):
        gimg, nc = frame_to_numpy(f, v)
        ok = match_with_n_contrib(gimg, nc, cands[v], ncand[v])
        bad += int((~ok).sum())
        for y, x in np.argwhere(~ok)[:4]:
            say("    view %d pixel (%d, %d): gpu rgb %s depth %.7g alpha %.7g n %d; %d oracle results:" % (
                v, y, x, gimg[y, x, :3], gimg[y, x, 3], gimg[y, x, 4], nc[y, x], ncand[v][y, x]))
            for c in cands[v][y, x, :abs(ncand[v][y, x])]:
                say("      rgb %s depth %.7g alpha %.7g n %d flips %d" % (c[:3], c[3], c[4], c[6], c[7]))
    say("  %s: K = %d, P2 bit-exact, P3 mismatched pixels %d" % (label, K, bad))
    assert bad == 0


def match_with_n_contrib(gimg, nc, cands, ncand):
    """A pixel matches when one enumerated result has its image within the
    tolerance and its n_contrib equal."""
    C = cands
    within = np.all(np.abs(C[..., :3] - gimg[..., None, :3]) <= TOL_RGB, -1)
    within &= np.abs(C[..., 3] - gimg[..., None, 3]) <= TOL_DEPTH_REL * np.maximum(1.0, np.abs(C[..., 3]))
    within &= np.abs(C[..., 4] - gimg[..., None, 4]) <= TOL_ALPHA
    within &= np.arange(C.shape[-2]) < np.abs(ncand)[..., None]
    within &= ~np.isnan(C[..., 0])
    return np.any(within & (C[..., 6] == nc[..., None]), -1)


def check_p3_independent(orc, gimg, g, cam, W, H, label):
    prm = orc.params(W, H)
    _, img_o, ncand, flags, cands, pairs = orc.render(g, cam, prm)
    ok, idx = pixel_match(gimg, cands, ncand)
    bad = ~ok & (flags == 0)
    frac = float((flags != 0).mean())
    say("  %s: P3' pairs %d, flagged %.4f%%, mismatched unflagged %d" % (label, pairs, 100 * frac, int(bad.sum())))
    assert not bad.any(), np.argwhere(bad)[:5]
    assert frac < 0.01


def test_full_size_headline_frame(dev, orc):
    """1M-Gaussian SH3 room, one 640x480 view: the benchmark's frame."""
    import torch
    from paper_2604_12626_amd import render
    cfg = synth.config(1)
    g = cfg["segments"][0]
    W, H = cfg["W"], cfg["H"]
    say("full-size headline frame: room1M 640x480 sh3")
    r = render.Renderer(W, H, capacity=1 << 22, device=dev)
    f = r.render([to_dev(g, dev)], torch.from_numpy(cfg["cams"]).to(dev), [[0]])
    torch.cuda.synchronize()
    check_p2_p3(orc, f, 1, W, H, "room1M")
    gimg, _ = frame_to_numpy(f, 0)
    check_p3_independent(orc, gimg, g, cfg["cams"][0], W, H, "room1M")


def test_batched_beyond_4096_tiles_default_path(dev, orc):
    """20 views at 256x256 over 3 scenes of uneven size: 5120 (view, tile)
    lists, past the 4096 tile counters that LDS holds, so the default
    binning counts in windows of whole views."""
    import torch
    from paper_2604_12626_amd import binding as B, render
    assert B.get_tuning()["sort_algorithm"] == 0  # default selection
    rng = np.random.default_rng(41)
    W = H = 256
    scenes = [synth.gaussians_room(n, rng, sh_degree=3) for n in (30000, 8000, 15000)]
    V = 20
    cams_np = np.stack([synth.camera_room(rng, W, H, fx=128.0) for _ in range(V)])
    vs = [[v % 3] for v in range(V)]
    r = render.Renderer(W, H, capacity=1 << 21, device=dev)
    assert V * r.T > 4096
    say("batched default path: %d views x 256 tiles, 3 scenes" % V)
    f = r.render([to_dev(s, dev) for s in scenes], torch.from_numpy(cams_np).to(dev), vs)
    torch.cuda.synchronize()
    check_p2_p3(orc, f, V, W, H, "batched 20 views")
    for v in (0, 1, 2, 19):
        gimg, _ = frame_to_numpy(f, v)
        check_p3_independent(orc, gimg, scenes[v % 3], cams_np[v], W, H, "view %d" % v)


def _posed(orc, scale):
    cfg = synth.config(4, scale=scale)
    av, skin = cfg["avatars"], cfg["skin"]
    w = orc.dense_weights(av["joint_idx"], av["weights"], synth.N_JOINTS)
    mo, co = orc.lbs(av["means"], av["log_scales"], av["quats"], w, av["avatar_of"], skin, synth.N_JOINTS)
    return av, {"means": mo.astype(F32), "cov6": co.astype(F32), "opacity": av["opacity"], "sh": av["sh"],
                "sh_degree": 3}


def test_avatar_union_and_avatar_only_passes(dev, orc):
    """Avatars posed by LBS (a covariance-given segment) rendered (a) in the
    same lists as a room scene (union), and (b) alone, the avatar pass of the
    paper's two-pass mode; both against the oracle."""
    import torch
    from paper_2604_12626_amd import render
    from test_gpu_gradients import avatar_cameras
    av, posed = _posed(orc, 0.04)
    room = synth.gaussians_room(40000, np.random.default_rng(43), sh_degree=3)
    W, H = 320, 240
    cams_np = avatar_cameras(posed, av["avatar_of"], W, H, 3, 44)
    tsegs = [to_dev(room, dev), to_dev(posed, dev)]
    cams = torch.from_numpy(cams_np).to(dev)
    r = render.Renderer(W, H, capacity=1 << 20, device=dev)
    say("avatar union: room 40k + %d posed avatar Gaussians, 3 views" % len(posed["means"]))
    f = r.render(tsegs, cams, [[0, 1]] * 3)
    torch.cuda.synchronize()
    check_p2_p3(orc, f, 3, W, H, "union")
    for v in range(3):
        gimg, _ = frame_to_numpy(f, v)
        check_p3_independent(orc, gimg, [room, posed], cams_np[v], W, H, "union view %d" % v)
    f = r.render([tsegs[1]], cams, [[0]] * 3)
    torch.cuda.synchronize()
    assert float(f.alpha.max().item()) > 0.5  # the avatars are in view
    check_p2_p3(orc, f, 3, W, H, "avatar pass")
    for v in range(3):
        gimg, _ = frame_to_numpy(f, v)
        check_p3_independent(orc, gimg, posed, cams_np[v], W, H, "avatar pass view %d" % v)
