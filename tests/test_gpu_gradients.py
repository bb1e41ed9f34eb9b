"""GPU parity of the gradients (gs_render_backward, gs_deform_lbs_backward and
the autograd function, through the C ABI) against the FP64 oracle's adjoint.

Sec. 2.2 of the paper: the rasterizer it builds on is differentiable.  The
oracle differentiates the branch the GPU took (its per-tile lists, its
n_contrib, and skip decisions inside their FP32 window chosen by reproducing
its image; discrete decisions are held fixed, O12), at its own FP64 values.
Bar: every parameter block of every Gaussian within 1e-4 of the block's
largest oracle gradient; every pixel's decisions accounted for (status 0 or
1, none unexplained)."""
import sys

import numpy as np
import pytest

from paper_2604_12626_amd import synth

from parity import gpu_decisions, grad_check, to_dev

pytestmark = pytest.mark.gpu

F32 = np.float32
SQ_FIELDS = ("means", "log_scales", "quats", "opacity", "sh")
COV_FIELDS = ("means", "cov6", "opacity", "sh")


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


def _np(d):
    return {k: v.cpu().numpy().astype(np.float64) for k, v in d.items()}


def _status_check(ref, n_pix):
    st = ref["pixel_status"]
    say("  pixels: GPU decisions = FP64 %d, inside their window %d, unexplained %d (of %d)" % (
        int((st == 0).sum()), int((st == 1).sum()), int((st == 2).sum()), n_pix))
    assert (st == 2).sum() == 0, np.argwhere(st == 2)[:5]


def _random_adjoints(rng, V, H, W):
    return [rng.standard_normal((V, H, W, 3)).astype(F32), rng.standard_normal((V, H, W)).astype(F32),
            rng.standard_normal((V, H, W)).astype(F32)]


@pytest.mark.parametrize("checkpoints", [False, True], ids=["whole_lists", "segmented"])
def test_backward_parity_sh3(dev, orc, checkpoints):
    """Gradients of <G, render> for random output adjoints G on a 100k-Gaussian
    room (scales x 1.65) at 256x256; lists walked whole, or in 64-entry
    segments from the forward's checkpoints (lists long enough to hold
    several)."""
    import torch
    from paper_2604_12626_amd import render
    cfg = synth.config(2, scale=0.2)
    W, H = cfg["W"], cfg["H"]
    g = dict(cfg["segments"][0])
    g["log_scales"] = (g["log_scales"] + F32(0.5)).astype(F32)
    say("backward parity: room100k 256x256 sh3, checkpoints", checkpoints)
    G = _random_adjoints(np.random.default_rng(5), 1, H, W)
    r = render.Renderer(W, H, capacity=1 << 18, device=dev, checkpoints=checkpoints)
    tg = to_dev(g, dev)
    cams = torch.from_numpy(cfg["cams"]).to(dev)
    f = r.render([tg], cams, [[0]])
    d = r.backward([tg], cams, [[0]], f, *[torch.from_numpy(x).to(dev) for x in G])[0]
    torch.cuda.synchronize()
    lens = (f.ranges[:, 1] - f.ranges[:, 0]).cpu().numpy()
    say("  lists: %d, longest %d, over 64 entries %d" % (len(lens), lens.max(), int((lens > 64).sum())))
    assert (lens > 2 * 64).sum() >= 8  # lists of several segments are differentiated
    prm = orc.params(W, H)
    ref = orc.backward(g, cfg["cams"], prm, *G, decisions=gpu_decisions(f, [0], [0], W, H))
    _status_check(ref, W * H)
    grad_check(say, _np(d), ref, SQ_FIELDS)


def test_backward_parity_2048_lists_whole_walk(dev, orc):
    """8 views x 256 tiles = 2048 (view, tile) lists with checkpoints off: the
    launch takes the whole-list walk whose four quadrant waves sum their
    per-entry gradients in LDS before the global atomics."""
    import torch
    from paper_2604_12626_amd import render
    rng = np.random.default_rng(61)
    W = H = 256
    g = synth.gaussians_room(20000, rng, sh_degree=3)
    V = 8
    cams_np = np.stack([synth.camera_room(rng, W, H, fx=128.0) for _ in range(V)])
    r = render.Renderer(W, H, capacity=1 << 20, device=dev, checkpoints=False)
    tg = to_dev(g, dev)
    cams = torch.from_numpy(cams_np).to(dev)
    vs = [[0]] * V
    f = r.render([tg], cams, vs)
    n_items = V * r.T
    say("backward parity: %d lists, whole-list walk" % n_items)
    assert n_items >= 2048 and f.ckpt is None
    G = _random_adjoints(np.random.default_rng(62), V, H, W)
    d = r.backward([tg], cams, vs, f, *[torch.from_numpy(x).to(dev) for x in G])[0]
    torch.cuda.synchronize()
    n = len(g["means"])
    prm = orc.params(W, H)
    ref = orc.backward(g, cams_np, prm, *G, decisions=gpu_decisions(f, range(V), [v * n for v in range(V)], W, H))
    _status_check(ref, V * W * H)
    grad_check(say, _np(d), ref, SQ_FIELDS)


def test_config2_full_size_l2_loss_and_finite_differences(dev, orc):
    """The fwd+bwd workload at full size: 500k room Gaussians, SH3, 256x256.
    L = sum |rgb - rgb*|^2 + (D - D*)^2 against the oracle's render of the
    parameters perturbed by N(0, 0.01) on every field.  (a) The GPU's
    gradient of its own loss against the oracle's adjoint along the GPU's
    branch, every Gaussian; (b) the GPU's gradient with the oracle's output
    adjoints against FP64 central finite differences of the oracle's loss on
    256 random visible Gaussians x all 59 parameters."""
    import torch
    from paper_2604_12626_amd import render
    cfg = synth.config(2)
    W, H = cfg["W"], cfg["H"]
    g = cfg["segments"][0]
    cam = cfg["cams"][0]
    prm = orc.params(W, H)
    tgt_params = synth.perturb(g, cfg["perturb_rng"])
    _, tgt_img, *_ = orc.render(tgt_params, cam, prm, want_cands=False)
    tgt = tgt_img[..., :5].astype(F32).astype(np.float64)  # the target is an FP32 image
    say("config 2 full size: 500k, 256x256, L2 loss")
    r = render.Renderer(W, H, capacity=1 << 21, device=dev, checkpoints="auto")
    tg = to_dev(g, dev)
    cams = torch.from_numpy(cfg["cams"]).to(dev)
    f = r.render([tg], cams, [[0]])
    t_rgb = torch.from_numpy(tgt[..., :3].astype(F32)).to(dev)[None]
    t_d = torch.from_numpy(tgt[..., 3].astype(F32)).to(dev)[None]
    d_rgb = (2.0 * (f.rgb - t_rgb)).contiguous()
    d_d = (2.0 * (f.depth - t_d)).contiguous()
    d_a = torch.zeros_like(f.alpha)
    d = r.backward([tg], cams, [[0]], f, d_rgb, d_d, d_a)[0]
    torch.cuda.synchronize()
    G = [x.cpu().numpy() for x in (d_rgb, d_d, d_a)]
    ref = orc.backward(g, cfg["cams"], prm, *G, decisions=gpu_decisions(f, [0], [0], W, H))
    _status_check(ref, W * H)
    grad_check(say, _np(d), ref, SQ_FIELDS, label="(a) GPU loss")
    # (b) output adjoints of the oracle's own forward, the same for both sides
    pr, img, *_ = orc.render(g, cam, prm, want_cands=False)
    Go = [(2.0 * (img[None, ..., :3] - tgt[None, ..., :3])).astype(F32),
          (2.0 * (img[None, ..., 3] - tgt[None, ..., 3])).astype(F32), np.zeros((1, H, W), F32)]
    d2 = _np(r.backward([tg], cams, [[0]], f, *[torch.from_numpy(x).to(dev) for x in Go])[0])
    torch.cuda.synchronize()
    scale_ref = orc.backward(g, cfg["cams"], prm, *Go)
    drawn = np.nonzero(np.abs(scale_ref["opacity"]) > 0)[0]
    rng = np.random.default_rng(202)
    sel = rng.choice(drawn, 256, replace=False)
    fields = [("means", 3), ("log_scales", 3), ("quats", 4), ("opacity", 1), ("sh", 48)]
    samples, hs = [], []
    for i in sel:
        for fld, m in fields:
            for c in range(m):
                samples.append((i, orc.param_index(fld, c, 3)))
                x0 = float(g[fld].reshape(len(g["means"]), -1)[i, c])
                hs.append(1e-6 * max(abs(x0), 1.0))
    fd, flag = orc.fd_loss(g, cam, prm, samples, np.array(hs), quad=[1.0, 1.0, 1.0, 1.0, 0.0], tgt=tgt)
    say("  FD samples %d, rejected (a decision flips within +-h) %d" % (len(fd), int((flag != 0).sum())))
    assert (flag != 0).sum() <= 0.01 * len(flag)
    k = 0
    worst = {}
    for i in sel:
        for fld, m in fields:
            gg = d2[fld].reshape(len(g["means"]), -1)
            scale = np.abs(scale_ref[fld]).max()
            for c in range(m):
                if flag[k] == 0:
                    e = abs(gg[i, c] - fd[k]) / scale
                    worst[fld] = max(worst.get(fld, 0.0), e)
                k += 1
    say("  (b) max |g_gpu - g_fd| / max |g_ref| over the FD samples:", {k: "%.2e" % v for k, v in worst.items()})
    for fld, v in worst.items():
        assert v <= 1e-4, (fld, v)


def _posed_avatars(orc, scale, seed=0):
    """Workload-4 avatars posed by the oracle's LBS (cast to FP32): the same
    covariance-given segment feeds the GPU and the oracle."""
    cfg = synth.config(4, scale=scale)
    av, skin = cfg["avatars"], cfg["skin"]
    w = orc.dense_weights(av["joint_idx"], av["weights"], synth.N_JOINTS)
    mo, co = orc.lbs(av["means"], av["log_scales"], av["quats"], w, av["avatar_of"], skin, synth.N_JOINTS)
    posed = {"means": mo.astype(F32), "cov6": co.astype(F32), "opacity": av["opacity"], "sh": av["sh"],
             "sh_degree": 3}
    return cfg, av, skin, w, posed


def look_at(target, dist, yaw, W, H, height=0.4):
    """Camera `dist` metres from `target` (horizontally, direction `yaw`),
    `height` above it, looking at it; 90 degree horizontal field of view."""
    target = np.asarray(target, np.float64)
    pos = target + np.array([-dist * np.cos(yaw), -dist * np.sin(yaw), height])
    d = target - pos
    return synth.look_camera(pos, np.arctan2(d[1], d[0]), np.arctan2(d[2], np.hypot(d[0], d[1])), W / 2.0, W / 2.0,
                             W / 2.0, H / 2.0)


def avatar_cameras(posed, avatar_of, W, H, n_views, seed):
    """One camera per view, each looking at the centroid of a posed avatar."""
    rng = np.random.default_rng(seed)
    cams = []
    for v in range(n_views):
        a = v % (int(avatar_of.max()) + 1)
        c = posed["means"][avatar_of == a].astype(np.float64).mean(0)
        cams.append(look_at(c, rng.uniform(1.5, 3.0), rng.uniform(0, 2 * np.pi), W, H))
    return np.stack(cams)


def test_avatar_union_backward_through_lbs(dev, orc):
    """Posed avatars (covariance-given segment) in the same lists as a room
    scene, 2 views: d_means / d_cov6 / opacity / SH of the avatars and the
    scene's gradients against the oracle; then the LBS backward of the GPU's
    (d_means, d_cov6) against the oracle's LBS adjoint of its own."""
    import torch
    from paper_2604_12626_amd import binding as B, render
    cfg, av, skin, w, posed = _posed_avatars(orc, 0.02)
    rng = np.random.default_rng(71)
    room = synth.gaussians_room(20000, rng, sh_degree=3)
    W, H = 320, 240
    cams_np = avatar_cameras(posed, av["avatar_of"], W, H, 2, 72)
    segs_np = [room, posed]
    tsegs = [to_dev(room, dev), to_dev(posed, dev)]
    cams = torch.from_numpy(cams_np).to(dev)
    vs = [[0, 1], [0, 1]]
    r = render.Renderer(W, H, capacity=1 << 20, device=dev, checkpoints="auto")
    f = r.render(tsegs, cams, vs)
    offs = B.instance_offsets(tsegs, vs)
    G = _random_adjoints(np.random.default_rng(73), 2, H, W)
    d_room, d_av = r.backward(tsegs, cams, vs, f, *[torch.from_numpy(x).to(dev) for x in G])
    torch.cuda.synchronize()
    n_room = len(room["means"])
    drawn_av = int((f.tiles_touched[n_room:offs[1]] > 0).sum().item())
    say("avatar union backward: room 20k + %d avatar Gaussians (%d drawn in view 0), 2 views at %dx%d" % (
        len(posed["means"]), drawn_av, W, H))
    assert drawn_av > 100
    prm = orc.params(W, H)
    ref = orc.backward(segs_np, cams_np, prm, *G, decisions=gpu_decisions(f, [0, 1], offs[:2], W, H))
    _status_check(ref, 2 * W * H)
    cut = lambda d, lo, hi: {k: v[lo:hi] for k, v in d.items() if k != "pixel_status"}
    ref_room, ref_av = cut(ref, 0, n_room), cut(ref, n_room, None)
    grad_check(say, _np(d_room), ref_room, SQ_FIELDS, label="scene")
    grad_check(say, _np(d_av), ref_av, COV_FIELDS, label="avatars")
    # through the skinning: canonical means, log-scales and quaternions
    t = to_dev(av, dev)
    n = len(av["means"])
    dm, ds, dq = (torch.empty(n, k, device=dev) for k in (3, 3, 4))
    B.deform_lbs_backward(t["means"], t["log_scales"], t["quats"], t["joint_idx"], t["weights"], t["avatar_of"],
                          torch.from_numpy(skin).to(dev), d_av["means"].contiguous(), d_av["cov6"].contiguous(),
                          dm, ds, dq)
    rm, rs, rq = orc.lbs_backward(av["means"], av["log_scales"], av["quats"], w, av["avatar_of"], skin,
                                  synth.N_JOINTS, ref_av["means"].astype(F32), ref_av["cov6"].astype(F32))
    torch.cuda.synchronize()
    grad_check(say, {"means": dm.cpu().numpy(), "log_scales": ds.cpu().numpy(), "quats": dq.cpu().numpy()},
               {"means": rm, "log_scales": rs, "quats": rq}, ("means", "log_scales", "quats"), label="canonical")


def test_rasterize_autograd_function(dev, orc):
    """render.rasterize (torch.autograd.Function): torch.autograd.grad gives
    exactly Renderer.backward's gradients, and they match the oracle."""
    import torch
    from paper_2604_12626_amd import render
    cfg = synth.config(2, scale=0.03)
    W, H = cfg["W"], cfg["H"]
    g = cfg["segments"][0]
    tg = to_dev(g, dev)
    cams = torch.from_numpy(cfg["cams"]).to(dev)
    leaves = {k: tg[k].clone().requires_grad_(True) for k in SQ_FIELDS}
    r = render.Renderer(W, H, capacity=1 << 18, device=dev)
    rgb, depth, alpha = render.rasterize(leaves["means"], leaves["log_scales"], leaves["quats"], leaves["opacity"],
                                         leaves["sh"], cams, r)
    rng = np.random.default_rng(81)
    G = [torch.from_numpy(x).to(dev) for x in _random_adjoints(rng, 1, H, W)]
    loss = (rgb * G[0]).sum() + (depth * G[1]).sum() + (alpha * G[2]).sum()
    grads = torch.autograd.grad(loss, [leaves[k] for k in SQ_FIELDS])
    # the same frame rendered again and differentiated directly
    r2 = render.Renderer(W, H, capacity=1 << 18, device=dev)
    f2 = r2.render([tg], cams, [[0]], checkpoints="auto")
    assert torch.equal(f2.rgb, rgb) and torch.equal(f2.depth, depth) and torch.equal(f2.alpha, alpha)
    d = r2.backward([tg], cams, [[0]], f2, *G)[0]
    torch.cuda.synchronize()
    # the same gradients up to the order of the float atomics that sum them
    for k, a in zip(SQ_FIELDS, grads):
        err = float((a - d[k]).abs().max() / d[k].abs().max().clamp_min(1e-30))
        assert err <= 1e-5, (k, err)
    say("rasterize autograd: gradients equal Renderer.backward up to the atomics' summation order")
    prm = orc.params(W, H)
    ref = orc.backward(g, cfg["cams"], prm, *[x.cpu().numpy() for x in G],
                       decisions=gpu_decisions(f2, [0], [0], W, H))
    _status_check(ref, W * H)
    grad_check(say, _np(d), ref, SQ_FIELDS)


def test_segmented_backward_with_a_short_checkpoint_buffer(dev, orc):
    """A checkpoint buffer sized for about a third of the frame's keys: the
    segments whose checkpoints lie past it walk from the end of their list
    and add only their own entries, so the gradients still equal the
    whole-list walk's up to rounding, and the oracle's."""
    import torch
    from paper_2604_12626_amd import binding as B, render
    cfg = synth.config(2, scale=0.2)
    W, H = cfg["W"], cfg["H"]
    g = dict(cfg["segments"][0])
    g["log_scales"] = (g["log_scales"] + F32(0.5)).astype(F32)
    tg = to_dev(g, dev)
    cams = torch.from_numpy(cfg["cams"]).to(dev)
    G = [torch.from_numpy(x).to(dev) for x in _random_adjoints(np.random.default_rng(15), 1, H, W)]
    r = render.Renderer(W, H, capacity=1 << 18, device=dev, checkpoints=True)
    f = r.render([tg], cams, [[0]])
    K = int(f.num.item())
    full = f.ckpt
    d_full = {k: v.clone() for k, v in r.backward([tg], cams, [[0]], f, *G)[0].items()}
    f.ckpt = full[:B.checkpoint_floats(K // 3)]
    say("short checkpoint buffer: %d keys, checkpoints for %d" % (K, K // 3))
    d_short = {k: v.clone() for k, v in r.backward([tg], cams, [[0]], f, *G)[0].items()}
    rw = render.Renderer(W, H, capacity=1 << 18, device=dev, checkpoints=False)
    fw = rw.render([tg], cams, [[0]])
    d_whole = rw.backward([tg], cams, [[0]], fw, *G)[0]
    torch.cuda.synchronize()
    ref = orc.backward(g, cfg["cams"], orc.params(W, H), *[x.cpu().numpy() for x in G],
                       decisions=gpu_decisions(f, [0], [0], W, H))
    _status_check(ref, W * H)
    res = [grad_check(say, _np(d), ref, SQ_FIELDS, label=lb, check=False)
           for d, lb in ((d_whole, "whole lists"), (d_full, "all checkpoints"), (d_short, "short buffer"))]
    # the worst Gaussians' conditioning (kappa of the 2D covariance) and screen size
    pr = orc.project(g, cfg["cams"][0], orc.params(W, H))
    for (_, where), lb in zip(res, ("whole", "full", "short")):
        for k, (i, rel) in where.items():
            a, b_, c = pr[i, 26], pr[i, 27], pr[i, 28]
            say("    %s %s: Gaussian %d kappa %.3g radius %d opacity %.3f" % (
                lb, k, i, (a * c + b_ * b_) / (a * c - b_ * b_), pr[i, 11], pr[i, 7]))
    for w, _ in res:
        for k, v in w.items():
            assert v <= 1e-4, (k, v)
    # GPU against GPU: the summation order of the float atomics differs
    for k in SQ_FIELDS:
        err = float((d_short[k] - d_whole[k]).abs().max() / d_whole[k].abs().max())
        assert err <= 1e-4, (k, err)
