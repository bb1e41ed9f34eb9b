#!/usr/bin/env python3
"""Benchmark of the Habitat-GS sensor-rendering hot path on one MI355X.

Headline (`value`): forward frames/s of one 640x480 view of a 1M-Gaussian SH3
room scene (synthetic stand-in for an indoor 3DGS capture), the whole
per-frame path -- projection + SH, binning (tile counts, bucket sort by
tile and depth, ranges, work order), compositing -- replayed from one HIP
graph with inputs resident in HBM (the eager launch sequence is reported
beside it).  Further lines of the metric (fwd+bwd, batched multi-view vs
plain per-view, avatars) are reported under "extras", each with its stage
roofline (algorithmic bytes, flops and exponentials of every stage from the
run's own counts, against the HBM, FP32 and transcendental peaks).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras]
                       [--no-cpu-baseline] [--profile] [--profile-fwd-bwd]
                       [--profile-batched] [--profile-avatars] [--copy-calib]
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# MI355X vector FP32 peak: the roofline fraction is taken against it.
FP32_PEAK_TFLOPS = 157.3
# 256 CU x 64 FP32 lanes x 2 flop (FMA) x 2.4 GHz without packed FP32
# instructions (this library is built without them): informational.
FP32_NONPACKED_TFLOPS = 78.6
# transcendentals (v_exp_f32) issue at a quarter of the lane rate
EXP_PEAK_TPS = 256 * 64 * 2.4e9 / 4 / 1e12
# Algorithmic work of one evaluated (pixel, list entry) pair of front-to-back
# compositing: offset (2), quadratic form (9), o * exp (1), clamp (1), skip
# test (1), T (1 - alpha) (2), stop test (1), alpha T (1), colour and depth
# accumulation (4 FMA = 8); the exponential itself is counted apart.
FLOPS_PER_PAIR = 26
# per pair of the backward walk: T recovery, the alpha and colour adjoints,
# the exponent's gradient and the ten wave sums (one exp, one reciprocal)
BWD_FLOPS_PER_PAIR = 70
COUNTERS_FILE = os.path.join(ROOT, "profiles", "composite_room1M_640x480_counters.txt")
COMPOSITE_SOURCES = [os.path.join(ROOT, "paper_2604_12626_amd", "csrc", n)
                     for n in ("gs_composite.hip", "gs_internal.hpp")]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile", action="store_true", help="headline workload only, for rocprofv3 runs")
    ap.add_argument("--copy-calib", action="store_true", help="also run a 512 MiB device copy (counter scale)")
    ap.add_argument("--profile-fwd-bwd", action="store_true",
                    help="forward + backward of the 256x256 500k-Gaussian view only, for rocprofv3 runs")
    ap.add_argument("--profile-batched", action="store_true",
                    help="the 64-view batched frame only (graph replays), for rocprofv3 runs")
    ap.add_argument("--profile-avatars", action="store_true",
                    help="the 16-view avatar frame only (forward and forward + backward), for rocprofv3 runs")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def to_dev(g, dev):
    import torch
    return {k: (torch.from_numpy(np.ascontiguousarray(v)).to(dev) if isinstance(v, np.ndarray) else v)
            for k, v in g.items()}


class Timer:
    """HIP events on torch's current stream (the stream libgs launches on)."""

    def __init__(self):
        import torch
        self.torch = torch
        self.acc = {}

    def run(self, name, fn):
        torch = self.torch
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        self.acc.setdefault(name, []).append((a, b))

    def means_ms(self):
        self.torch.cuda.synchronize()
        return {k: float(np.mean([a.elapsed_time(b) for a, b in v])) for k, v in self.acc.items()}


def sh_bytes(D):
    return 12 * (D + 1) ** 2


def stage_roofline(c):
    """Algorithmic bytes, flops and exponentials of each stage of one step and
    the roofline time: sum over stages of max(bytes / HBM, flops / FP32 peak,
    exps / transcendental rate).  c: measured counts -- N (Gaussians read,
    each scene once), I (instances: Gaussians x the views drawing them),
    n_vis (visible instances), K (tile instances), V, HW (pixels per view),
    T (tiles per view), D (SH degree), pairs (evaluated (pixel, entry) pairs
    of compositing); for a backward also pairs_b (pairs walked back),
    n_drawn and N_grad (dense gradient rows); n_av (skinned Gaussians)."""
    D = c["D"]
    sh = sh_bytes(D)
    st = {
        "project": (c["N"] * 12 + c["I"] * 4 + c["n_vis"] * (32 + sh + 48), 250 * c["n_vis"], 0),
        # binning's least traffic: tile counts and the drawn instances' rects
        # read once, every key and value written once, the ranges
        "bin_sort": (c["I"] * 4 + c["n_vis"] * 20 + c["K"] * 12 + c["V"] * c["T"] * 8, 0, 0),
        "composite": (c["K"] * 52 + c["V"] * c["HW"] * 28, FLOPS_PER_PAIR * c["pairs"], c["pairs"]),
    }
    if c.get("pairs_b") is not None:
        st["bwd_composite"] = (c["V"] * c["HW"] * 28 + c["K"] * 52 + c["n_vis"] * 80,
                               BWD_FLOPS_PER_PAIR * c["pairs_b"], 2 * c["pairs_b"])
        st["bwd_project"] = (c["n_drawn"] * (32 + sh + 80 + 48) + c["N_grad"] * 4 * (11 + 3 * (D + 1) ** 2),
                             600 * c["n_drawn"], 0)
    if c.get("n_av"):
        st["lbs"] = (c["n_av"] * 96, 90 * c["n_av"], 0)
        if c.get("pairs_b") is not None:
            st["lbs_backward"] = (c["n_av"] * 140, 200 * c["n_av"], 0)
    out = {}
    total = 0.0
    for k, (by, fl, ex) in st.items():
        t = max(by / (HBM_PEAK_GBS * 1e9), fl / (FP32_PEAK_TFLOPS * 1e12), ex / (EXP_PEAK_TPS * 1e12)) * 1e3
        out[k] = {"bytes": int(by), "flops": int(fl), "exps": int(ex), "ms": t}
        total += t
    return total, out


def roofline_block(counts, measured_ms, pairs_source):
    rt, stages = stage_roofline(counts)
    return {"roofline_ms": rt, "measured_ms": measured_ms, "frac": rt / measured_ms, "pairs_source": pairs_source,
            "counts": {k: (int(v) if isinstance(v, (int, np.integer)) else v) for k, v in counts.items()},
            "stages": stages}


def oracle_pairs(views):
    """Evaluated (pixel, entry) pairs of the oracle's render: views is a list
    of (gaussian dict of numpy arrays, camera, W, H)."""
    import oracle
    total = 0
    for g, cam, W, H in views:
        prm = oracle.params(W, H, max_flips=0)
        proj = oracle.project(g, cam, prm)
        total += oracle.render_view(proj, prm, want_cands=False)[4]
    return total


def _time_seq(fn, warmup, steps):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def _frame_counts(f, n_views, T, HW, D, N, I):
    import torch
    return {"N": int(N), "I": int(I), "n_vis": int((f.tiles_touched > 0).sum().item()), "K": int(f.num.item()),
            "V": int(n_views), "HW": int(HW), "T": int(T), "D": int(D)}


def bench_forward(args, dev):
    """The headline frame: 1M-Gaussian SH3 room, one 640x480 view.  Timed as
    replays of the captured frame (one HIP graph: projection, binning and
    compositing, inputs resident) and as the eager launch sequence, whose
    compositing launches are bracketed by HIP events on their stream."""
    import torch
    from paper_2604_12626_amd import render, synth
    cfg = synth.config(1)
    g = cfg["segments"][0]
    N, D = len(g["means"]), g["sh_degree"]
    W, H = cfg["W"], cfg["H"]
    segs = [to_dev(g, dev)]
    cams = torch.from_numpy(cfg["cams"]).to(dev)
    vs = [[0]]
    r = render.Renderer(W, H, capacity=1 << 22, device=dev)
    f = r.render(segs, cams, vs)  # sizes the key capacity (grows on overflow)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        r.enqueue(segs, cams, vs, f)
    torch.cuda.synchronize()
    comp_ev = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r.project(segs, cams, vs, f)
        r.bin_sort(f, 1)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        r.composite(f, 1)
        b.record()
        comp_ev.append((a, b))
    torch.cuda.synchronize()
    ms_eager = (time.perf_counter() - t0) * 1e3 / args.steps
    composite_ms = float(np.mean([a.elapsed_time(b) for a, b in comp_ev]))
    assert int(f.overflow.item()) == 0, "key capacity overflow during the timed region"
    cap = render.CapturedRender(render.Renderer(W, H, capacity=r.capacity, device=dev), segs, cams, vs)
    ms_graph = _time_seq(cap.replay, args.warmup, args.steps)
    assert not cap.overflowed()
    assert torch.equal(cap.frame.rgb, f.rgb) and torch.equal(cap.frame.depth, f.depth)
    tm = Timer()
    for _ in range(max(5, args.steps // 2)):
        tm.run("project", lambda: r.project(segs, cams, vs, f))
        tm.run("bin_sort", lambda: r.bin_sort(f, 1))
    stages = tm.means_ms()
    stages["composite"] = composite_ms
    counts = _frame_counts(f, 1, r.T, W * H, D, N, N)
    info = {"stage_ms": stages, "counts": counts, "ms_eager": ms_eager,
            "n_contrib_sum": int(f.n_contrib.to(torch.int64).sum().item()),
            "layout_ab": layout_ab(r, g, cams, vs, f, dev)}
    return ms_graph, info


def bench_fwd_bwd(args, dev, steps, want_pairs=True):
    """Forward + backward of one 256x256 view of a 500k-Gaussian SH3 room:
    L = sum |rgb - rgb*|^2 + sum (D - D*)^2 against the render of the
    perturbed parameters; one step = forward (recording segment checkpoints),
    loss adjoint, backward with dense gradients of every parameter, replayed
    from one HIP graph."""
    import torch
    from paper_2604_12626_amd import render, synth
    cfg = synth.config(2)
    g = cfg["segments"][0]
    W, H = cfg["W"], cfg["H"]
    segs = [to_dev(g, dev)]
    tgt = [to_dev(synth.perturb(g, cfg["perturb_rng"]), dev)]
    cams = torch.from_numpy(cfg["cams"]).to(dev)
    vs = [[0]]
    r = render.Renderer(W, H, capacity=1 << 21, device=dev, checkpoints="auto")
    ft = r.render(tgt, cams, vs)
    # the loss adjoint 2 (x - x*) as one fused kernel per output: -2 x* is
    # formed once, then d = -2 x* + 2 x into buffers of their own (measured:
    # one multi-tensor launch for both outputs took longer than the two)
    neg2_rgb_t, neg2_depth_t = -2.0 * ft.rgb, -2.0 * ft.depth
    d_rgb, d_depth = torch.empty_like(ft.rgb), torch.empty_like(ft.depth)
    r.render(segs, cams, vs)  # sizes the key capacity for the timed parameters

    def after(f2):
        torch.add(neg2_rgb_t, f2.rgb, alpha=2.0, out=d_rgb)
        torch.add(neg2_depth_t, f2.depth, alpha=2.0, out=d_depth)
        return r.backward(segs, cams, vs, f2, d_rgb, d_depth, None)

    # the whole step -- forward, loss adjoint, backward -- replayed from one graph
    cap = render.CapturedRender(r, segs, cams, vs, checkpoints="auto", after=after)
    ms = _time_seq(cap.replay, max(2, args.warmup // 2), steps)
    assert not cap.overflowed()
    f = r.render(segs, cams, vs)
    torch.cuda.synchronize()
    c = _frame_counts(f, 1, r.T, W * H, g["sh_degree"], len(g["means"]), len(g["means"]))
    c["pairs_b"] = int(f.n_contrib.to(torch.int64).sum().item())
    c["n_drawn"] = c["n_vis"]
    c["N_grad"] = len(g["means"])
    c["pairs"] = oracle_pairs([(g, cfg["cams"][0], W, H)]) if want_pairs else c["pairs_b"]
    src = "oracle count (forward); backward: sum of n_contrib" if want_pairs else "lower bound: sum of n_contrib"
    return ms, roofline_block(c, ms, src)


def bench_batched(args, dev, steps, want_pairs=True):
    """64 views at 256x256 of 8 room scenes (view v shows scene v mod 8,
    scenes of 1e5..2e6 Gaussians): one batched frame (scene-major projection,
    one sort and one persistent compositing launch for all views) captured
    into one HIP graph, vs the same views rendered one call at a time (plain,
    each view its own captured graph); eager launch sequences for reference."""
    import torch
    from paper_2604_12626_amd import autotune, binding as B, render, synth
    cfg = synth.config(3)
    segs = [to_dev(g, dev) for g in cfg["segments"]]
    cams = torch.from_numpy(cfg["cams"]).to(dev)
    vs = cfg["view_segs"]
    W, H = cfg["W"], cfg["H"]
    rb = render.Renderer(W, H, capacity=1 << 24, device=dev)
    fb = rb.render(segs, cams, vs)
    best, _ = autotune.tune_composite(rb, fb, len(vs))
    ms_b_eager = _time_seq(lambda: rb.enqueue(segs, cams, vs, fb), args.warmup, steps)
    cap = render.CapturedRender(render.Renderer(W, H, capacity=rb.capacity, device=dev), segs, cams, vs)
    ms_b = _time_seq(cap.replay, args.warmup, steps)
    assert not cap.overflowed()
    assert torch.equal(cap.frame.rgb, fb.rgb)
    # the per-view frames are another workload: the default schedule (a
    # captured graph keeps the launch shapes of its capture)
    B.set_tuning()
    plain = []
    for v in range(len(vs)):
        sv = [segs[vs[v][0]]]
        plain.append(render.CapturedRender(render.Renderer(W, H, capacity=1 << 20, device=dev), sv,
                                           cams[v:v + 1].contiguous(), [[0]]))

    def all_plain():
        for c in plain:
            c.replay()

    ms_p = _time_seq(all_plain, args.warmup, steps)
    assert not any(c.overflowed() for c in plain)
    ms_p_eager = _time_seq(lambda: [c.renderer.enqueue(c.segs, c.cams, c.view_segs, c.frame) for c in plain],
                           args.warmup, steps)
    Ns = [len(g["means"]) for g in cfg["segments"]]
    counts = _frame_counts(fb, len(vs), rb.T, W * H, 3, sum(Ns), sum(Ns[v[0]] for v in vs))
    if want_pairs:
        counts["pairs"] = oracle_pairs([(cfg["segments"][vs[v][0]], cfg["cams"][v], W, H) for v in range(len(vs))])
        src = "oracle count"
    else:
        counts["pairs"] = int(fb.n_contrib.to(torch.int64).sum().item())
        src = "lower bound: sum of n_contrib"
    res = {"ms_batched": ms_b, "ms_plain": ms_p, "ms_batched_eager": ms_b_eager, "ms_plain_eager": ms_p_eager,
           "n_views": len(vs), "groups_per_cu": best, "roofline": roofline_block(counts, ms_b, src)}
    return res


def bench_avatars(args, dev, steps, want_pairs=True):
    """1M room + 8 avatars x 50k Gaussians, 16 views at 640x480: LBS of the
    avatar Gaussians, then all views of room + posed avatars in one call
    (forward, captured with the skinning into one HIP graph), and the same
    with the backward through the renderer and LBS to the canonical avatar
    parameters (fwd+bwd, also one graph; checkpoints "auto", which leaves
    them off for 19200 tile lists)."""
    import torch
    from paper_2604_12626_amd import autotune, binding as B, render
    from paper_2604_12626_amd import synth
    cfg = synth.config(4)
    room = to_dev(cfg["segments"][0], dev)
    av = to_dev(cfg["avatars"], dev)
    skin = torch.from_numpy(cfg["skin"]).to(dev)
    n_av = av["means"].shape[0]
    posed = {"means": torch.empty(n_av, 3, device=dev), "cov6": torch.empty(n_av, 6, device=dev),
             "opacity": av["opacity"], "sh": av["sh"], "sh_degree": 3}
    cams = torch.from_numpy(cfg["cams"]).to(dev)
    vs = cfg["view_segs"]
    W, H = cfg["W"], cfg["H"]
    r = render.Renderer(W, H, capacity=1 << 24, device=dev)
    d_means = torch.empty(n_av, 3, device=dev)
    d_ls = torch.empty(n_av, 3, device=dev)
    d_q = torch.empty(n_av, 4, device=dev)

    def lbs():
        B.deform_lbs(av["means"], av["log_scales"], av["quats"], av["joint_idx"], av["weights"], av["avatar_of"],
                     skin, posed["means"], posed["cov6"])

    lbs()
    f = r.render([room, posed], cams, vs)
    autotune.tune_composite(r, f, len(vs))  # the compositing schedule for this workload
    target = torch.rand_like(f.rgb)

    def frame():
        lbs()
        r.enqueue([room, posed], cams, vs, f)

    ms_eager = _time_seq(frame, args.warmup, steps)
    cap = render.CapturedRender(render.Renderer(W, H, capacity=r.capacity, device=dev), [room, posed], cams, vs,
                                before=lbs)
    ms = _time_seq(cap.replay, args.warmup, steps)
    assert not cap.overflowed()
    rb = render.Renderer(W, H, capacity=r.capacity, device=dev, checkpoints="auto")
    neg2_target = -2.0 * target
    d_rgb = torch.empty_like(target)

    def after(fb):
        # loss adjoint 2 (rgb - target), backward through the renderer, then LBS
        torch.add(neg2_target, fb.rgb, alpha=2.0, out=d_rgb)
        gr = rb.backward([room, posed], cams, vs, fb, d_rgb, None, None)
        B.deform_lbs_backward(av["means"], av["log_scales"], av["quats"], av["joint_idx"], av["weights"],
                              av["avatar_of"], skin, gr[1]["means"], gr[1]["cov6"], d_means, d_ls, d_q)
        return gr

    # skinning, forward, loss adjoint and the whole backward replayed from one graph
    cap_b = render.CapturedRender(rb, [room, posed], cams, vs, checkpoints="auto", before=lbs, after=after)
    ms_b = _time_seq(cap_b.replay, max(2, args.warmup // 2), max(3, steps // 2))
    fb = cap_b.frame
    assert int(f.overflow.item()) == 0 and not cap_b.overflowed()
    N_room = int(room["means"].shape[0])
    counts = _frame_counts(f, len(vs), r.T, W * H, 3, N_room + n_av, len(vs) * (N_room + n_av))
    counts["n_av"] = int(n_av)
    if want_pairs:
        posed_np = {"means": posed["means"].cpu().numpy(), "cov6": posed["cov6"].cpu().numpy(),
                    "opacity": cfg["avatars"]["opacity"], "sh": cfg["avatars"]["sh"], "sh_degree": 3}
        import oracle
        both = oracle.concat_segments([cfg["segments"][0], posed_np])
        counts["pairs"] = oracle_pairs([(both, cfg["cams"][v], W, H) for v in range(len(vs))])
        src = "oracle count"
    else:
        counts["pairs"] = int(f.n_contrib.to(torch.int64).sum().item())
        src = "lower bound: sum of n_contrib"
    roof_f = roofline_block(dict(counts), ms, src)
    cb = dict(counts)
    cb["pairs_b"] = int(fb.n_contrib.to(torch.int64).sum().item())
    cb["n_drawn"] = min(counts["n_vis"], N_room + n_av)
    cb["N_grad"] = N_room + n_av
    roof_b = roofline_block(cb, ms_b, src + "; backward: sum of n_contrib")
    # skinning alone, with fixed joint matrices and with each avatar's matrices
    # interpolated in a 90-frame walking clip at its current time
    clip, first, nfr = synth.avatar_clips(np.random.default_rng(5), [90] * int(skin.shape[0]))
    tclip = [torch.from_numpy(x).to(dev) for x in (clip, first, nfr)]
    fpos = torch.linspace(0.3, 80.7, int(skin.shape[0]), device=dev)

    def lbs_clip():
        B.deform_lbs_clip(av["means"], av["log_scales"], av["quats"], av["joint_idx"], av["weights"],
                          av["avatar_of"], *tclip, fpos, posed["means"], posed["cov6"])

    lbs_ms = {k: _event_ms(fn, 20 * steps) for k, fn in (("fixed", lbs), ("clip", lbs_clip))}
    return {"ms": ms, "ms_eager": ms_eager, "ms_bwd": ms_b, "n_views": len(vs), "lbs_ms": lbs_ms, "n_av": n_av,
            "roofline_fwd": roof_f, "roofline_fwd_bwd": roof_b}


def _planar(g):
    """The segment g (numpy rows) component-major, every attribute [components][n]."""
    n = len(g["means"])
    out = {"sh_degree": g["sh_degree"], "layout": "planes"}
    for k in ("means", "log_scales", "quats", "cov6", "opacity", "sh"):
        if g.get(k) is not None:
            a = np.asarray(g[k], np.float32).reshape(n, -1)
            out[k] = np.ascontiguousarray(a.T if a.shape[1] > 1 else a[:, 0])
    return out


def layout_ab(r, g, cams, vs, f, dev, reps=20):
    """Projection of the same Gaussians stored in rows and in planes (device
    time per launch, HIP events); the records must agree bit for bit."""
    import torch
    rows, planes = [to_dev(g, dev)], [to_dev(_planar(g), dev)]
    r.project(rows, cams, vs, f)
    tt0, rec0 = f.tiles_touched.clone(), f.rec.clone()
    r.project(planes, cams, vs, f)
    torch.cuda.synchronize()
    vis = (tt0 > 0).nonzero().squeeze(1)
    assert torch.equal(tt0, f.tiles_touched) and torch.equal(rec0[vis], f.rec[vis])
    ms_r = _event_ms(lambda: r.project(rows, cams, vs, f), reps)
    ms_p = _event_ms(lambda: r.project(planes, cams, vs, f), reps)
    r.project(rows, cams, vs, f)
    return {"rows_ms": ms_r, "planes_ms": ms_p}


def _event_ms(fn, reps):
    """Mean device time per call of a short launch sequence (HIP events on
    the current stream around reps back-to-back calls)."""
    import torch
    for _ in range(3):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_sensor(args, dev, steps):
    """Sensor hand-off of 16 views at 640x480 against a mesh pass: HBM-bound,
    28 B read + 8 B written per pixel.  Returns (ms per call, fraction of the
    HBM peak)."""
    import torch
    from paper_2604_12626_amd import render, synth
    d = synth.sensor_inputs(7, 16, 480, 640, mesh=True)
    t = {k: torch.from_numpy(v).to(dev) for k, v in d.items()}
    out = render.observation(t["rgb"], t["depth"], t["alpha"], t["mesh_rgba"], t["mesh_depth"])
    reps = 20 * steps
    for _ in range(args.warmup):
        render.observation(t["rgb"], t["depth"], t["alpha"], t["mesh_rgba"], t["mesh_depth"], out=out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        render.observation(t["rgb"], t["depth"], t["alpha"], t["mesh_rgba"], t["mesh_depth"], out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    n_px = 16 * 480 * 640
    return ms, n_px * 36 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS


def bench_capsules(args, dev, steps):
    """Capsule queries of 4096 agents against 8 walking avatars (184
    capsules, 90-frame clips): clearance, nearest capsule and a swept 0.25 m
    step per agent.  Returns ms per call."""
    import torch
    from paper_2604_12626_amd import binding as B, synth
    rng = np.random.default_rng(41)
    clip, first, nfr = synth.avatar_clips(rng, [90] * 8)
    caps = synth.capsule_clips(clip)
    now = np.stack([caps[first[a]] for a in range(8)])
    pos, nxt = synth.agents_near_avatars(rng, now, 4096)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    tp, tn, ta = t(pos), t(nxt), t(np.tile(np.array([0, 8], np.int32), (4096, 1)))
    tc, tf, tnf, tfp = t(caps), t(first), t(nfr), t(np.linspace(0.3, 80.7, 8).astype(np.float32))
    cl = torch.empty(4096, device=dev)
    nn = torch.empty(4096, dtype=torch.int32, device=dev)
    sg = torch.empty(4096, device=dev)
    bl = torch.empty(4096, dtype=torch.uint8, device=dev)

    def q():
        B.capsule_queries(tp, tn, ta, 0.1, 1.5, tc, tf, tnf, tfp, cl, nn, sg, bl)

    return _event_ms(q, 20 * steps)


def source_digest(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic():
    """HBM bytes per compositing launch from the committed FETCH_SIZE /
    WRITE_SIZE counter summary, scaled by the plain-copy calibration in the
    same file; None when the summary is absent or the kernel's sources have
    changed since the counters were taken."""
    if not os.path.exists(COUNTERS_FILE):
        return None, "no counter summary"
    kv = {}
    with open(COUNTERS_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        if kv.get("kernel_source_sha256") != source_digest(COMPOSITE_SOURCES):
            return None, "kernel changed since the counters were taken"
        fetch = float(kv["fetch_kib_per_dispatch"]) * float(kv["fetch_scale"])
        write = float(kv["write_kib_per_dispatch"]) * float(kv["write_scale"])
    except (KeyError, ValueError):
        return None, "unreadable counter summary"
    return (fetch + write) * 1024.0, "FETCH_SIZE x %s + WRITE_SIZE x %s" % (kv["fetch_scale"], kv["write_scale"])


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _time_cpu(fn, min_seconds):
    n = 0
    t0 = time.perf_counter()
    while True:
        fn()
        n += 1
        el = time.perf_counter() - t0
        if el >= min_seconds:
            return n, el


def cpu_baseline(leg_seconds=5.0):
    """The FP64 oracle as it stands (no candidate enumeration) on the host's
    cores, on all of its OpenMP threads and on one: the headline frame
    (projection of all 1M Gaussians and compositing of all 640x480 pixels),
    the fwd+bwd step of the 500k view (forward, L2 adjoint, backward to every
    parameter) and a sample of the batched workload (views 0-7: one per
    scene, 256x256 each).  Each leg repeats for at least `leg_seconds`."""
    import oracle
    from paper_2604_12626_amd import synth
    n_all = oracle.set_threads(1)
    oracle.set_threads(n_all)
    c1 = synth.config(1)
    g1, W1, H1 = c1["segments"][0], c1["W"], c1["H"]
    p1 = oracle.params(W1, H1, max_flips=0)

    def fwd():
        oracle.render_view(oracle.project(g1, c1["cams"][0], p1), p1, want_cands=False)

    c2 = synth.config(2)
    g2, W2, H2 = c2["segments"][0], c2["W"], c2["H"]
    p2 = oracle.params(W2, H2, max_flips=0)
    _, timg, *_ = oracle.render(synth.perturb(g2, c2["perturb_rng"]), c2["cams"][0], p2, want_cands=False)

    def fwd_bwd():
        _, img, *_ = oracle.render(g2, c2["cams"][0], p2, want_cands=False)
        G = [2.0 * (img[None, ..., :3] - timg[None, ..., :3]), 2.0 * (img[None, ..., 3] - timg[None, ..., 3]),
             np.zeros((1, H2, W2))]
        oracle.backward(g2, c2["cams"], p2, *G)

    c3 = synth.config(3)
    p3 = oracle.params(c3["W"], c3["H"], max_flips=0)
    sample = list(range(8))

    def batched():
        for v in sample:
            oracle.render_view(oracle.project(c3["segments"][c3["view_segs"][v][0]], c3["cams"][v], p3), p3,
                               want_cands=False)

    legs = {}
    for name, fn, per in (("fwd_frames_per_s", fwd, 1), ("fwd_bwd_steps_per_s", fwd_bwd, 1),
                          ("batched_views_per_s", batched, len(sample))):
        legs[name] = {}
        for label, nt in (("all_threads", n_all), ("one_thread", 1)):
            oracle.set_threads(nt)
            n, el = _time_cpu(fn, leg_seconds)
            legs[name][label] = per * n / el
    oracle.set_threads(n_all)
    return {"value": legs["fwd_frames_per_s"]["all_threads"], "unit": "frames/s", "cores": n_all, "kind": "oracle",
            "cpu_model": cpu_model(), "legs": legs,
            "sample": "FP64 oracle, OpenMP over Gaussians and tiles; value: the full headline frame (projection of "
                      "1M Gaussians + all 640x480 pixels) on %d threads; legs on %d threads and on 1: that frame, "
                      "the 500k / 256x256 forward + L2 adjoint + backward step, and views 0-7 of the 64-view "
                      "batch (one per scene); each leg >= %.0f s" % (n_all, n_all, leg_seconds)}


def copy_calibration(dev):
    import torch
    n = 512 << 20
    a = torch.empty(n // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    return n


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only (the renderer runs on a single MI355X); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_2604_12626_amd import binding
    binding.load()
    dev = torch.device("cuda:0")
    if args.copy_calib:
        log("copy calibration: 512 MiB x 3")
        copy_calibration(dev)
    if args.profile_fwd_bwd:
        log("fwd+bwd only: 256x256, 500k Gaussians")
        ms, _ = bench_fwd_bwd(args, dev, args.steps, want_pairs=False)
        print(json.dumps({"fwd_bwd_256x256_500k_ms": ms, "steps": args.steps, "warmup": args.warmup}), flush=True)
        return
    if args.profile_batched:
        log("batched only: 64 views x 256x256, 8 scenes")
        res = bench_batched(args, dev, args.steps, want_pairs=False)
        print(json.dumps({k: v for k, v in res.items() if k != "roofline"}), flush=True)
        return
    if args.profile_avatars:
        log("avatars only: 1M room + 8 x 50k avatars, 16 views x 640x480")
        res = bench_avatars(args, dev, args.steps, want_pairs=False)
        print(json.dumps({k: v for k, v in res.items() if not k.startswith("roofline")}), flush=True)
        return
    log("forward: 640x480, 1M Gaussians, SH3")
    ms, info = bench_forward(args, dev)
    fps = 1e3 / ms
    st = info["stage_ms"]
    counts = info["counts"]
    want_pairs = not args.profile
    if want_pairs:
        from paper_2604_12626_amd import synth
        c1 = synth.config(1)
        counts["pairs"] = oracle_pairs([(c1["segments"][0], c1["cams"][0], c1["W"], c1["H"])])
        pair_src = "oracle count of evaluated pairs, same frame"
    else:
        counts["pairs"] = int(info["n_contrib_sum"])
        pair_src = "lower bound: sum of n_contrib over pixels"
    _, stages_alg = stage_roofline(counts)
    extras = {"stage_ms": st, "eager_fps": 1e3 / info["ms_eager"], "N": counts["N"], "visible": counts["n_vis"],
              "tile_instances": counts["K"],
              "stage_hbm_frac": {k: stages_alg[k]["bytes"] / (st[k] * 1e-3) / 1e9 / HBM_PEAK_GBS for k in st},
              "frame_roofline": roofline_block(counts, ms, pair_src),
              "project_layout_ab": info["layout_ab"]}
    if not args.profile and not args.no_extras:
        steps2 = max(5, args.steps // 5)
        log("fwd+bwd: 256x256, 500k Gaussians")
        ms_fb, roof_fb = bench_fwd_bwd(args, dev, steps2)
        extras["fwd_bwd_256x256_500k_fps"] = 1e3 / ms_fb
        extras["fwd_bwd_roofline"] = roof_fb
        log("batched vs plain: 64 views x 256x256, 8 scenes")
        rb = bench_batched(args, dev, steps2)
        nv = rb["n_views"]
        extras["batched_64x256x256_8scenes_fps"] = nv * 1e3 / rb["ms_batched"]
        extras["plain_64x256x256_8scenes_fps"] = nv * 1e3 / rb["ms_plain"]
        extras["batched_eager_fps"] = nv * 1e3 / rb["ms_batched_eager"]
        extras["plain_eager_fps"] = nv * 1e3 / rb["ms_plain_eager"]
        extras["batched_composite_groups_per_cu"] = rb["groups_per_cu"]
        extras["batched_roofline"] = rb["roofline"]
        log("avatars: 1M room + 8 x 50k avatars, 16 views x 640x480")
        ra = bench_avatars(args, dev, steps2)
        nva = ra["n_views"]
        extras["avatars_16x640x480_fwd_fps"] = nva * 1e3 / ra["ms"]
        extras["avatars_16x640x480_fwd_eager_fps"] = nva * 1e3 / ra["ms_eager"]
        extras["avatars_16x640x480_fwd_bwd_fps"] = nva * 1e3 / ra["ms_bwd"]
        extras["avatars_fwd_roofline"] = ra["roofline_fwd"]
        extras["avatars_fwd_bwd_roofline"] = ra["roofline_fwd_bwd"]
        extras["lbs_400k_fixed_ms"] = ra["lbs_ms"]["fixed"]
        extras["lbs_400k_clip_ms"] = ra["lbs_ms"]["clip"]
        extras["lbs_400k_clip_hbm_frac"] = ra["n_av"] * 96 / (ra["lbs_ms"]["clip"] * 1e-3) / 1e9 / HBM_PEAK_GBS
        log("sensor hand-off: 16 views x 640x480 with a mesh pass")
        ms_s, frac_s = bench_sensor(args, dev, steps2)
        extras["sensor_16x640x480_mesh_ms"] = ms_s
        extras["sensor_16x640x480_mesh_hbm_frac"] = frac_s
        log("capsule queries: 4096 agents x 8 avatars")
        extras["capsule_queries_4096x184_ms"] = bench_capsules(args, dev, steps2)
    cpu = None
    if not args.profile and not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline()
    # roofline of the dominant kernel: compositing, plain FP32 VALU work per
    # evaluated pair (the pair count from the oracle's render of the same
    # frame), its duration from the events around its launches in the timed loop
    pairs = counts["pairs"]
    t_comp = st["composite"] * 1e-3
    achieved = pairs * FLOPS_PER_PAIR / t_comp / 1e12
    traffic, traffic_src = counter_traffic()
    roof = {"bound": "alu", "kernel": "composite_kernel", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS, "traffic": traffic,
            "traffic_source": traffic_src, "pairs": pairs, "pairs_source": pair_src,
            "flops_per_pair": FLOPS_PER_PAIR, "exp_per_pair": 1, "avg_launch_ms": st["composite"],
            "alg_bytes_per_launch": stages_alg["composite"]["bytes"],
            "frac_of_nonpacked_peak": achieved / FP32_NONPACKED_TFLOPS}
    out = {"metric": "frames/s 640x480 1M-Gaussian SH3: fwd, fwd+bwd, batched vs plain", "value": fps,
           "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded room-shaped 3DGS scene; no dataset)",
           "config": {"workload": "room1M_640x480_sh3: 1 view, 1M Gaussians, SH degree 3, forward frame "
                                  "(projection, binning, compositing) replayed from one HIP graph",
                      "global_batch": 1, "parallelism": "none (1 GPU)"},
           "roofline": roof, "extras": extras}
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
