#!/usr/bin/env python3
"""Benchmark of the Habitat-GS sensor-rendering hot path on one MI355X.

Headline (`value`): forward frames/s of one 640x480 view of a 1M-Gaussian SH3
room scene (synthetic stand-in for an indoor 3DGS capture), the whole
per-frame path -- projection + SH, scan/emit, onesweep sort, ranges,
compositing -- enqueued back to back on one stream with no host
synchronisation and inputs resident in HBM.  Further lines of the metric
(fwd+bwd, batched multi-view vs plain per-view, avatars) are reported under
"extras".

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras]
                       [--no-cpu-baseline] [--profile] [--profile-fwd-bwd]
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
# 256 CU x 64 FP32 lanes x 2 flop (FMA) x 2.4 GHz.  The chip's 157.3 TFLOP/s
# needs packed FP32 instructions, which this library is built without.
FP32_NONPACKED_TFLOPS = 78.6
FP32_PACKED_TFLOPS = 157.3
# Algorithmic work of one evaluated (pixel, list entry) pair of front-to-back
# compositing: offset (2), quadratic form (9), o * exp (1), clamp (1), skip
# test (1), T (1 - alpha) (2), stop test (1), alpha T (1), colour and depth
# accumulation (4 FMA = 8); the exponential itself is counted apart.
FLOPS_PER_PAIR = 26
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


def algorithmic_bytes(N, n_vis, K, passes, V, HW, T, D):
    """Bytes each stage must move at minimum (reads + writes), per call."""
    return {
        # means of every Gaussian (near-plane cull) + scale/rotation/opacity and SH of the
        # visible ones + tiles_touched of all + the 48-B record of the visible ones
        "project": N * 12 + n_vis * (32 + sh_bytes(D)) + N * 4 + n_vis * 48,
        # scan (tiles_touched read twice, offsets written), emission (counts, offsets,
        # the 16-B head + view of visible records, 12 B per key), histogram (8 B per key),
        # P passes of 24 B per key, ranges (8 B per key + 8 B per tile)
        "bin_sort": N * 16 + n_vis * 20 + K * 12 + K * 8 + passes * K * 24 + K * 8 + V * T * 8,
        # values + gathered 48-B records + 28 B of outputs per pixel
        "composite": K * 52 + V * HW * 28,
    }


def bench_forward(args, dev, timer_steps):
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
    K = int(f.num.item())
    n_vis = int((f.tiles_touched > 0).sum().item())
    # the whole forward frame as a launch sequence on one stream, no host sync
    for _ in range(args.warmup):
        r.enqueue(segs, cams, vs, f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r.enqueue(segs, cams, vs, f)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert int(f.overflow.item()) == 0, "key capacity overflow during the timed region"
    ms = (t1 - t0) * 1e3 / args.steps
    # per-stage durations (eager launches bracketed by events on the same stream)
    tm = Timer()
    for _ in range(timer_steps):
        tm.run("project", lambda: r.project(segs, cams, vs, f))
        tm.run("bin_sort", lambda: r.bin_sort(f, 1))
        tm.run("composite", lambda: r.composite(f, 1))
    stages = tm.means_ms()
    T = r.T
    tile_bits = max(1, int(np.ceil(np.log2(T))))
    passes = (32 + tile_bits + 7) // 8
    nbytes = algorithmic_bytes(N, n_vis, K, passes, 1, W * H, T, D)
    info = {"N": N, "n_vis": n_vis, "K": K, "sort_passes": passes, "stage_ms": stages, "alg_bytes": nbytes,
            "capacity": r.capacity, "n_contrib_sum": int(f.n_contrib.to(torch.int64).sum().item())}
    return ms, info, (r, f, segs, cams, vs)


def bench_fwd_bwd(args, dev, steps):
    """Forward + backward of one 256x256 view of a 500k-Gaussian SH3 room:
    L = sum |rgb - rgb*|^2 + sum (D - D*)^2 against the render of the
    perturbed parameters; one step = forward (recording segment checkpoints),
    loss adjoint, backward with dense gradients of every parameter."""
    import torch
    from paper_2604_12626_amd import render, synth
    cfg = synth.config(2)
    g = cfg["segments"][0]
    segs = [to_dev(g, dev)]
    tgt = [to_dev(synth.perturb(g, cfg["perturb_rng"]), dev)]
    cams = torch.from_numpy(cfg["cams"]).to(dev)
    vs = [[0]]
    r = render.Renderer(cfg["W"], cfg["H"], capacity=1 << 21, device=dev, checkpoints="auto")
    ft = r.render(tgt, cams, vs)
    rgb_t, depth_t = ft.rgb.clone(), ft.depth.clone()
    r.render(segs, cams, vs)  # sizes the key capacity for the timed parameters

    def step():
        f2 = r.render(segs, cams, vs, sync_check=False)
        r.backward(segs, cams, vs, f2, 2.0 * (f2.rgb - rgb_t), 2.0 * (f2.depth - depth_t), None)

    ms = _time_seq(step, max(2, args.warmup // 2), steps)
    assert int(r._bufs["ovf"][0].item()) == 0
    return ms


def bench_batched(args, dev, steps):
    """64 views at 256x256 of 8 room scenes (view v shows scene v mod 8,
    scenes of 1e5..2e6 Gaussians): one batched call (scene-major projection,
    one sort and one persistent compositing launch for all views) vs the same
    views rendered one call at a time (plain)."""
    import torch
    from paper_2604_12626_amd import autotune, render, synth
    cfg = synth.config(3)
    segs = [to_dev(g, dev) for g in cfg["segments"]]
    cams = torch.from_numpy(cfg["cams"]).to(dev)
    vs = cfg["view_segs"]
    W, H = cfg["W"], cfg["H"]
    rb = render.Renderer(W, H, capacity=1 << 24, device=dev)
    fb = rb.render(segs, cams, vs)
    best, _ = autotune.tune_composite(rb, fb, len(vs))
    ms_b = _time_seq(lambda: rb.enqueue(segs, cams, vs, fb), args.warmup, steps)
    plain = []
    for v in range(len(vs)):
        rp = render.Renderer(W, H, capacity=1 << 20, device=dev)
        sv = [segs[vs[v][0]]]
        fp = rp.render(sv, cams[v:v + 1], [[0]])
        plain.append((rp, fp, sv, v))

    def all_plain():
        for rp, fp, sv, v in plain:
            rp.enqueue(sv, cams[v:v + 1], [[0]], fp)

    ms_p = _time_seq(all_plain, args.warmup, steps)
    assert int(fb.overflow.item()) == 0 and all(int(fp.overflow.item()) == 0 for _, fp, _, _ in plain)
    return ms_b, ms_p, len(vs), int(fb.num.item()), best


def bench_avatars(args, dev, steps):
    """1M room + 8 avatars x 50k Gaussians, 16 views at 640x480: LBS of the
    avatar Gaussians, then all views of room + posed avatars in one call
    (forward), and the same with the backward through the renderer and LBS
    to the canonical avatar parameters (fwd+bwd; checkpoints "auto", which
    leaves them off for 19200 tile lists)."""
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
    r = render.Renderer(cfg["W"], cfg["H"], capacity=1 << 24, device=dev)
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

    rb = render.Renderer(cfg["W"], cfg["H"], capacity=1 << 24, device=dev, checkpoints="auto")
    fb = rb.render([room, posed], cams, vs)

    def frame_bwd():
        lbs()
        rb.enqueue([room, posed], cams, vs, fb)
        gr = rb.backward([room, posed], cams, vs, fb, 2.0 * (fb.rgb - target), None, None)
        B.deform_lbs_backward(av["means"], av["log_scales"], av["quats"], av["joint_idx"], av["weights"],
                              av["avatar_of"], skin, gr[1]["means"], gr[1]["cov6"], d_means, d_ls, d_q)

    ms = _time_seq(frame, args.warmup, steps)
    ms_b = _time_seq(frame_bwd, max(2, args.warmup // 2), max(3, steps // 2))
    assert int(f.overflow.item()) == 0 and int(fb.overflow.item()) == 0
    # skinning alone, with fixed joint matrices and with each avatar's matrices
    # interpolated in a 90-frame walking clip at its current time
    clip, first, nfr = synth.avatar_clips(np.random.default_rng(5), [90] * int(skin.shape[0]))
    tclip = [torch.from_numpy(x).to(dev) for x in (clip, first, nfr)]
    fpos = torch.linspace(0.3, 80.7, int(skin.shape[0]), device=dev)

    def lbs_clip():
        B.deform_lbs_clip(av["means"], av["log_scales"], av["quats"], av["joint_idx"], av["weights"],
                          av["avatar_of"], *tclip, fpos, posed["means"], posed["cov6"])

    lbs_ms = {k: _event_ms(fn, 20 * steps) for k, fn in (("fixed", lbs), ("clip", lbs_clip))}
    return ms, ms_b, len(vs), lbs_ms, n_av


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


def cpu_baseline(min_seconds=10.0):
    """The FP64 oracle (as it stands, no candidate enumeration) rendering the
    headline frame -- projection of all 1M Gaussians and compositing of all
    640x480 pixels -- repeated until at least `min_seconds` of CPU work."""
    import oracle
    from paper_2604_12626_amd import synth
    cfg = synth.config(1)
    g = cfg["segments"][0]
    W, H = cfg["W"], cfg["H"]
    prm = oracle.params(W, H, max_flips=0)
    frames = 0
    pairs = None
    t0 = time.perf_counter()
    while True:
        proj = oracle.project(g, cfg["cams"][0], prm)
        _, _, _, _, npairs = oracle.render_view(proj, prm, want_cands=False)
        pairs = npairs if pairs is None else pairs
        frames += 1
        el = time.perf_counter() - t0
        if el >= min_seconds:
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": frames / el, "unit": "frames/s", "cores": cores, "kind": "oracle",
            "sample": "FP64 oracle, full headline frame (projection of 1M Gaussians + all 640x480 pixels) "
                      "x %d frames in %.1f s, OpenMP over Gaussians and tiles" % (frames, el)}, pairs


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
    if args.profile_fwd_bwd:
        log("fwd+bwd only: 256x256, 500k Gaussians")
        ms = bench_fwd_bwd(args, dev, args.steps)
        print(json.dumps({"fwd_bwd_256x256_500k_ms": ms, "steps": args.steps, "warmup": args.warmup}), flush=True)
        return
    if args.copy_calib:
        log("copy calibration: 512 MiB x 3")
        copy_calibration(dev)
    log("forward: 640x480, 1M Gaussians, SH3")
    ms, info, _ = bench_forward(args, dev, timer_steps=max(5, args.steps // 2))
    fps = 1e3 / ms
    st = info["stage_ms"]
    extras = {"stage_ms": st, "N": info["N"], "visible": info["n_vis"], "tile_instances": info["K"],
              "sort_passes": info["sort_passes"],
              "stage_hbm_frac": {k: info["alg_bytes"][k] / (st[k] * 1e-3) / 1e9 / HBM_PEAK_GBS for k in st}}
    if not args.profile and not args.no_extras:
        steps2 = max(5, args.steps // 5)
        log("fwd+bwd: 256x256, 500k Gaussians")
        extras["fwd_bwd_256x256_500k_fps"] = 1e3 / bench_fwd_bwd(args, dev, steps2)
        log("batched vs plain: 64 views x 256x256, 8 scenes")
        ms_b, ms_p, nv, kb, best = bench_batched(args, dev, steps2)
        extras["batched_64x256x256_8scenes_fps"] = nv * 1e3 / ms_b
        extras["plain_64x256x256_8scenes_fps"] = nv * 1e3 / ms_p
        extras["batched_tile_instances"] = kb
        extras["batched_composite_groups_per_cu"] = best
        log("avatars: 1M room + 8 x 50k avatars, 16 views x 640x480")
        ms_a, ms_ab, nva, lbs_ms, n_av = bench_avatars(args, dev, steps2)
        extras["avatars_16x640x480_fwd_fps"] = nva * 1e3 / ms_a
        extras["avatars_16x640x480_fwd_bwd_fps"] = nva * 1e3 / ms_ab
        extras["lbs_400k_fixed_ms"] = lbs_ms["fixed"]
        extras["lbs_400k_clip_ms"] = lbs_ms["clip"]
        extras["lbs_400k_clip_hbm_frac"] = n_av * 96 / (lbs_ms["clip"] * 1e-3) / 1e9 / HBM_PEAK_GBS
        log("sensor hand-off: 16 views x 640x480 with a mesh pass")
        ms_s, frac_s = bench_sensor(args, dev, steps2)
        extras["sensor_16x640x480_mesh_ms"] = ms_s
        extras["sensor_16x640x480_mesh_hbm_frac"] = frac_s
        log("capsule queries: 4096 agents x 8 avatars")
        extras["capsule_queries_4096x184_ms"] = bench_capsules(args, dev, steps2)
    cpu, pairs = None, None
    if not args.profile and not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu, pairs = cpu_baseline()
    # roofline of the dominant kernel (compositing: plain FP32 VALU work per
    # evaluated pair, the pair count taken from the oracle's render of the same
    # frame; without it, the composited entries n_contrib summed over pixels,
    # a lower bound)
    pair_src = "oracle count of evaluated pairs, same frame"
    if pairs is None:
        pairs = int(info["n_contrib_sum"])
        pair_src = "lower bound: sum of n_contrib over pixels"
    t_comp = st["composite"] * 1e-3
    achieved = pairs * FLOPS_PER_PAIR / t_comp / 1e12
    traffic, traffic_src = counter_traffic()
    roof = {"bound": "alu", "kernel": "composite_kernel", "achieved": achieved, "peak": FP32_NONPACKED_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP32_NONPACKED_TFLOPS, "traffic": traffic,
            "traffic_source": traffic_src, "pairs": pairs, "pairs_source": pair_src,
            "flops_per_pair": FLOPS_PER_PAIR, "exp_per_pair": 1, "avg_launch_ms": st["composite"],
            "alg_bytes_per_launch": info["alg_bytes"]["composite"],
            "frac_of_packed_peak": achieved / FP32_PACKED_TFLOPS}
    out = {"metric": "frames/s 640x480 1M-Gaussian SH3: fwd, fwd+bwd, batched vs plain", "value": fps,
           "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded room-shaped 3DGS scene; no dataset)",
           "config": {"workload": "room1M_640x480_sh3: 1 view, 1M Gaussians, SH degree 3, forward",
                      "global_batch": 1, "parallelism": "none (1 GPU)"},
           "roofline": roof, "extras": extras}
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
