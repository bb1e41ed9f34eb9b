"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bars: integer/index results (tile rects, keys, values, ranges, counts)
bit-exact; images within 1e-4 max-abs (depth 1e-4 * max(1, |D|)) of one of
the oracle's enumerated results for near-threshold decisions; pixels the
oracle flags (ambiguous rect / depth near-tie) are excluded and counted."""
import sys
import zlib

import numpy as np
import pytest

from paper_2604_12626_amd import synth

from parity import TOL_RGB, frame_to_numpy, pixel_match, to_dev

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


def _project_gpu(dev, segs, cams, view_segs, W, H):
    import torch
    from paper_2604_12626_amd import binding as B
    tsegs = [to_dev(g, dev) for g in segs]
    tc = torch.from_numpy(np.ascontiguousarray(cams, dtype=F32)).to(dev)
    n_inst = B.instance_offsets(tsegs, view_segs)[-1]
    tt = torch.zeros(n_inst, dtype=torch.int32, device=dev)
    rec = torch.zeros(n_inst, 12, dtype=torch.float32, device=dev)
    prm = B.make_params(W, H)
    B.project(tsegs, tc, view_segs, prm, tt, rec)
    torch.cuda.synchronize()
    return tt.cpu().numpy().view(np.uint32), rec.cpu().numpy()


PROJECT_CASES = [
    ("cube10k_128x128_sh0", lambda: synth.config(0)),
    ("room50k_640x480_sh3", lambda: synth.config(1, scale=0.05)),
    ("room30k_200x150_sh3_ragged", lambda: dict(synth.config(1, scale=0.03), W=200, H=150,
                                                cams=synth.camera_room(np.random.default_rng(9), 200, 150)[None])),
]


@pytest.mark.parametrize("name,make", PROJECT_CASES, ids=[c[0] for c in PROJECT_CASES])
def test_project_parity(dev, orc, name, make):
    cfg = make()
    W, H = cfg["W"], cfg["H"]
    g = cfg["segments"][0]
    say("project parity:", name, len(g["means"]))
    tt, rec = _project_gpu(dev, [g], cfg["cams"][:1], [[0]], W, H)
    prm = orc.params(W, H)
    pr = orc.project(g, cfg["cams"][0], prm)
    vis_o, amb = pr[:, 0] > 0, pr[:, 21] > 0
    vis_g = tt > 0
    assert np.all((vis_o == vis_g) | amb), np.nonzero((vis_o != vis_g) & ~amb)[0][:10]
    both = vis_o & vis_g
    assert both.sum() > 100
    r, o = rec[both].astype(np.float64), pr[both]
    # tiles and radius: exact unless the oracle flags an integer decision in its margin
    sure = ~amb[both]
    assert np.array_equal(tt[both][sure], ((o[:, 13] - o[:, 12]) * (o[:, 15] - o[:, 14]))[sure].astype(np.uint32))
    rad_g = rec[both][:, 3].view(np.int32)
    rad_sure = o[:, 18] > 1e-5
    assert np.array_equal(rad_g[rad_sure], o[rad_sure, 11].astype(np.int32))
    # continuous values, against an FP32 error model of the camera transform:
    # each camera coordinate carries ~eps * (sum_j |R_ij mu_j| + |t_i|)
    cam = cfg["cams"][0].astype(np.float64)
    R, t = cam[:9].reshape(3, 3), cam[9:12]
    mu = g["means"][both].astype(np.float64)
    mag = np.abs(mu) @ np.abs(R).T + np.abs(t)
    eps = 4 * 2.0 ** -24
    tz = o[:, 3]
    tol_u = eps * (np.abs(o[:, 1] - cam[14]) * mag[:, 2] + cam[12] * mag[:, 0]) / tz + 8 * eps * np.abs(o[:, 1]) + 1e-5
    tol_v = eps * (np.abs(o[:, 2] - cam[15]) * mag[:, 2] + cam[13] * mag[:, 1]) / tz + 8 * eps * np.abs(o[:, 2]) + 1e-5
    assert np.all(np.abs(r[:, 0] - o[:, 1]) <= tol_u)
    assert np.all(np.abs(r[:, 1] - o[:, 2]) <= tol_v)
    assert np.all(np.abs(r[:, 2] - o[:, 3]) <= eps * mag[:, 2])
    # conic = inverse of the 2D covariance [[a, b], [b, c]]: relative errors
    # of its entries (FP32 rounding in the projection chain, a few 2^-24 of
    # their magnitudes) reach the conic amplified by kappa = (ac + b^2) / det
    scale = np.abs(o[:, 4]) + np.abs(o[:, 6])
    cerr = np.max(np.abs(r[:, 4:7] - o[:, 4:7]), axis=1) / scale
    a, b, c = o[:, 26], o[:, 27], o[:, 28]
    kappa = (a * c + b * b) / (a * c - b * b)
    ratio = np.maximum(cerr - 1e-4, 0.0) / (2.0 ** -24 * kappa)
    say("  conic rel err: max %.3g p99.9 %.3g; kappa max %.3g; max (err - 1e-4) / (2^-24 kappa) = %.3g" % (
        cerr.max(), np.quantile(cerr, 0.999), kappa.max(), ratio.max()))
    assert np.quantile(cerr, 0.999) < 1e-4
    assert np.all(cerr <= 1e-4 + 256 * 2.0 ** -24 * kappa)
    assert np.array_equal(r[:, 7], o[:, 7])
    assert np.abs(r[:, 8:11] - o[:, 8:11]).max() <= 1e-5
    assert np.all(rec[both][:, 11].view(np.int32) == 0)


BIN_CASES = [
    ("1view_128x128_5k", [5000], 128, 128),
    ("4views_ragged_100x70", [3000, 0, 2500, 10], 100, 70),
    ("single_instance", [1], 16, 16),
    ("empty", [0], 32, 32),
    ("1view_640x480_200k", [200000], 640, 480),
    ("16views_256x256_60k", [4000] * 15 + [100], 256, 256),
    # past 4096 tiles: tile counters in a window of whole views (16 of 256
    # tiles here) that moves with the views
    ("64views_256x256_windowed", [3000] * 63 + [500], 256, 256),
    # one emission block draws 40 views: the keys past its window take the
    # tiles' last slots
    ("40views_256x256_block_past_window", [90] * 40, 256, 256),
    # 475 tiles a view: a window of 8 views, the ring wraps at 3800 tiles
    ("10views_400x300_ring", [6000] * 10, 400, 300),
]


@pytest.mark.parametrize("name,counts,W,H", BIN_CASES, ids=[c[0] for c in BIN_CASES])
def test_bin_sort_bit_exact(dev, orc, name, counts, W, H):
    import torch
    from paper_2604_12626_amd import binding as B
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    rec, vis = synth.synthetic_records(rng, counts, W, H)
    V = len(counts)
    tt_o, keys_o, vals_o, ranges_o, K = orc.bin_records(rec, vis, W, H, V)
    say("bin_sort:", name, "instances", len(rec), "K", K)
    prm = B.make_params(W, H)
    # both sort algorithms, and every onesweep configuration the tuner may
    # pick, sort identically
    one = {"sort_algorithm": 1}
    runs = [(K + 1000, 0, {}), (K + 1000, 0, one),
            (K + 1000, 0, dict(one, sort_partition_keys=8192, sort_lookback=64)),
            (K + 1000, 0, dict(one, sort_partition_keys=4096, sort_lookback=32)),
            (max(1, K // 2), 1 if K > max(1, K // 2) else 0, {}),
            (max(1, K // 2), 1 if K > max(1, K // 2) else 0, one)]
    prev = B.get_tuning()
    try:
        for cap, expect_ovf, knobs in runs:
            B.set_tuning(**dict(prev, **knobs))
            _bin_sort_case(dev, B, rec, tt_o, keys_o, vals_o, ranges_o, K, V, W, H, prm, cap, expect_ovf)
    finally:
        B.set_tuning(**prev)


LONG_BUCKET_CASES = [
    # 20 views of 256x256: 5120 tiles, the windowed counters and the five
    # sort classes with the run merge kernel
    ("windowed_20views", [80000, 30000] + [2000] * 18, 20),
    # 4 views: 1024 tiles, the two-launch sort (up to 2048 entries; longer,
    # with runs merged by their own workgroup)
    ("two_launch_4views", [80000, 39000, 2000, 2000], 4),
]


@pytest.mark.parametrize("name,counts,V", LONG_BUCKET_CASES, ids=[c[0] for c in LONG_BUCKET_CASES])
def test_bin_sort_long_buckets_bit_exact(dev, orc, name, counts, V):
    """Buckets longer than one LDS sort (16384 entries): sorted as runs and
    merged, one with two runs, one with four and a ragged fifth, next to
    buckets of every shorter class."""
    from paper_2604_12626_amd import binding as B
    rng = np.random.default_rng(77)
    W = H = 256
    rec, vis = synth.synthetic_records(rng, counts, W, H)
    # view 0: every instance in tile 0; view 1: 30000 in tile 5, then (if
    # there are more) 3000 in tile 9 and 6000 in tile 12
    place = {0: [((0, 0), None)], 1: [((5, 0), 30000), ((9, 0), 3000), ((12, 0), 6000)]}
    for v, spots in place.items():
        idx = np.flatnonzero(rec[:, 11].view(np.int32) == v)
        at = 0
        for (tx, ty), k in spots:
            sel = idx[at:] if k is None else idx[at:at + k]
            at += len(sel)
            n = len(sel)
            if n == 0:
                continue
            rec[sel, 0] = 16 * tx + rng.uniform(4.0, 12.0, n)
            rec[sel, 1] = 16 * ty + rng.uniform(4.0, 12.0, n)
            rec[sel, 3] = np.ones(n, np.int32).view(np.float32)
    assert len(counts) == V
    tt_o, keys_o, vals_o, ranges_o, K = orc.bin_records(rec, vis, W, H, V)
    lens = ranges_o.reshape(-1, 2).astype(np.int64)
    lens = lens[:, 1] - lens[:, 0]
    say("long buckets %s: K %d, longest lists %s" % (name, K, np.sort(lens)[-5:]))
    assert lens[0] > 4 * 16384 and 16384 < lens[256 + 5] <= 2 * 16384
    if V * 256 <= 4096:  # the classes between: (2048, 4096] and (4096, 8192]
        assert 2048 < lens[256 + 9] <= 4096 and 4096 < lens[256 + 12] <= 8192
    prm = B.make_params(W, H)
    prev = B.get_tuning()
    try:
        for knobs in ({}, {"sort_algorithm": 1}):
            B.set_tuning(**dict(prev, **knobs))
            _bin_sort_case(dev, B, rec, tt_o, keys_o, vals_o, ranges_o, K, V, W, H, prm, K + 1000, 0)
    finally:
        B.set_tuning(**prev)


def _bin_sort_case(dev, B, rec, tt_o, keys_o, vals_o, ranges_o, K, V, W, H, prm, cap, expect_ovf):
    import torch
    tt = torch.from_numpy(tt_o.view(np.int32).copy()).to(dev)
    r = torch.from_numpy(rec).to(dev)
    keys = torch.zeros(cap, dtype=torch.int64, device=dev)
    vals = torch.zeros(cap, dtype=torch.int32, device=dev)
    T = ((W + 15) // 16) * ((H + 15) // 16)
    ranges = torch.full((V * T, 2), 7, dtype=torch.int32, device=dev)
    num = torch.zeros(1, dtype=torch.int64, device=dev)
    ovf = torch.full((1,), 5, dtype=torch.int32, device=dev)
    ws = torch.empty(B.bin_sort_workspace(len(rec), cap, V, prm), dtype=torch.uint8, device=dev)
    order = torch.full((B.tile_order_words(V, prm),), -1, dtype=torch.int32, device=dev)
    B.bin_sort(tt, r, V, prm, ws, keys, vals, ranges, num, ovf, order=order)
    torch.cuda.synchronize()
    assert int(num.item()) == K and int(ovf.item()) == expect_ovf
    if expect_ovf:
        assert np.all(ranges.cpu().numpy() == 0)
        check_tile_order(order.cpu().numpy(), np.zeros(V * T, np.int64))
        return
    assert np.array_equal(keys.cpu().numpy()[:K].view(np.uint64), keys_o)
    assert np.array_equal(vals.cpu().numpy()[:K].view(np.uint32), vals_o)
    assert np.array_equal(ranges.cpu().numpy().view(np.uint32), ranges_o)
    ro = ranges_o.reshape(-1, 2).astype(np.int64)
    check_tile_order(order.cpu().numpy(), ro[:, 1] - ro[:, 0])


def check_tile_order(order, lens):
    """The compositing work order: queue q (items t = q mod 8) lists each of
    its items once from word q * ceil(n / 8) on, in descending list length
    counted in chunks of 64 entries (63 chunks and more tie)."""
    n = len(lens)
    qs = (n + 7) // 8
    assert len(order) == 8 * qs
    chunks = np.minimum(lens // 64, 63)
    for q in range(8):
        mine = np.arange(q, n, 8)
        got = order[q * qs: q * qs + len(mine)].astype(np.int64)
        assert np.array_equal(np.sort(got), mine), "queue %d is not a permutation of its items" % q
        assert np.all(np.diff(chunks[got]) <= 0), "queue %d not in descending list chunks" % q


COMPOSITE_CASES = [
    ("1view_96x80_4k", [4000], 96, 80, 8.0, 0.7),
    ("2views_256x160_35k", [20000, 15000], 256, 160, 6.0, 0.7),
    ("1view_64x64_big_radii", [600], 64, 64, 30.0, 0.7),
    ("1view_128x96_needles", [3000], 128, 96, 10.0, 1.5),
]


@pytest.mark.parametrize("pairs", [1, 2], ids=["one_wave", "wave_pairs"])
@pytest.mark.parametrize("name,counts,W,H,rmed,aniso", COMPOSITE_CASES, ids=[c[0] for c in COMPOSITE_CASES])
def test_composite_parity(dev, orc, name, counts, W, H, rmed, aniso, pairs):
    """Both compositing walks (one wave per quadrant, and a producer /
    consumer pair of waves) against the oracle."""
    from paper_2604_12626_amd import binding as B
    prev = B.set_tuning(composite_pairs=pairs)
    try:
        _composite_parity_case(dev, orc, name, counts, W, H, rmed, aniso)
    finally:
        B.set_tuning(**prev)


def _composite_parity_case(dev, orc, name, counts, W, H, rmed, aniso):
    import torch
    from paper_2604_12626_amd import binding as B
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    rec, vis = synth.synthetic_records(rng, counts, W, H, r_median=rmed, aniso_sigma=aniso)
    V = len(counts)
    tt_o, keys_o, vals_o, ranges_o, K = orc.bin_records(rec, vis, W, H, V)
    say("composite:", name, "K", K)
    prm_o = orc.params(W, H, bg=(0.1, 0.2, 0.3))
    img_o, ncand, cands = orc.composite(rec, vals_o, ranges_o, V, prm_o)
    prm = B.make_params(W, H, bg=(0.1, 0.2, 0.3))
    T = ((W + 15) // 16) * ((H + 15) // 16)
    tt = torch.from_numpy(tt_o.view(np.int32).copy()).to(dev)
    r = torch.from_numpy(rec).to(dev)
    keys = torch.zeros(K + 16, dtype=torch.int64, device=dev)
    vals = torch.zeros(K + 16, dtype=torch.int32, device=dev)
    ranges = torch.zeros((V * T, 2), dtype=torch.int32, device=dev)
    num = torch.zeros(1, dtype=torch.int64, device=dev)
    ovf = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = torch.empty(B.bin_sort_workspace(len(rec), K + 16, V, prm), dtype=torch.uint8, device=dev)
    order = torch.empty(B.tile_order_words(V, prm), dtype=torch.int32, device=dev)
    B.bin_sort(tt, r, V, prm, ws, keys, vals, ranges, num, ovf, order=order)
    rgb = torch.zeros(V, H, W, 3, device=dev)
    depth = torch.zeros(V, H, W, device=dev)
    alpha = torch.zeros(V, H, W, device=dev)
    tfin = torch.zeros(V, H, W, device=dev)
    ncon = torch.zeros(V, H, W, dtype=torch.int32, device=dev)
    cws = torch.zeros(B.composite_workspace(V, prm), dtype=torch.uint8, device=dev)
    B.composite(r, vals, ranges, V, prm, cws, rgb, depth, alpha, tfin, ncon)
    torch.cuda.synchronize()
    # the call (its own work order) leaves its queue counters (the first 2048
    # bytes) at zero, and a second call over the same workspace, popping tiles
    # in the order the binning wrote, gives the same images
    assert int(cws[:2048].to(torch.int32).abs().sum().item()) == 0, "composite counters not returned to zero"
    rgb2 = torch.full_like(rgb, -1.0)
    ncon2 = torch.full_like(ncon, -1)
    B.composite(r, vals, ranges, V, prm, cws, rgb2, depth, alpha, tfin, ncon2, order=order)
    torch.cuda.synchronize()
    assert torch.equal(rgb, rgb2) and torch.equal(ncon, ncon2)
    gimg = np.concatenate([rgb.cpu().numpy(), depth.cpu().numpy()[..., None], alpha.cpu().numpy()[..., None]],
                          -1).astype(np.float64)
    ok, idx = pixel_match(gimg, cands, ncand)
    say("  max |rgb - primary| = %.3g, alternative-branch pixels: %d" % (
        np.abs(gimg[..., :3] - img_o[..., :3]).max(), int((idx > 0).sum())))
    assert ok.all(), np.argwhere(~ok)[:5]
    nsel = np.take_along_axis(cands[..., 6], np.maximum(idx, 0)[..., None], -1)[..., 0]
    assert np.array_equal(ncon.cpu().numpy(), nsel.astype(np.int32))
    assert np.allclose(tfin.cpu().numpy(), 1 - alpha.cpu().numpy(), atol=1e-6)


RENDER_CASES = [
    ("cube10k_128x128_sh0", lambda: synth.config(0)),
    ("room50k_640x480_sh3", lambda: synth.config(1, scale=0.05)),
    ("room20k_256x256_sh3", lambda: synth.config(2, scale=0.04)),
]


@pytest.mark.parametrize("name,make", RENDER_CASES, ids=[c[0] for c in RENDER_CASES])
def test_render_end_to_end(dev, orc, name, make):
    import torch
    from paper_2604_12626_amd import render
    cfg = make()
    W, H = cfg["W"], cfg["H"]
    g = cfg["segments"][0]
    say("render end-to-end:", name)
    r = render.Renderer(W, H, capacity=1 << 18, device=dev)
    cams = torch.from_numpy(cfg["cams"][:1]).to(dev)
    f = r.render([to_dev(g, dev)], cams, [[0]])
    torch.cuda.synchronize()
    gimg, _ = frame_to_numpy(f, 0)
    prm = orc.params(W, H)
    _, img_o, ncand, flags, cands, pairs = orc.render(g, cfg["cams"][0], prm)
    ok, idx = pixel_match(gimg, cands, ncand)
    bad = ~ok & (flags == 0)
    frac_flag = float((flags != 0).mean())
    say("  pairs %d, flagged %.4f%%, mismatched unflagged %d, max|rgb diff| unflagged %.3g" % (
        pairs, 100 * frac_flag, int(bad.sum()), np.abs(gimg[..., :3] - img_o[..., :3])[flags == 0].max()))
    assert not bad.any(), np.argwhere(bad)[:5]
    assert frac_flag < 0.01


def test_render_deterministic_and_batched_equals_plain(dev):
    import torch
    from paper_2604_12626_amd import render
    cfg = synth.config(3, scale=0.02)
    W, H = cfg["W"], cfg["H"]
    views = [0, 1, 2, 9, 10]
    segs = [to_dev(g, dev) for g in cfg["segments"]]
    cams = torch.from_numpy(cfg["cams"][views]).to(dev)
    vs = [cfg["view_segs"][v] for v in views]
    say("batched vs plain: views", views)
    r = render.Renderer(W, H, capacity=1 << 18, device=dev)
    f = r.render(segs, cams, vs)
    a1 = (f.rgb.clone(), f.depth.clone(), f.alpha.clone())
    f = r.render(segs, cams, vs)
    a2 = (f.rgb.clone(), f.depth.clone(), f.alpha.clone())
    for x, y in zip(a1, a2):
        assert torch.equal(x, y)
    for k, v in enumerate(views):
        r1 = render.Renderer(W, H, capacity=1 << 18, device=dev)
        f1 = r1.render([segs[vs[k][0]]], cams[k:k + 1], [[0]])
        assert torch.equal(f1.rgb[0], a1[0][k]) and torch.equal(f1.depth[0], a1[1][k])
        assert torch.equal(f1.alpha[0], a1[2][k])


def test_composite_schedule_does_not_change_results(dev):
    """Every launch configuration the autotuner may pick (persistent groups
    per CU) gives bit-identical images; the tuner leaves one of them set."""
    import torch
    from paper_2604_12626_amd import autotune, binding as B, render
    cfg = synth.config(3, scale=0.02)
    W, H = cfg["W"], cfg["H"]
    segs = [to_dev(g, dev) for g in cfg["segments"]]
    cams = torch.from_numpy(cfg["cams"][:12]).to(dev)
    vs = cfg["view_segs"][:12]
    r = render.Renderer(W, H, capacity=1 << 18, device=dev)
    prev = B.set_tuning(8)
    try:
        f = r.render(segs, cams, vs)
        ref = (f.rgb.clone(), f.depth.clone(), f.n_contrib.clone())
        for c in (1, 3, 32):
            say("composite groups per CU", c)
            B.set_tuning(c)
            r.composite(f, len(vs))
            torch.cuda.synchronize()
            assert torch.equal(f.rgb, ref[0]) and torch.equal(f.depth, ref[1]) and torch.equal(f.n_contrib, ref[2])
        # without the binning's work order (computed inside the call)
        B.composite(f.rec, f.vals, f.ranges, len(vs), r.params, f.comp_ws, f.rgb, f.depth, f.alpha, f.t_final,
                    f.n_contrib)
        torch.cuda.synchronize()
        assert torch.equal(f.rgb, ref[0]) and torch.equal(f.depth, ref[1]) and torch.equal(f.n_contrib, ref[2])
        best, times = autotune.tune_composite(r, f, len(vs), candidates=(2, 8), reps=2)
        assert best in (2, 8) and B.get_tuning()["composite_groups_per_cu"] == best
    finally:
        B.set_tuning(**prev)


def test_composite_pairs_bit_identical(dev):
    """The pair walk (one wave evaluates a chunk's alphas, the other
    accumulates the chunk before) gives the single wave's results bit for
    bit: images, T_final, n_contrib and the segment checkpoints.  On the
    500k-Gaussian 256x256 view (1024 quadrant items: one pair each, lists of
    many chunks, early stops) and on 12 views of 256x256 with pairs forced,
    so that every pair walks many items in turn."""
    import torch
    from paper_2604_12626_amd import binding as B, render
    prev = B.get_tuning()
    try:
        cfg = synth.config(2)
        cases = [("500k_256x256", cfg, [to_dev(cfg["segments"][0], dev)], cfg["cams"], [[0]], True)]
        c3 = synth.config(3, scale=0.02)
        cases.append(("12views_256x256", c3, [to_dev(g, dev) for g in c3["segments"]], c3["cams"][:12],
                      c3["view_segs"][:12], False))
        for name, c, segs, cams_np, vs, ck in cases:
            W, H = c["W"], c["H"]
            say("pairs vs one wave:", name)
            r = render.Renderer(W, H, capacity=1 << 21, device=dev)
            f = r.render(segs, torch.from_numpy(np.ascontiguousarray(cams_np)).to(dev), vs, checkpoints=ck)
            torch.cuda.synchronize()
            lens = (f.ranges[:, 1] - f.ranges[:, 0]).cpu().numpy()
            out = {}
            for mode in (1, 2):
                B.set_tuning(composite_pairs=mode)
                if f.ckpt is not None:
                    f.ckpt.fill_(-7.0)
                f.rgb.fill_(-1.0)
                f.n_contrib.fill_(-1)
                r.composite(f, len(vs))
                torch.cuda.synchronize()
                out[mode] = [f.rgb.clone(), f.depth.clone(), f.alpha.clone(), f.t_final.clone(), f.n_contrib.clone()]
                if f.ckpt is not None:
                    out[mode].append(f.ckpt.clone())
            for a, b in zip(out[1], out[2]):
                assert torch.equal(a, b), name
            # the paths this reached
            if ck:  # lists of several chunks, opaque pixels, checkpoints written
                assert lens.max() > 4 * 64, lens.max()
                assert (out[1][3].cpu().numpy() < 1e-3).any() and out[1][4].cpu().numpy().max() > 64
                assert (out[1][5] != -7.0).any()
            else:  # many more quadrant items than pairs of waves
                assert 4 * len(lens) > 4 * 256 * 4 and (lens > 64).any()
    finally:
        B.set_tuning(**prev)


def _planes(g):
    """The same segment component-major: every attribute [components][n]."""
    n = len(g["means"])
    out = {"sh_degree": g["sh_degree"], "layout": "planes"}
    for k in ("means", "log_scales", "quats", "cov6", "opacity", "sh"):
        if g.get(k) is not None:
            a = np.asarray(g[k], np.float32).reshape(n, -1)
            out[k] = np.ascontiguousarray(a.T if a.shape[1] > 1 else a[:, 0])
    return out


def test_project_planes_equals_rows(dev):
    """A segment stored component-major (planes) projects to exactly the
    records of the same segment stored in rows -- a scene with rotations and
    scales and a segment given by covariances -- and so renders the same
    images; the backward refuses a planar segment."""
    import torch
    from paper_2604_12626_amd import binding as B, render
    rng = np.random.default_rng(91)
    W, H = 256, 192
    scene = synth.gaussians_room(30000, rng, sh_degree=3)
    n2 = 5000
    A = rng.normal(0.0, 0.03, (n2, 3, 3)).astype(np.float64)
    S = A @ np.transpose(A, (0, 2, 1)) + 1e-5 * np.eye(3)
    cov = np.stack([S[:, 0, 0], S[:, 0, 1], S[:, 0, 2], S[:, 1, 1], S[:, 1, 2], S[:, 2, 2]], 1).astype(np.float32)
    other = synth.gaussians_room(n2, rng, sh_degree=1)
    covseg = {"means": other["means"], "cov6": cov, "opacity": other["opacity"], "sh": other["sh"], "sh_degree": 1}
    cams = torch.from_numpy(np.stack([synth.camera_room(rng, W, H) for _ in range(2)])).to(dev)
    vs = [[0, 1], [0, 1]]
    out = []
    for layout in ("rows", "planes"):
        segs = [scene, covseg] if layout == "rows" else [_planes(scene), _planes(covseg)]
        r = render.Renderer(W, H, capacity=1 << 20, device=dev)
        f = r.render([to_dev(g, dev) for g in segs], cams, vs)
        torch.cuda.synchronize()
        out.append((f.tiles_touched.clone(), f.rec.clone(), f.rgb.clone(), f.depth.clone(), f.n_contrib.clone(), r, f))
    tt0 = out[0][0]
    assert int((tt0 > 0).sum().item()) > 1000
    vis = (tt0 > 0).nonzero().squeeze(1)
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][1][vis], out[1][1][vis])
    for a, b in zip(out[0][2:5], out[1][2:5]):
        assert torch.equal(a, b)
    r, f = out[1][5], out[1][6]
    planar = [to_dev(g, dev) for g in (_planes(scene), _planes(covseg))]
    with pytest.raises(B.GSError):
        r.backward(planar, cams, vs, f, torch.zeros_like(f.rgb), None, None)


def test_union_equals_concatenation(dev):
    import torch
    from paper_2604_12626_amd import render
    rng = np.random.default_rng(77)
    a = synth.gaussians_room(20000, rng, sh_degree=3)
    b = synth.gaussians_room(7000, rng, sh_degree=3)
    cat = {k: (np.concatenate([a[k], b[k]]) if isinstance(a[k], np.ndarray) else a[k]) for k in a}
    cam = synth.camera_room(rng, 160, 128)
    cams = torch.from_numpy(cam[None]).to(dev)
    r = render.Renderer(160, 128, capacity=1 << 18, device=dev)
    f = r.render([to_dev(a, dev), to_dev(b, dev)], cams, [[0, 1]])
    u = (f.rgb.clone(), f.depth.clone(), f.alpha.clone())
    f = r.render([to_dev(cat, dev)], cams, [[0]])
    assert torch.equal(u[0], f.rgb) and torch.equal(u[1], f.depth) and torch.equal(u[2], f.alpha)


def test_full_size_room_keys_are_a_valid_binning(dev):
    """Config of the benchmark (1M Gaussians, 640x480, SH3): keys sorted, values
    a permutation of the instance multiset, ranges consistent, K = sum tiles."""
    import torch
    from paper_2604_12626_amd import render
    cfg = synth.config(1)
    g = cfg["segments"][0]
    say("full-size binning properties: room1M 640x480")
    r = render.Renderer(640, 480, capacity=1 << 22, device=dev)
    f = r.render([to_dev(g, dev)], torch.from_numpy(cfg["cams"]).to(dev), [[0]])
    torch.cuda.synchronize()
    K = int(f.num.item())
    tt = f.tiles_touched.cpu().numpy().view(np.uint32).astype(np.int64)
    assert K == tt.sum() and int(f.overflow.item()) == 0
    keys = f.keys.cpu().numpy()[:K].view(np.uint64)
    vals = f.vals.cpu().numpy()[:K].view(np.uint32)
    assert np.all(keys[1:] >= keys[:-1])
    eq = keys[1:] == keys[:-1]
    assert np.all(vals[1:][eq] > vals[:-1][eq])  # ties in ascending instance order
    assert np.array_equal(np.bincount(vals, minlength=len(tt)), tt)
    rec = f.rec.cpu().numpy()
    assert np.array_equal((keys & np.uint64(0xFFFFFFFF)).astype(np.uint32), rec[vals, 2].view(np.uint32))
    ranges = f.ranges.cpu().numpy().view(np.uint32)
    tiles = (keys >> np.uint64(32)).astype(np.int64)
    starts = np.searchsorted(tiles, np.arange(1200), "left")
    ends = np.searchsorted(tiles, np.arange(1200), "right")
    empty = starts == ends
    assert np.array_equal(ranges[~empty, 0], starts[~empty]) and np.array_equal(ranges[~empty, 1], ends[~empty])
    assert np.all(ranges[empty] == 0)
    say("  K = %d, visible = %d" % (K, int((tt > 0).sum())))


def test_segmented_backward_matches_whole_lists(dev):
    """With lists of thousands of entries (many segments each, and some longer
    than the segment grid holds: 1M room Gaussians at five times their
    scale, 256x256), the segmented backward equals the whole-list walk up to
    rounding, on every parameter block, and the forward images do not depend
    on whether checkpoints are recorded."""
    import torch
    from paper_2604_12626_amd import render
    cfg = synth.config(2, scale=2.0)
    W, H = cfg["W"], cfg["H"]
    g0 = dict(cfg["segments"][0])
    g0["log_scales"] = (g0["log_scales"] + np.log(5.0)).astype(F32)
    g = to_dev(g0, dev)
    # two views: the work list spans several views' tiles
    cam2 = synth.camera_room(np.random.default_rng(21), W, H, fx=128.0)[None]
    cams = torch.from_numpy(np.concatenate([cfg["cams"], cam2]).astype(F32)).to(dev)
    V = 2
    rng = np.random.default_rng(9)
    G = [torch.from_numpy(rng.standard_normal(sh).astype(F32)).to(dev) for sh in ((V, H, W, 3), (V, H, W), (V, H, W))]
    out = {}
    for ck in (False, True):
        r = render.Renderer(W, H, capacity=1 << 22, device=dev, checkpoints=ck)
        f = r.render([g], cams, [[0]] * V)
        img = (f.rgb.clone(), f.depth.clone(), f.alpha.clone())
        d = r.backward([g], cams, [[0]] * V, f, *G)[0]
        torch.cuda.synchronize()
        out[ck] = (img, {k: v.cpu().numpy().astype(np.float64) for k, v in d.items()})
        lens = (f.ranges[:, 1] - f.ranges[:, 0]).cpu().numpy()
    say("  list length max %d, lists over 8 segments: %d" % (lens.max(), int((lens > 8 * 64).sum())))
    assert lens.max() > 64 * 64, "the case must exceed the segment grid"
    for a, b in zip(out[False][0], out[True][0]):
        assert torch.equal(a, b)
    for k, ref in out[False][1].items():
        err = np.abs(out[True][1][k] - ref).max() / max(np.abs(ref).max(), 1e-30)
        say("  %s: max |seg - whole| / max |whole| = %.2e" % (k, err))
        assert err <= 1e-4, (k, err)
    # and both against the oracle along the GPU's branch (segments longer
    # than 64 entries: lists of more than 64 x 64 entries)
    import oracle
    from parity import gpu_decisions, grad_check
    n = len(g0["means"])
    ref = oracle.backward(g0, cams.cpu().numpy(), oracle.params(W, H), *[x.cpu().numpy() for x in G],
                          decisions=gpu_decisions(f, [0, 1], [0, n], W, H))
    assert (ref["pixel_status"] == 2).sum() == 0
    grad_check(say, out[True][1], ref, ("means", "log_scales", "quats", "opacity", "sh"), label="segmented vs oracle")


def test_segmented_backward_many_lists(dev):
    """Checkpoints forced on a launch of more than 2048 lists (9 views of
    256x256: the segment list gets a launch of its own instead of being built
    by the accumulator clear): the segmented backward equals the whole-list
    walk up to rounding."""
    import torch
    from paper_2604_12626_amd import render
    cfg = synth.config(2, scale=0.2)
    W, H = cfg["W"], cfg["H"]
    g = to_dev(cfg["segments"][0], dev)
    rng = np.random.default_rng(33)
    V = 9
    cams = torch.from_numpy(np.stack([synth.camera_room(rng, W, H, fx=128.0) for _ in range(V)]).astype(F32)).to(dev)
    G = [torch.from_numpy(rng.standard_normal(sh).astype(F32)).to(dev) for sh in ((V, H, W, 3), (V, H, W), (V, H, W))]
    out = {}
    for ck in (False, True):
        r = render.Renderer(W, H, capacity=1 << 21, device=dev, checkpoints=ck)
        f = r.render([g], cams, [[0]] * V)
        assert (f.ckpt is not None) == ck
        d = r.backward([g], cams, [[0]] * V, f, *G)[0]
        torch.cuda.synchronize()
        out[ck] = {k: v.cpu().numpy().astype(np.float64) for k, v in d.items()}
        lens = (f.ranges[:, 1] - f.ranges[:, 0]).cpu().numpy()
    assert len(lens) > 2048 and lens.max() > 64
    for k, ref in out[False].items():
        err = np.abs(out[True][k] - ref).max() / max(np.abs(ref).max(), 1e-30)
        say("  %s: max |seg - whole| / max |whole| = %.2e" % (k, err))
        assert err <= 1e-4, (k, err)


def test_lbs_parity(dev, orc):
    import torch
    from paper_2604_12626_amd import binding as B
    cfg = synth.config(4, scale=0.02)  # 8 avatars x 1000 Gaussians (room unused here)
    av, skin = cfg["avatars"], cfg["skin"]
    n, J = len(av["means"]), synth.N_JOINTS
    say("lbs parity:", n, "avatar gaussians")
    t = to_dev(av, dev)
    tskin = torch.from_numpy(skin).to(dev)
    mo = torch.empty(n, 3, device=dev)
    co = torch.empty(n, 6, device=dev)
    B.deform_lbs(t["means"], t["log_scales"], t["quats"], t["joint_idx"], t["weights"], t["avatar_of"], tskin, mo, co)
    w = orc.dense_weights(av["joint_idx"], av["weights"], J)
    mo_o, co_o = orc.lbs(av["means"], av["log_scales"], av["quats"], w, av["avatar_of"], skin, J)
    torch.cuda.synchronize()
    assert np.abs(mo.cpu().numpy() - mo_o).max() <= 1e-5 * max(1.0, np.abs(mo_o).max())
    cs = np.abs(co_o).max(1, keepdims=True)
    assert np.all(np.abs(co.cpu().numpy() - co_o) <= 1e-5 * cs + 1e-12)
    rng = np.random.default_rng(3)
    gm = rng.standard_normal((n, 3)).astype(F32)
    gc = (rng.standard_normal((n, 6)) * 1e3).astype(F32)
    dm, ds, dq = (torch.empty(n, k, device=dev) for k in (3, 3, 4))
    B.deform_lbs_backward(t["means"], t["log_scales"], t["quats"], t["joint_idx"], t["weights"], t["avatar_of"], tskin,
                          torch.from_numpy(gm).to(dev), torch.from_numpy(gc).to(dev), dm, ds, dq)
    rm, rs, rq = orc.lbs_backward(av["means"], av["log_scales"], av["quats"], w, av["avatar_of"], skin, J, gm, gc)
    torch.cuda.synchronize()
    for a, b in ((dm, rm), (ds, rs), (dq, rq)):
        a = a.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(a - b) <= 1e-4 * np.abs(b).max(1, keepdims=True) + 1e-9), np.abs(a - b).max()



@pytest.mark.parametrize("n_avatars", [8, 16], ids=["lds_sums", "global_sums"])
def test_lbs_joint_matrix_gradient_parity(dev, orc, n_avatars):
    # adjoint w.r.t. the joint matrices; 16 avatars x 24 joints exceed the
    # 16-KB workgroup copy, so the kernel sums into the output directly
    import torch
    from paper_2604_12626_amd import binding as B
    cfg = synth.config(4, scale=0.02)
    av = cfg["avatars"]
    n, J = len(av["means"]), synth.N_JOINTS
    rng = np.random.default_rng(91)
    skin = np.stack([synth.skinning_matrices(*synth.avatar_pose(rng)) for _ in range(n_avatars)]).astype(F32)
    aof = (np.arange(n) % n_avatars).astype(np.int32)
    say("lbs joint-matrix gradient:", n, "gaussians,", n_avatars, "avatars")
    t = to_dev(av, dev)
    gm = rng.standard_normal((n, 3)).astype(F32)
    gc = (rng.standard_normal((n, 6)) * 1e3).astype(F32)
    d_skin = torch.full((n_avatars, J, 12), 7.0, device=dev)
    B.deform_lbs_backward_joints(t["means"], t["log_scales"], t["quats"], t["joint_idx"], t["weights"],
                                 torch.from_numpy(aof).to(dev), torch.from_numpy(skin).to(dev),
                                 torch.from_numpy(gm).to(dev), torch.from_numpy(gc).to(dev), d_skin)
    w = orc.dense_weights(av["joint_idx"], av["weights"], J)
    ref = orc.lbs_backward_joints(av["means"], av["log_scales"], av["quats"], w, aof, skin, J, gm, gc)
    torch.cuda.synchronize()
    got = d_skin.cpu().numpy().astype(np.float64)
    assert np.abs(got - ref).max() <= 2e-4 * np.abs(ref).max(), np.abs(got - ref).max() / np.abs(ref).max()
    assert np.all(got[ref == 0] == 0)  # joints no Gaussian blends stay exactly zero


@pytest.mark.parametrize("n_avatars", [8, 131], ids=["8", "131_ragged"])
def test_forward_kinematics_parity(dev, orc, n_avatars):
    import torch
    from paper_2604_12626_amd import binding as B
    J = synth.N_JOINTS
    rng = np.random.default_rng(101)
    pose = rng.normal(0.0, 0.6, (n_avatars, J, 3)).astype(F32)
    pose[0] = 0.0                                   # rest pose
    pose[1, :, :] = rng.normal(0.0, 1e-4, (J, 3))   # tiny angles (series branch of sin t / t)
    pose[2, 5] = [0.0, 3.1, 0.0]                    # near pi
    roots = np.stack([np.concatenate([synth.rodrigues(rng.normal(0, 1, 3)), rng.uniform(-4, 4, (3, 1))], 1)
                      .reshape(12) for _ in range(n_avatars)]).astype(F32)
    say("forward kinematics:", n_avatars, "avatars")
    out = torch.full((n_avatars, J, 12), 7.0, device=dev)
    B.forward_kinematics(synth.PARENTS, torch.from_numpy(synth.REST.astype(F32)).to(dev),
                         torch.from_numpy(pose).to(dev), torch.from_numpy(roots).to(dev), out)
    ref = orc.forward_kinematics(synth.PARENTS, synth.REST.astype(F32).astype(np.float64), pose, roots)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref) <= 2e-5 * np.maximum(1.0, np.abs(ref))), np.abs(got - ref).max()
    # the matrices drive the skinning kernel like any others
    cfg = synth.config(4, scale=0.02)
    av = to_dev(cfg["avatars"], dev)
    n = av["means"].shape[0]
    mo, co = torch.empty(n, 3, device=dev), torch.empty(n, 6, device=dev)
    B.deform_lbs(av["means"], av["log_scales"], av["quats"], av["joint_idx"], av["weights"], av["avatar_of"],
                 out[:8].contiguous(), mo, co)
    torch.cuda.synchronize()
    assert torch.isfinite(mo).all() and torch.isfinite(co).all()


CLIP_POSITIONS = [
    ("fractions", [0.0, 0.4, 2.5, 7.75, 13.2, 28.9, 1.0, 5.5]),
    ("integers_and_ends", [0.0, 1.0, 3.0, 8.0, 0.0, 29.0, 2.0, 11.0]),
    ("clamped", [-3.0, 100.0, float("nan"), -0.5, 1e9, 29.0001, float("inf"), -float("inf")]),
]


@pytest.mark.parametrize("name,pos", CLIP_POSITIONS, ids=[c[0] for c in CLIP_POSITIONS])
def test_lbs_clip_parity(dev, orc, name, pos):
    # 8 avatars x 1000 Gaussians, walking clips of 1 to 30 frames sampled at
    # fractional, integer and out-of-range times
    import torch
    from paper_2604_12626_amd import binding as B
    cfg = synth.config(4, scale=0.02)
    av = cfg["avatars"]
    n, J = len(av["means"]), synth.N_JOINTS
    clip, first, nfr = synth.avatar_clips(np.random.default_rng(17), [1, 2, 4, 9, 3, 30, 6, 12])
    fpos = np.array(pos, np.float32)
    say("lbs clip parity:", name, n, "avatar gaussians,", len(clip), "clip frames")
    t = to_dev(av, dev)
    tc = [torch.from_numpy(x).to(dev) for x in (clip, first, nfr, fpos)]
    mo = torch.empty(n, 3, device=dev)
    co = torch.empty(n, 6, device=dev)
    B.deform_lbs_clip(t["means"], t["log_scales"], t["quats"], t["joint_idx"], t["weights"], t["avatar_of"], *tc,
                      mo, co)
    w = orc.dense_weights(av["joint_idx"], av["weights"], J)
    mo_o, co_o = orc.lbs_clip(av["means"], av["log_scales"], av["quats"], w, av["avatar_of"], clip, first, nfr, fpos)
    torch.cuda.synchronize()
    assert np.abs(mo.cpu().numpy() - mo_o).max() <= 1e-5 * max(1.0, np.abs(mo_o).max())
    cs = np.abs(co_o).max(1, keepdims=True)
    assert np.all(np.abs(co.cpu().numpy() - co_o) <= 1e-5 * cs + 1e-12)
    rng = np.random.default_rng(4)
    gm = rng.standard_normal((n, 3)).astype(F32)
    gc = (rng.standard_normal((n, 6)) * 1e3).astype(F32)
    dm, ds, dq = (torch.empty(n, k, device=dev) for k in (3, 3, 4))
    B.deform_lbs_clip_backward(t["means"], t["log_scales"], t["quats"], t["joint_idx"], t["weights"], t["avatar_of"],
                               *tc, torch.from_numpy(gm).to(dev), torch.from_numpy(gc).to(dev), dm, ds, dq)
    rm, rs, rq = orc.lbs_clip_backward(av["means"], av["log_scales"], av["quats"], w, av["avatar_of"], clip, first,
                                       nfr, fpos, gm, gc)
    torch.cuda.synchronize()
    for a, b in ((dm, rm), (ds, rs), (dq, rq)):
        a = a.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(a - b) <= 1e-4 * np.abs(b).max(1, keepdims=True) + 1e-9), np.abs(a - b).max()
    # at integer times the clip path equals the plain path on that frame's matrices, bit for bit
    if name == "integers_and_ends":
        skin = np.stack([clip[first[a] + int(pos[a])] for a in range(len(first))])
        mp, cp = torch.empty_like(mo), torch.empty_like(co)
        B.deform_lbs(t["means"], t["log_scales"], t["quats"], t["joint_idx"], t["weights"], t["avatar_of"],
                     torch.from_numpy(skin).to(dev), mp, cp)
        torch.cuda.synchronize()
        assert torch.equal(mp, mo) and torch.equal(cp, co)