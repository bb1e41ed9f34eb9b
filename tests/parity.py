"""Helpers shared by the GPU parity tests: moving seeded inputs to the device
and comparing device results with the oracle's (its candidate enumeration
for near-threshold compositing decisions and its flags for ambiguous rects
and depth ties)."""
import numpy as np

TOL_RGB = 1e-4      # max-abs per channel (FP32 path vs FP64 oracle)
TOL_ALPHA = 1e-4
TOL_DEPTH_REL = 1e-4  # depth in metres: 1e-4 * max(1, |D|)


def to_dev(g, dev):
    import torch
    out = {}
    for k, v in g.items():
        if isinstance(v, np.ndarray):
            out[k] = torch.from_numpy(np.ascontiguousarray(v)).to(dev)
        else:
            out[k] = v
    return out


def pixel_match(gpu_img, cands, ncand):
    """gpu_img [..., 5] (r, g, b, depth, alpha) vs candidate table [..., MAXC, 10].
    Returns (match mask, index of the matching candidate or -1)."""
    n = np.abs(ncand)
    C = cands[..., :5]
    d = np.abs(C - gpu_img[..., None, :])
    tol = np.empty_like(d)
    tol[..., :3] = TOL_RGB
    tol[..., 3] = TOL_DEPTH_REL * np.maximum(1.0, np.abs(C[..., 3]))
    tol[..., 4] = TOL_ALPHA
    ok = np.all(d <= tol, axis=-1)
    ok &= np.arange(ok.shape[-1]) < n[..., None]
    ok &= ~np.isnan(C[..., 0])
    idx = np.where(ok.any(-1), ok.argmax(-1), -1)
    return ok.any(-1), idx


def frame_to_numpy(f, view):
    rgb = f.rgb[view].cpu().numpy().astype(np.float64)
    depth = f.depth[view].cpu().numpy().astype(np.float64)
    alpha = f.alpha[view].cpu().numpy().astype(np.float64)
    img = np.concatenate([rgb, depth[..., None], alpha[..., None]], -1)
    nc = f.n_contrib[view].cpu().numpy().astype(np.int64)
    return img, nc


def gpu_decisions(f, views, bases, W, H):
    """The GPU frame's discrete decisions per view, in the form the oracle's
    branch-following adjoint takes: its per-tile lists (vals, ranges of the
    view), the instance id of the view's first Gaussian, n_contrib and its
    image (r, g, b, depth, alpha)."""
    T = ((W + 15) // 16) * ((H + 15) // 16)
    K = int(f.num.item())
    vals = f.vals[:K].cpu().numpy().view(np.uint32)
    ranges = f.ranges.cpu().numpy().view(np.uint32)
    out = []
    for v, base in zip(views, bases):
        img, nc = frame_to_numpy(f, v)
        out.append({"vals": vals, "ranges": ranges[v * T:(v + 1) * T], "base": int(base), "n_contrib": nc,
                    "img": img})
    return out


def grad_check(say, got, ref, fields, tol=1e-4, label="", check=True):
    """max |g_gpu - g_ref| <= tol * max |g_ref| per parameter block, on every
    Gaussian.  got: dict of numpy arrays, ref: the oracle's dict.  A block
    over the bar also reports its worst Gaussian (index, its own largest
    |g_ref| relative to the block's)."""
    worst, where = {}, {}
    for k in fields:
        g = np.asarray(got[k], np.float64).reshape(ref[k].shape)
        scale = np.abs(ref[k]).max()
        assert scale > 0, (label, k)
        err = np.abs(g - ref[k]).reshape(len(g), -1).max(1)
        i = int(err.argmax())
        worst[k] = err[i] / scale
        where[k] = (i, float(np.abs(ref[k]).reshape(len(g), -1)[i].max() / scale))
    say("  %s max |g_gpu - g_ref| / max |g_ref|:" % label, {k: "%.2e" % v for k, v in worst.items()})
    for k, v in worst.items():
        if v > tol:
            say("    %s: worst Gaussian %d, its |g_ref| / block max %.3g" % ((k,) + where[k]))
    if check:
        for k, v in worst.items():
            assert v <= tol, (label, k, v)
    return worst, where
