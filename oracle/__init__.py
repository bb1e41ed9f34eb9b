"""FP64 CPU oracle for the Habitat-GS sensor-rendering path (arXiv 2604.12626).

TEST INFRASTRUCTURE ONLY: the test-suite, the package smoke check and the
benchmark's CPU-baseline leg are the only callers.  The product (the HIP
library and its binding) never imports this module, and this module imports
nothing from the product.

The arithmetic lives in ``gs_oracle.c`` (plain C, double precision, OpenMP);
this file builds it with gcc, loads it with ctypes and marshals numpy arrays.

Each function names the passage it follows:
  * Sec. 2.2 / Sec. 3.2 of the paper: explicit anisotropic 3D Gaussians
    rendered by tile-based rasterization into colour and depth; scene and all
    avatars in one rasterization pass.
  * Sec. 3.1 / Sec. 3.3: canonical avatar Gaussians posed by linear blend
    skinning with per-frame joint matrices.
The numeric readings where the paper is silent (camera axes, pixel centres,
near plane 0.2, low-pass 0.3, 3-sigma radius, rect rule, SH convention,
thresholds as FP32 values) are listed in the design notes.

Parity pins: every function here is checked by ``tests/test_oracle_*.py``
against closed forms, invariants, brute force and independent derivations.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

PROJ_STRIDE = 40
MAXC = 8
CAND_STRIDE = 10

# The compositing thresholds are FP32 values promoted to double.
ALPHA_MAX = float(np.float32(0.99))
ALPHA_MIN = float(np.float32(1.0 / 255.0))
T_MIN = float(np.float32(1e-4))


def build(force: bool = True) -> str:
    """Compile gs_oracle.c with gcc into liboracle.so (next to the source)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64, i32, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.or_sh_basis.argtypes = [i32, P, P, P]
    lib.or_project.argtypes = [i64, i32, P, P, P, P, P, P, P, P, P, P]
    lib.or_bin.argtypes = [i64, P, P, i32, i32, i32, i32, P, P, P, i64, P]
    lib.or_bin.restype = i64
    lib.or_composite.argtypes = [i32, P, P, P, P, P, P, P]
    lib.or_render_view.argtypes = [i64, P, P, P, P, P, P, P]
    lib.or_backward_2d.argtypes = [i64, P, P, P, P, P, P, P, P, i64, P, P, P]
    lib.or_backward_3d.argtypes = [i64, i32, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P]
    lib.or_fd_loss.argtypes = [i64, i32, P, P, P, P, P, P, P, P, P, P, P, P, P, i64, P, P, P, P, P]
    lib.or_lbs.argtypes = [i64, P, P, P, P, P, P, i32, P, P]
    lib.or_lbs_backward.argtypes = [i64, P, P, P, P, P, P, i32, P, P, P, P, P]
    lib.or_version.restype = i32
    lib.or_set_threads.argtypes = [i32]
    lib.or_get_threads.restype = i32
    lib.or_cov3d.argtypes = [i64, P, P, P]
    _ = f64
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


def params(width, height, near=0.2, lowpass=0.3, sigma_cut=3.0, fov_clamp=1.3, bg=(0.0, 0.0, 0.0), tile=16,
           d_skip=1e-4, d_stop=1e-4, d_near=1e-5, d_int=1e-5, d_tie=1e-6, max_flips=3, img_tol=1e-4):
    """Rendering constants plus the oracle's decision margins (all double).

    The constants near/lowpass/sigma_cut/fov_clamp are FP32 values on the GPU
    side; they are promoted from FP32 here too so both sides use one value.
    d_skip / d_stop: relative windows around the alpha and transmittance
    thresholds inside which an FP32 implementation may take the other branch
    (its projected means and conics carry FP32 error that moves the exponent
    by ~1e-5..1e-4 relative, see the design notes); d_near / d_int: windows of
    the near-plane test and of the integer radius / floor; d_tie: relative
    depth gap under which two entries' order may swap; img_tol: the image
    tolerance a branch must meet to be taken as an implementation's."""
    f = lambda x: float(np.float32(x))
    return np.array([width, height, f(near), f(lowpass), f(sigma_cut), f(fov_clamp), ALPHA_MAX, ALPHA_MIN, T_MIN,
                     f(bg[0]), f(bg[1]), f(bg[2]), tile, d_skip, d_stop, d_near, d_int, d_tie, max_flips, img_tol],
                    dtype=np.float64)


def cam_array(cam):
    """Camera as 16 doubles: R (row-major world->camera, OpenCV axes), t, fx, fy, cx, cy.

    Accepts the 16-float32 camera record the GPU path reads; promoted exactly."""
    return np.ascontiguousarray(np.asarray(cam, dtype=np.float32).astype(np.float64).reshape(16))


def sh_basis(D, dirs):
    """Real SH (Condon-Shortley phase, l-major, m=-l..l) and gradients at unit directions."""
    lib = _load()
    dirs = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    K = (D + 1) ** 2
    Y = np.zeros((len(dirs), K))
    dY = np.zeros((len(dirs), K, 3))
    for i in range(len(dirs)):
        y = np.zeros(K)
        dy = np.zeros((K, 3))
        lib.or_sh_basis(D, _p(dirs[i]), _p(y), _p(dy))
        Y[i], dY[i] = y, dy
    return Y, dY


def cov3d(log_scales, quats):
    """O1/O2: 3D covariance rows (xx, xy, xz, yy, yz, zz) in double."""
    lib = _load()
    lsc, q = _f32(log_scales).reshape(-1, 3), _f32(quats).reshape(-1, 4)
    out = np.zeros((len(lsc), 6))
    lib.or_cov3d(len(lsc), _p(lsc), _p(q), _p(out))
    return out


def project(g, cam, prm):
    """Per-Gaussian projection of one gaussian set into one camera (O1-O9).

    g: dict with means [n,3], log_scales [n,3], quats [n,4], opacity [n],
    sh [n,K,3], sh_degree, optional cov6 [n,6] and use_cov6 [n] (uint8).
    Returns the [n, PROJ_STRIDE] double table (column meaning in gs_oracle.c)."""
    lib = _load()
    n = len(g["means"])
    D = int(g["sh_degree"])
    means = _f32(g["means"])
    lsc = _f32(g.get("log_scales"))
    quats = _f32(g.get("quats"))
    cov6 = _f32(g.get("cov6"))
    use = g.get("use_cov6")
    use = None if use is None else np.ascontiguousarray(use, dtype=np.uint8)
    opac = _f32(g["opacity"])
    sh = _f32(g["sh"])
    out = np.zeros((n, PROJ_STRIDE))
    lib.or_project(n, D, _p(means), _p(lsc), _p(quats), _p(cov6), _p(use), _p(opac), _p(sh), _p(cam_array(cam)),
                   _p(prm), _p(out))
    return out


def bin_records(rec, visible, W, H, n_views, tile=16, capacity=None):
    """Plain binning of FP32 records: tiles_touched, sorted keys/vals, ranges, K."""
    lib = _load()
    rec = np.ascontiguousarray(rec, dtype=np.float32).reshape(-1, 12)
    m = len(rec)
    vis = np.ascontiguousarray(visible, dtype=np.uint8)
    TX, TY = (W + tile - 1) // tile, (H + tile - 1) // tile
    tt = np.zeros(m, np.uint32)
    # first pass for K
    if capacity is None:
        ranges = np.zeros((n_views * TX * TY, 2), np.uint32)
        K = lib.or_bin(m, _p(rec), _p(vis), W, H, tile, n_views, _p(tt), None, None, 0, _p(ranges))
        capacity = K
    keys = np.zeros(max(capacity, 1), np.uint64)
    vals = np.zeros(max(capacity, 1), np.uint32)
    ranges = np.zeros((n_views * TX * TY, 2), np.uint32)
    K = lib.or_bin(m, _p(rec), _p(vis), W, H, tile, n_views, _p(tt), _p(keys), _p(vals), capacity, _p(ranges))
    return tt, keys[:min(K, capacity)], vals[:min(K, capacity)], ranges, K


def composite(rec, vals, ranges, n_views, prm, want_cands=True):
    """O11 compositing of FP32 records along given per-tile lists.

    Returns img [V,H,W,10] (r, g, b, depth, alpha, T, n_contrib, flips,
    composited count, composited-set signature), ncand [V,H,W] and the
    candidate table [V,H,W,MAXC,10] (NaN rows unused) or None."""
    lib = _load()
    W, H = int(prm[0]), int(prm[1])
    rec = np.ascontiguousarray(rec, dtype=np.float32).reshape(-1, 12)
    vals = np.ascontiguousarray(vals, dtype=np.uint32)
    ranges = np.ascontiguousarray(ranges, dtype=np.uint32)
    img = np.zeros((n_views, H, W, CAND_STRIDE))
    ncand = np.zeros((n_views, H, W), np.int32)
    cands = np.zeros((n_views, H, W, MAXC, CAND_STRIDE)) if want_cands else None
    lib.or_composite(n_views, _p(rec), _p(vals if len(vals) else np.zeros(1, np.uint32)), _p(ranges), _p(prm),
                     _p(img), _p(ncand), _p(cands))
    return img, ncand, cands


def render_view(proj, prm, want_cands=True):
    """Independent FP64 render of one view from the oracle's own projection.

    Returns img [H,W,10], ncand [H,W], flags [H,W] (bit0 rect/visibility
    ambiguity, bit1 depth near-tie), cands or None, pairs."""
    lib = _load()
    W, H = int(prm[0]), int(prm[1])
    proj = np.ascontiguousarray(proj, dtype=np.float64)
    img = np.zeros((H, W, CAND_STRIDE))
    ncand = np.zeros((H, W), np.int32)
    flags = np.zeros((H, W), np.uint8)
    cands = np.zeros((H, W, MAXC, CAND_STRIDE)) if want_cands else None
    pairs = np.zeros(1, np.int64)
    lib.or_render_view(len(proj), _p(proj), _p(prm), _p(img), _p(ncand), _p(flags), _p(cands), _p(pairs))
    return img, ncand, flags, cands, int(pairs[0])


def set_threads(n):
    """Number of OpenMP threads of the oracle's loops; returns the previous one."""
    lib = _load()
    prev = int(lib.or_get_threads())
    lib.or_set_threads(int(n))
    return prev


def concat_segments(segs):
    """Union of gaussian sets in segment order (the instance order of a view).

    Segments given by covariance (cov6) and by scale/rotation may be mixed; the
    result carries use_cov6 per Gaussian.  Pure data marshalling."""
    D = max(int(s["sh_degree"]) for s in segs)
    K = (D + 1) ** 2
    out = {"sh_degree": D}
    n = [len(s["means"]) for s in segs]
    out["means"] = np.concatenate([_f32(s["means"]) for s in segs])
    out["opacity"] = np.concatenate([_f32(s["opacity"]) for s in segs])
    shs = []
    for s in segs:
        sh = _f32(s["sh"]).reshape(len(s["means"]), -1, 3)
        pad = np.zeros((sh.shape[0], K, 3), np.float32)
        pad[:, :sh.shape[1]] = sh
        shs.append(pad)
    out["sh"] = np.concatenate(shs)
    out["log_scales"] = np.concatenate([_f32(s["log_scales"]) if s.get("log_scales") is not None
                                        else np.zeros((k, 3), np.float32) for s, k in zip(segs, n)])
    out["quats"] = np.concatenate([_f32(s["quats"]) if s.get("quats") is not None
                                   else np.tile(np.float32([1, 0, 0, 0]), (k, 1)) for s, k in zip(segs, n)])
    if any(s.get("cov6") is not None for s in segs):
        out["cov6"] = np.concatenate([_f32(s["cov6"]) if s.get("cov6") is not None else np.zeros((k, 6), np.float32)
                                      for s, k in zip(segs, n)])
        out["use_cov6"] = np.concatenate([np.full(k, s.get("cov6") is not None, np.uint8) for s, k in zip(segs, n)])
    return out


def render(g, cam, prm, want_cands=True):
    """Project + render one view of gaussian set g (or a list of segments)."""
    if isinstance(g, (list, tuple)):
        g = concat_segments(g)
    proj = project(g, cam, prm)
    return (proj,) + render_view(proj, prm, want_cands)


def _flat_gaussians(g):
    n = len(g["means"])
    use = g.get("use_cov6")
    return (n, int(g["sh_degree"]), _f32(g["means"]), _f32(g.get("log_scales")), _f32(g.get("quats")),
            _f32(g.get("cov6")), None if use is None else np.ascontiguousarray(use, dtype=np.uint8),
            _f32(g["opacity"]), _f32(g["sh"]))


def backward(g, cams, prm, d_rgb, d_depth, d_alpha, decisions=None):
    """O12 adjoint summed over the views in `cams` (all of the same gaussian set).

    d_rgb [V,H,W,3], d_depth [V,H,W], d_alpha [V,H,W].  Returns a dict of
    double gradients with the input layouts (means, log_scales, quats, opacity,
    sh, cov6 when present).

    decisions (optional): an implementation's discrete decisions per view, a
    list of dicts with "vals" and "ranges" (its per-tile lists for that view:
    ranges [T, 2] into vals), "base" (the instance id of the view's first
    Gaussian), "n_contrib" [H,W] and "img" [H,W,5] (r, g, b, depth, alpha).
    The adjoint then differentiates the branch that implementation took (see
    or_backward_2d) and the result also holds "pixel_status" [V,H,W]:
    0 same decisions as FP64, 1 decisions differing only inside their
    windows with the image reproduced, 2 otherwise."""
    lib = _load()
    if isinstance(g, (list, tuple)):
        g = concat_segments(g)
    n, D, means, lsc, quats, cov6, use, opac, sh = _flat_gaussians(g)
    K = (D + 1) ** 2
    out = {"means": np.zeros((n, 3)), "log_scales": np.zeros((n, 3)), "quats": np.zeros((n, 4)),
           "opacity": np.zeros(n), "sh": np.zeros((n, K, 3)), "cov6": np.zeros((n, 6))}
    cams = np.asarray(cams, dtype=np.float32).reshape(-1, 16)
    W, H = int(prm[0]), int(prm[1])
    if decisions is not None:
        out["pixel_status"] = np.zeros((len(cams), H, W), np.uint8)
    for v in range(len(cams)):
        cam = cam_array(cams[v])
        proj = np.zeros((n, PROJ_STRIDE))
        lib.or_project(n, D, _p(means), _p(lsc), _p(quats), _p(cov6), _p(use), _p(opac), _p(sh), _p(cam), _p(prm),
                       _p(proj))
        g2d = np.zeros((n, 10))
        dr = _f32(d_rgb[v])
        dd = _f32(d_depth[v])
        da = _f32(d_alpha[v])
        if decisions is None:
            lib.or_backward_2d(n, _p(proj), _p(prm), _p(dr), _p(dd), _p(da), _p(g2d), None, None, 0, None, None, None)
        else:
            dv = decisions[v]
            vals = np.ascontiguousarray(dv["vals"], dtype=np.uint32)
            ranges = np.ascontiguousarray(dv["ranges"], dtype=np.uint32).reshape(-1, 2)
            assert len(ranges) == ((W + 15) // 16) * ((H + 15) // 16)
            nc = np.ascontiguousarray(dv["n_contrib"], dtype=np.int32).reshape(H, W)
            img = _f32(dv["img"]).reshape(H, W, 5)
            st = np.zeros((H, W), np.uint8)
            lib.or_backward_2d(n, _p(proj), _p(prm), _p(dr), _p(dd), _p(da), _p(g2d),
                               _p(vals if len(vals) else np.zeros(1, np.uint32)), _p(ranges), int(dv["base"]),
                               _p(nc), _p(img), _p(st))
            out["pixel_status"][v] = st
        lib.or_backward_3d(n, D, _p(means), _p(lsc), _p(quats), _p(cov6), _p(use), _p(opac), _p(sh), _p(cam), _p(prm),
                           _p(g2d), _p(out["means"]), _p(out["log_scales"]), _p(out["quats"]), _p(out["opacity"]),
                           _p(out["sh"]), _p(out["cov6"]))
    return out


def backward_2d(proj, prm, d_rgb, d_depth, d_alpha):
    """Per-Gaussian screen-space adjoints [n,10] (u, v, A, B, C, o, r, g, b, z) of one view."""
    lib = _load()
    n = len(proj)
    g2d = np.zeros((n, 10))
    lib.or_backward_2d(n, _p(np.ascontiguousarray(proj)), _p(prm), _p(_f32(d_rgb)), _p(_f32(d_depth)),
                       _p(_f32(d_alpha)), _p(g2d), None, None, 0, None, None, None)
    return g2d


def param_index(field, comp, sh_degree):
    """Index of one parameter in the flat per-Gaussian vector of fd_loss:
    means 0..2, log_scales 3..5, quats 6..9, opacity 10, sh 11.. (coefficient
    k, channel c at 11 + 3 k + c), cov6 after the SH."""
    K = (sh_degree + 1) ** 2
    base = {"means": 0, "log_scales": 3, "quats": 6, "opacity": 10, "sh": 11, "cov6": 11 + 3 * K}[field]
    return base + int(comp)


def fd_loss(g, cam, prm, samples, h, lin=None, quad=None, tgt=None):
    """Central finite differences (double precision) of the image loss
    L = sum_pix sum_k lin[..., k] y_k + quad[k] (y_k - tgt[..., k])^2 over
    y = (r, g, b, depth, alpha) of the oracle's render of one view, w.r.t.
    the parameters `samples` = [(gaussian, param_index), ...] with steps h.
    Only the tiles the perturbed Gaussian covers are re-rendered.  Returns
    (fd [S], flag [S]); flag 1 marks a sample whose discrete decisions change
    within +-h (no derivative there)."""
    lib = _load()
    if isinstance(g, (list, tuple)):
        g = concat_segments(g)
    n, D, means, lsc, quats, cov6, use, opac, sh = _flat_gaussians(g)
    W, H = int(prm[0]), int(prm[1])
    camd = cam_array(cam)
    proj = np.zeros((n, PROJ_STRIDE))
    lib.or_project(n, D, _p(means), _p(lsc), _p(quats), _p(cov6), _p(use), _p(opac), _p(sh), _p(camd), _p(prm),
                   _p(proj))
    lin = np.zeros((H, W, 5)) if lin is None else np.ascontiguousarray(lin, dtype=np.float64).reshape(H, W, 5)
    quad = np.zeros(5) if quad is None else np.ascontiguousarray(quad, dtype=np.float64).reshape(5)
    tgt = np.zeros((H, W, 5)) if tgt is None else np.ascontiguousarray(tgt, dtype=np.float64).reshape(H, W, 5)
    samples = np.asarray(samples, dtype=np.int64).reshape(-1, 2)
    gi = np.ascontiguousarray(samples[:, 0])
    pi = np.ascontiguousarray(samples[:, 1].astype(np.int32))
    hh = np.ascontiguousarray(np.broadcast_to(np.asarray(h, np.float64), (len(samples),)))
    fd = np.zeros(len(samples))
    flag = np.zeros(len(samples), np.int32)
    lib.or_fd_loss(n, D, _p(means), _p(lsc), _p(quats), _p(cov6), _p(use), _p(opac), _p(sh), _p(camd), _p(prm),
                   _p(proj), _p(lin), _p(quad), _p(tgt), len(samples), _p(gi), _p(pi), _p(hh), _p(fd), _p(flag))
    return fd, flag


def dense_weights(joint_idx, weights, n_joints):
    """Scatter sparse (joint index, weight) pairs into dense [n, J] rows (marshalling)."""
    n = len(joint_idx)
    w = np.zeros((n, n_joints), np.float64)
    for k in range(joint_idx.shape[1]):
        np.add.at(w, (np.arange(n), joint_idx[:, k].astype(np.int64)), weights[:, k].astype(np.float64))
    return w


def lbs(means, log_scales, quats, w_dense, avatar_of, skin, n_joints):
    """O13 linear blend skinning with dense weights: (means' [n,3], cov6' [n,6]) in double."""
    lib = _load()
    n = len(means)
    mo = np.zeros((n, 3))
    co = np.zeros((n, 6))
    w = np.ascontiguousarray(w_dense, dtype=np.float64)
    lib.or_lbs(n, _p(_f32(means)), _p(_f32(log_scales)), _p(_f32(quats)), _p(w),
               _p(np.ascontiguousarray(avatar_of, dtype=np.int32)), _p(_f32(skin)), n_joints, _p(mo), _p(co))
    return mo, co


def lbs_backward(means, log_scales, quats, w_dense, avatar_of, skin, n_joints, d_means_out, d_cov6_out):
    """Adjoint of lbs w.r.t. canonical means, log-scales and quaternions (double)."""
    lib = _load()
    n = len(means)
    dm = np.zeros((n, 3))
    ds = np.zeros((n, 3))
    dq = np.zeros((n, 4))
    w = np.ascontiguousarray(w_dense, dtype=np.float64)
    lib.or_lbs_backward(n, _p(_f32(means)), _p(_f32(log_scales)), _p(_f32(quats)), _p(w),
                        _p(np.ascontiguousarray(avatar_of, dtype=np.int32)), _p(_f32(skin)), n_joints,
                        _p(_f32(d_means_out)), _p(_f32(d_cov6_out)), _p(dm), _p(ds), _p(dq))
    return dm, ds, dq


def sensor_compose(rgb, depth, alpha, mesh_rgba=None, mesh_depth=None):
    """Sensor hand-off: the observation the RGB and depth sensors deliver.

    Sec. 3.4 asks for RGB and depth in the mesh renderer's format (8-bit RGBA
    and metric depth); Sec. 3.2 resolves occlusion against a mesh pass by
    keeping, per pixel, the nearer of the 3DGS fragment (C_g, D_g) and the
    mesh fragment (C_m, D_m), the mesh winning ties.  Because this turns
    floats into byte codes and a comparison, it is written in FP32 (the
    precision the decision is taken in), pixel-wise:
      3DGS fragment where alpha > 0, D_g = depth / alpha;
      bytes rint(clip(c, 0, 1) * 255) (nearest even; NaN -> 0), fourth byte 255;
      mesh fragment where mesh_depth > 0 (NaN: none), bytes copied;
      neither: the 3DGS colour and depth 0.
    Shapes: rgb [..., 3], depth and alpha [...], mesh_rgba uint8 [..., 4],
    mesh_depth [...].  Returns (rgba uint8 [..., 4], depth float32 [...]).
    """
    rgb = np.asarray(rgb, np.float32)
    depth = np.asarray(depth, np.float32)
    alpha = np.asarray(alpha, np.float32)
    one, zero = np.float32(1.0), np.float32(0.0)
    clipped = np.where(rgb > zero, np.minimum(rgb, one), zero)
    codes = np.rint(clipped * np.float32(255.0)).astype(np.uint8)
    out_rgba = np.empty(depth.shape + (4,), np.uint8)
    out_rgba[..., :3] = codes
    out_rgba[..., 3] = 255
    gs_frag = alpha > zero
    d_g = np.zeros_like(depth)
    np.divide(depth, alpha, out=d_g, where=gs_frag)
    out_depth = np.where(gs_frag, d_g, zero).astype(np.float32)
    if mesh_rgba is not None:
        mesh_rgba = np.asarray(mesh_rgba, np.uint8)
        mesh_depth = np.asarray(mesh_depth, np.float32)
        with np.errstate(invalid="ignore"):
            mesh_frag = mesh_depth > zero
            nearer = d_g < mesh_depth
        keep_gs = gs_frag & (~mesh_frag | nearer)
        take_mesh = mesh_frag & ~keep_gs
        out_rgba[take_mesh] = mesh_rgba[take_mesh]
        out_depth[take_mesh] = mesh_depth[take_mesh]
    return out_rgba, out_depth


def clip_frames(frame_pos, clip_first, clip_frames, clip_total):
    """Sec. 3.3 (GAMMA trajectory): each avatar's joint matrices at the
    current time are interpolated between the two clip frames around its
    fractional frame position.  Reading: linear interpolation of the matrices
    ((1 - s) M[f] + s M[f + 1], f = floor(p), s = p - f), p clamped to the
    clip (NaN -> 0), a one-frame clip holding its pose; clip_first clamped
    into the clip array, clip_frames to [1, frames left].  Returns per avatar
    (absolute frame f0, absolute frame f1, s) with s in double."""
    out = []
    for a in range(len(clip_first)):
        first = min(max(int(clip_first[a]), 0), clip_total - 1)
        F = min(max(int(clip_frames[a]), 1), clip_total - first)
        p = float(np.float32(frame_pos[a]))
        p = min(p, float(F - 1)) if p > 0 else 0.0
        if F > 1:
            f0 = min(int(math.floor(p)), F - 2)
            out.append((first + f0, first + f0 + 1, p - f0))
        else:
            out.append((first, first, 0.0))
    return out


def _clip_as_lbs(w_dense, avatar_of, clip, frames):
    """The interpolated blend as a blend over 2J matrices per avatar (the
    frames f0 and f1 of every joint) with weights w (1 - s) and w s: exact,
    since interpolation and blend are both linear in the matrices."""
    J = clip.shape[1]
    skin2 = np.zeros((len(frames), 2 * J, 12), np.float32)
    s_av = np.zeros(len(frames))
    for a, (f0, f1, s) in enumerate(frames):
        skin2[a, :J] = clip[f0]
        skin2[a, J:] = clip[f1]
        s_av[a] = s
    sa = s_av[np.asarray(avatar_of, np.int64)][:, None]
    w2 = np.concatenate([w_dense * (1.0 - sa), w_dense * sa], 1)
    return skin2, w2, 2 * J


def lbs_clip(means, log_scales, quats, w_dense, avatar_of, clip, clip_first, clip_frames_, frame_pos):
    """LBS (O13) with each avatar's joint matrices interpolated at its frame
    position (see clip_frames); double precision."""
    frames = clip_frames(frame_pos, clip_first, clip_frames_, len(clip))
    skin2, w2, J2 = _clip_as_lbs(w_dense, avatar_of, clip, frames)
    return lbs(means, log_scales, quats, w2, avatar_of, skin2, J2)


def lbs_clip_backward(means, log_scales, quats, w_dense, avatar_of, clip, clip_first, clip_frames_, frame_pos,
                      d_means_out, d_cov6_out):
    """Adjoint of lbs_clip w.r.t. canonical means, log-scales, quaternions."""
    frames = clip_frames(frame_pos, clip_first, clip_frames_, len(clip))
    skin2, w2, J2 = _clip_as_lbs(w_dense, avatar_of, clip, frames)
    return lbs_backward(means, log_scales, quats, w2, avatar_of, skin2, J2, d_means_out, d_cov6_out)


# --------------------------------------------------------------------------
# Avatar capsule queries (Sec. 3.3 dynamic NavMesh blocking, Sec. 3.4 query
# APIs): clearance to the nearest avatar capsule and whether a step is
# blocked.  Plain double-precision geometry, one agent at a time.
# --------------------------------------------------------------------------
def point_segment_distance(x, a, b):
    """min over t in [0, 1] of |x - (a + t (b - a))| (the minimiser of a
    one-dimensional convex quadratic, clamped to the interval)."""
    x, a, b = (np.asarray(v, np.float64) for v in (x, a, b))
    d = b - a
    dd = float(d @ d)
    t = 0.0 if dd == 0.0 else min(max(float((x - a) @ d) / dd, 0.0), 1.0)
    return float(np.linalg.norm(x - (a + t * d)))


def segment_segment_distance(p0, p1, q0, q1):
    """min over (s, t) in [0, 1]^2 of |p(s) - q(t)|: a convex quadratic over a
    square, so the minimum is its stationary point when that lies inside,
    else on one of the four sides (each a point-segment distance)."""
    p0, p1, q0, q1 = (np.asarray(v, np.float64) for v in (p0, p1, q0, q1))
    u, v, w = p1 - p0, q1 - q0, p0 - q0
    a, b, c, d, e = u @ u, u @ v, v @ v, u @ w, v @ w
    best = min(point_segment_distance(p0, q0, q1), point_segment_distance(p1, q0, q1),
               point_segment_distance(q0, p0, p1), point_segment_distance(q1, p0, p1))
    den = a * c - b * b
    if den > 1e-12 * a * c:
        s = (b * e - c * d) / den
        t = (a * e - b * d) / den
        if 0.0 <= s <= 1.0 and 0.0 <= t <= 1.0:
            best = min(best, float(np.linalg.norm(w + s * u - t * v)))
    return best


def segment_parallelogram_distance(s0, s1, o, U, V):
    """Distance between the segment [s0, s1] and the parallelogram
    {o + a U + b V : a, b in [0, 1]}: zero where the segment crosses it,
    else attained at a segment end point (against the parallelogram) or on
    one of its four edges (against the segment)."""
    s0, s1, o, U, V = (np.asarray(x, np.float64) for x in (s0, s1, o, U, V))
    edges = [(o, o + U), (o + V, o + U + V), (o, o + V), (o + U, o + U + V)]
    best = min(segment_segment_distance(s0, s1, e0, e1) for e0, e1 in edges)
    g11, g12, g22 = U @ U, U @ V, V @ V
    gd = g11 * g22 - g12 * g12
    if gd > 1e-12 * g11 * g22:  # a proper parallelogram: end points over its interior
        n = np.cross(U, V)
        for x in (s0, s1):
            r = x - o
            a = (g22 * (r @ U) - g12 * (r @ V)) / gd
            b = (g11 * (r @ V) - g12 * (r @ U)) / gd
            if 0.0 <= a <= 1.0 and 0.0 <= b <= 1.0:
                best = min(best, abs(float(r @ n)) / float(np.linalg.norm(n)))
        # the segment crossing the interior: s0 + l (s1 - s0) = o + a U + b V
        M = np.stack([s1 - s0, -U, -V], 1)
        det = float(np.linalg.det(M))
        scale = float(np.linalg.norm(s1 - s0) * np.linalg.norm(U) * np.linalg.norm(V))
        if abs(det) > 1e-6 * scale:
            lab = np.linalg.solve(M, o - s0)
            if np.all(lab >= 0.0) and np.all(lab <= 1.0):
                best = 0.0
    return best


def capsule_queries(agent_pos, agent_next, agent_avatars, radius, height, caps, clip_first, clip_frames_,
                    frame_pos, n_caps):
    """Per agent e (a vertical capsule: axis from agent_pos[e] up `height`,
    radius `radius`), against the capsules of avatars agent_avatars[e] =
    (first, count):
      clearance[e] = min over capsules of dist(agent axis, capsule axis)
                     - radius - r_c (negative: overlap), +inf with no capsule;
      nearest[e]   = the capsule attaining it (avatar * n_caps + c), -1 if none;
      step_gap[e]  = the same minimum for the step from agent_pos[e] to
                     agent_next[e]: the agent axis swept along the step is the
                     parallelogram {p0 + a (p1 - p0) + b height z}.
    Capsule endpoints (and radius) are interpolated linearly in each avatar's
    clip at its frame position, with the clip rules of clip_frames.
    caps: [frames][n_caps][8] = (a.xyz, r, b.xyz, unused)."""
    caps = np.asarray(caps, np.float64)
    frames = clip_frames(frame_pos, clip_first, clip_frames_, len(caps))
    A = len(frames)
    cur = np.zeros((A, n_caps, 7))
    for a, (f0, f1, s) in enumerate(frames):
        cur[a] = (1.0 - s) * caps[f0, :, :7] + s * caps[f1, :, :7]
    E = len(agent_pos)
    clearance = np.full(E, np.inf)
    nearest = np.full(E, -1, np.int64)
    step_gap = np.full(E, np.inf)
    zup = np.array([0.0, 0.0, float(height)])
    for e in range(E):
        first, count = int(agent_avatars[e][0]), int(agent_avatars[e][1])
        p0 = np.asarray(agent_pos[e], np.float64)
        for av in range(max(first, 0), min(first + count, A)):
            for c in range(n_caps):
                ca, r, cb = cur[av, c, 0:3], cur[av, c, 3], cur[av, c, 4:7]
                g = segment_segment_distance(p0, p0 + zup, ca, cb) - radius - r
                if g < clearance[e]:
                    clearance[e], nearest[e] = g, av * n_caps + c
                if agent_next is not None:
                    p1 = np.asarray(agent_next[e], np.float64)
                    gs = segment_parallelogram_distance(ca, cb, p0, p1 - p0, zup) - radius - r
                    step_gap[e] = min(step_gap[e], gs)
    return clearance, nearest, step_gap


def lbs_backward_joints(means, log_scales, quats, w_dense, avatar_of, skin, n_joints, d_means_out, d_cov6_out):
    """Adjoint of lbs (O13) w.r.t. the joint matrices: d_skin [A][J][12] in
    double.  Per Gaussian, with A = sum_j w_j M_j (3x4) and G the symmetric
    adjoint of the posed covariance (off-diagonal cov6 adjoints halved):
    dL/dA[:, :3] = g mean^T + 2 G A3 Sigma, dL/dA[:, 3] = g; then
    dL/dM_j += w_j dL/dA for the Gaussian's avatar."""
    means = np.asarray(means, np.float64)
    Sig = cov3d(log_scales, quats)  # [n, 6] (xx, xy, xz, yy, yz, zz)
    n = len(means)
    A_av = int(np.asarray(skin).shape[0])
    sk = np.asarray(skin, np.float64).reshape(A_av, n_joints, 3, 4)
    aof = np.asarray(avatar_of, np.int64)
    w = np.asarray(w_dense, np.float64)
    gm = np.asarray(d_means_out, np.float64)
    gc = np.asarray(d_cov6_out, np.float64)
    out = np.zeros((A_av, n_joints, 3, 4))
    for i in range(n):
        A = np.einsum("j,jrc->rc", w[i], sk[aof[i]])
        S = np.array([[Sig[i, 0], Sig[i, 1], Sig[i, 2]], [Sig[i, 1], Sig[i, 3], Sig[i, 4]],
                      [Sig[i, 2], Sig[i, 4], Sig[i, 5]]])
        G = np.array([[gc[i, 0], gc[i, 1] / 2, gc[i, 2] / 2], [gc[i, 1] / 2, gc[i, 3], gc[i, 4] / 2],
                      [gc[i, 2] / 2, gc[i, 4] / 2, gc[i, 5]]])
        dA = np.zeros((3, 4))
        dA[:, :3] = np.outer(gm[i], means[i]) + 2.0 * G @ A[:, :3] @ S
        dA[:, 3] = gm[i]
        out[aof[i]] += w[i][:, None, None] * dA[None]
    return out.reshape(A_av, n_joints, 12)


def axis_angle_matrix(w):
    """Rotation by |w| about w / |w| (Rodrigues' formula), double."""
    w = np.asarray(w, np.float64)
    th = float(np.linalg.norm(w))
    if th == 0.0:
        return np.eye(3)
    k = w / th
    K = np.array([[0.0, -k[2], k[1]], [k[2], 0.0, -k[0]], [-k[1], k[0], 0.0]])
    return np.eye(3) + math.sin(th) * K + (1.0 - math.cos(th)) * (K @ K)


def forward_kinematics(parents, rest, pose, root):
    """Skinning matrices of posed skeletons (the forward-kinematics step that
    turns joint rotations into the per-frame joint matrices of Sec. 3.3):
    joint k's world transform is its parent's (the root transform for the
    root) times [R(pose_k) | rest_k - rest_parent] (rest_k for the root), and
    its skinning matrix is that transform times [I | -rest_k], i.e. relative
    to the rest pose.  pose [A][J][3] axis-angle, root [A][12] (3x4),
    rest [J][3].  Returns [A][J][12] double."""
    rest = np.asarray(rest, np.float64)
    A, J = len(pose), len(parents)
    out = np.zeros((A, J, 12))
    for a in range(A):
        Rt = np.eye(4)
        Rt[:3, :] = np.asarray(root[a], np.float64).reshape(3, 4)
        G = [None] * J
        for k in range(J):
            L = np.eye(4)
            L[:3, :3] = axis_angle_matrix(pose[a][k])
            p = int(parents[k])
            L[:3, 3] = rest[k] - (rest[p] if p >= 0 else 0.0)
            G[k] = (Rt if p < 0 else G[p]) @ L
            to_rest = np.eye(4)
            to_rest[:3, 3] = -rest[k]
            out[a, k] = (G[k] @ to_rest)[:3, :].reshape(12)
    return out
