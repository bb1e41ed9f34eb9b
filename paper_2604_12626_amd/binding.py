"""ctypes binding of libgs.so (the C ABI in include/gs.h) for torch tensors.

Argument marshalling only: every step of the rendering path runs in the HIP
kernels of libgs.so.  Device memory and streams come from PyTorch (ROCm); each
call enqueues on torch's current stream.  If the library is missing this
module raises when first used -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgs.so")

GS_OK, GS_ERR_INVALID_ARGUMENT, GS_ERR_UNSUPPORTED, GS_ERR_WORKSPACE_TOO_SMALL, GS_ERR_HIP = range(5)
TILE = 16
REC_FLOATS = 12
MAX_SEGMENTS = 32
MAX_CAPACITY = (1 << 30) - 1
G2D = 10

P = ctypes.c_void_p


class Camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float)]


class Params(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("near_plane", ctypes.c_float),
                ("lowpass", ctypes.c_float), ("sigma_cut", ctypes.c_float), ("fov_clamp", ctypes.c_float),
                ("alpha_max", ctypes.c_float), ("alpha_min", ctypes.c_float), ("t_min", ctypes.c_float),
                ("bg", ctypes.c_float * 3)]


class Gaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("means", P), ("log_scales", P), ("quats", P), ("cov6", P), ("opacity", P), ("sh", P)]


class GaussiansGrad(ctypes.Structure):
    _fields_ = [("means", P), ("log_scales", P), ("quats", P), ("cov6", P), ("opacity", P), ("sh", P)]


class Projected(ctypes.Structure):
    _fields_ = [("n_instances", ctypes.c_int64), ("tiles_touched", P), ("rec", P)]


class Tuning(ctypes.Structure):
    _fields_ = [("composite_groups_per_cu", ctypes.c_int32), ("sort_partition_keys", ctypes.c_int32),
                ("sort_lookback", ctypes.c_int32), ("sort_algorithm", ctypes.c_int32),
                ("composite_pairs", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


TUNING_FIELDS = ("composite_groups_per_cu", "sort_partition_keys", "sort_lookback", "sort_algorithm",
                 "composite_pairs")


EXPORTS = ["gs_status_string", "gs_last_error", "gs_version", "gs_default_params", "gs_set_tuning", "gs_get_tuning",
           "gs_instance_offsets",
           "gs_deform_lbs", "gs_deform_lbs_backward", "gs_deform_lbs_backward_joints", "gs_forward_kinematics", "gs_deform_lbs_clip", "gs_deform_lbs_clip_backward", "gs_project", "gs_bin_sort_workspace", "gs_tile_order_words", "gs_bin_sort",
           "gs_composite_workspace", "gs_composite", "gs_composite_noalloc", "gs_checkpoint_floats", "gs_render_backward_workspace", "gs_render_backward",
           "gs_sensor_compose", "gs_capsule_queries"]

_lib = None


class GSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (status, msg))
        self.status = status


def load():
    """Load libgs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libgs.so is not built (%s); run __graft_entry__.build() or "
                           "python -m paper_2604_12626_amd.build" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    lib.gs_status_string.restype = ctypes.c_char_p
    lib.gs_status_string.argtypes = [ctypes.c_int]
    lib.gs_last_error.restype = ctypes.c_char_p
    lib.gs_version.restype = i32
    lib.gs_default_params.argtypes = [ctypes.POINTER(Params), i32, i32]
    lib.gs_instance_offsets.argtypes = [ctypes.POINTER(Gaussians), i32, i32, P, P]
    lib.gs_deform_lbs.argtypes = [i64, P, P, P, P, P, P, P, i32, i32, P, P, P]
    lib.gs_deform_lbs_backward.argtypes = [i64, P, P, P, P, P, P, P, i32, i32, P, P, P, P, P, P]
    lib.gs_deform_lbs_backward_joints.argtypes = [i64, P, P, P, P, P, P, P, i32, i32, P, P, P, P]
    lib.gs_forward_kinematics.argtypes = [i32, i32, P, P, P, P, P, P]
    lib.gs_deform_lbs_clip.argtypes = [i64, P, P, P, P, P, P, P, i32, P, P, P, i32, i32, P, P, P]
    lib.gs_deform_lbs_clip_backward.argtypes = [i64, P, P, P, P, P, P, P, i32, P, P, P, i32, i32, P, P, P, P, P, P]
    lib.gs_project.argtypes = [ctypes.POINTER(Gaussians), i32, P, i32, P, ctypes.POINTER(Params),
                               ctypes.POINTER(Projected), P]
    lib.gs_bin_sort_workspace.restype = sz
    lib.gs_bin_sort_workspace.argtypes = [i64, i64, i32, ctypes.POINTER(Params)]
    lib.gs_tile_order_words.restype = sz
    lib.gs_tile_order_words.argtypes = [i32, ctypes.POINTER(Params)]
    lib.gs_bin_sort.argtypes = [ctypes.POINTER(Projected), i32, ctypes.POINTER(Params), P, sz, P, P, i64, P, P, P, P,
                                P]
    lib.gs_composite_workspace.restype = sz
    lib.gs_composite_workspace.argtypes = [i32, ctypes.POINTER(Params)]
    lib.gs_composite.argtypes = [ctypes.POINTER(Projected), P, P, P, i32, ctypes.POINTER(Params), P, sz, P, P, P, P,
                                 P, P, sz, P]
    lib.gs_composite_noalloc.argtypes = [ctypes.POINTER(Projected), P, P, P, i32, ctypes.POINTER(Params), P, P, P, P,
                                         P, P, sz, P]
    lib.gs_checkpoint_floats.restype = sz
    lib.gs_checkpoint_floats.argtypes = [i64]
    lib.gs_render_backward_workspace.restype = sz
    lib.gs_render_backward_workspace.argtypes = [i64]
    lib.gs_render_backward.argtypes = [ctypes.POINTER(Gaussians), i32, P, i32, P, ctypes.POINTER(Params),
                                       ctypes.POINTER(Projected), P, P, P, P, P, P, sz, P, P, P, P, sz,
                                       ctypes.POINTER(GaussiansGrad), P]
    lib.gs_sensor_compose.argtypes = [i32, i32, i32, P, P, P, P, P, P, P, P]
    f32 = ctypes.c_float
    lib.gs_capsule_queries.argtypes = [i32, P, P, P, f32, f32, P, i32, i32, P, P, P, i32, P, P, P, P, P]
    lib.gs_set_tuning.argtypes = [ctypes.POINTER(Tuning)]
    lib.gs_get_tuning.argtypes = [ctypes.POINTER(Tuning)]
    lib.gs_get_tuning.restype = None
    for f in ("gs_deform_lbs", "gs_deform_lbs_backward", "gs_deform_lbs_backward_joints", "gs_forward_kinematics", "gs_deform_lbs_clip", "gs_deform_lbs_clip_backward",
              "gs_project", "gs_bin_sort", "gs_composite", "gs_composite_noalloc",
              "gs_render_backward", "gs_instance_offsets", "gs_set_tuning", "gs_sensor_compose",
              "gs_capsule_queries"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(st):
    if st != GS_OK:
        lib = load()
        raise GSError(lib.gs_status_string(st).decode(), lib.gs_last_error().decode())


def ptr(t):
    """Device (or host) address of a tensor, or None."""
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def stream_handle(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def make_params(width, height, bg=(0.0, 0.0, 0.0), **overrides):
    lib = load()
    p = Params()
    lib.gs_default_params(ctypes.byref(p), int(width), int(height))
    for k, v in overrides.items():
        setattr(p, k, v)
    p.bg[0], p.bg[1], p.bg[2] = (float(x) for x in bg)
    return p


def _req(t, dtype, what):
    if t is None:
        return
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (what, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)


def make_segment(g):
    """gs_gaussians for a dict of device tensors (means, log_scales, quats,
    opacity, sh[, cov6], sh_degree[, layout]).  layout "planes" (gs_project
    only): every attribute component-major, means [3][n], sh [3 (D+1)^2][n]."""
    for k in ("means", "log_scales", "quats", "opacity", "sh", "cov6"):
        _req(g.get(k), torch.float32, k)
    planes = g.get("layout", "rows") == "planes"
    s = Gaussians()
    s.n = int(g["means"].shape[1] if planes else g["means"].shape[0])
    s.layout = 1 if planes else 0
    s.sh_degree = int(g["sh_degree"])
    s.means = ptr(g["means"])
    s.log_scales = ptr(g.get("log_scales"))
    s.quats = ptr(g.get("quats"))
    s.cov6 = ptr(g.get("cov6"))
    s.opacity = ptr(g["opacity"])
    s.sh = ptr(g["sh"])
    return s


def seg_array(segs):
    arr = (Gaussians * len(segs))()
    for i, g in enumerate(segs):
        arr[i] = make_segment(g)
    return arr


def mask_array(view_segs):
    """uint32 masks from per-view lists of segment indices."""
    m = (ctypes.c_uint32 * len(view_segs))()
    for v, ss in enumerate(view_segs):
        x = 0
        for s in ss:
            x |= 1 << int(s)
        m[v] = x
    return m


def instance_offsets(segs, view_segs):
    lib = load()
    arr = seg_array(segs)
    masks = mask_array(view_segs)
    off = (ctypes.c_int64 * (len(view_segs) + 1))()
    _check(lib.gs_instance_offsets(arr, len(segs), len(view_segs), masks, off))
    return list(off)


def project(segs, cams, view_segs, params, tiles_touched, rec):
    """gs_project: cams is a [V,16] float32 device tensor."""
    lib = load()
    _req(cams, torch.float32, "cams")
    arr = seg_array(segs)
    masks = mask_array(view_segs)
    out = Projected(int(rec.shape[0]), ptr(tiles_touched), ptr(rec))
    _check(lib.gs_project(arr, len(segs), ptr(cams), len(view_segs), masks, ctypes.byref(params), ctypes.byref(out),
                          stream_handle()))


def bin_sort_workspace(n_instances, capacity, n_views, params):
    return int(load().gs_bin_sort_workspace(int(n_instances), int(capacity), int(n_views), ctypes.byref(params)))


def tile_order_words(n_views, params):
    return int(load().gs_tile_order_words(int(n_views), ctypes.byref(params)))


def bin_sort(tiles_touched, rec, n_views, params, ws, keys, vals, ranges, d_num, d_overflow, order=None):
    lib = load()
    proj = Projected(int(rec.shape[0]), ptr(tiles_touched), ptr(rec))
    _check(lib.gs_bin_sort(ctypes.byref(proj), int(n_views), ctypes.byref(params), ptr(ws), ws.numel() * ws.element_size(),
                           ptr(keys), ptr(vals), int(keys.shape[0]), ptr(ranges), ptr(order), ptr(d_num),
                           ptr(d_overflow), stream_handle()))


def composite_workspace(n_views, params):
    return int(load().gs_composite_workspace(int(n_views), ctypes.byref(params)))


def checkpoint_floats(capacity):
    return int(load().gs_checkpoint_floats(int(capacity)))


def composite(rec, vals, ranges, n_views, params, ws, rgb, depth, alpha, t_final=None, n_contrib=None, order=None,
              ckpt=None):
    lib = load()
    proj = Projected(int(rec.shape[0]), None, ptr(rec))
    _check(lib.gs_composite(ctypes.byref(proj), ptr(vals), ptr(ranges), ptr(order), int(n_views), ctypes.byref(params),
                            ptr(ws), ws.numel() * ws.element_size(), ptr(rgb), ptr(depth), ptr(alpha), ptr(t_final),
                            ptr(n_contrib), ptr(ckpt), 0 if ckpt is None else ckpt.numel(), stream_handle()))


def composite_noalloc(rec, vals, ranges, n_views, params, rgb, depth, alpha, t_final=None, n_contrib=None, order=None,
                      ckpt=None):
    """gs_composite_noalloc: gs_composite with its workspace in the library's
    own per-GPU scratch (nothing allocated by the call)."""
    lib = load()
    proj = Projected(int(rec.shape[0]), None, ptr(rec))
    _check(lib.gs_composite_noalloc(ctypes.byref(proj), ptr(vals), ptr(ranges), ptr(order), int(n_views),
                                    ctypes.byref(params), ptr(rgb), ptr(depth), ptr(alpha), ptr(t_final),
                                    ptr(n_contrib), ptr(ckpt), 0 if ckpt is None else ckpt.numel(), stream_handle()))


def render_backward_workspace(n_instances):
    return int(load().gs_render_backward_workspace(int(n_instances)))


def render_backward(segs, cams, view_segs, params, tiles_touched, rec, vals, ranges, t_final, n_contrib, d_rgb,
                    d_depth, d_alpha, ws, grads, ckpt=None, order=None):
    """grads: list (per segment) of dicts of output tensors (means, log_scales, quats, cov6, opacity, sh)."""
    lib = load()
    arr = seg_array(segs)
    masks = mask_array(view_segs)
    garr = (GaussiansGrad * len(segs))()
    for i, g in enumerate(grads):
        garr[i] = GaussiansGrad(ptr(g.get("means")), ptr(g.get("log_scales")), ptr(g.get("quats")), ptr(g.get("cov6")),
                                ptr(g.get("opacity")), ptr(g.get("sh")))
    proj = Projected(int(rec.shape[0]), ptr(tiles_touched), ptr(rec))
    _check(lib.gs_render_backward(arr, len(segs), ptr(cams), len(view_segs), masks, ctypes.byref(params),
                                  ctypes.byref(proj), ptr(vals), ptr(ranges), ptr(order), ptr(t_final),
                                  ptr(n_contrib), ptr(ckpt),
                                  0 if ckpt is None else ckpt.numel(), ptr(d_rgb), ptr(d_depth), ptr(d_alpha), ptr(ws),
                                  ws.numel() * ws.element_size(), garr, stream_handle()))


def deform_lbs(means_c, log_scales_c, quats_c, joint_idx, weights, avatar_of, skin_mats, means_out, cov6_out):
    lib = load()
    A, J = int(skin_mats.shape[0]), int(skin_mats.shape[1])
    _check(lib.gs_deform_lbs(int(means_c.shape[0]), ptr(means_c), ptr(log_scales_c), ptr(quats_c), ptr(joint_idx),
                             ptr(weights), ptr(avatar_of), ptr(skin_mats), A, J, ptr(means_out), ptr(cov6_out),
                             stream_handle()))


def deform_lbs_backward(means_c, log_scales_c, quats_c, joint_idx, weights, avatar_of, skin_mats, d_means_out,
                        d_cov6_out, d_means, d_log_scales, d_quats):
    lib = load()
    A, J = int(skin_mats.shape[0]), int(skin_mats.shape[1])
    _check(lib.gs_deform_lbs_backward(int(means_c.shape[0]), ptr(means_c), ptr(log_scales_c), ptr(quats_c),
                                      ptr(joint_idx), ptr(weights), ptr(avatar_of), ptr(skin_mats), A, J,
                                      ptr(d_means_out), ptr(d_cov6_out), ptr(d_means), ptr(d_log_scales),
                                      ptr(d_quats), stream_handle()))


def sensor_compose(rgb, depth, alpha, out_rgba, out_depth, mesh_rgba=None, mesh_depth=None):
    """gs_sensor_compose on [V, H, W] views: rgb [V, H, W, 3], depth / alpha
    [V, H, W], optional mesh_rgba uint8 [V, H, W, 4] and mesh_depth; writes
    out_rgba uint8 [V, H, W, 4] and out_depth [V, H, W]."""
    lib = load()
    V, H, W = (int(x) for x in depth.shape)
    _check(lib.gs_sensor_compose(V, H, W, ptr(rgb), ptr(depth), ptr(alpha), ptr(mesh_rgba), ptr(mesh_depth),
                                 ptr(out_rgba), ptr(out_depth), stream_handle()))


def deform_lbs_backward_joints(means_c, log_scales_c, quats_c, joint_idx, weights, avatar_of, skin_mats, d_means_out,
                               d_cov6_out, d_skin_mats):
    lib = load()
    A, J = int(skin_mats.shape[0]), int(skin_mats.shape[1])
    _check(lib.gs_deform_lbs_backward_joints(int(means_c.shape[0]), ptr(means_c), ptr(log_scales_c), ptr(quats_c),
                                             ptr(joint_idx), ptr(weights), ptr(avatar_of), ptr(skin_mats), A, J,
                                             ptr(d_means_out), ptr(d_cov6_out), ptr(d_skin_mats), stream_handle()))


def forward_kinematics(parents, rest, pose, root, skin_out):
    """gs_forward_kinematics: parents is a host sequence of ints; rest [J, 3],
    pose [A, J, 3], root [A, 12] and skin_out [A, J, 12] on the device."""
    lib = load()
    par = (ctypes.c_int32 * len(parents))(*[int(p) for p in parents])
    _check(lib.gs_forward_kinematics(int(pose.shape[0]), len(parents), par, ptr(rest), ptr(pose), ptr(root),
                                     ptr(skin_out), stream_handle()))


def deform_lbs_clip(means_c, log_scales_c, quats_c, joint_idx, weights, avatar_of, clip, clip_first, clip_frames,
                    frame_pos, means_out, cov6_out):
    """gs_deform_lbs_clip: clip [frames, J, 12]; clip_first, clip_frames int32
    [A] and frame_pos float32 [A] on the device."""
    lib = load()
    _check(lib.gs_deform_lbs_clip(int(means_c.shape[0]), ptr(means_c), ptr(log_scales_c), ptr(quats_c),
                                  ptr(joint_idx), ptr(weights), ptr(avatar_of), ptr(clip), int(clip.shape[0]),
                                  ptr(clip_first), ptr(clip_frames), ptr(frame_pos), int(clip_first.shape[0]),
                                  int(clip.shape[1]), ptr(means_out), ptr(cov6_out), stream_handle()))


def deform_lbs_clip_backward(means_c, log_scales_c, quats_c, joint_idx, weights, avatar_of, clip, clip_first,
                             clip_frames, frame_pos, d_means_out, d_cov6_out, d_means, d_log_scales, d_quats):
    lib = load()
    _check(lib.gs_deform_lbs_clip_backward(int(means_c.shape[0]), ptr(means_c), ptr(log_scales_c), ptr(quats_c),
                                           ptr(joint_idx), ptr(weights), ptr(avatar_of), ptr(clip),
                                           int(clip.shape[0]), ptr(clip_first), ptr(clip_frames), ptr(frame_pos),
                                           int(clip_first.shape[0]), int(clip.shape[1]), ptr(d_means_out),
                                           ptr(d_cov6_out), ptr(d_means), ptr(d_log_scales), ptr(d_quats),
                                           stream_handle()))


def capsule_queries(agent_pos, agent_next, agent_avatars, radius, height, caps, clip_first, clip_frames, frame_pos,
                    clearance, nearest=None, step_gap=None, blocked=None):
    """gs_capsule_queries: agent_pos / agent_next [E, 3], agent_avatars int32
    [E, 2], caps [frames, n_caps, 8], clip_first / clip_frames int32 [A],
    frame_pos [A]; writes clearance [E] (and nearest int32 [E], step_gap [E],
    blocked uint8 [E])."""
    lib = load()
    _check(lib.gs_capsule_queries(int(agent_pos.shape[0]), ptr(agent_pos), ptr(agent_next), ptr(agent_avatars),
                                  float(radius), float(height), ptr(caps), int(caps.shape[0]), int(caps.shape[1]),
                                  ptr(clip_first), ptr(clip_frames), ptr(frame_pos), int(clip_first.shape[0]),
                                  ptr(clearance), ptr(nearest), ptr(step_gap), ptr(blocked), stream_handle()))


def set_tuning(composite_groups_per_cu=None, **kw):
    """Set launch knobs (others keep their current values); with no
    arguments, restore the defaults.  Returns the previous configuration."""
    lib = load()
    prev = get_tuning()
    if composite_groups_per_cu is None and not kw:
        _check(lib.gs_set_tuning(None))
        return prev
    cur = dict(prev)
    if composite_groups_per_cu is not None:
        cur["composite_groups_per_cu"] = composite_groups_per_cu
    for k, v in kw.items():
        if k not in TUNING_FIELDS:
            raise KeyError(k)
        cur[k] = v
    t = Tuning()
    for k in TUNING_FIELDS:
        setattr(t, k, int(cur[k]))
    _check(lib.gs_set_tuning(ctypes.byref(t)))
    return prev


def get_tuning():
    t = Tuning()
    load().gs_get_tuning(ctypes.byref(t))
    return {k: int(getattr(t, k)) for k in TUNING_FIELDS}
