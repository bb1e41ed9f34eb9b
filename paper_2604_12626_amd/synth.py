"""Seeded synthetic inputs shaped like the paper's workloads.

This module draws inputs only: Gaussian sets, cameras, skinning assets and
projected-record stand-ins.  It contains none of the renderer's arithmetic and
serves the HIP path and the oracle alike.

Stand-ins (the paper's assets are not available):
  * indoor 3DGS captures (InteriorGS / self-reconstructions, 300K-7M
    Gaussians, Sec. 4.1 and Table 6) -> a room-shaped 8 x 6 x 3 m box with 70%
    of the Gaussians within 5 cm of its floor and walls;
  * AnimatableGaussians avatars posed by SMPL-X joint matrices (Sec. 3.1,
    Sec. 3.3) -> a synthetic 24-joint humanoid with Gaussians along its bones;
    the per-frame joint matrices come from forward kinematics of random joint
    rotations, standing in for the offline GAMMA -> FK stage the paper runs
    before rendering.

All draws use numpy's PCG64 with ``SeedSequence(seed).spawn(k)`` children, one
per scene / view / avatar.  Values are drawn in float64 and stored as float32;
both sides consume the same float32 arrays.

Layouts (row-major, one row per Gaussian): means [n,3], log_scales [n,3],
quats [n,4] (w,x,y,z), opacity [n], sh [n,(D+1)^2,3], cov6 [n,6]
(xx,xy,xz,yy,yz,zz).  A camera is 16 float32: R (world->camera, OpenCV axes,
row-major), t, fx, fy, cx, cy.
"""
from __future__ import annotations

import math

import numpy as np

ROOM = (8.0, 6.0, 3.0)


def _rngs(seed, k):
    return [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(seed).spawn(k)]


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _unit_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def gaussians_cube(n, rng, sh_degree=0, center=(0.0, 0.0, 3.0)):
    """Means uniform in [-1,1]^3 + center; log-scales N(-4, 0.5); unit quats;
    opacity sigmoid(N(0,1)); DC ~ N(0, 0.3), higher bands N(0, 0.05)."""
    K = (sh_degree + 1) ** 2
    means = rng.uniform(-1.0, 1.0, (n, 3)) + np.asarray(center)
    lsc = rng.normal(-4.0, 0.5, (n, 3))
    q = _unit_quats(rng, n)
    op = _sigmoid(rng.standard_normal(n))
    sh = np.zeros((n, K, 3))
    sh[:, 0, :] = rng.normal(0.0, 0.3, (n, 3))
    if K > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.05, (n, K - 1, 3))
    return _pack(means, lsc, q, op, sh, sh_degree)


def gaussians_room(n, rng, sh_degree=3, log_scale_mu=-4.5, log_scale_sigma=0.7):
    """Room-shaped scene: 70% of the means on the floor/walls (face chosen in
    proportion to its area, inward offset U[0, 0.05] m), 30% uniform in the box."""
    L, Wd, Hh = ROOM
    K = (sh_degree + 1) ** 2
    n_surf = int(round(0.7 * n))
    faces = np.array([L * Wd, L * Hh, L * Hh, Wd * Hh, Wd * Hh])  # floor, y=0, y=W, x=0, x=L
    face = rng.choice(5, size=n_surf, p=faces / faces.sum())
    a = rng.uniform(0.0, 1.0, n_surf)
    b = rng.uniform(0.0, 1.0, n_surf)
    off = rng.uniform(0.0, 0.05, n_surf)
    P = np.zeros((n_surf, 3))
    m = face == 0
    P[m] = np.stack([a[m] * L, b[m] * Wd, off[m]], 1)
    m = face == 1
    P[m] = np.stack([a[m] * L, off[m], b[m] * Hh], 1)
    m = face == 2
    P[m] = np.stack([a[m] * L, Wd - off[m], b[m] * Hh], 1)
    m = face == 3
    P[m] = np.stack([off[m], a[m] * Wd, b[m] * Hh], 1)
    m = face == 4
    P[m] = np.stack([L - off[m], a[m] * Wd, b[m] * Hh], 1)
    Q = rng.uniform(0.0, 1.0, (n - n_surf, 3)) * np.array([L, Wd, Hh])
    means = np.concatenate([P, Q])
    lsc = rng.normal(log_scale_mu, log_scale_sigma, (n, 3))
    q = _unit_quats(rng, n)
    op = _sigmoid(rng.standard_normal(n))
    sh = np.zeros((n, K, 3))
    sh[:, 0, :] = rng.normal(0.0, 0.3, (n, 3))
    if K > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.05, (n, K - 1, 3))
    return _pack(means, lsc, q, op, sh, sh_degree)


def _pack(means, lsc, q, op, sh, D):
    f = lambda x: np.ascontiguousarray(x, dtype=np.float32)
    return {"means": f(means), "log_scales": f(lsc), "quats": f(q), "opacity": f(op), "sh": f(sh),
            "sh_degree": int(D)}


def look_camera(pos, yaw, pitch, fx, fy, cx, cy):
    """World->camera record (OpenCV axes) for a z-up world, looking along
    (cos p cos y, cos p sin y, sin p) with zero roll."""
    f = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
    up = np.array([0.0, 0.0, 1.0])
    right = np.cross(f, up)
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    R = np.stack([right, down, f])
    t = -R @ np.asarray(pos, dtype=np.float64)
    return np.concatenate([R.reshape(9), t, [fx, fy, cx, cy]]).astype(np.float32)


def camera_room(rng, W, H, fx=None):
    """Camera inside the room box shrunk by 0.5 m, yaw U[0, 2pi), pitch
    U[-20, 20] deg, roll 0; 90 deg horizontal FOV unless fx is given."""
    L, Wd, Hh = ROOM
    pos = rng.uniform(0.0, 1.0, 3) * (np.array([L, Wd, Hh]) - 1.0) + 0.5
    yaw = rng.uniform(0.0, 2 * math.pi)
    pitch = math.radians(rng.uniform(-20.0, 20.0))
    if fx is None:
        fx = W / 2.0
    return look_camera(pos, yaw, pitch, fx, fx, W / 2.0, H / 2.0)


def identity_camera(fx, fy, cx, cy):
    return np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, fx, fy, cx, cy], np.float32)


# --------------------------------------------------------------------------
# avatars: synthetic 24-joint humanoid, canonical Gaussians, skinning weights
# --------------------------------------------------------------------------
# joint: (name, parent, rest position [m]); z-up, 1.7 m tall, T-pose along +-y
SKELETON = [
    ("pelvis", -1, (0.0, 0.0, 0.95)),
    ("spine1", 0, (0.0, 0.0, 1.05)),
    ("spine2", 1, (0.0, 0.0, 1.20)),
    ("spine3", 2, (0.0, 0.0, 1.35)),
    ("neck", 3, (0.0, 0.0, 1.50)),
    ("head", 4, (0.0, 0.0, 1.60)),
    ("l_collar", 3, (0.0, 0.07, 1.42)),
    ("l_shoulder", 6, (0.0, 0.18, 1.42)),
    ("l_elbow", 7, (0.0, 0.45, 1.42)),
    ("l_wrist", 8, (0.0, 0.70, 1.42)),
    ("l_hand", 9, (0.0, 0.78, 1.42)),
    ("r_collar", 3, (0.0, -0.07, 1.42)),
    ("r_shoulder", 11, (0.0, -0.18, 1.42)),
    ("r_elbow", 12, (0.0, -0.45, 1.42)),
    ("r_wrist", 13, (0.0, -0.70, 1.42)),
    ("r_hand", 14, (0.0, -0.78, 1.42)),
    ("l_hip", 0, (0.0, 0.09, 0.90)),
    ("l_knee", 16, (0.0, 0.09, 0.50)),
    ("l_ankle", 17, (0.0, 0.09, 0.08)),
    ("l_foot", 18, (0.10, 0.09, 0.02)),
    ("r_hip", 0, (0.0, -0.09, 0.90)),
    ("r_knee", 20, (0.0, -0.09, 0.50)),
    ("r_ankle", 21, (0.0, -0.09, 0.08)),
    ("r_foot", 22, (0.10, -0.09, 0.02)),
]
N_JOINTS = len(SKELETON)
PARENTS = np.array([p for _, p, _ in SKELETON], np.int64)
REST = np.array([x for _, _, x in SKELETON], np.float64)


def avatar_canonical(n, rng, sh_degree=3):
    """Canonical avatar Gaussians: uniform along the bones (bone picked in
    proportion to its length) within a 6 cm ball, plus a head cluster; skinning
    weights Dirichlet(1,1,1,1) over 4 distinct uniform-random joints."""
    K = (sh_degree + 1) ** 2
    bones = [(PARENTS[k], k) for k in range(1, N_JOINTS)]
    seg_a = np.array([REST[p] for p, _ in bones])
    seg_b = np.array([REST[c] for _, c in bones])
    length = np.linalg.norm(seg_b - seg_a, axis=1)
    n_head = n // 10
    which = rng.choice(len(bones), size=n - n_head, p=length / length.sum())
    t = rng.uniform(0.0, 1.0, n - n_head)[:, None]
    d = rng.standard_normal((n - n_head, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rad = 0.06 * rng.uniform(0.0, 1.0, n - n_head) ** (1.0 / 3.0)
    P = seg_a[which] + t * (seg_b[which] - seg_a[which]) + d * rad[:, None]
    hd = rng.standard_normal((n_head, 3))
    hd /= np.linalg.norm(hd, axis=1, keepdims=True)
    H = REST[5] + np.array([0.0, 0.0, 0.02]) + hd * 0.1 * rng.uniform(0.0, 1.0, n_head)[:, None] ** (1.0 / 3.0)
    means = np.concatenate([P, H])
    lsc = rng.normal(-5.0, 0.5, (n, 3))
    q = _unit_quats(rng, n)
    op = _sigmoid(rng.standard_normal(n))
    sh = np.zeros((n, K, 3))
    sh[:, 0, :] = rng.normal(0.0, 0.3, (n, 3))
    if K > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.05, (n, K - 1, 3))
    g = _pack(means, lsc, q, op, sh, sh_degree)
    idx = np.argsort(rng.random((n, N_JOINTS)), axis=1)[:, :4]  # 4 distinct uniform joints
    w = rng.dirichlet(np.ones(4), size=n)
    g["joint_idx"] = idx.astype(np.uint8)
    g["weights"] = w.astype(np.float32)
    return g


def rodrigues(w):
    """Rotation matrix of an axis-angle vector (exp of its skew matrix)."""
    th = float(np.linalg.norm(w))
    Kx = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])
    if th < 1e-12:
        return np.eye(3) + Kx
    return np.eye(3) + math.sin(th) / th * Kx + (1.0 - math.cos(th)) / (th * th) * (Kx @ Kx)


def skinning_matrices(pose, root_R, root_t):
    """Forward kinematics of the synthetic skeleton (offline asset preparation
    in the paper): G_0 = [root_R | root_t] [R(w_0) | j_0],
    G_k = G_parent [R(w_k) | j_k - j_parent], skin_k = G_k [I | -j_k].
    Returns [J, 12] float64 (3x4 row-major)."""
    G = np.zeros((N_JOINTS, 4, 4))
    root = np.eye(4)
    root[:3, :3] = root_R
    root[:3, 3] = root_t
    for k in range(N_JOINTS):
        L = np.eye(4)
        L[:3, :3] = rodrigues(pose[k])
        p = PARENTS[k]
        L[:3, 3] = REST[k] - (REST[p] if p >= 0 else 0.0)
        G[k] = (root if p < 0 else G[p]) @ L
    out = np.zeros((N_JOINTS, 12))
    for k in range(N_JOINTS):
        inv_rest = np.eye(4)
        inv_rest[:3, 3] = -REST[k]
        out[k] = (G[k] @ inv_rest)[:3, :].reshape(12)
    return out


def avatar_pose(rng, sigma=0.3):
    """Per-joint axis-angle ~ N(0, sigma^2 I3); root at a random floor
    position in the room with a random yaw."""
    pose = rng.normal(0.0, sigma, (N_JOINTS, 3))
    yaw = rng.uniform(0.0, 2 * math.pi)
    Rz = np.array([[math.cos(yaw), -math.sin(yaw), 0.0], [math.sin(yaw), math.cos(yaw), 0.0], [0.0, 0.0, 1.0]])
    pos = np.array([rng.uniform(1.0, ROOM[0] - 1.0), rng.uniform(1.0, ROOM[1] - 1.0), 0.0])
    return pose, Rz, pos


def avatar_clips(rng, frames, fps=30.0, speed=1.2):
    """Per-frame skinning matrices of walking avatars, standing in for the
    offline GAMMA -> forward-kinematics clips (Sec. 3.3): avatar a has
    frames[a] frames; its root walks in a straight line at `speed` m/s from a
    random floor position with a random yaw, and its joint angles swing
    sinusoidally (amplitude ~0.3 rad, random phase per joint, 1 Hz).
    Returns (clip [sum(frames), 24, 12] float32, first int32 [A],
    frames int32 [A])."""
    mats, first = [], []
    for F in frames:
        pose0, Rz, pos = avatar_pose(rng)
        amp = rng.normal(0.0, 0.3, (N_JOINTS, 3))
        phase = rng.uniform(0.0, 2 * math.pi, (N_JOINTS, 1))
        heading = Rz @ np.array([1.0, 0.0, 0.0])
        first.append(sum(len(m) for m in mats))
        clip = []
        for f in range(F):
            t = f / fps
            pose = 0.3 * pose0 + amp * np.sin(2 * math.pi * t + phase)
            clip.append(skinning_matrices(pose, Rz, pos + speed * t * heading))
        mats.append(np.stack(clip))
    return (np.concatenate(mats).astype(np.float32), np.array(first, np.int32),
            np.array(list(frames), np.int32))


def capsule_clips(clip):
    """Per-frame proxy capsules of the bones of the synthetic skeleton
    (Sec. 3.3: capsules derived from the skeletal bones, world positions
    pre-computed per frame), from the skinning matrices of avatar_clips:
    one capsule per non-root joint k, from the posed parent joint to the posed
    joint k, radius 0.05 m + 0.1 x its rest length.  The posed position of
    joint k is skin_k [rest_k, 1].  Returns [frames, 23, 8] float32 rows
    (a.xyz, r, b.xyz, 0)."""
    clip = np.asarray(clip, np.float64).reshape(len(clip), N_JOINTS, 3, 4)
    joints = np.einsum("fkij,kj->fki", clip[..., :3], REST) + clip[..., 3]
    kids = [k for k in range(N_JOINTS) if PARENTS[k] >= 0]
    out = np.zeros((len(clip), len(kids), 8))
    for c, k in enumerate(kids):
        p = PARENTS[k]
        out[:, c, 0:3] = joints[:, p]
        out[:, c, 3] = 0.05 + 0.1 * np.linalg.norm(REST[k] - REST[p])
        out[:, c, 4:7] = joints[:, k]
    return out.astype(np.float32)


def agents_near_avatars(rng, caps_now, n_agents, height=1.5, step=0.25):
    """Agents standing on the floor around the avatars (positions within
    1.5 m of a random avatar's pelvis capsule), each with a candidate forward
    step of `step` m in a random heading; a quarter of them placed right
    against a capsule.  caps_now: [A, n_caps, 8] capsules at the current time.
    Returns (pos [E, 3], next [E, 3]) float32."""
    A = len(caps_now)
    pos = np.zeros((n_agents, 3))
    for e in range(n_agents):
        a = rng.integers(0, A)
        base = caps_now[a, 0, 0:3].astype(np.float64)
        if rng.random() < 0.25:
            c = caps_now[a, rng.integers(0, caps_now.shape[1])].astype(np.float64)
            pos[e, :2] = (c[0:2] + c[4:6]) / 2 + rng.normal(0.0, 0.1, 2)
        else:
            pos[e, :2] = base[:2] + rng.uniform(-1.5, 1.5, 2)
    heading = rng.uniform(0.0, 2 * math.pi, n_agents)
    nxt = pos + step * np.stack([np.cos(heading), np.sin(heading), np.zeros(n_agents)], 1)
    return pos.astype(np.float32), nxt.astype(np.float32)


# --------------------------------------------------------------------------
# projected-record stand-ins (inputs of the binning and compositing calls)
# --------------------------------------------------------------------------
def synthetic_records(rng, counts, W, H, tie_frac=0.05, vis_frac=0.9, r_median=8.0, aniso_sigma=0.7):
    """FP32 projected records [m,12] (u, v, depth, radius-bits, A, B, C,
    opacity, r, g, b, view-bits) for views with `counts[v]` instances each,
    plus a visibility mask.  u, v uniform over the image plus a margin;
    integer radius log-normal around r_median; the conic is the inverse of a
    random 2D covariance of comparable extent (drawn independently of the
    radius: these are inputs, not projections); depth U[0.3, 10] with a
    fraction of exact depth ties to exercise the index tie-break."""
    m = int(np.sum(counts))
    view = np.repeat(np.arange(len(counts)), counts)
    r = np.maximum(1, np.round(np.exp(rng.normal(math.log(r_median), 0.8, m)))).astype(np.int32)
    u = rng.uniform(-40.0, W + 40.0, m)
    v = rng.uniform(-40.0, H + 40.0, m)
    z = rng.uniform(0.3, 10.0, m)
    tie = rng.uniform(0.0, 1.0, m) < tie_frac
    src = rng.integers(0, m, m)
    z[tie] = z[src[tie]]
    s1 = np.exp(rng.normal(math.log(r_median / 3.0), 0.5, m))
    s2 = s1 * np.exp(-np.abs(rng.normal(0.0, aniso_sigma, m)))
    th = rng.uniform(0.0, math.pi, m)
    c, s = np.cos(th), np.sin(th)
    a = c * c * s1 * s1 + s * s * s2 * s2 + 0.3
    b = c * s * (s1 * s1 - s2 * s2)
    cc = s * s * s1 * s1 + c * c * s2 * s2 + 0.3
    det = a * cc - b * b
    rec = np.zeros((m, 12), np.float32)
    rec[:, 0] = u
    rec[:, 1] = v
    rec[:, 2] = z
    rec[:, 3] = r.view(np.float32)
    rec[:, 4] = cc / det
    rec[:, 5] = -b / det
    rec[:, 6] = a / det
    rec[:, 7] = _sigmoid(rng.standard_normal(m))
    rec[:, 8:11] = rng.uniform(0.0, 1.0, (m, 3))
    rec[:, 11] = view.astype(np.int32).view(np.float32)
    visible = (rng.uniform(0.0, 1.0, m) < vis_frac).astype(np.uint8)
    return rec, visible


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
def sensor_inputs(seed, n_views, H, W, mesh=True):
    """Compositing-output and mesh-pass stand-ins for the sensor hand-off:
    rgb in [-0.1, 1.1] with a few special values (NaN, +-inf, exact k/255
    steps), alpha 0 on 20% of the pixels and 1 on 10%, accumulated depth
    alpha * U[0.3, 10], mesh depth U[0.3, 10] with 15% zeros, 3% negatives
    and 2% NaN, and on 5% of the pixels (those with alpha 1) a mesh depth equal
    to the accumulated depth (exact ties).  Returns a dict of float32 / uint8
    arrays [V, H, W(, C)]."""
    rng = np.random.default_rng(seed)
    shp = (n_views, H, W)
    rgb = rng.uniform(-0.1, 1.1, shp + (3,))
    u = rng.random(shp + (3,))
    rgb[u < 0.02] = np.round(rgb[u < 0.02] * 255.0) / 255.0
    rgb = rgb.astype(np.float32)
    flat = rgb.reshape(-1)
    sp = rng.integers(0, flat.size, max(4, flat.size // 500))
    flat[sp] = np.array([np.nan, np.inf, -np.inf, 0.5], np.float32)[np.arange(sp.size) % 4]
    a = rng.random(shp)
    alpha = np.where(a < 0.2, 0.0, np.where(a < 0.3, 1.0, rng.uniform(1e-4, 1.0, shp))).astype(np.float32)
    depth = (alpha.astype(np.float64) * rng.uniform(0.3, 10.0, shp)).astype(np.float32)
    out = {"rgb": rgb, "depth": depth, "alpha": alpha}
    if mesh:
        m = rng.random(shp)
        md = rng.uniform(0.3, 10.0, shp)
        md[m < 0.15] = 0.0
        md[(m >= 0.15) & (m < 0.18)] = -1.0
        md[(m >= 0.18) & (m < 0.20)] = np.nan
        md = md.astype(np.float32)
        tie = (alpha == 1.0) & (rng.random(shp) < 0.5)
        md[tie] = depth[tie]
        out["mesh_depth"] = md
        out["mesh_rgba"] = rng.integers(0, 256, shp + (4,), dtype=np.uint8)
    return out


def config(idx, scale=1.0):
    """Inputs of workload `idx` (0..4).  `scale` < 1 shrinks Gaussian counts
    (for the oracle-sized parity cases); resolutions and structure are kept.

    Returns dict: segments (list of gaussian dicts), cams [V,16] float32,
    view_segs (list of segment-index lists per view), W, H, plus avatar assets
    for workload 4."""
    sc = lambda n: max(1, int(round(n * scale)))
    if idx == 0:
        (r,) = _rngs(0, 1)
        g = gaussians_cube(sc(10_000), r, sh_degree=0)
        cams = identity_camera(128.0, 128.0, 64.0, 64.0)[None]
        return {"segments": [g], "cams": cams, "view_segs": [[0]], "W": 128, "H": 128, "name": "cube10k_128"}
    if idx == 1:
        rs = _rngs(1, 2)
        g = gaussians_room(sc(1_000_000), rs[0], sh_degree=3)
        cams = camera_room(rs[1], 640, 480)[None]
        return {"segments": [g], "cams": cams, "view_segs": [[0]], "W": 640, "H": 480, "name": "room1M_640x480_sh3"}
    if idx == 2:
        rs = _rngs(2, 3)
        g = gaussians_room(sc(500_000), rs[0], sh_degree=3)
        cams = camera_room(rs[1], 256, 256, fx=128.0)[None]
        return {"segments": [g], "cams": cams, "view_segs": [[0]], "W": 256, "H": 256, "perturb_rng": rs[2],
                "name": "room500k_256_fwdbwd"}
    if idx == 3:
        rs = _rngs(3, 8 + 64 + 1)
        sizes = [int(round(math.exp(rs[0].uniform(math.log(1e5), math.log(2e6))))) for _ in range(8)]
        segs = [gaussians_room(sc(sizes[s]), rs[1 + s], sh_degree=3) for s in range(8)]
        cams = np.stack([camera_room(rs[9 + v], 256, 256, fx=128.0) for v in range(64)])
        return {"segments": segs, "cams": cams, "view_segs": [[v % 8] for v in range(64)], "W": 256, "H": 256,
                "name": "batched64x256_8scenes"}
    if idx == 4:
        rs = _rngs(4, 2 + 8 + 16)
        room = gaussians_room(sc(1_000_000), rs[0], sh_degree=3)
        avs = [avatar_canonical(sc(50_000), rs[2 + a], sh_degree=3) for a in range(8)]
        poses = [avatar_pose(rs[2 + a]) for a in range(8)]
        skin = np.stack([skinning_matrices(*p) for p in poses]).astype(np.float32)
        cat = lambda k: np.concatenate([a[k] for a in avs])
        av = {"means": cat("means"), "log_scales": cat("log_scales"), "quats": cat("quats"),
              "opacity": cat("opacity"), "sh": cat("sh"), "sh_degree": 3, "joint_idx": cat("joint_idx"),
              "weights": cat("weights"),
              "avatar_of": np.repeat(np.arange(8), [len(a["means"]) for a in avs]).astype(np.int32)}
        cams = np.stack([camera_room(rs[10 + v], 640, 480) for v in range(16)])
        return {"segments": [room], "avatars": av, "skin": skin, "cams": cams, "view_segs": [[0, 1]] * 16,
                "W": 640, "H": 480, "name": "room1M_8avatars_16x640x480"}
    raise ValueError(idx)


def perturb(g, rng, sigma=0.01):
    """N(0, sigma) on every field: means, log-scales, quaternions (then
    renormalised), opacity logit, SH (the fwd+bwd target parameters)."""
    f = lambda x: np.ascontiguousarray(x, dtype=np.float32)
    n = len(g["means"])
    q = g["quats"].astype(np.float64) + rng.normal(0, sigma, (n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    o = g["opacity"].astype(np.float64)
    logit = np.log(o / (1 - o)) + rng.normal(0, sigma, n)
    return {"means": f(g["means"] + rng.normal(0, sigma, (n, 3))),
            "log_scales": f(g["log_scales"] + rng.normal(0, sigma, (n, 3))),
            "quats": f(q), "opacity": f(_sigmoid(logit)), "sh": f(g["sh"] + rng.normal(0, sigma, g["sh"].shape)),
            "sh_degree": g["sh_degree"]}
