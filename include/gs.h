/*
 * gs.h -- C ABI of the MI355X (gfx950) tile-based 3D Gaussian Splatting
 * sensor renderer: the rendering and avatar-deformation hot path of
 * Habitat-GS (arXiv 2604.12626).
 *
 * The paper renders scenes stored as explicit anisotropic 3D Gaussians with
 * tile-based rasterization (Sec. 2.2, Sec. 3.2), deforms canonical avatar
 * Gaussians to the current pose with linear blend skinning every frame
 * (Sec. 3.1, Sec. 3.3) and rasterizes all avatars in one pass together with
 * the scene, producing colour and depth (Sec. 3.2).  The five calls below are
 * that path:
 *
 *   gs_deform_lbs       canonical avatar Gaussians -> posed means + covariances
 *   gs_project          EWA projection, SH colour, tile rect per (view, Gaussian)
 *   gs_bin_sort         tile binning: scan, (tile, depth) key emission, onesweep
 *                       LSD radix sort, per-tile ranges
 *   gs_composite        per-tile front-to-back alpha compositing -> RGB, depth, alpha
 *                       (gs_composite_noalloc: the same with library-owned scratch)
 *   gs_render_backward  gradients of an image loss w.r.t. the Gaussian parameters
 *
 * Around it, the pieces the paper puts directly before and after the path:
 *
 *   gs_deform_lbs_clip  the same skinning with each avatar's joint matrices
 *                       interpolated in its clip at the current time (Sec. 3.3)
 *   gs_deform_lbs_backward_joints
 *                       gradients w.r.t. the joint matrices (pose fitting)
 *   gs_forward_kinematics  joint rotations -> joint (skinning) matrices
 *   gs_sensor_compose   8-bit RGBA + metric depth observation, nearer-fragment
 *                       select against a mesh pass (Sec. 3.2, Sec. 3.4)
 *   gs_capsule_queries  clearance to the nearest avatar capsule and blocked
 *                       steps for a batch of agents (Sec. 3.3, Sec. 3.4)
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Memory.  Every array argument is a DEVICE pointer owned by the caller,
 *    unless the comment says "host".  The library never allocates or frees
 *    device memory; scratch space is a caller-provided workspace whose size
 *    the *_workspace_bytes() helpers report.  The one exception is
 *    gs_composite_noalloc, whose workspace is a static device array of
 *    GS_NOALLOC_SCRATCH_BYTES per GPU (loaded with the code object, held until
 *    the process ends) for callers that cannot allocate.
 *  - Asynchrony.  Each call validates its arguments on the host, then only
 *    enqueues kernels on `stream` (a hipStream_t; NULL is the default
 *    stream) and returns.  Results are ready when the stream reaches them.
 *  - Errors.  A call returns GS_OK or an error status.  Invalid arguments
 *    return before anything is enqueued.  A failed launch returns GS_ERR_HIP.
 *    gs_last_error() gives a thread-local message for the last failure.  No
 *    C++ exception crosses this boundary.  Data-dependent overflow (more tile
 *    instances than the key buffers hold) is reported on the device (see
 *    gs_bin_sort) so that no call needs a host synchronisation.
 *  - Layouts.  Row-major, one row per Gaussian: means [n][3],
 *    log_scales [n][3], quats [n][4] as (w, x, y, z), opacity [n] (activated,
 *    in (0,1)), sh [n][(D+1)^2][3] (real SH, Condon-Shortley phase, l-major,
 *    m = -l..l), cov6 [n][6] as (xx, xy, xz, yy, yz, zz).  gs_project
 *    also takes a segment in planes (layout GS_LAYOUT_PLANES), component-
 *    major: means [3][n], log_scales [3][n], quats [4][n], cov6 [6][n],
 *    opacity [n], sh [3 (D+1)^2][n] (plane 3 k + channel); gs_render_backward
 *    returns GS_ERR_UNSUPPORTED for such a segment.  Images are
 *    [view][y][x] with RGB interleaved: rgb [V][H][W][3], depth [V][H][W],
 *    alpha [V][H][W].  Dtypes are FP32 except where noted.
 *  - Instances.  One call renders V views.  Each view draws a set of
 *    gaussian segments (bit s of view_seg_mask[v] set = segment s drawn;
 *    a scene and the posed avatars are two segments of one view, Sec. 3.2).
 *    Instance g = base[v] + offset of segment s within view v + i numbers the
 *    pair (view v, Gaussian i of segment s), with segments in ascending index
 *    order inside a view and base[v] = sum of the previous views' counts; see
 *    gs_instance_offsets().
 */
#ifndef GS_H_
#define GS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* A hipStream_t, passed as an opaque handle (NULL = default stream). */
typedef void *gs_stream_t;

typedef enum gs_status {
    GS_OK = 0,
    GS_ERR_INVALID_ARGUMENT = 1,   /* a pointer, size or parameter is invalid */
    GS_ERR_UNSUPPORTED = 2,        /* valid but outside this library's limits */
    GS_ERR_WORKSPACE_TOO_SMALL = 3,
    GS_ERR_HIP = 4                 /* a HIP runtime call or launch failed */
} gs_status;

#define GS_TILE 16            /* tile edge in pixels (part of the image definition) */
#define GS_REC_FLOATS 12      /* projected record: 3 x float4, see gs_projected */
#define GS_MAX_SEGMENTS 32    /* bits of view_seg_mask */
#define GS_MAX_VIEWS 4096
#define GS_MAX_SH_DEGREE 3
#define GS_MAX_CAPACITY ((1LL << 30) - 1) /* tile-instance limit of one gs_bin_sort call */
#define GS_SEGMENT 64         /* list entries per segment of the segmented backward */
/* gs_composite_noalloc: most (view, tile) items per call, and the bytes of
 * its library-owned scratch on each GPU (2048 B of queue counters + a work
 * order of 8 x GS_NOALLOC_MAX_ITEMS / 8 words) */
#define GS_NOALLOC_MAX_ITEMS 65536
#define GS_NOALLOC_SCRATCH_BYTES (2048 + 4 * GS_NOALLOC_MAX_ITEMS)

/* Pinhole camera, world -> camera with OpenCV axes (x right, y down, z
 * forward): p_cam = R p_world + t, R row-major.  Pixel (x, y) samples the
 * image-plane point (x + 1/2, y + 1/2); u = fx X/Z + cx, v = fy Y/Z + cy.
 * 64 bytes; the cameras of a call live in a device array of n_views. */
typedef struct gs_camera {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
} gs_camera;

/* Rendering constants (host struct, by pointer).  Defaults in brackets are
 * those of the 3DGS lineage the paper cites; gs_default_params() fills them. */
typedef struct gs_params {
    int32_t width, height; /* image size shared by all views of a call */
    float near_plane;      /* cull if !(z_cam > near_plane)        [0.2] */
    float lowpass;         /* added to the 2D covariance diagonal  [0.3] */
    float sigma_cut;       /* radius = ceil(sigma_cut sqrt(lambda_max)) [3] */
    float fov_clamp;       /* Jacobian tangent clamp, x half-FOV   [1.3] */
    float alpha_max;       /* alpha = min(alpha_max, o G)          [0.99] */
    float alpha_min;       /* skip the entry if alpha < alpha_min  [1/255] */
    float t_min;           /* stop before T(1-alpha) < t_min       [1e-4] */
    float bg[3];           /* background colour, added as T_final bg [0] */
} gs_params;

/* One gaussian segment (device pointers).  If cov6 is non-NULL it gives the
 * 3D covariance directly (posed avatars) and log_scales/quats are ignored.
 * layout: GS_LAYOUT_ROWS (0, one row per Gaussian) or GS_LAYOUT_PLANES (1,
 * one plane per component; gs_project only), see Layouts above; any other
 * value is GS_ERR_INVALID_ARGUMENT. */
#define GS_LAYOUT_ROWS 0
#define GS_LAYOUT_PLANES 1
typedef struct gs_gaussians {
    int64_t n;
    int32_t sh_degree; /* 0..3 */
    int32_t layout;
    const float *means, *log_scales, *quats, *cov6, *opacity, *sh;
} gs_gaussians;

/* Gradients of one segment, same layouts as gs_gaussians (device pointers).
 * cov6 is written when the segment was given by cov6, log_scales and quats
 * otherwise; the unused ones may be NULL. */
typedef struct gs_gaussians_grad {
    float *means, *log_scales, *quats, *cov6, *opacity, *sh;
} gs_gaussians_grad;

/* Projected instances (device arrays of n_instances).
 *  tiles_touched[g]: number of tiles of g's rect; 0 = culled (16-byte aligned).
 *  rec[g] (12 floats, 16-byte aligned, written only when g is visible):
 *    [0] u  [1] v  [2] camera-space depth z  [3] radius (int32 bits)
 *    [4] A  [5] B  [6] C   (conic = inverse 2D covariance [[A,B],[B,C]])
 *    [7] opacity  [8..10] rgb  [11] view (int32 bits) */
typedef struct gs_projected {
    int64_t n_instances;
    uint32_t *tiles_touched;
    float *rec;
} gs_projected;

/* ---------------------------------------------------------------------- */
/* helpers                                                                 */
/* ---------------------------------------------------------------------- */
const char *gs_status_string(gs_status s);
const char *gs_last_error(void); /* thread-local; "" if none */
/* ABI version: 2 adds the sensor hand-off, the capsule queries, the clip,
 * joint-gradient and forward-kinematics skinning calls. */
int32_t gs_version(void);
void gs_default_params(gs_params *p, int32_t width, int32_t height);

/* Launch configuration (host-side, process-wide; it changes scheduling only,
 * never a result).
 *  composite_groups_per_cu: persistent 4-wave groups per compute unit in
 *    gs_composite (1..32, default 3); each wave of the grid pops (view, tile,
 *    quadrant) work items until none is left.
 *  sort_partition_keys: keys per onesweep partition in gs_bin_sort (4096 or
 *    8192, default 4096).
 *  sort_lookback: predecessor partitions read per round trip of the onesweep
 *    look-back (16, 32 or 64, default 16).
 *  sort_algorithm: 0 (default) sorts by tile buckets (count per tile,
 *    scatter into buckets, sort each bucket by (depth, instance) in LDS)
 *    when every view has at most 4096 tiles and the launch at most 2^18
 *    tiles over all views (beyond 4096 in all, the counts are taken in a
 *    sliding window of whole views), and with the onesweep radix sort
 *    otherwise; 1 always uses the onesweep radix sort.  Both give the same
 *    keys, values, ranges and work order.
 *  composite_pairs: 0 (default) lets gs_composite walk each quadrant's list
 *    with a pair of waves (one evaluates the alphas of a chunk while the
 *    other accumulates the previous chunk) when the launch has at most
 *    16 x (compute units) quadrant items, and with one wave otherwise; 1
 *    always uses one wave, 2 always a pair.  The images are bit-identical.
 * gs_set_tuning(NULL) restores the defaults; invalid values return
 * GS_ERR_INVALID_ARGUMENT and change nothing.  Meant for an autotuner that
 * times the candidates on the target workload.
 * The settings are process-wide: one set shared by every caller, stream and
 * device of the process (atomic, so reading and writing never tear).  A call
 * reads them when it enqueues its launches, so a change affects only later
 * calls, and a captured HIP graph keeps the launch shapes of its capture.
 * Renderers that want different settings must take turns (set, enqueue,
 * restore); results never depend on them. */
typedef struct gs_tuning {
    int32_t composite_groups_per_cu;
    int32_t sort_partition_keys;
    int32_t sort_lookback;
    int32_t sort_algorithm;
    int32_t composite_pairs;
    int32_t reserved[3];
} gs_tuning;
gs_status gs_set_tuning(const gs_tuning *t);
void gs_get_tuning(gs_tuning *t);

/* Host helper: offsets[v] = first instance of view v, offsets[n_views] =
 * total (host arrays; offsets has n_views + 1 entries). */
gs_status gs_instance_offsets(const gs_gaussians *segs, int32_t n_segs, int32_t n_views,
                              const uint32_t *view_seg_mask, int64_t *offsets);

/* ---------------------------------------------------------------------- */
/* avatars: linear blend skinning (Sec. 3.3)                               */
/* ---------------------------------------------------------------------- */
/* For each canonical avatar Gaussian i: A_i = sum_k weights[i][k] *
 * skin_mats[avatar_of[i]][joint_idx[i][k]] (a blend of 3x4 joint matrices,
 * k < 4; the weights are used as given), then
 *   means_out[i] = A3 means_c[i] + a,   cov6_out[i] = A3 Sigma A3^T,
 * Sigma = R(q) diag(exp(2 s)) R(q)^T from log_scales_c / quats_c.
 *  joint_idx uint8 [n][4], weights [n][4], avatar_of int32 [n],
 *  skin_mats [n_avatars][n_joints][12] (row-major 3x4), n_joints <= 255.
 * Outputs [n][3] and [n][6] feed gs_project as a cov6 segment.  The joint
 * matrices are read from device memory at run time, so a captured graph
 * replays with new poses.  Errors: GS_ERR_INVALID_ARGUMENT for NULL arrays
 * with n > 0 or non-positive joint/avatar counts. */
gs_status gs_deform_lbs(int64_t n, const float *means_c, const float *log_scales_c, const float *quats_c,
                        const uint8_t *joint_idx, const float *weights, const int32_t *avatar_of,
                        const float *skin_mats, int32_t n_avatars, int32_t n_joints, float *means_out,
                        float *cov6_out, gs_stream_t stream);

/* Adjoint of gs_deform_lbs w.r.t. the canonical means, log-scales and
 * quaternions, given d_means_out [n][3] and d_cov6_out [n][6] (for example
 * the cov6 gradients gs_render_backward writes).  Outputs are overwritten.
 * Joint matrices and weights are held fixed. */
gs_status gs_deform_lbs_backward(int64_t n, const float *means_c, const float *log_scales_c,
                                 const float *quats_c, const uint8_t *joint_idx, const float *weights,
                                 const int32_t *avatar_of, const float *skin_mats, int32_t n_avatars,
                                 int32_t n_joints, const float *d_means_out, const float *d_cov6_out,
                                 float *d_means_c, float *d_log_scales_c, float *d_quats_c, gs_stream_t stream);

/* Adjoint of gs_deform_lbs w.r.t. the joint matrices: d_skin_mats
 * [n_avatars][n_joints][12] (overwritten) = sum over the Gaussians of each
 * avatar of w_k dL/dA for the joints they blend, with dL/dA[:, :3] =
 * g mean^T + 2 G A3 Sigma and dL/dA[:, 3] = g (g = d_means_out, G the
 * symmetric adjoint of the posed covariance from d_cov6_out).  For fitting
 * poses through the renderer; the paper prepares the matrices offline.
 * Summed with float atomics (per-workgroup partial sums first when all
 * matrices fit in 16 KB), so the order of the additions, and the last bits,
 * vary from run to run.  Arguments and errors as gs_deform_lbs_backward;
 * n == 0 clears d_skin_mats. */
gs_status gs_deform_lbs_backward_joints(int64_t n, const float *means_c, const float *log_scales_c,
                                        const float *quats_c, const uint8_t *joint_idx, const float *weights,
                                        const int32_t *avatar_of, const float *skin_mats, int32_t n_avatars,
                                        int32_t n_joints, const float *d_means_out, const float *d_cov6_out,
                                        float *d_skin_mats, gs_stream_t stream);

/* Skinning matrices of posed skeletons: the forward-kinematics step that
 * turns per-joint rotations into the joint matrices gs_deform_lbs consumes
 * (the paper runs it offline on the GAMMA poses, Sec. 3.3; here it can run
 * per frame on the device).  Joint k's world transform is its parent's (the
 * root transform for a root) times [R(pose_k) | rest_k - rest_parent]
 * (rest_k for a root); its skinning matrix is that times [I | -rest_k].
 *  parents  HOST int32 [n_joints]: -1 for a root, else a joint < k
 *  rest     [n_joints][3] rest-pose joint positions
 *  pose     [n_avatars][n_joints][3] axis-angle rotations
 *  root     [n_avatars][12] root transforms (row-major 3x4)
 *  skin_out [n_avatars][n_joints][12], overwritten.
 * One thread per avatar.  Errors: GS_ERR_INVALID_ARGUMENT for n_joints
 * outside 1..256, parents not before their children, NULL arrays. */
gs_status gs_forward_kinematics(int32_t n_avatars, int32_t n_joints, const int32_t *parents, const float *rest,
                                const float *pose, const float *root, float *skin_out, gs_stream_t stream);

/* The same deformation with each avatar's joint matrices taken at its
 * current time (Sec. 3.3, GAMMA trajectory: per-frame joint matrices
 * prepared offline by forward kinematics are interpolated at the current
 * simulation time before skinning).  The interpolation is linear in the
 * matrices, fused into the blend: with p = frame_pos[a] clamped to
 * [0, clip_frames[a] - 1] (NaN -> 0), f = floor(p) (at most
 * clip_frames[a] - 2) and s = p - f, joint j of avatar a uses
 * (1 - s) M_j[clip_first[a] + f] + s M_j[clip_first[a] + f + 1]; a clip of
 * one frame holds that pose.
 *  clip_mats [clip_total_frames][n_joints][12] (row-major 3x4, 16-byte
 *  aligned): the frames of all avatars' clips; clip_first, clip_frames
 *  int32 [n_avatars] and frame_pos [n_avatars] are device arrays (read at
 *  run time, so a captured graph replays with new times); clip_first is
 *  clamped to [0, clip_total_frames - 1] and clip_frames to [1, the frames
 *  left from there].  Other arguments and errors as gs_deform_lbs. */
gs_status gs_deform_lbs_clip(int64_t n, const float *means_c, const float *log_scales_c, const float *quats_c,
                             const uint8_t *joint_idx, const float *weights, const int32_t *avatar_of,
                             const float *clip_mats, int32_t clip_total_frames, const int32_t *clip_first,
                             const int32_t *clip_frames, const float *frame_pos, int32_t n_avatars,
                             int32_t n_joints, float *means_out, float *cov6_out, gs_stream_t stream);

/* Adjoint of gs_deform_lbs_clip w.r.t. the canonical means, log-scales and
 * quaternions (clip and times held fixed); arguments as
 * gs_deform_lbs_backward with the clip arguments of gs_deform_lbs_clip. */
gs_status gs_deform_lbs_clip_backward(int64_t n, const float *means_c, const float *log_scales_c,
                                      const float *quats_c, const uint8_t *joint_idx, const float *weights,
                                      const int32_t *avatar_of, const float *clip_mats, int32_t clip_total_frames,
                                      const int32_t *clip_first, const int32_t *clip_frames,
                                      const float *frame_pos, int32_t n_avatars, int32_t n_joints,
                                      const float *d_means_out, const float *d_cov6_out, float *d_means_c,
                                      float *d_log_scales_c, float *d_quats_c, gs_stream_t stream);

/* ---------------------------------------------------------------------- */
/* rasterizer (Sec. 2.2, Sec. 3.2)                                         */
/* ---------------------------------------------------------------------- */
/* Projection of every (view, Gaussian) instance: camera-space mean, cull if
 * !(z > near_plane); EWA 2D covariance J W Sigma W^T J^T + lowpass I with the
 * tangent-clamped Jacobian; conic; radius ceil(sigma_cut sqrt(lambda_max))
 * (0.1 floor under the eigenvalue root); rect of the tiles meeting the
 * square [u-r, u+r] x [v-r, v+r]; SH colour max(0, sum Y_lm(d) k_lm + 1/2)
 * with d the world-space direction from the camera centre.  Reads each
 * Gaussian's attributes once for all views that draw its segment.
 *  segs: host array of n_segs (<= GS_MAX_SEGMENTS) segment descriptors.
 *  cams: device array of n_views gs_camera.
 *  view_seg_mask: host array of n_views masks.
 *  out: n_instances must equal the total of gs_instance_offsets(); writes
 *       tiles_touched for every instance and rec for visible ones.
 * Errors: GS_ERR_INVALID_ARGUMENT (NULL/size mismatch, sh_degree > 3,
 * width/height <= 0, empty mask bits beyond n_segs), GS_ERR_UNSUPPORTED
 * (more than 2^32 - 1 instances). */
gs_status gs_project(const gs_gaussians *segs, int32_t n_segs, const gs_camera *cams, int32_t n_views,
                     const uint32_t *view_seg_mask, const gs_params *p, gs_projected *out, gs_stream_t stream);

/* Workspace bytes gs_bin_sort needs for n_instances projected instances,
 * `capacity` key slots and n_views views of p->width x p->height. */
size_t gs_bin_sort_workspace(int64_t n_instances, int64_t capacity, int32_t n_views, const gs_params *p);

/* Words of a tile work order (see gs_bin_sort) for n_views views of the
 * image size in p: 8 * ceil(n_views * T / 8) (0 for a NULL or invalid p or
 * n_views < 1). */
size_t gs_tile_order_words(int32_t n_views, const gs_params *p);

/* Tile binning of the projected instances.  Every visible instance g emits
 * one key per tile of its rect: key = ((view * T + tile) << 32) | bits(fp32
 * z), value = g (T = tiles per view; z > 0 so the bits order like z).  The
 * result is the (key, value) pairs in the order a stable sort by key of the
 * keys emitted in ascending instance order gives (ties in depth keep
 * ascending instance order), computed either by bucketing the keys by tile
 * and sorting each bucket (launches with up to 4096 tiles over all views,
 * unless gs_tuning selects the other path) or by a stable LSD radix sort
 * over the significant key bits (one hand-written onesweep pass per 8-bit
 * digit); both give identical output.
 *  keys uint64 [capacity], vals uint32 [capacity]: sorted output.
 *  tile_ranges uint32 [n_views * T][2]: [first, last + 1) of each (view,
 *  tile) run, (0, 0) if empty.
 *  tile_order uint32 [gs_tile_order_words()] or NULL: the work order
 *  gs_composite pops tiles in -- queue q = item mod 8 lists its (view, tile)
 *  items (item = view * T + tile) from word q * ceil(n_views * T / 8) on, by
 *  descending list length in chunks of 64 entries.  Always a permutation of
 *  the items, also after an overflow.
 *  d_num_instances (int64, device): K, the number of keys.  d_overflow
 *  (int32, device): set to 1 when K > capacity (then keys, values and the
 *  ranges' contents are invalid and every range is (0, 0)), else 0.  The
 *  caller re-runs with a larger capacity; nothing here synchronises with the
 *  host.
 * Errors: GS_ERR_INVALID_ARGUMENT, GS_ERR_WORKSPACE_TOO_SMALL,
 * GS_ERR_UNSUPPORTED (capacity > GS_MAX_CAPACITY, n_views * T > 2^31). */
gs_status gs_bin_sort(const gs_projected *proj, int32_t n_views, const gs_params *p, void *ws, size_t ws_bytes,
                      uint64_t *keys, uint32_t *vals, int64_t capacity, uint32_t *tile_ranges, uint32_t *tile_order,
                      int64_t *d_num_instances, int32_t *d_overflow, gs_stream_t stream);

/* Workspace bytes gs_composite needs for n_views views of the image size in
 * p (0 for a NULL or invalid p or n_views < 1): the persistent tile queues'
 * counters (the first 2048 bytes), then room for a tile work order (used
 * when the call gets none).  The counters must be zero-filled before the
 * workspace's first use; every call leaves them zero-filled again, so one
 * zeroing at allocation serves all later calls (calls sharing a workspace
 * must not overlap). */
size_t gs_composite_workspace(int32_t n_views, const gs_params *p);

/* Per-tile front-to-back compositing.  For each pixel p = (x + 1/2, y + 1/2)
 * and each entry i of its tile's sorted list: G = exp(-1/2 d^T Q d) with
 * d = p - (u, v); alpha = min(alpha_max, o G); skip if alpha < alpha_min;
 * stop (without compositing i) if T (1 - alpha) < t_min; else C += c alpha T,
 * D += z alpha T, T *= 1 - alpha.  Outputs rgb = C + T bg, depth = D (z-depth
 * accumulated, un-normalised), alpha = 1 - T; optional t_final = T and
 * n_contrib = 1 + list position of the last composited entry (the state the
 * backward pass starts from; pass NULL to skip them).
 * The tiles are processed by a persistent grid that pops (view, tile,
 * quadrant) work items from counters in `ws` (zero on entry, zero again when
 * the call completes) in the order of tile_order: the one gs_bin_sort wrote
 * for the same ranges, or NULL to have it computed here into `ws` (one more
 * small launch).  The order only affects timing, never a result.
 *  ckpt (optional, ckpt_floats floats; NULL to skip): the state of every
 *  pixel at each position b = m GS_SEGMENT (m >= 1) inside a tile list that
 *  its compositing walk crosses, for gs_render_backward: transmittance T_b in
 *  front of entry b, then the colour (3) and depth still to come from
 *  entries b.. (background included) divided by T_b.  Layout: slot (list
 *  start + b) / GS_SEGMENT, 8 x 8 quadrant (0..3, row-major in the tile),
 *  value (5), pixel of the quadrant (64, row-major).  Size it with
 *  gs_checkpoint_floats(capacity of the binning); writes past ckpt_floats
 *  are dropped.
 * Errors: GS_ERR_INVALID_ARGUMENT, GS_ERR_WORKSPACE_TOO_SMALL. */
gs_status gs_composite(const gs_projected *proj, const uint32_t *vals, const uint32_t *tile_ranges,
                       const uint32_t *tile_order, int32_t n_views, const gs_params *p, void *ws, size_t ws_bytes,
                       float *rgb, float *depth, float *alpha, float *t_final, uint32_t *n_contrib, float *ckpt,
                       size_t ckpt_floats, gs_stream_t stream);

/* gs_composite for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, results and errors as gs_composite, without the workspace:
 * the queue counters and (when tile_order is NULL) the work order live in a
 * library-owned device array of GS_NOALLOC_SCRATCH_BYTES on each GPU, held
 * until the process ends.  The call allocates nothing: it clears the
 * counters with a fill kernel on `stream`, then launches as gs_composite.
 * Call it with the stream's device current (the array's address is looked
 * up on the current device, once).
 * Limit: n_views x tiles per view <= GS_NOALLOC_MAX_ITEMS, else
 * GS_ERR_UNSUPPORTED before anything is enqueued.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other streams, other host threads) race and give wrong images;
 * serialise them. */
gs_status gs_composite_noalloc(const gs_projected *proj, const uint32_t *vals, const uint32_t *tile_ranges,
                               const uint32_t *tile_order, int32_t n_views, const gs_params *p, float *rgb,
                               float *depth, float *alpha, float *t_final, uint32_t *n_contrib, float *ckpt,
                               size_t ckpt_floats, gs_stream_t stream);

/* Floats of a compositing checkpoint buffer for `capacity` key slots:
 * (capacity / GS_SEGMENT + 1) * (4 * 5 * 64 + GS_SEGMENT + 2) + 1 (0 for
 * capacity < 1): the checkpoint slots, then room for gs_render_backward's
 * list of segments to walk (it rewrites that part; gs_composite never
 * touches it). */
size_t gs_checkpoint_floats(int64_t capacity);

/* Workspace bytes gs_render_backward needs for n_instances instances. */
size_t gs_render_backward_workspace(int64_t n_instances);

/* Gradients of L(rgb, depth, alpha) given dL/drgb [V][H][W][3],
 * dL/ddepth [V][H][W], dL/dalpha [V][H][W] (any may be NULL = zero), for the
 * forward described by the same segs/cams/masks/params and its outputs
 * (proj, vals, tile_ranges, t_final, n_contrib, and ckpt).  The transmittance
 * of each pixel is recovered back to front (T_i = T_{i+1} / (1 - alpha_i));
 * the discrete decisions of the forward (cull, rect, skip, stop, clamp) are
 * held fixed, so this is the derivative almost everywhere, and it is zero
 * through the alpha clamp.  Gradients are summed over the views that draw a
 * segment and written densely (zeros for Gaussians no view sees).
 *  ckpt: the checkpoints gs_composite wrote for this frame (ckpt_floats
 *  floats), or NULL.  With them each tile list is walked in segments of
 *  GS_SEGMENT entries (at most 64 per list, the last taking the rest) by a
 *  persistent grid that pops them from a list built here in the buffer's
 *  tail (so the buffer is written as well as read), each segment starting
 *  from the state at its end (the last segment, and every list without
 *  checkpoints, from t_final and the background), so long lists are
 *  differentiated in parallel; the two give the same gradients up to
 *  rounding.  A segment whose checkpoint lies past ckpt_floats (a buffer
 *  sized for a smaller capacity than the binning's) walks from the end of
 *  its list instead, adding only its own entries: the same gradients,
 *  slower.
 *  tile_order: the work order gs_bin_sort wrote for tile_ranges, or NULL.
 *  Without checkpoints each list is walked by one workgroup; with the order
 *  the workgroups take the lists longest first (queue by queue), so that the
 *  longest walks start at once; NULL takes them in (view, tile) order.  The
 *  gradients do not depend on it.
 *  grads: host array of n_segs gradient descriptors (device pointers),
 *  overwritten (zeros for a Gaussian no view draws).  ws: per-instance
 *  screen-space accumulators (FP64, 16-byte aligned: a large Gaussian sums
 *  thousands of largely cancelling per-pixel contributions); only the drawn
 *  instances' are cleared and used.
 * Errors: as gs_project, plus GS_ERR_WORKSPACE_TOO_SMALL. */
gs_status gs_render_backward(const gs_gaussians *segs, int32_t n_segs, const gs_camera *cams, int32_t n_views,
                             const uint32_t *view_seg_mask, const gs_params *p, const gs_projected *proj,
                             const uint32_t *vals, const uint32_t *tile_ranges, const uint32_t *tile_order,
                             const float *t_final, const uint32_t *n_contrib, float *ckpt, size_t ckpt_floats,
                             const float *d_rgb, const float *d_depth, const float *d_alpha, void *ws,
                             size_t ws_bytes, const gs_gaussians_grad *grads, gs_stream_t stream);

/* ---------------------------------------------------------------------- */
/* avatar capsule queries (Sec. 3.3 dynamic NavMesh blocking, Sec. 3.4)    */
/* ---------------------------------------------------------------------- */
/* The two avatar queries of the Habitat-Lab API for a batch of agents: the
 * clearance to the nearest avatar proxy capsule and whether a candidate
 * step is blocked.  An agent is a vertical capsule: axis from its base point
 * agent_pos[e] up agent_height, radius agent_radius.  It is checked against
 * the capsules of avatars agent_avatars[e] = (first, count) (clipped to
 * [0, n_avatars)).  Capsule endpoints and radius are interpolated linearly
 * in each avatar's clip at frame_pos, with the clip rules of
 * gs_deform_lbs_clip.
 *  caps [caps_total_frames][n_caps][8] (16-byte aligned): per frame and
 *  capsule (a.x, a.y, a.z, r, b.x, b.y, b.z, unused), the capsules of avatar
 *  a being frames clip_first[a] .. + clip_frames[a] - 1.
 *  out: clearance [n_agents] = min over capsules of dist(agent axis,
 *       capsule axis) - agent_radius - r (negative: overlap; +inf with no
 *       capsule); nearest int32 [n_agents] (or NULL) = the capsule attaining
 *       it, avatar * n_caps + capsule (smallest on ties; -1 if none);
 *       with agent_next [n_agents][3] (or NULL): step_gap [n_agents] = the
 *       same minimum for the agent's axis swept along the step, the
 *       parallelogram {p0 + a (p1 - p0) + b h z : a, b in [0, 1]}, and
 *       blocked uint8 [n_agents] = step_gap < 0.
 * One wave per agent.  Errors: GS_ERR_INVALID_ARGUMENT for negative
 * counts, non-finite or negative agent sizes, NULL arrays, agent_next /
 * step_gap / blocked not all given or all NULL, misaligned caps. */
gs_status gs_capsule_queries(int32_t n_agents, const float *agent_pos, const float *agent_next,
                             const int32_t *agent_avatars, float agent_radius, float agent_height,
                             const float *caps, int32_t caps_total_frames, int32_t n_caps,
                             const int32_t *clip_first, const int32_t *clip_frames, const float *frame_pos,
                             int32_t n_avatars, float *clearance, int32_t *nearest, float *step_gap,
                             uint8_t *blocked, gs_stream_t stream);

/* ---------------------------------------------------------------------- */
/* sensor hand-off (Sec. 3.2 occlusion rule, Sec. 3.4 sensor format)       */
/* ---------------------------------------------------------------------- */
/* Turns the compositing outputs of n_views views of height x width pixels
 * into what the simulator's RGB and depth sensors deliver, and optionally
 * resolves occlusion against a mesh pass by the nearer-fragment rule of
 * Sec. 3.2: per pixel, the colour and depth of whichever pass is nearer.
 *  in:  rgb [V][H][W][3], depth [V][H][W] (accumulated z-depth) and alpha
 *       [V][H][W], as gs_composite writes them;
 *       mesh_rgba uint8 [V][H][W][4] and mesh_depth [V][H][W] (metric
 *       depth) of a mesh pass, or both NULL when there is none.
 *  out: out_rgba uint8 [V][H][W][4], out_depth [V][H][W] (metric depth).
 * Per pixel, all in FP32:
 *  - the 3DGS fragment exists where alpha > 0; its depth is
 *    D_g = depth / alpha (correctly rounded division) and its colour bytes
 *    are rint(min(max(c, 0), 1) * 255) per channel (round to nearest even;
 *    NaN gives 0), with 255 in the fourth byte;
 *  - the mesh fragment exists where mesh_depth > 0 (0, negative values and
 *    NaN mark pixels the mesh pass did not cover); its bytes are copied;
 *  - the 3DGS fragment is kept where it exists and either there is no mesh
 *    fragment or D_g < D_m (the mesh wins ties); otherwise the mesh
 *    fragment where it exists; a pixel with neither gets the 3DGS colour
 *    (the background) and depth 0.
 * Outputs must not overlap the inputs.  Float arrays need 4-byte alignment
 * and the byte arrays 4-byte alignment; with every array 16-byte aligned
 * each thread moves four pixels with 16-byte accesses.  n_views == 0 is a
 * no-op.  Errors: GS_ERR_INVALID_ARGUMENT for negative or oversized sizes
 * (height or width above 65536, more than 2^38 pixels in all),
 * NULL arrays, only one of mesh_rgba / mesh_depth, or misalignment. */
gs_status gs_sensor_compose(int32_t n_views, int32_t height, int32_t width, const float *rgb, const float *depth,
                            const float *alpha, const uint8_t *mesh_rgba, const float *mesh_depth,
                            uint8_t *out_rgba, float *out_depth, gs_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* GS_H_ */
