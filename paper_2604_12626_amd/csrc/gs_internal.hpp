// Internal definitions shared by the gfx950 kernels of libgs (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <tuple>
#include <utility>

#include "gs.h"

namespace gs {

constexpr int kTile = GS_TILE;
constexpr int kTilePixels = kTile * kTile;     // 256 pixels = 4 wave64 per tile
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kCoordClamp = 1048576.0f;       // |u|, |v| clamped to 2^20 before floor
constexpr float kRadiusCap = 16777216.0f;       // 2^24: covers every tile of any image
constexpr int kProjViews = 64;                  // views handled by one projection launch

// screen-space gradient slots accumulated per instance by the backward pass
enum { kGU = 0, kGV, kGA, kGB, kGC, kGO, kGR, kGG, kGBl, kGZ, kG2D };

// ---------------------------------------------------------------------------
// launch argument blocks (passed by value as kernel arguments)
// ---------------------------------------------------------------------------
struct ProjectArgs {
    gs_gaussians seg;
    const gs_camera *cams;
    uint32_t *tiles_touched;
    float4 *rec;
    int64_t base[kProjViews];  // first instance of this segment in each view
    int32_t view[kProjViews];  // view index
    int32_t nv;
    int32_t W, H, TX, TY;
    float near_plane, lowpass, sigma_cut, fov_clamp;
};

struct BackwardProjectArgs {
    gs_gaussians seg;
    gs_gaussians_grad grad;
    const gs_camera *cams;
    const uint32_t *tiles_touched;
    const double *g2d;  // [instances][kG2D]
    int64_t base[kProjViews];
    int32_t view[kProjViews];
    int32_t nv;
    int32_t first;     // 1: overwrite the gradients, 0: accumulate (later chunk of views)
    int32_t zeroed;    // the planes are zeroed already (by B1): list only
    int32_t W, H;
    float near_plane, lowpass, sigma_cut, fov_clamp;
    uint32_t *list;   // [seg.n]: Gaussians with an instance drawn in one of the views (compacted)
    uint32_t *count;  // number of entries of `list` (zero before the compaction)
};

struct CompositeArgs {
    const float4 *rec;
    const uint32_t *vals;
    const uint2 *ranges;
    uint32_t *counter;  // 8 queue heads + workgroups finished, 128 B apart; zero on entry and on exit
    const uint32_t *order;  // [8][qstride] items of each queue, longest list first
    int64_t qstride;        // order_stride(n_items)
    int64_t n_items;    // n_views * T
    uint32_t n_groups;  // workgroups in the grid (set by the launcher)
    int32_t W, H, TX, T;
    float alpha_max, alpha_min, t_min;
    float bg0, bg1, bg2;
    float *rgb, *depth, *alpha, *t_final;
    uint32_t *n_contrib;
    float *ckpt;          // segment checkpoints (optional)
    uint64_t ckpt_slots;  // checkpoint slots the buffer holds
};

// Segmented backward.  Checkpoint buffer: S slots of [quadrant][kCkptVals][64]
// floats, then the backward's work list (a count, then up to kListPerSlot
// entries per slot: a list has at most ceil(L / kSegment) segments, and the L
// sum to at most 64 S keys), S taken from the buffer's size.
constexpr uint32_t kSegment = GS_SEGMENT;
constexpr int kCkptVals = 5;      // T, then colour r g b and depth behind, over T
constexpr int kMaxSegments = 64;  // segments per list at most
constexpr uint64_t kCkptSlotFloats = 4 * kCkptVals * 64;
constexpr uint64_t kListPerSlot = kSegment + 2;
__host__ __device__ inline uint64_t ckpt_slots(uint64_t floats) {
    return floats > 0 ? (floats - 1) / (kCkptSlotFloats + kListPerSlot) : 0;
}
// Segment length of a list of L entries: kSegment, or the multiple of it
// that keeps the list to kMaxSegments segments (each segment then starts from
// the checkpoint at its end, which sits on a multiple of kSegment).
__host__ __device__ inline uint32_t seg_len_of(uint32_t L) {
    const uint32_t chunks = (L + kSegment - 1) / kSegment;
    const uint32_t per = (chunks + (uint32_t)kMaxSegments - 1) / (uint32_t)kMaxSegments;
    return (per > 0 ? per : 1u) * kSegment;
}
__host__ __device__ inline uint64_t ckpt_index(uint64_t slot, int quad, int val, int lane) {
    return ((slot * 4 + (uint64_t)quad) * kCkptVals + (uint64_t)val) * 64 + (uint64_t)lane;
}

constexpr int kZeroPlanes = 12;  // two segments' gradient planes

struct BackwardTileArgs {
    const float4 *rec;
    const uint32_t *vals;
    const uint2 *ranges;
    const float *t_final;
    const uint32_t *n_contrib;
    const float *d_rgb, *d_depth, *d_alpha;
    double *g2d;  // [instances][kG2D], FP64 accumulators
    const float *ckpt;   // segment checkpoints, or null (one walk per list)
    uint64_t ckpt_slots;
    uint32_t *seg_list;  // (item << 6 | segment) of every segment to walk, after a count
    const uint32_t *order;  // whole lists: the binning's work order (longest first per queue), or null
    uint32_t n_groups;   // workgroups of the persistent grid (set by the launcher)
    int64_t n_items;
    int32_t W, H, TX, T;
    float alpha_max, alpha_min;
    float bg0, bg1, bg2;
    // dense gradient planes to zero while the tiles are walked (the
    // gradients' first writer, B2, then only overwrites the drawn Gaussians)
    float *zero_ptr[kZeroPlanes];
    int64_t zero_n[kZeroPlanes];  // floats
    int32_t n_zero;
};

struct LbsArgs {
    int64_t n;
    const float *means, *log_scales, *quats;
    const uint8_t *joint_idx;
    const float *weights;
    const int32_t *avatar_of;
    const float *skin;
    int32_t n_avatars, n_joints;
    float *means_out, *cov6_out;
    // backward
    const float *d_means_out, *d_cov6_out;
    float *d_means, *d_log_scales, *d_quats;
    // clip mode (skin == NULL): per-frame joint matrices of all avatars'
    // clips [clip_total][n_joints][12], avatar a's clip is frames
    // clip_first[a] .. + clip_frames[a] - 1, sampled at frame_pos[a]
    const float *clip;
    const int32_t *clip_first, *clip_frames;
    const float *frame_pos;
    int32_t clip_total;
};

// forward kinematics: one thread per avatar, joints in parent-first order
constexpr int kFkMaxJoints = 256;
struct FkArgs {
    int32_t n_avatars, n_joints;
    int16_t parents[kFkMaxJoints];
    const float *rest;  // [J][3]
    const float *pose;  // [A][J][3] axis-angle
    const float *root;  // [A][12]
    float *out;         // [A][J][12]
};

// sensor hand-off: n_px pixels of compositing outputs (and an optional mesh
// pass) in, packed RGBA bytes and metric depth out
struct SensorArgs {
    int64_t n_px;
    const float *rgb, *depth, *alpha;
    const uint32_t *mesh_rgba;  // NULL: no mesh pass (mesh_depth NULL too)
    const float *mesh_depth;
    uint32_t *out_rgba;
    float *out_depth;
};

// avatar capsule queries: agents [n_agents] against the capsules of their
// avatars, interpolated in per-avatar clips
struct CapsuleArgs {
    int64_t n_agents;
    const float *agent_pos, *agent_next;  // [n][3]; agent_next NULL: no step query
    const int32_t *agent_avatars;         // [n][2] (first, count)
    float radius, height;
    const float *caps;  // [clip_total][n_caps][8] (a.xyz, r, b.xyz, -)
    int32_t clip_total, n_caps, n_avatars;
    const int32_t *clip_first, *clip_frames;
    const float *frame_pos;
    float *clearance, *step_gap;
    int32_t *nearest;
    uint8_t *blocked;
};

struct SortPlan {
    int64_t n, capacity, n_tiles_total;
    int tile_bits, passes;
    int part_keys, lookback;  // onesweep partition size (4096 / 8192) and look-back window (16 / 32 / 64)
    bool bucket_ok, use_bucket;  // bucket-by-tile path available / chosen (else onesweep)
    bool windowed;               // bucket path with its tile counters in a window of whole views
    int64_t T;                   // tiles per view
    int win_views;               // views per window
    int64_t bucket_blocks;
    int64_t scan_blocks, sort_parts;
    // workspace layout (byte offsets)
    size_t off_part, off_keys2, off_vals2, off_rows, off_dbase, off_tcnt, off_tcount, off_tover, off_tstart, off_comp,
        off_compn, off_slist, off_sctl, off_rlist, off_hist, off_status, off_ticket, total;
};

// launchers (one per translation unit)
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_project(const ProjectArgs &a, hipStream_t s);
SortPlan make_sort_plan(int64_t n, int64_t capacity, int64_t tiles_per_view, int64_t n_views);
hipError_t run_bin_sort(const SortPlan &P, const uint32_t *tt, const float4 *rec, int TX, int TY, char *ws,
                        uint64_t *keys, uint32_t *vals, uint32_t *ranges, uint32_t *order, int64_t *d_num,
                        int32_t *d_overflow, int n_cu, hipStream_t s);
// Tile work order for the compositing queues: queue q (items t = q mod
// kOrderQueues) lists its items from order[q * order_stride(n_items)] on, by
// descending list length in chunks of 64 entries (kOrderBins bins, the last
// holding every list of 63 chunks or more).
constexpr int kOrderQueues = 8, kOrderBins = 64;
__host__ __device__ constexpr int64_t order_stride(int64_t n_items) { return (n_items + kOrderQueues - 1) / kOrderQueues; }
hipError_t launch_tile_order(const uint32_t *ranges, int64_t n_items, uint32_t *order, hipStream_t s);
hipError_t launch_composite(CompositeArgs a, int grid, hipStream_t s);
hipError_t launch_composite_pairs(CompositeArgs a, int grid, hipStream_t s);  // grid: 2-wave workgroups
hipError_t launch_backward_tiles(BackwardTileArgs a, int n_cu, hipStream_t s);
hipError_t launch_backward_project(const BackwardProjectArgs &a, hipStream_t s);
// zeroes the screen-space accumulators of the drawn instances (tiles_touched
// > 0) and the n_counts list counters
hipError_t launch_clear_g2d(const uint32_t *tiles_touched, int64_t n_instances, double *g2d, uint32_t *counts,
                            int n_counts, const uint2 *ranges, int64_t n_items, uint32_t *seg_list, uint64_t seg_cap,
                            hipStream_t s);  // seg_list: the tile pass's work list, built too when non-NULL
hipError_t launch_lbs(const LbsArgs &a, bool backward, hipStream_t s);
hipError_t launch_lbs_joint_grad(const LbsArgs &a, float *d_skin, int n_cu, hipStream_t s);
hipError_t launch_fk(const FkArgs &a, hipStream_t s);
hipError_t launch_sensor(const SensorArgs &a, bool vec4, hipStream_t s);
hipError_t launch_capsule_queries(const CapsuleArgs &a, hipStream_t s);

// Launch a kernel through hipLaunchKernel so that the call returns the status
// of this launch itself (never a stale error of an earlier runtime call).  The
// arguments are converted to the kernel's parameter types first.
template <typename... KArgs, typename... Args>
inline hipError_t launch_kernel(void (*kernel)(KArgs...), dim3 grid, dim3 block, hipStream_t s, Args &&...args) {
    static_assert(sizeof...(KArgs) == sizeof...(Args), "kernel argument count");
    if (grid.x == 0 || grid.y == 0 || grid.z == 0) return hipSuccess;
    struct Pack {
        std::tuple<KArgs...> t;
    } pack{std::tuple<KArgs...>(std::forward<Args>(args)...)};
    void *argv[sizeof...(KArgs) > 0 ? sizeof...(KArgs) : 1];
    std::apply([&](auto &...x) {
        int k = 0;
        ((argv[k++] = static_cast<void *>(&x)), ...);
    }, pack.t);
    return hipLaunchKernel(reinterpret_cast<const void *>(kernel), grid, block, argv, 0, s);
}

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int floor_div_tile(int a) { return a >> 4; }  // floor(a / 16), arithmetic shift

struct Rect {
    int x0, x1, y0, y1;
};

// Tiles whose pixel extent [16 t, 16 t + 16) meets the closed square
// [u - r, u + r] x [v - r, v + r]; exact for an integer r given floor(u), floor(v).
__device__ __forceinline__ Rect tile_rect(float u, float v, int r, int TX, int TY) {
    const int ix = (int)floorf(fminf(fmaxf(u, -kCoordClamp), kCoordClamp));
    const int iy = (int)floorf(fminf(fmaxf(v, -kCoordClamp), kCoordClamp));
    Rect R;
    R.x0 = max(0, floor_div_tile(ix - r));
    R.x1 = min(TX, floor_div_tile(ix + r) + 1);
    R.y0 = max(0, floor_div_tile(iy - r));
    R.y1 = min(TY, floor_div_tile(iy + r) + 1);
    return R;
}

// Real spherical harmonics up to l = 3 with the Condon-Shortley phase, l-major,
// m = -l..l, evaluated at a unit direction (x, y, z) as polynomials.
// Constants: sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) times the polynomial
// normalisation, e.g. Y_1,-1 = -sqrt(3/(4 pi)) y.
struct SH {
    static constexpr float C0 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
    static constexpr float C1 = 0.48860251190291992f;   // sqrt(3/(4 pi))
    static constexpr float C2a = 1.0925484305920792f;   // sqrt(15/(4 pi))
    static constexpr float C2b = 0.31539156525252005f;  // sqrt(5/(16 pi))
    static constexpr float C2c = 0.54627421529603959f;  // sqrt(15/(16 pi))
    static constexpr float C3a = 0.59004358992664352f;  // sqrt(35/(32 pi))
    static constexpr float C3b = 2.8906114426405538f;   // sqrt(105/(4 pi))
    static constexpr float C3c = 0.45704579946446572f;  // sqrt(21/(32 pi))
    static constexpr float C3d = 0.37317633259011540f;  // sqrt(7/(16 pi))
    static constexpr float C3e = 1.4453057213202769f;   // sqrt(105/(16 pi))
};

template <int D>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float *Y) {
    Y[0] = SH::C0;
    if (D >= 1) {
        Y[1] = -SH::C1 * y;
        Y[2] = SH::C1 * z;
        Y[3] = -SH::C1 * x;
    }
    if (D >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = SH::C2a * x * y;
        Y[5] = -SH::C2a * y * z;
        Y[6] = SH::C2b * (2.0f * zz - xx - yy);
        Y[7] = -SH::C2a * x * z;
        Y[8] = SH::C2c * (xx - yy);
        if (D >= 3) {
            Y[9] = -SH::C3a * y * (3.0f * xx - yy);
            Y[10] = SH::C3b * x * y * z;
            Y[11] = -SH::C3c * y * (4.0f * zz - xx - yy);
            Y[12] = SH::C3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
            Y[13] = -SH::C3c * x * (4.0f * zz - xx - yy);
            Y[14] = SH::C3e * z * (xx - yy);
            Y[15] = -SH::C3a * x * (xx - 3.0f * yy);
        }
    }
}

// Gradient of the polynomials of sh_basis w.r.t. (x, y, z): dY[k] = (dx, dy, dz).
template <int D>
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, float3 *dY) {
    dY[0] = make_float3(0.f, 0.f, 0.f);
    if (D >= 1) {
        dY[1] = make_float3(0.f, -SH::C1, 0.f);
        dY[2] = make_float3(0.f, 0.f, SH::C1);
        dY[3] = make_float3(-SH::C1, 0.f, 0.f);
    }
    if (D >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        dY[4] = make_float3(SH::C2a * y, SH::C2a * x, 0.f);
        dY[5] = make_float3(0.f, -SH::C2a * z, -SH::C2a * y);
        dY[6] = make_float3(-2.f * SH::C2b * x, -2.f * SH::C2b * y, 4.f * SH::C2b * z);
        dY[7] = make_float3(-SH::C2a * z, 0.f, -SH::C2a * x);
        dY[8] = make_float3(2.f * SH::C2c * x, -2.f * SH::C2c * y, 0.f);
        if (D >= 3) {
            dY[9] = make_float3(-SH::C3a * 6.f * x * y, -SH::C3a * (3.f * xx - 3.f * yy), 0.f);
            dY[10] = make_float3(SH::C3b * y * z, SH::C3b * x * z, SH::C3b * x * y);
            dY[11] = make_float3(SH::C3c * 2.f * x * y, -SH::C3c * (4.f * zz - xx - 3.f * yy), -SH::C3c * 8.f * y * z);
            dY[12] = make_float3(-SH::C3d * 6.f * x * z, -SH::C3d * 6.f * y * z, SH::C3d * (6.f * zz - 3.f * xx - 3.f * yy));
            dY[13] = make_float3(-SH::C3c * (4.f * zz - 3.f * xx - yy), SH::C3c * 2.f * x * y, -SH::C3c * 8.f * x * z);
            dY[14] = make_float3(SH::C3e * 2.f * x * z, -SH::C3e * 2.f * y * z, SH::C3e * (xx - yy));
            dY[15] = make_float3(-SH::C3a * (3.f * xx - 3.f * yy), SH::C3a * 6.f * x * y, 0.f);
        }
    }
}

// Unit quaternion (w, x, y, z) -> rotation matrix (row-major).  A quaternion
// with |q|^2 < 1e-24 stands for the identity.  Templated on the arithmetic
// type: FP32 where the forward's decisions are made, FP64 in the backward's
// chain through the projection.
template <typename F>
struct RotT {
    F R[9];
    F q[4];   // normalised
    F inv_n;  // 1/|q|, 0 for the identity fallback
};
using Rot = RotT<float>;

template <typename F>
__device__ __forceinline__ RotT<F> quat_rot_t(F w, F x, F y, F z) {
    RotT<F> o;
    const F n2 = w * w + x * x + y * y + z * z;
    if (!(n2 >= (F)1e-24f)) {
        w = (F)1;
        x = y = z = (F)0;
        o.inv_n = (F)0;
    } else {
        const F inv = (F)1 / sqrt(n2);
        w *= inv;
        x *= inv;
        y *= inv;
        z *= inv;
        o.inv_n = inv;
    }
    o.q[0] = w;
    o.q[1] = x;
    o.q[2] = y;
    o.q[3] = z;
    o.R[0] = (F)1 - (F)2 * (y * y + z * z);
    o.R[1] = (F)2 * (x * y - w * z);
    o.R[2] = (F)2 * (x * z + w * y);
    o.R[3] = (F)2 * (x * y + w * z);
    o.R[4] = (F)1 - (F)2 * (x * x + z * z);
    o.R[5] = (F)2 * (y * z - w * x);
    o.R[6] = (F)2 * (x * z - w * y);
    o.R[7] = (F)2 * (y * z + w * x);
    o.R[8] = (F)1 - (F)2 * (x * x + y * y);
    return o;
}
__device__ __forceinline__ Rot quat_rot(float w, float x, float y, float z) { return quat_rot_t<float>(w, x, y, z); }

// Sigma = R diag(s^2) R^T as (xx, xy, xz, yy, yz, zz)
template <typename F>
__device__ __forceinline__ void cov_from_rot_scale(const F *R, const F *s, F *c6) {
    F M[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) M[3 * i + j] = R[3 * i + j] * s[j];
    c6[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
    c6[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
    c6[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
    c6[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
    c6[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
    c6[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
}

// Adjoint of Sigma = (R S)(R S)^T w.r.t. log-scales and the raw quaternion,
// given the symmetric adjoint dS (full 3x3, row-major).
template <typename F>
__device__ __forceinline__ void cov_backward(const RotT<F> &rot, const F *s, const F *dS, F *dlog_s, F *dq) {
    F M[9], dM[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) M[3 * i + j] = rot.R[3 * i + j] * s[j];
    // dM = (dS + dS^T) M
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            F acc = (F)0;
#pragma unroll
            for (int k = 0; k < 3; ++k) acc += (dS[3 * i + k] + dS[3 * k + i]) * M[3 * k + j];
            dM[3 * i + j] = acc;
        }
#pragma unroll
    for (int k = 0; k < 3; ++k)
        dlog_s[k] = s[k] * (rot.R[k] * dM[k] + rot.R[3 + k] * dM[3 + k] + rot.R[6 + k] * dM[6 + k]);
    if (rot.inv_n == (F)0) {
        dq[0] = dq[1] = dq[2] = dq[3] = (F)0;
        return;
    }
    F dR[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) dR[3 * i + j] = dM[3 * i + j] * s[j];
    const F w = rot.q[0], x = rot.q[1], y = rot.q[2], z = rot.q[3];
    F g[4];
    g[0] = (F)2 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    g[1] = (F)2 * (y * dR[1] + z * dR[2] + y * dR[3] - (F)2 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] -
                   (F)2 * x * dR[8]);
    g[2] = (F)2 * (-(F)2 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] -
                   (F)2 * y * dR[8]);
    g[3] = (F)2 * (-(F)2 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - (F)2 * z * dR[4] + y * dR[5] + x * dR[6] +
                   y * dR[7]);
    const F qd = w * g[0] + x * g[1] + y * g[2] + z * g[3];
#pragma unroll
    for (int c = 0; c < 4; ++c) dq[c] = (g[c] - rot.q[c] * qd) * rot.inv_n;
}

// Compositing entry as staged in LDS: exponent coefficients pre-scaled by
// log2(e) so that G = exp2(a dx^2 + c dy^2 + b dx dy).
struct Entry {
    float u, v, a, b, c, o, z, r, g, bl;
};

__device__ __forceinline__ Entry make_entry(const float4 q0, const float4 q1, const float4 q2) {
    Entry e;
    e.u = q0.x;
    e.v = q0.y;
    e.z = q0.z;
    e.a = -0.5f * kLog2e * q1.x;
    e.b = -kLog2e * q1.y;
    e.c = -0.5f * kLog2e * q1.z;
    e.o = q1.w;
    e.r = q2.x;
    e.g = q2.y;
    e.bl = q2.z;
    return e;
}

// Conservative reach of an entry: can it get alpha >= alpha_min at any pixel
// centre of the box [bx0, bx1] x [by0, by1]?  o G >= alpha_min needs
// d^T Q d <= 2 tau with tau = ln(o / alpha_min); the test uses the bounding
// box of that ellipse with tau widened by 1% + 0.1 + 1e-5 cond(Q), which
// exceeds the FP32 rounding of the exponent the compositing loop evaluates,
// so culling never changes a result.  The bound is evaluated with the
// hardware reciprocal, logarithm and square root (errors of a few ulp, far
// inside the widening), since it runs for every list entry of every quadrant.
__device__ __forceinline__ bool entry_reaches_box(float u, float v, float A, float B, float C, float o,
                                                  float alpha_min, float bx0, float by0, float bx1, float by1) {
    if (!(o >= alpha_min)) return false;
    const float detq = A * C - B * B;
    if (!(detq > 0.0f)) return true;
    const float rdet = __builtin_amdgcn_rcpf(detq);
    constexpr float kLn2 = 0.693147180559945f;
    const float tau = (__builtin_amdgcn_logf(o) - __builtin_amdgcn_logf(alpha_min)) * kLn2;
    const float tr = A + C;
    const float t2 = fmaf(1.01f, tau, 0.1f) + 1e-5f * (tr * tr * rdet);
    const float inv = 2.0f * t2 * rdet;
    const float ex = fmaf(__builtin_amdgcn_sqrtf(inv * C), 1.01f, 0.02f);
    const float ey = fmaf(__builtin_amdgcn_sqrtf(inv * A), 1.01f, 0.02f);
    if (!(u + ex >= bx0 && u - ex <= bx1 && v + ey >= by0 && v - ey <= by1)) return false;
    // The box meets the ellipse's bounding box; test the ellipse itself: the
    // minimum over the box of 1/2 d^T Q d (centre inside: 0; else on one of
    // the four edges, where it is a clamped one-dimensional minimum) against
    // the same widened threshold t2, on a box widened by the same 0.02 px.
    const float x0 = bx0 - 0.02f, x1 = bx1 + 0.02f, y0 = by0 - 0.02f, y1 = by1 + 0.02f;
    if (u >= x0 && u <= x1 && v >= y0 && v <= y1) return true;
    const float lx0 = x0 - u, lx1 = x1 - u, ly0 = y0 - v, ly1 = y1 - v;
    // A, C > 0 here (A C > B^2 >= 0); the slopes of the best point on an edge
    const float sy = -B * __builtin_amdgcn_rcpf(C), sx = -B * __builtin_amdgcn_rcpf(A);
    float qmin = INFINITY;
    {  // vertical edges: dx fixed, best dy = -B dx / C
        const float dx[2] = {lx0, lx1};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const float dy = fminf(fmaxf(sy * dx[k], ly0), ly1);
            qmin = fminf(qmin, 0.5f * (A * dx[k] * dx[k] + C * dy * dy) + B * dx[k] * dy);
        }
    }
    {  // horizontal edges: dy fixed, best dx = -B dy / A
        const float dy[2] = {ly0, ly1};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const float dx = fminf(fmaxf(sx * dy[k], lx0), lx1);
            qmin = fminf(qmin, 0.5f * (A * dx * dx + C * dy[k] * dy[k]) + B * dx * dy[k]);
        }
    }
    return !(qmin > t2);
}

// 2^x with the hardware instruction (v_exp_f32); the forward and the backward
// use this same function so that every alpha decision repeats exactly
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// exponent (base 2) at pixel offset (dx, dy); clamped to <= 0
__device__ __forceinline__ float entry_power2(float a, float b, float c, float dx, float dy) {
    // a dx^2 + b dx dy + c dy^2 = dx (a dx + b dy) + (c dy) dy
    const float p = fmaf(dx, fmaf(a, dx, b * dy), (c * dy) * dy);
    return fminf(p, 0.0f);
}

}  // namespace gs
