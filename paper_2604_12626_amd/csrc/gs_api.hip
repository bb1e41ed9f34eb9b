// Host side of the C ABI declared in include/gs.h: argument validation,
// workspace layout, instance bookkeeping and kernel launches.  Nothing here
// allocates device memory or synchronises with the device.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include <cmath>

#include "gs_internal.hpp"

namespace {

thread_local std::string g_last_error;

gs_status fail(gs_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

gs_status hip_fail(hipError_t e, const char *where) {
    return fail(GS_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

void clear_error() { g_last_error.clear(); }

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int tiles_x(const gs_params *p) { return (p->width + GS_TILE - 1) / GS_TILE; }
int tiles_y(const gs_params *p) { return (p->height + GS_TILE - 1) / GS_TILE; }

gs_status check_params(const gs_params *p) {
    if (!p) return fail(GS_ERR_INVALID_ARGUMENT, "params is NULL");
    if (p->width <= 0 || p->height <= 0 || p->width > 32768 || p->height > 32768)
        return fail(GS_ERR_INVALID_ARGUMENT, "image size %dx%d outside [1, 32768]", p->width, p->height);
    if (!(p->alpha_max > 0.f && p->alpha_max < 1.f) || !(p->alpha_min >= 0.f) || !(p->t_min >= 0.f) ||
        !(p->near_plane > 0.f) || !(p->lowpass >= 0.f) || !(p->sigma_cut > 0.f) || !(p->fov_clamp > 0.f))
        return fail(GS_ERR_INVALID_ARGUMENT, "rendering constants out of range");
    return GS_OK;
}

gs_status check_segments(const gs_gaussians *segs, int32_t n_segs) {
    if (n_segs < 1 || n_segs > GS_MAX_SEGMENTS)
        return fail(GS_ERR_INVALID_ARGUMENT, "n_segs=%d outside [1, %d]", n_segs, GS_MAX_SEGMENTS);
    if (!segs) return fail(GS_ERR_INVALID_ARGUMENT, "segs is NULL");
    for (int s = 0; s < n_segs; ++s) {
        const gs_gaussians &g = segs[s];
        if (g.n < 0) return fail(GS_ERR_INVALID_ARGUMENT, "segment %d: n < 0", s);
        if (g.sh_degree < 0 || g.sh_degree > GS_MAX_SH_DEGREE)
            return fail(GS_ERR_INVALID_ARGUMENT, "segment %d: sh_degree %d outside [0, 3]", s, g.sh_degree);
        if (g.layout != GS_LAYOUT_ROWS && g.layout != GS_LAYOUT_PLANES)
            return fail(GS_ERR_INVALID_ARGUMENT, "segment %d: layout %d (rows 0 or planes 1)", s, g.layout);
        if (g.n == 0) continue;
        if (!g.means || !g.opacity || !g.sh)
            return fail(GS_ERR_INVALID_ARGUMENT, "segment %d: means/opacity/sh is NULL", s);
        if (!g.cov6 && (!g.log_scales || !g.quats))
            return fail(GS_ERR_INVALID_ARGUMENT, "segment %d: needs cov6 or log_scales + quats", s);
        const bool rows = g.layout == GS_LAYOUT_ROWS;
        if (rows && !g.cov6 && !aligned(g.quats, 16))
            return fail(GS_ERR_INVALID_ARGUMENT, "segment %d: quats must be 16-byte aligned", s);
        const int K3 = 3 * (g.sh_degree + 1) * (g.sh_degree + 1);
        if (rows && K3 % 4 == 0 && !aligned(g.sh, 16))
            return fail(GS_ERR_INVALID_ARGUMENT, "segment %d: sh must be 16-byte aligned", s);
        if (!aligned(g.means, 4) || !aligned(g.opacity, 4) || !aligned(g.sh, 4) || (g.cov6 && !aligned(g.cov6, 4)) ||
            (!g.cov6 && (!aligned(g.quats, 4) || !aligned(g.log_scales, 4))))
            return fail(GS_ERR_INVALID_ARGUMENT, "segment %d: arrays must be 4-byte aligned", s);
    }
    return GS_OK;
}

gs_status check_views(const gs_camera *cams, int32_t n_views, const uint32_t *mask, int32_t n_segs) {
    if (n_views < 1 || n_views > GS_MAX_VIEWS)
        return fail(GS_ERR_INVALID_ARGUMENT, "n_views=%d outside [1, %d]", n_views, GS_MAX_VIEWS);
    if (!cams || !mask) return fail(GS_ERR_INVALID_ARGUMENT, "cams/view_seg_mask is NULL");
    if (!aligned(cams, 4)) return fail(GS_ERR_INVALID_ARGUMENT, "cams must be 4-byte aligned");
    const uint32_t allowed = n_segs >= 32 ? 0xFFFFFFFFu : ((1u << n_segs) - 1u);
    for (int v = 0; v < n_views; ++v)
        if (mask[v] & ~allowed)
            return fail(GS_ERR_INVALID_ARGUMENT, "view %d draws segment bits 0x%x beyond n_segs=%d", v, mask[v], n_segs);
    return GS_OK;
}

// offsets[v] (host) for every view, offsets[n_views] = total
void instance_offsets(const gs_gaussians *segs, int32_t n_segs, int32_t n_views, const uint32_t *mask,
                      int64_t *off) {
    int64_t acc = 0;
    for (int v = 0; v < n_views; ++v) {
        off[v] = acc;
        for (int s = 0; s < n_segs; ++s)
            if (mask[v] & (1u << s)) acc += segs[s].n;
    }
    off[n_views] = acc;
}

int64_t seg_offset_in_view(const gs_gaussians *segs, uint32_t mask, int s) {
    int64_t o = 0;
    for (int t = 0; t < s; ++t)
        if (mask & (1u << t)) o += segs[t].n;
    return o;
}

std::atomic<int> g_comp_groups{3};
std::atomic<int> g_sort_part_keys{4096};
std::atomic<int> g_sort_lookback{16};
std::atomic<int> g_sort_algorithm{0};
std::atomic<int> g_comp_pairs{0};

std::mutex g_dev_mu;
int g_cu_count[64] = {0};

int cu_count() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (g_cu_count[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        g_cu_count[dev] = n;
    }
    return g_cu_count[dev];
}

// Library-owned workspace of gs_composite_noalloc: the queue counters, then
// room for a work order of up to GS_NOALLOC_MAX_ITEMS items.  One copy per GPU
// (a file-scope device array, zero-initialised when the code object loads),
// held until the process ends; its device address is looked up once per
// device, with that device current, and used for every launch argument.
constexpr size_t kCompCounterBytes = 2048;
constexpr int kPairsPerCu = 4;  // two-wave compositing workgroups per CU in pair mode (their LDS)
constexpr int kPairsAutoItemsPerCu = 16;  // quadrant items per CU up to which the default takes pairs
constexpr size_t kNoallocScratchBytes =
    kCompCounterBytes + (size_t)gs::kOrderQueues * gs::order_stride(GS_NOALLOC_MAX_ITEMS) * sizeof(uint32_t);
static_assert(kNoallocScratchBytes == GS_NOALLOC_SCRATCH_BYTES, "gs.h states the scratch size");
static __device__ __align__(256) uint8_t scratch[kNoallocScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {nullptr};

hipError_t scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

const char *gs_status_string(gs_status s) {
    switch (s) {
        case GS_OK: return "GS_OK";
        case GS_ERR_INVALID_ARGUMENT: return "GS_ERR_INVALID_ARGUMENT";
        case GS_ERR_UNSUPPORTED: return "GS_ERR_UNSUPPORTED";
        case GS_ERR_WORKSPACE_TOO_SMALL: return "GS_ERR_WORKSPACE_TOO_SMALL";
        case GS_ERR_HIP: return "GS_ERR_HIP";
    }
    return "GS_ERR_UNKNOWN";
}

const char *gs_last_error(void) { return g_last_error.c_str(); }

int32_t gs_version(void) { return 2; }

void gs_default_params(gs_params *p, int32_t width, int32_t height) {
    if (!p) return;
    p->width = width;
    p->height = height;
    p->near_plane = 0.2f;
    p->lowpass = 0.3f;
    p->sigma_cut = 3.0f;
    p->fov_clamp = 1.3f;
    p->alpha_max = 0.99f;
    p->alpha_min = 1.0f / 255.0f;
    p->t_min = 1e-4f;
    p->bg[0] = p->bg[1] = p->bg[2] = 0.0f;
}

gs_status gs_set_tuning(const gs_tuning *t) {
    clear_error();
    if (!t) {
        g_comp_groups.store(3);
        g_sort_part_keys.store(4096);
        g_sort_lookback.store(16);
        g_sort_algorithm.store(0);
        g_comp_pairs.store(0);
        return GS_OK;
    }
    if (t->composite_groups_per_cu < 1 || t->composite_groups_per_cu > 32)
        return fail(GS_ERR_INVALID_ARGUMENT, "composite_groups_per_cu=%d outside [1, 32]", t->composite_groups_per_cu);
    if (t->sort_partition_keys != 4096 && t->sort_partition_keys != 8192)
        return fail(GS_ERR_INVALID_ARGUMENT, "sort_partition_keys=%d (4096 or 8192)", t->sort_partition_keys);
    if (t->sort_lookback != 16 && t->sort_lookback != 32 && t->sort_lookback != 64)
        return fail(GS_ERR_INVALID_ARGUMENT, "sort_lookback=%d (16, 32 or 64)", t->sort_lookback);
    if (t->sort_algorithm != 0 && t->sort_algorithm != 1)
        return fail(GS_ERR_INVALID_ARGUMENT, "sort_algorithm=%d (0 or 1)", t->sort_algorithm);
    if (t->composite_pairs < 0 || t->composite_pairs > 2)
        return fail(GS_ERR_INVALID_ARGUMENT, "composite_pairs=%d (0, 1 or 2)", t->composite_pairs);
    g_comp_groups.store(t->composite_groups_per_cu);
    g_sort_part_keys.store(t->sort_partition_keys);
    g_sort_lookback.store(t->sort_lookback);
    g_sort_algorithm.store(t->sort_algorithm);
    g_comp_pairs.store(t->composite_pairs);
    return GS_OK;
}

void gs_get_tuning(gs_tuning *t) {
    if (!t) return;
    memset(t, 0, sizeof(*t));
    t->composite_groups_per_cu = g_comp_groups.load();
    t->sort_partition_keys = g_sort_part_keys.load();
    t->sort_lookback = g_sort_lookback.load();
    t->sort_algorithm = g_sort_algorithm.load();
    t->composite_pairs = g_comp_pairs.load();
}

gs_status gs_instance_offsets(const gs_gaussians *segs, int32_t n_segs, int32_t n_views,
                              const uint32_t *view_seg_mask, int64_t *offsets) {
    clear_error();
    gs_status st;
    if ((st = check_segments(segs, n_segs)) != GS_OK) return st;
    if (n_views < 1 || n_views > GS_MAX_VIEWS || !view_seg_mask || !offsets)
        return fail(GS_ERR_INVALID_ARGUMENT, "bad views/mask/offsets");
    instance_offsets(segs, n_segs, n_views, view_seg_mask, offsets);
    return GS_OK;
}

// ---------------------------------------------------------------------------
gs_status gs_deform_lbs(int64_t n, const float *means_c, const float *log_scales_c, const float *quats_c,
                        const uint8_t *joint_idx, const float *weights, const int32_t *avatar_of,
                        const float *skin_mats, int32_t n_avatars, int32_t n_joints, float *means_out,
                        float *cov6_out, gs_stream_t stream) {
    clear_error();
    if (n < 0) return fail(GS_ERR_INVALID_ARGUMENT, "n < 0");
    if (n_avatars < 1 || n_joints < 1 || n_joints > 256)
        return fail(GS_ERR_INVALID_ARGUMENT, "n_avatars=%d / n_joints=%d invalid", n_avatars, n_joints);
    if (n == 0) return GS_OK;
    if (!means_c || !log_scales_c || !quats_c || !joint_idx || !weights || !avatar_of || !skin_mats || !means_out ||
        !cov6_out)
        return fail(GS_ERR_INVALID_ARGUMENT, "NULL array");
    if (!aligned(quats_c, 16) || !aligned(weights, 16) || !aligned(skin_mats, 16) || !aligned(joint_idx, 4))
        return fail(GS_ERR_INVALID_ARGUMENT, "quats/weights/skin_mats need 16-byte, joint_idx 4-byte alignment");
    gs::LbsArgs a = {};
    a.n = n;
    a.means = means_c;
    a.log_scales = log_scales_c;
    a.quats = quats_c;
    a.joint_idx = joint_idx;
    a.weights = weights;
    a.avatar_of = avatar_of;
    a.skin = skin_mats;
    a.n_avatars = n_avatars;
    a.n_joints = n_joints;
    a.means_out = means_out;
    a.cov6_out = cov6_out;
    hipError_t e = gs::launch_lbs(a, false, (hipStream_t)stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_deform_lbs");
}

gs_status gs_deform_lbs_backward(int64_t n, const float *means_c, const float *log_scales_c, const float *quats_c,
                                 const uint8_t *joint_idx, const float *weights, const int32_t *avatar_of,
                                 const float *skin_mats, int32_t n_avatars, int32_t n_joints,
                                 const float *d_means_out, const float *d_cov6_out, float *d_means_c,
                                 float *d_log_scales_c, float *d_quats_c, gs_stream_t stream) {
    clear_error();
    if (n < 0) return fail(GS_ERR_INVALID_ARGUMENT, "n < 0");
    if (n_avatars < 1 || n_joints < 1 || n_joints > 256)
        return fail(GS_ERR_INVALID_ARGUMENT, "n_avatars=%d / n_joints=%d invalid", n_avatars, n_joints);
    if (n == 0) return GS_OK;
    if (!means_c || !log_scales_c || !quats_c || !joint_idx || !weights || !avatar_of || !skin_mats ||
        !d_means_out || !d_cov6_out || !d_means_c || !d_log_scales_c || !d_quats_c)
        return fail(GS_ERR_INVALID_ARGUMENT, "NULL array");
    if (!aligned(quats_c, 16) || !aligned(weights, 16) || !aligned(skin_mats, 16) || !aligned(joint_idx, 4) ||
        !aligned(d_quats_c, 16))
        return fail(GS_ERR_INVALID_ARGUMENT, "quats/weights/skin_mats/d_quats need 16-byte alignment");
    gs::LbsArgs a = {};
    a.n = n;
    a.means = means_c;
    a.log_scales = log_scales_c;
    a.quats = quats_c;
    a.joint_idx = joint_idx;
    a.weights = weights;
    a.avatar_of = avatar_of;
    a.skin = skin_mats;
    a.n_avatars = n_avatars;
    a.n_joints = n_joints;
    a.d_means_out = d_means_out;
    a.d_cov6_out = d_cov6_out;
    a.d_means = d_means_c;
    a.d_log_scales = d_log_scales_c;
    a.d_quats = d_quats_c;
    hipError_t e = gs::launch_lbs(a, true, (hipStream_t)stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_deform_lbs_backward");
}

// ---------------------------------------------------------------------------
gs_status gs_project(const gs_gaussians *segs, int32_t n_segs, const gs_camera *cams, int32_t n_views,
                     const uint32_t *view_seg_mask, const gs_params *p, gs_projected *out, gs_stream_t stream) {
    clear_error();
    gs_status st;
    if ((st = check_params(p)) != GS_OK) return st;
    if ((st = check_segments(segs, n_segs)) != GS_OK) return st;
    if ((st = check_views(cams, n_views, view_seg_mask, n_segs)) != GS_OK) return st;
    if (!out) return fail(GS_ERR_INVALID_ARGUMENT, "out is NULL");
    std::vector<int64_t> off(n_views + 1);
    instance_offsets(segs, n_segs, n_views, view_seg_mask, off.data());
    if (out->n_instances != off[n_views])
        return fail(GS_ERR_INVALID_ARGUMENT, "out->n_instances=%lld but the views draw %lld instances",
                    (long long)out->n_instances, (long long)off[n_views]);
    if (off[n_views] > 0xFFFFFFFFll) return fail(GS_ERR_UNSUPPORTED, "more than 2^32-1 instances");
    if (off[n_views] == 0) return GS_OK;
    if (!out->tiles_touched || !out->rec) return fail(GS_ERR_INVALID_ARGUMENT, "out arrays are NULL");
    if (!aligned(out->rec, 16)) return fail(GS_ERR_INVALID_ARGUMENT, "rec must be 16-byte aligned");
    for (int s = 0; s < n_segs; ++s) {
        std::vector<int> views;
        for (int v = 0; v < n_views; ++v)
            if (view_seg_mask[v] & (1u << s)) views.push_back(v);
        for (size_t c = 0; c < views.size(); c += gs::kProjViews) {
            gs::ProjectArgs a = {};
            a.seg = segs[s];
            a.cams = cams;
            a.tiles_touched = out->tiles_touched;
            a.rec = reinterpret_cast<float4 *>(out->rec);
            a.nv = (int)std::min(views.size() - c, (size_t)gs::kProjViews);
            for (int k = 0; k < a.nv; ++k) {
                const int v = views[c + k];
                a.view[k] = v;
                a.base[k] = off[v] + seg_offset_in_view(segs, view_seg_mask[v], s);
            }
            a.W = p->width;
            a.H = p->height;
            a.TX = tiles_x(p);
            a.TY = tiles_y(p);
            a.near_plane = p->near_plane;
            a.lowpass = p->lowpass;
            a.sigma_cut = p->sigma_cut;
            a.fov_clamp = p->fov_clamp;
            hipError_t e = gs::launch_project(a, (hipStream_t)stream);
            if (e != hipSuccess) return hip_fail(e, "gs_project");
        }
    }
    return GS_OK;
}

// ---------------------------------------------------------------------------
size_t gs_bin_sort_workspace(int64_t n_instances, int64_t capacity, int32_t n_views, const gs_params *p) {
    if (!p || n_views < 1 || capacity < 1 || n_instances < 0) return 0;
    const int64_t T = (int64_t)tiles_x(p) * tiles_y(p);
    return gs::make_sort_plan(n_instances, capacity, T, n_views).total;
}

size_t gs_tile_order_words(int32_t n_views, const gs_params *p) {
    if (!p || n_views < 1 || check_params(p) != GS_OK) return 0;
    return (size_t)gs::kOrderQueues * gs::order_stride((int64_t)tiles_x(p) * tiles_y(p) * n_views);
}

gs_status gs_bin_sort(const gs_projected *proj, int32_t n_views, const gs_params *p, void *ws, size_t ws_bytes,
                      uint64_t *keys, uint32_t *vals, int64_t capacity, uint32_t *tile_ranges, uint32_t *tile_order,
                      int64_t *d_num_instances, int32_t *d_overflow, gs_stream_t stream) {
    clear_error();
    gs_status st;
    if ((st = check_params(p)) != GS_OK) return st;
    if (!proj || proj->n_instances < 0) return fail(GS_ERR_INVALID_ARGUMENT, "proj is NULL or has n < 0");
    if (n_views < 1 || n_views > GS_MAX_VIEWS) return fail(GS_ERR_INVALID_ARGUMENT, "n_views=%d", n_views);
    if (capacity < 1) return fail(GS_ERR_INVALID_ARGUMENT, "capacity < 1");
    if (capacity > GS_MAX_CAPACITY) return fail(GS_ERR_UNSUPPORTED, "capacity above %lld", (long long)GS_MAX_CAPACITY);
    if (proj->n_instances > 0 && (!proj->tiles_touched || !proj->rec || !aligned(proj->rec, 16) ||
                                  !aligned(proj->tiles_touched, 16)))
        return fail(GS_ERR_INVALID_ARGUMENT, "proj arrays NULL or rec/tiles_touched not 16-byte aligned");
    if (!keys || !vals || !tile_ranges || !d_num_instances || !d_overflow || !ws)
        return fail(GS_ERR_INVALID_ARGUMENT, "NULL output or workspace");
    if (!aligned(keys, 8) || !aligned(tile_ranges, 8) || !aligned(d_num_instances, 8) || !aligned(ws, 256) ||
        !aligned(tile_order, 4))
        return fail(GS_ERR_INVALID_ARGUMENT, "keys/ranges/counter need 8-byte, order 4-byte, ws 256-byte alignment");
    const int64_t T = (int64_t)tiles_x(p) * tiles_y(p);
    if (T * n_views > (1ll << 31)) return fail(GS_ERR_UNSUPPORTED, "more than 2^31 tiles");
    gs::SortPlan plan = gs::make_sort_plan(proj->n_instances, capacity, T, n_views);
    plan.part_keys = g_sort_part_keys.load();
    plan.lookback = g_sort_lookback.load();
    plan.use_bucket = plan.bucket_ok && g_sort_algorithm.load() == 0;
    if (ws_bytes < plan.total)
        return fail(GS_ERR_WORKSPACE_TOO_SMALL, "workspace %zu < %zu bytes", ws_bytes, plan.total);
    hipError_t e = gs::run_bin_sort(plan, proj->tiles_touched, reinterpret_cast<const float4 *>(proj->rec),
                                    tiles_x(p), tiles_y(p), static_cast<char *>(ws), keys, vals, tile_ranges,
                                    tile_order, d_num_instances, d_overflow, cu_count(), (hipStream_t)stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_bin_sort");
}

// ---------------------------------------------------------------------------
// nine counters (one 128-B line each), then room for a tile work order
size_t gs_composite_workspace(int32_t n_views, const gs_params *p) {
    const size_t words = gs_tile_order_words(n_views, p);
    return words ? kCompCounterBytes + words * sizeof(uint32_t) : 0;
}

size_t gs_checkpoint_floats(int64_t capacity) {
    if (capacity < 1) return 0;
    return (size_t)(capacity / (int64_t)gs::kSegment + 1) * (gs::kCkptSlotFloats + gs::kListPerSlot) + 1;
}

}  // extern "C"

namespace {

// gs_composite and gs_composite_noalloc: validation, then the launches with
// the queue counters and work-order room at `counter` / `own_order`.
gs_status composite_checks(const gs_projected *proj, const uint32_t *vals, const uint32_t *tile_ranges,
                           const uint32_t *tile_order, int32_t n_views, const gs_params *p, float *rgb, float *depth,
                           float *alpha, const float *ckpt) {
    gs_status st;
    if ((st = check_params(p)) != GS_OK) return st;
    if (!proj || !vals || !tile_ranges || !rgb || !depth || !alpha)
        return fail(GS_ERR_INVALID_ARGUMENT, "NULL argument");
    if (n_views < 1 || n_views > GS_MAX_VIEWS) return fail(GS_ERR_INVALID_ARGUMENT, "n_views=%d", n_views);
    if (proj->n_instances > 0 && (!proj->rec || !aligned(proj->rec, 16)))
        return fail(GS_ERR_INVALID_ARGUMENT, "rec NULL or not 16-byte aligned");
    if (!aligned(tile_ranges, 8) || !aligned(tile_order, 4) || !aligned(ckpt, 4))
        return fail(GS_ERR_INVALID_ARGUMENT, "misaligned ranges/order/ckpt");
    return GS_OK;
}

gs_status composite_launch(const char *who, const gs_projected *proj, const uint32_t *vals,
                           const uint32_t *tile_ranges, const uint32_t *tile_order, int32_t n_views,
                           const gs_params *p, uint32_t *counter, uint32_t *own_order, bool clear_counters,
                           float *rgb, float *depth, float *alpha, float *t_final, uint32_t *n_contrib, float *ckpt,
                           size_t ckpt_floats, hipStream_t stream) {
    gs::CompositeArgs a = {};
    a.rec = reinterpret_cast<const float4 *>(proj->rec);
    a.vals = vals;
    a.ranges = reinterpret_cast<const uint2 *>(tile_ranges);
    a.counter = counter;
    a.order = tile_order ? tile_order : own_order;
    a.W = p->width;
    a.H = p->height;
    a.TX = tiles_x(p);
    a.T = tiles_x(p) * tiles_y(p);
    a.n_items = (int64_t)a.T * n_views;
    a.qstride = gs::order_stride(a.n_items);
    a.alpha_max = p->alpha_max;
    a.alpha_min = p->alpha_min;
    a.t_min = p->t_min;
    a.bg0 = p->bg[0];
    a.bg1 = p->bg[1];
    a.bg2 = p->bg[2];
    a.rgb = rgb;
    a.depth = depth;
    a.alpha = alpha;
    a.t_final = t_final;
    a.n_contrib = n_contrib;
    a.ckpt_slots = gs::ckpt_slots(ckpt_floats);
    a.ckpt = a.ckpt_slots ? ckpt : nullptr;
    hipError_t e;
    // persistent waves: a tunable number of four-wave groups per CU, never
    // more waves than quadrant work items; or, with few items, pairs of
    // waves (the LDS of a pair allows four per CU), whose shorter walks win
    // while the longest lists bound the kernel (measured: 256 x 256 views,
    // 1024 to 4096 quadrant items, 0.72-0.75 of the single-wave time; a
    // 640 x 480 view, 4800 items, 1.35 of it)
    const int pairs_mode = g_comp_pairs.load();
    const bool pairs =
        pairs_mode == 2 || (pairs_mode == 0 && 4 * a.n_items <= (int64_t)kPairsAutoItemsPerCu * cu_count());
    int64_t grid = (int64_t)cu_count() * (pairs ? kPairsPerCu : g_comp_groups.load());
    if (grid > (pairs ? 4 : 1) * a.n_items) grid = (pairs ? 4 : 1) * a.n_items;
    if (clear_counters &&
        (e = gs::launch_fill_u32(counter, 0u, (int64_t)(kCompCounterBytes / sizeof(uint32_t)), stream)) != hipSuccess)
        return hip_fail(e, who);
    if (!tile_order && (e = gs::launch_tile_order(tile_ranges, a.n_items, own_order, stream)) != hipSuccess)
        return hip_fail(e, who);
    e = pairs ? gs::launch_composite_pairs(a, (int)grid, stream) : gs::launch_composite(a, (int)grid, stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, who);
}

}  // namespace

extern "C" {

gs_status gs_composite(const gs_projected *proj, const uint32_t *vals, const uint32_t *tile_ranges,
                       const uint32_t *tile_order, int32_t n_views, const gs_params *p, void *ws, size_t ws_bytes,
                       float *rgb, float *depth, float *alpha, float *t_final, uint32_t *n_contrib, float *ckpt,
                       size_t ckpt_floats, gs_stream_t stream) {
    clear_error();
    gs_status st = composite_checks(proj, vals, tile_ranges, tile_order, n_views, p, rgb, depth, alpha, ckpt);
    if (st != GS_OK) return st;
    if (!ws) return fail(GS_ERR_INVALID_ARGUMENT, "NULL workspace");
    if (!aligned(ws, 4)) return fail(GS_ERR_INVALID_ARGUMENT, "misaligned workspace");
    if (ws_bytes < gs_composite_workspace(n_views, p)) return fail(GS_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
    uint32_t *own_order = reinterpret_cast<uint32_t *>(static_cast<char *>(ws) + kCompCounterBytes);
    return composite_launch("gs_composite", proj, vals, tile_ranges, tile_order, n_views, p,
                            static_cast<uint32_t *>(ws), own_order, false, rgb, depth, alpha, t_final, n_contrib,
                            ckpt, ckpt_floats, (hipStream_t)stream);
}

gs_status gs_composite_noalloc(const gs_projected *proj, const uint32_t *vals, const uint32_t *tile_ranges,
                               const uint32_t *tile_order, int32_t n_views, const gs_params *p, float *rgb,
                               float *depth, float *alpha, float *t_final, uint32_t *n_contrib, float *ckpt,
                               size_t ckpt_floats, gs_stream_t stream) {
    clear_error();
    gs_status st = composite_checks(proj, vals, tile_ranges, tile_order, n_views, p, rgb, depth, alpha, ckpt);
    if (st != GS_OK) return st;
    const int64_t n_items = (int64_t)tiles_x(p) * tiles_y(p) * n_views;
    if (n_items > GS_NOALLOC_MAX_ITEMS)
        return fail(GS_ERR_UNSUPPORTED, "gs_composite_noalloc: %lld (view, tile) items exceed its scratch (%d)",
                    (long long)n_items, GS_NOALLOC_MAX_ITEMS);
    void *base = nullptr;
    hipError_t e = scratch_address(&base);
    if (e != hipSuccess) return hip_fail(e, "gs_composite_noalloc: scratch address");
    uint32_t *counter = static_cast<uint32_t *>(base);
    uint32_t *own_order = reinterpret_cast<uint32_t *>(static_cast<char *>(base) + kCompCounterBytes);
    return composite_launch("gs_composite_noalloc", proj, vals, tile_ranges, tile_order, n_views, p, counter,
                            own_order, true, rgb, depth, alpha, t_final, n_contrib, ckpt, ckpt_floats,
                            (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// workspace: per-instance screen-space accumulators, then the compacted
// Gaussian list of one projection launch, then its counters (one per launch)
static size_t bwd_list_offset(int64_t n_instances) {
    return ((size_t)(n_instances > 0 ? n_instances : 1) * gs::kG2D * sizeof(double) + 255) & ~(size_t)255;
}
static size_t bwd_count_offset(int64_t n_instances) {
    return bwd_list_offset(n_instances) +
           (((size_t)(n_instances > 0 ? n_instances : 1) * sizeof(uint32_t) + 255) & ~(size_t)255);
}
constexpr int kBwdMaxLaunches = GS_MAX_SEGMENTS * ((GS_MAX_VIEWS + gs::kProjViews - 1) / gs::kProjViews);

size_t gs_render_backward_workspace(int64_t n_instances) {
    if (n_instances < 0) return 0;
    return bwd_count_offset(n_instances) + sizeof(uint32_t) * kBwdMaxLaunches;
}

gs_status gs_render_backward(const gs_gaussians *segs, int32_t n_segs, const gs_camera *cams, int32_t n_views,
                             const uint32_t *view_seg_mask, const gs_params *p, const gs_projected *proj,
                             const uint32_t *vals, const uint32_t *tile_ranges, const uint32_t *tile_order,
                             const float *t_final, const uint32_t *n_contrib, float *ckpt, size_t ckpt_floats,
                             const float *d_rgb, const float *d_depth, const float *d_alpha, void *ws,
                             size_t ws_bytes, const gs_gaussians_grad *grads, gs_stream_t stream) {
    clear_error();
    gs_status st;
    if ((st = check_params(p)) != GS_OK) return st;
    if ((st = check_segments(segs, n_segs)) != GS_OK) return st;
    if ((st = check_views(cams, n_views, view_seg_mask, n_segs)) != GS_OK) return st;
    if (!proj || !vals || !tile_ranges || !t_final || !n_contrib || !ws || !grads)
        return fail(GS_ERR_INVALID_ARGUMENT, "NULL argument");
    if (!aligned(ckpt, 4) || !aligned(ws, 16) || !aligned(tile_order, 4))
        return fail(GS_ERR_INVALID_ARGUMENT, "ckpt, tile_order or ws misaligned");
    std::vector<int64_t> off(n_views + 1);
    instance_offsets(segs, n_segs, n_views, view_seg_mask, off.data());
    if (proj->n_instances != off[n_views])
        return fail(GS_ERR_INVALID_ARGUMENT, "proj->n_instances does not match the views");
    if (ws_bytes < gs_render_backward_workspace(proj->n_instances))
        return fail(GS_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
    for (int s = 0; s < n_segs; ++s)
        if (segs[s].layout != GS_LAYOUT_ROWS)
            return fail(GS_ERR_UNSUPPORTED, "segment %d: the backward takes rows (layout 0)", s);
    for (int s = 0; s < n_segs; ++s) {
        if (segs[s].n == 0) continue;
        const gs_gaussians_grad &g = grads[s];
        if (!g.means || !g.opacity || !g.sh) return fail(GS_ERR_INVALID_ARGUMENT, "segment %d: NULL gradient", s);
        if (!segs[s].cov6 && g.quats && !aligned(g.quats, 16))
            return fail(GS_ERR_INVALID_ARGUMENT, "segment %d: quats gradient must be 16-byte aligned", s);
    }
    hipStream_t sm = (hipStream_t)stream;
    // screen-space adjoints accumulate in FP64: a large Gaussian sums thousands
    // of per-pixel contributions that largely cancel
    double *g2d = static_cast<double *>(ws);
    uint32_t *list = reinterpret_cast<uint32_t *>(static_cast<char *>(ws) + bwd_list_offset(proj->n_instances));
    uint32_t *counts = reinterpret_cast<uint32_t *>(static_cast<char *>(ws) + bwd_count_offset(proj->n_instances));
    hipError_t e;
    int launch_no = 0;
    gs::BackwardTileArgs b = {};
    b.rec = reinterpret_cast<const float4 *>(proj->rec);
    b.vals = vals;
    b.ranges = reinterpret_cast<const uint2 *>(tile_ranges);
    b.t_final = t_final;
    b.n_contrib = n_contrib;
    b.d_rgb = d_rgb;
    b.d_depth = d_depth;
    b.d_alpha = d_alpha;
    b.g2d = g2d;
    b.ckpt_slots = gs::ckpt_slots(ckpt_floats);
    b.ckpt = b.ckpt_slots ? ckpt : nullptr;
    // the work list lives behind the checkpoints (the backward's own part of the buffer)
    b.seg_list = b.ckpt ? reinterpret_cast<uint32_t *>(ckpt + b.ckpt_slots * gs::kCkptSlotFloats)
                        : nullptr;
    b.order = tile_order;
    b.W = p->width;
    b.H = p->height;
    b.TX = tiles_x(p);
    b.T = tiles_x(p) * tiles_y(p);
    b.n_items = (int64_t)b.T * n_views;
    if (b.seg_list && b.n_items >= (int64_t)1 << 26) b.seg_list = nullptr;  // item ids need 26 bits
    // only the drawn instances' accumulators are used, so only those are
    // cleared, together with the list counters; the same launch builds the
    // tile pass's segment list
    e = gs::launch_clear_g2d(proj->tiles_touched, proj->n_instances, g2d, counts, kBwdMaxLaunches, b.ranges,
                             b.n_items, b.seg_list, (uint64_t)(b.ckpt_slots * gs::kListPerSlot), sm);
    if (e != hipSuccess) return hip_fail(e, "gs_render_backward");
    b.alpha_max = p->alpha_max;
    b.alpha_min = p->alpha_min;
    b.bg0 = p->bg[0];
    b.bg1 = p->bg[1];
    b.bg2 = p->bg[2];
    // the tile pass also clears the dense gradient planes of the first
    // segments (as many as its arguments hold); B2 clears the others itself
    std::vector<int> zeroed(n_segs, 0);
    if (proj->n_instances > 0) {
        for (int s = 0; s < n_segs; ++s) {
            if (segs[s].n == 0) continue;
            const gs_gaussians_grad &g = grads[s];
            const int64_t n = segs[s].n, K = (int64_t)(segs[s].sh_degree + 1) * (segs[s].sh_degree + 1);
            float *ptr[6] = {g.means, g.opacity, g.sh, segs[s].cov6 ? g.cov6 : nullptr,
                             segs[s].cov6 ? nullptr : g.log_scales, segs[s].cov6 ? nullptr : g.quats};
            const int64_t w[6] = {3, 1, 3 * K, 6, 3, 4};
            int need = 0;
            for (int k = 0; k < 6; ++k) need += ptr[k] ? 1 : 0;
            if (b.n_zero + need > gs::kZeroPlanes) break;
            for (int k = 0; k < 6; ++k)
                if (ptr[k]) {
                    b.zero_ptr[b.n_zero] = ptr[k];
                    b.zero_n[b.n_zero] = w[k] * n;
                    ++b.n_zero;
                }
            zeroed[s] = 1;
        }
        e = gs::launch_backward_tiles(b, cu_count(), sm);
        if (e != hipSuccess) return hip_fail(e, "gs_render_backward (tiles)");
    }
    for (int s = 0; s < n_segs; ++s) {
        std::vector<int> views;
        for (int v = 0; v < n_views; ++v)
            if (view_seg_mask[v] & (1u << s)) views.push_back(v);
        size_t c = 0;
        do {
            gs::BackwardProjectArgs a = {};
            a.seg = segs[s];
            a.grad = grads[s];
            a.cams = cams;
            a.tiles_touched = proj->tiles_touched;
            a.g2d = g2d;
            a.nv = (int)std::min(views.size() - c, (size_t)gs::kProjViews);
            for (int k = 0; k < a.nv; ++k) {
                const int v = views[c + k];
                a.view[k] = v;
                a.base[k] = off[v] + seg_offset_in_view(segs, view_seg_mask[v], s);
            }
            a.first = (c == 0) ? 1 : 0;
            a.zeroed = zeroed[s];
            a.W = p->width;
            a.H = p->height;
            a.near_plane = p->near_plane;
            a.lowpass = p->lowpass;
            a.sigma_cut = p->sigma_cut;
            a.fov_clamp = p->fov_clamp;
            a.list = list;
            a.count = counts + launch_no++;
            e = gs::launch_backward_project(a, sm);
            if (e != hipSuccess) return hip_fail(e, "gs_render_backward (projection)");
            c += gs::kProjViews;
        } while (c < views.size());
    }
    return GS_OK;
}

gs_status gs_deform_lbs_backward_joints(int64_t n, const float *means_c, const float *log_scales_c,
                                        const float *quats_c, const uint8_t *joint_idx, const float *weights,
                                        const int32_t *avatar_of, const float *skin_mats, int32_t n_avatars,
                                        int32_t n_joints, const float *d_means_out, const float *d_cov6_out,
                                        float *d_skin_mats, gs_stream_t stream) {
    clear_error();
    if (n < 0) return fail(GS_ERR_INVALID_ARGUMENT, "n < 0");
    if (n_avatars < 1 || n_joints < 1 || n_joints > 256)
        return fail(GS_ERR_INVALID_ARGUMENT, "n_avatars=%d / n_joints=%d invalid", n_avatars, n_joints);
    if (!d_skin_mats) return fail(GS_ERR_INVALID_ARGUMENT, "NULL d_skin_mats");
    if (n > 0 && (!means_c || !log_scales_c || !quats_c || !joint_idx || !weights || !avatar_of || !skin_mats ||
                  !d_means_out || !d_cov6_out))
        return fail(GS_ERR_INVALID_ARGUMENT, "NULL array");
    if (!aligned(quats_c, 16) || !aligned(weights, 16) || !aligned(skin_mats, 16) || !aligned(joint_idx, 4))
        return fail(GS_ERR_INVALID_ARGUMENT, "quats/weights/skin_mats need 16-byte, joint_idx 4-byte alignment");
    gs::LbsArgs a = {};
    a.n = n;
    a.means = means_c;
    a.log_scales = log_scales_c;
    a.quats = quats_c;
    a.joint_idx = joint_idx;
    a.weights = weights;
    a.avatar_of = avatar_of;
    a.skin = skin_mats;
    a.n_avatars = n_avatars;
    a.n_joints = n_joints;
    a.d_means_out = d_means_out;
    a.d_cov6_out = d_cov6_out;
    hipError_t e = gs::launch_lbs_joint_grad(a, d_skin_mats, cu_count(), (hipStream_t)stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_deform_lbs_backward_joints");
}

gs_status gs_forward_kinematics(int32_t n_avatars, int32_t n_joints, const int32_t *parents, const float *rest,
                                const float *pose, const float *root, float *skin_out, gs_stream_t stream) {
    clear_error();
    if (n_avatars < 0 || n_joints < 1 || n_joints > gs::kFkMaxJoints)
        return fail(GS_ERR_INVALID_ARGUMENT, "n_avatars=%d / n_joints=%d invalid", n_avatars, n_joints);
    if (!parents) return fail(GS_ERR_INVALID_ARGUMENT, "NULL parents (host array)");
    gs::FkArgs f = {};
    for (int k = 0; k < n_joints; ++k) {
        if (parents[k] < -1 || parents[k] >= k)
            return fail(GS_ERR_INVALID_ARGUMENT, "parents[%d]=%d: parents must come before their children", k,
                        parents[k]);
        f.parents[k] = (int16_t)parents[k];
    }
    if (n_avatars == 0) return GS_OK;
    if (!rest || !pose || !root || !skin_out) return fail(GS_ERR_INVALID_ARGUMENT, "NULL array");
    f.n_avatars = n_avatars;
    f.n_joints = n_joints;
    f.rest = rest;
    f.pose = pose;
    f.root = root;
    f.out = skin_out;
    hipError_t e = gs::launch_fk(f, (hipStream_t)stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_forward_kinematics");
}

// the clip-mode arguments shared by gs_deform_lbs_clip and its backward
static gs_status clip_args(gs::LbsArgs &a, const float *clip_mats, int32_t clip_total_frames,
                           const int32_t *clip_first, const int32_t *clip_frames, const float *frame_pos) {
    if (clip_total_frames < 1) return fail(GS_ERR_INVALID_ARGUMENT, "clip_total_frames=%d", clip_total_frames);
    if (!clip_mats || !clip_first || !clip_frames || !frame_pos) return fail(GS_ERR_INVALID_ARGUMENT, "NULL clip array");
    if (!aligned(clip_mats, 16)) return fail(GS_ERR_INVALID_ARGUMENT, "clip_mats needs 16-byte alignment");
    a.skin = nullptr;
    a.clip = clip_mats;
    a.clip_total = clip_total_frames;
    a.clip_first = clip_first;
    a.clip_frames = clip_frames;
    a.frame_pos = frame_pos;
    return GS_OK;
}

gs_status gs_deform_lbs_clip(int64_t n, const float *means_c, const float *log_scales_c, const float *quats_c,
                             const uint8_t *joint_idx, const float *weights, const int32_t *avatar_of,
                             const float *clip_mats, int32_t clip_total_frames, const int32_t *clip_first,
                             const int32_t *clip_frames, const float *frame_pos, int32_t n_avatars,
                             int32_t n_joints, float *means_out, float *cov6_out, gs_stream_t stream) {
    clear_error();
    if (n < 0) return fail(GS_ERR_INVALID_ARGUMENT, "n < 0");
    if (n_avatars < 1 || n_joints < 1 || n_joints > 256)
        return fail(GS_ERR_INVALID_ARGUMENT, "n_avatars=%d / n_joints=%d invalid", n_avatars, n_joints);
    if (n == 0) return GS_OK;
    if (!means_c || !log_scales_c || !quats_c || !joint_idx || !weights || !avatar_of || !means_out || !cov6_out)
        return fail(GS_ERR_INVALID_ARGUMENT, "NULL array");
    if (!aligned(quats_c, 16) || !aligned(weights, 16) || !aligned(joint_idx, 4))
        return fail(GS_ERR_INVALID_ARGUMENT, "quats/weights need 16-byte, joint_idx 4-byte alignment");
    gs::LbsArgs a = {};
    gs_status st = clip_args(a, clip_mats, clip_total_frames, clip_first, clip_frames, frame_pos);
    if (st != GS_OK) return st;
    a.n = n;
    a.means = means_c;
    a.log_scales = log_scales_c;
    a.quats = quats_c;
    a.joint_idx = joint_idx;
    a.weights = weights;
    a.avatar_of = avatar_of;
    a.n_avatars = n_avatars;
    a.n_joints = n_joints;
    a.means_out = means_out;
    a.cov6_out = cov6_out;
    hipError_t e = gs::launch_lbs(a, false, (hipStream_t)stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_deform_lbs_clip");
}

gs_status gs_deform_lbs_clip_backward(int64_t n, const float *means_c, const float *log_scales_c,
                                      const float *quats_c, const uint8_t *joint_idx, const float *weights,
                                      const int32_t *avatar_of, const float *clip_mats, int32_t clip_total_frames,
                                      const int32_t *clip_first, const int32_t *clip_frames,
                                      const float *frame_pos, int32_t n_avatars, int32_t n_joints,
                                      const float *d_means_out, const float *d_cov6_out, float *d_means_c,
                                      float *d_log_scales_c, float *d_quats_c, gs_stream_t stream) {
    clear_error();
    if (n < 0) return fail(GS_ERR_INVALID_ARGUMENT, "n < 0");
    if (n_avatars < 1 || n_joints < 1 || n_joints > 256)
        return fail(GS_ERR_INVALID_ARGUMENT, "n_avatars=%d / n_joints=%d invalid", n_avatars, n_joints);
    if (n == 0) return GS_OK;
    if (!means_c || !log_scales_c || !quats_c || !joint_idx || !weights || !avatar_of || !d_means_out ||
        !d_cov6_out || !d_means_c || !d_log_scales_c || !d_quats_c)
        return fail(GS_ERR_INVALID_ARGUMENT, "NULL array");
    if (!aligned(quats_c, 16) || !aligned(weights, 16) || !aligned(joint_idx, 4) || !aligned(d_quats_c, 16))
        return fail(GS_ERR_INVALID_ARGUMENT, "quats/weights/d_quats need 16-byte alignment");
    gs::LbsArgs a = {};
    gs_status st = clip_args(a, clip_mats, clip_total_frames, clip_first, clip_frames, frame_pos);
    if (st != GS_OK) return st;
    a.n = n;
    a.means = means_c;
    a.log_scales = log_scales_c;
    a.quats = quats_c;
    a.joint_idx = joint_idx;
    a.weights = weights;
    a.avatar_of = avatar_of;
    a.n_avatars = n_avatars;
    a.n_joints = n_joints;
    a.d_means_out = d_means_out;
    a.d_cov6_out = d_cov6_out;
    a.d_means = d_means_c;
    a.d_log_scales = d_log_scales_c;
    a.d_quats = d_quats_c;
    hipError_t e = gs::launch_lbs(a, true, (hipStream_t)stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_deform_lbs_clip_backward");
}

gs_status gs_capsule_queries(int32_t n_agents, const float *agent_pos, const float *agent_next,
                             const int32_t *agent_avatars, float agent_radius, float agent_height,
                             const float *caps, int32_t caps_total_frames, int32_t n_caps,
                             const int32_t *clip_first, const int32_t *clip_frames, const float *frame_pos,
                             int32_t n_avatars, float *clearance, int32_t *nearest, float *step_gap,
                             uint8_t *blocked, gs_stream_t stream) {
    clear_error();
    if (n_agents < 0) return fail(GS_ERR_INVALID_ARGUMENT, "n_agents < 0");
    if (n_agents == 0) return GS_OK;
    if (n_avatars < 1 || n_caps < 1 || caps_total_frames < 1)
        return fail(GS_ERR_INVALID_ARGUMENT, "n_avatars=%d n_caps=%d caps_total_frames=%d invalid", n_avatars,
                    n_caps, caps_total_frames);
    if (!(agent_radius >= 0.0f) || !(agent_height >= 0.0f) || !std::isfinite(agent_radius) ||
        !std::isfinite(agent_height))
        return fail(GS_ERR_INVALID_ARGUMENT, "agent radius / height must be finite and >= 0");
    if (!agent_pos || !agent_avatars || !caps || !clip_first || !clip_frames || !frame_pos || !clearance)
        return fail(GS_ERR_INVALID_ARGUMENT, "NULL array");
    if ((agent_next == nullptr) != (step_gap == nullptr) || (agent_next == nullptr) != (blocked == nullptr))
        return fail(GS_ERR_INVALID_ARGUMENT, "agent_next, step_gap and blocked must all be given or all be NULL");
    if (!aligned(caps, 16)) return fail(GS_ERR_INVALID_ARGUMENT, "caps needs 16-byte alignment");
    gs::CapsuleArgs a = {};
    a.n_agents = n_agents;
    a.agent_pos = agent_pos;
    a.agent_next = agent_next;
    a.agent_avatars = agent_avatars;
    a.radius = agent_radius;
    a.height = agent_height;
    a.caps = caps;
    a.clip_total = caps_total_frames;
    a.n_caps = n_caps;
    a.n_avatars = n_avatars;
    a.clip_first = clip_first;
    a.clip_frames = clip_frames;
    a.frame_pos = frame_pos;
    a.clearance = clearance;
    a.nearest = nearest;
    a.step_gap = step_gap;
    a.blocked = blocked;
    hipError_t e = gs::launch_capsule_queries(a, (hipStream_t)stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_capsule_queries");
}

gs_status gs_sensor_compose(int32_t n_views, int32_t height, int32_t width, const float *rgb, const float *depth,
                            const float *alpha, const uint8_t *mesh_rgba, const float *mesh_depth,
                            uint8_t *out_rgba, float *out_depth, gs_stream_t stream) {
    clear_error();
    if (n_views < 0 || height < 1 || width < 1 || height > (1 << 16) || width > (1 << 16))
        return fail(GS_ERR_INVALID_ARGUMENT, "n_views=%d height=%d width=%d invalid", n_views, height, width);
    if (n_views == 0) return GS_OK;
    if (!rgb || !depth || !alpha || !out_rgba || !out_depth)
        return fail(GS_ERR_INVALID_ARGUMENT, "NULL array");
    if ((mesh_rgba == nullptr) != (mesh_depth == nullptr))
        return fail(GS_ERR_INVALID_ARGUMENT, "mesh_rgba and mesh_depth must both be given or both be NULL");
    const void *arrays[7] = {rgb, depth, alpha, mesh_rgba, mesh_depth, out_rgba, out_depth};
    bool vec4 = true;
    for (const void *q : arrays) {
        if (q && !aligned(q, 4)) return fail(GS_ERR_INVALID_ARGUMENT, "arrays need 4-byte alignment");
        if (q && !aligned(q, 16)) vec4 = false;
    }
    gs::SensorArgs a = {};
    a.n_px = (int64_t)n_views * height * width;
    if (a.n_px > ((int64_t)1 << 38))  // keeps the one-pixel-per-thread grid within 2^30 workgroups
        return fail(GS_ERR_INVALID_ARGUMENT, "%lld pixels: too many for one call", (long long)a.n_px);
    a.rgb = rgb;
    a.depth = depth;
    a.alpha = alpha;
    a.mesh_rgba = reinterpret_cast<const uint32_t *>(mesh_rgba);
    a.mesh_depth = mesh_depth;
    a.out_rgba = reinterpret_cast<uint32_t *>(out_rgba);
    a.out_depth = out_depth;
    hipError_t e = gs::launch_sensor(a, vec4, (hipStream_t)stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_sensor_compose");
}

}  // extern "C"
