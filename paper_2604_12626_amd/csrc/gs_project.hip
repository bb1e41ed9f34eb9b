// gs_project kernel: per (view, Gaussian) EWA projection, SH colour and tile
// rect.  One thread per Gaussian of a segment; the thread reads the
// Gaussian's attributes once and projects it into every view of the launch
// (the cameras are staged in LDS), so a scene drawn by many views is read from
// HBM once.  Attribute reads are row-per-Gaussian (means 12 B, scales 12 B,
// quats 16 B, SH 12 (D+1)^2 B contiguous), so a Gaussian culled in every view
// never pulls its SH rows (the 32 B of rotation, scales and opacity are read
// with the mean, to overlap their latency).  PLANES: the same reads from a
// segment stored component-major (plane k of an attribute at k n), where
// each load of a wave is one coalesced stretch of a plane.
#include "gs_ewa.hpp"

namespace gs {

template <int D, bool PLANES>
__global__ void __launch_bounds__(256) project_kernel(const ProjectArgs a) {
    constexpr int K = (D + 1) * (D + 1);
    __shared__ float s_cam[kProjViews * kCamStride];
    for (int k = threadIdx.x; k < a.nv * 16; k += 256) {
        const int vi = k >> 4, f = k & 15;
        s_cam[vi * kCamStride + f] = reinterpret_cast<const float *>(a.cams + a.view[vi])[f];
    }
    __syncthreads();
    for (int vi = threadIdx.x; vi < a.nv; vi += 256) {
        float *c = s_cam + vi * kCamStride;
        // camera centre -R^T t
#pragma unroll
        for (int j = 0; j < 3; ++j) c[16 + j] = -(c[j] * c[9] + c[3 + j] * c[10] + c[6 + j] * c[11]);
    }
    __syncthreads();

    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = a.seg.n;
    if (i >= n) return;
    // component k of Gaussian i in an attribute of w components
    auto at = [&](const float *p, int w, int k) { return PLANES ? p[(int64_t)k * n + i] : p[w * i + k]; };

    const float mx = at(a.seg.means, 3, 0), my = at(a.seg.means, 3, 1), mz = at(a.seg.means, 3, 2);
    // the small attribute rows (rotation, scales, opacity: 32 B) are requested
    // together with the mean, so their latency overlaps; the SH rows are read
    // only once the Gaussian is known to land in a view
    float4 q4 = make_float4(1.0f, 0.0f, 0.0f, 0.0f);
    float ls[3] = {0.0f, 0.0f, 0.0f};
    float S[6];
    if (a.seg.cov6) {
#pragma unroll
        for (int k = 0; k < 6; ++k) S[k] = at(a.seg.cov6, 6, k);
    } else {
        if (PLANES)
            q4 = make_float4(at(a.seg.quats, 4, 0), at(a.seg.quats, 4, 1), at(a.seg.quats, 4, 2), at(a.seg.quats, 4, 3));
        else
            q4 = reinterpret_cast<const float4 *>(a.seg.quats)[i];
#pragma unroll
        for (int k = 0; k < 3; ++k) ls[k] = at(a.seg.log_scales, 3, k);
    }
    const float opac = a.seg.opacity[i];
    // near-plane test from the mean alone: a Gaussian behind every camera of
    // the launch never reads its SH rows
    bool any_front = false;
    for (int vi = 0; vi < a.nv; ++vi) {
        const float *c = s_cam + vi * kCamStride;
        const float tz = c[6] * mx + c[7] * my + c[8] * mz + c[11];
        any_front |= tz > a.near_plane;
    }
    if (!any_front) {
        for (int vi = 0; vi < a.nv; ++vi) a.tiles_touched[a.base[vi] + i] = 0u;
        return;
    }
    if (!a.seg.cov6) {
        const Rot rot = quat_rot(q4.x, q4.y, q4.z, q4.w);
        float s[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) s[k] = expf(ls[k]);
        cov_from_rot_scale(rot.R, s, S);
    }
    if (!isfinite(opac)) {  // non-finite input is culled, never rendered
        for (int vi = 0; vi < a.nv; ++vi) a.tiles_touched[a.base[vi] + i] = 0u;
        return;
    }

    const float *shp = a.seg.sh + (PLANES ? (size_t)i : (size_t)(3 * K) * i);
    for (int vi = 0; vi < a.nv; ++vi) {
        const int64_t inst = a.base[vi] + i;
        const float *cam = s_cam + vi * kCamStride;
        ViewProj p;
        if (!ewa_project(cam, mx, my, mz, S, a.W, a.H, a.TX, a.TY, a.near_plane, a.lowpass, a.sigma_cut,
                         a.fov_clamp, p)) {
            a.tiles_touched[inst] = 0u;
            continue;
        }
        // view direction in world space, from the camera centre to the mean
        float dx = mx - cam[16], dy = my - cam[17], dz = mz - cam[18];
        const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
        dx *= inv;
        dy *= inv;
        dz *= inv;
        float Y[K];
        sh_basis<D>(dx, dy, dz, Y);
        // colour straight from the SH rows (16-B loads when the row allows;
        // later views of the same Gaussian hit the caches), accumulated per
        // channel in basis order
        float col[3] = {0.0f, 0.0f, 0.0f};
        if (PLANES) {
#pragma unroll
            for (int f = 0; f < 3 * K; ++f) col[f % 3] += Y[f / 3] * shp[(int64_t)f * n];
        } else if ((3 * K) % 4 == 0) {
#pragma unroll
            for (int k4 = 0; k4 < 3 * K / 4; ++k4) {
                const float4 t = reinterpret_cast<const float4 *>(shp)[k4];
                const float v4[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int f = 4 * k4 + m;  // coefficient f = 3 k + ch
                    col[f % 3] += Y[f / 3] * v4[m];
                }
            }
        } else {
#pragma unroll
            for (int f = 0; f < 3 * K; ++f) col[f % 3] += Y[f / 3] * shp[f];
        }
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) col[ch] = fmaxf(col[ch] + 0.5f, 0.0f);
        float4 *r = a.rec + 3 * inst;
        r[0] = make_float4(p.u, p.v, p.tz, __int_as_float(p.radius));
        r[1] = make_float4(p.A, p.B, p.C, opac);
        r[2] = make_float4(col[0], col[1], col[2], __int_as_float(a.view[vi]));
        a.tiles_touched[inst] = (uint32_t)((p.rect.x1 - p.rect.x0) * (p.rect.y1 - p.rect.y0));
    }
}

hipError_t launch_project(const ProjectArgs &a, hipStream_t s) {
    if (a.seg.n == 0 || a.nv == 0) return hipSuccess;
    const unsigned grid = (unsigned)((a.seg.n + 255) / 256);
    if (a.seg.layout == GS_LAYOUT_PLANES) {
        switch (a.seg.sh_degree) {
            case 0: return launch_kernel(project_kernel<0, true>, dim3(grid), dim3(256), s, a);
            case 1: return launch_kernel(project_kernel<1, true>, dim3(grid), dim3(256), s, a);
            case 2: return launch_kernel(project_kernel<2, true>, dim3(grid), dim3(256), s, a);
            default: return launch_kernel(project_kernel<3, true>, dim3(grid), dim3(256), s, a);
        }
    }
    switch (a.seg.sh_degree) {
        case 0: return launch_kernel(project_kernel<0, false>, dim3(grid), dim3(256), s, a);
        case 1: return launch_kernel(project_kernel<1, false>, dim3(grid), dim3(256), s, a);
        case 2: return launch_kernel(project_kernel<2, false>, dim3(grid), dim3(256), s, a);
        default: return launch_kernel(project_kernel<3, false>, dim3(grid), dim3(256), s, a);
    }
}

}  // namespace gs
