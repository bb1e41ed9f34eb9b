// gs_sensor_compose kernel: the sensor hand-off after compositing.
//
// Per pixel it turns the compositing outputs into the observation the RGB
// and depth sensors deliver (8-bit RGBA, metric depth) and, when a mesh pass
// is given, keeps the nearer of the 3DGS and the mesh fragment (Sec. 3.2).
// The kernel streams 20 B in (28 B with a mesh pass) and 8 B out per pixel,
// so it is HBM-bound: each thread handles four consecutive pixels with
// 16-B loads and stores when every array is 16-B aligned (the usual case for
// whole tensors), one pixel at a time otherwise.
#include "gs_internal.hpp"

namespace gs {

// One 8-bit code of a colour channel: clamp to [0, 1] (NaN -> 0), scale by
// 255 and round to nearest even, all in FP32.
__device__ __forceinline__ uint32_t channel_code(float c) {
    const float s = c > 0.0f ? fminf(c, 1.0f) : 0.0f;
    return (uint32_t)__builtin_rintf(s * 255.0f);
}

// The observation of one pixel: packed RGBA bytes (R in the low byte) and
// metric depth.
__device__ __forceinline__ void sensor_pixel(float r, float g, float b, float d, float al, bool has_mesh,
                                             uint32_t mesh_rgba, float mesh_d, uint32_t &out_rgba, float &out_d) {
    const bool gs_frag = al > 0.0f;
    const float dg = gs_frag ? d / al : 0.0f;
    const bool mesh_frag = has_mesh && mesh_d > 0.0f;  // NaN: no fragment
    const bool keep_gs = gs_frag && !(mesh_frag && !(dg < mesh_d));
    if (mesh_frag && !keep_gs) {
        out_rgba = mesh_rgba;
        out_d = mesh_d;
    } else {
        out_rgba = channel_code(r) | (channel_code(g) << 8) | (channel_code(b) << 16) | 0xff000000u;
        out_d = dg;
    }
}

template <bool MESH>
__global__ void __launch_bounds__(256) sensor_vec4_kernel(const SensorArgs a) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t p0 = 4 * i;
    if (p0 >= a.n_px) return;
    if (p0 + 4 <= a.n_px) {
        const float4 *rgb4 = reinterpret_cast<const float4 *>(a.rgb) + 3 * i;
        const float4 c0 = rgb4[0], c1 = rgb4[1], c2 = rgb4[2];
        const float4 d = reinterpret_cast<const float4 *>(a.depth)[i];
        const float4 al = reinterpret_cast<const float4 *>(a.alpha)[i];
        uint4 m = make_uint4(0u, 0u, 0u, 0u);
        float4 md = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (MESH) {
            m = reinterpret_cast<const uint4 *>(a.mesh_rgba)[i];
            md = reinterpret_cast<const float4 *>(a.mesh_depth)[i];
        }
        uint4 o;
        float4 od;
        sensor_pixel(c0.x, c0.y, c0.z, d.x, al.x, MESH, m.x, md.x, o.x, od.x);
        sensor_pixel(c0.w, c1.x, c1.y, d.y, al.y, MESH, m.y, md.y, o.y, od.y);
        sensor_pixel(c1.z, c1.w, c2.x, d.z, al.z, MESH, m.z, md.z, o.z, od.z);
        sensor_pixel(c2.y, c2.z, c2.w, d.w, al.w, MESH, m.w, md.w, o.w, od.w);
        reinterpret_cast<uint4 *>(a.out_rgba)[i] = o;
        reinterpret_cast<float4 *>(a.out_depth)[i] = od;
        return;
    }
    for (int64_t p = p0; p < a.n_px; ++p) {  // the last one to three pixels
        uint32_t o;
        float od;
        sensor_pixel(a.rgb[3 * p], a.rgb[3 * p + 1], a.rgb[3 * p + 2], a.depth[p], a.alpha[p], MESH,
                     MESH ? a.mesh_rgba[p] : 0u, MESH ? a.mesh_depth[p] : 0.0f, o, od);
        a.out_rgba[p] = o;
        a.out_depth[p] = od;
    }
}

template <bool MESH>
__global__ void __launch_bounds__(256) sensor_scalar_kernel(const SensorArgs a) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= a.n_px) return;
    uint32_t o;
    float od;
    sensor_pixel(a.rgb[3 * p], a.rgb[3 * p + 1], a.rgb[3 * p + 2], a.depth[p], a.alpha[p], MESH,
                 MESH ? a.mesh_rgba[p] : 0u, MESH ? a.mesh_depth[p] : 0.0f, o, od);
    a.out_rgba[p] = o;
    a.out_depth[p] = od;
}

hipError_t launch_sensor(const SensorArgs &a, bool vec4, hipStream_t s) {
    if (a.n_px <= 0) return hipSuccess;
    const bool mesh = a.mesh_rgba != nullptr;
    if (vec4) {
        const unsigned grid = (unsigned)((a.n_px + 1023) / 1024);
        return mesh ? launch_kernel(sensor_vec4_kernel<true>, dim3(grid), dim3(256), s, a)
                    : launch_kernel(sensor_vec4_kernel<false>, dim3(grid), dim3(256), s, a);
    }
    const unsigned grid = (unsigned)((a.n_px + 255) / 256);
    return mesh ? launch_kernel(sensor_scalar_kernel<true>, dim3(grid), dim3(256), s, a)
                : launch_kernel(sensor_scalar_kernel<false>, dim3(grid), dim3(256), s, a);
}

}  // namespace gs
