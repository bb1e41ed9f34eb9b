// gs_composite kernel: per-tile front-to-back alpha compositing.
//
// A persistent grid of 256-thread workgroups (one thread per pixel of a
// 16 x 16 tile, four wave64) pops (view, tile) work items from an atomic
// counter.  For each item the workgroup walks the tile's sorted list in
// batches of 256 entries: every thread gathers one record (48 B) into LDS,
// then every pixel thread evaluates the batch from LDS.  A pixel stops at the
// transmittance threshold; the workgroup leaves the list as soon as all 256
// pixels have stopped (a block-wide count after each batch).
#include "gs_internal.hpp"

namespace gs {



constexpr int kBatch = 256;

__global__ void __launch_bounds__(kTilePixels) composite_kernel(const CompositeArgs a) {
    __shared__ int64_t s_item;
    __shared__ float s_u[kBatch], s_v[kBatch], s_a[kBatch], s_b[kBatch], s_c[kBatch], s_o[kBatch], s_z[kBatch],
        s_r[kBatch], s_g[kBatch], s_bl[kBatch];
    const int tid = threadIdx.x;
    const int lx = tid & (kTile - 1), ly = tid >> 4;
    while (true) {
        if (tid == 0) s_item = (int64_t)atomicAdd(a.counter, 1u);
        __syncthreads();
        const int64_t item = s_item;
        if (item >= a.n_items) break;
        const int view = (int)(item / a.T);
        const int tile = (int)(item - (int64_t)view * a.T);
        const int px = (tile % a.TX) * kTile + lx;
        const int py = (tile / a.TX) * kTile + ly;
        const bool inside = px < a.W && py < a.H;
        const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
        const uint2 range = a.ranges[item];
        float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f, dd = 0.0f;
        uint32_t last = 0;
        bool done = !inside;
        for (uint32_t b0 = range.x; b0 < range.y; b0 += kBatch) {
            const uint32_t j = b0 + tid;
            if (j < range.y) {
                const uint32_t g = a.vals[j];
                const float4 q0 = a.rec[3 * (size_t)g], q1 = a.rec[3 * (size_t)g + 1], q2 = a.rec[3 * (size_t)g + 2];
                const Entry e = make_entry(q0, q1, q2);
                s_u[tid] = e.u;
                s_v[tid] = e.v;
                s_a[tid] = e.a;
                s_b[tid] = e.b;
                s_c[tid] = e.c;
                s_o[tid] = e.o;
                s_z[tid] = e.z;
                s_r[tid] = e.r;
                s_g[tid] = e.g;
                s_bl[tid] = e.bl;
            }
            __syncthreads();
            const int nb = (int)min((uint32_t)kBatch, range.y - b0);
            if (!done) {
                for (int k = 0; k < nb; ++k) {
                    const float dx = fx - s_u[k], dy = fy - s_v[k];
                    const float p2 = entry_power2(s_a[k], s_b[k], s_c[k], dx, dy);
                    const float al = fminf(a.alpha_max, s_o[k] * exp2f(p2));
                    if (al < a.alpha_min) continue;
                    const float Tn = T * (1.0f - al);
                    if (Tn < a.t_min) {
                        done = true;
                        break;
                    }
                    const float w = al * T;
                    cr += w * s_r[k];
                    cg += w * s_g[k];
                    cb += w * s_bl[k];
                    dd += w * s_z[k];
                    T = Tn;
                    last = b0 - range.x + (uint32_t)k + 1u;
                }
            }
            const int n_done = __syncthreads_count(done);
            if (n_done == kTilePixels) break;
        }
        if (inside) {
            const size_t pix = ((size_t)view * a.H + py) * a.W + px;
            a.rgb[3 * pix + 0] = cr + T * a.bg0;
            a.rgb[3 * pix + 1] = cg + T * a.bg1;
            a.rgb[3 * pix + 2] = cb + T * a.bg2;
            a.depth[pix] = dd;
            a.alpha[pix] = 1.0f - T;
            if (a.t_final) a.t_final[pix] = T;
            if (a.n_contrib) a.n_contrib[pix] = last;
        }
        __syncthreads();
    }
}

hipError_t launch_composite(const CompositeArgs &a, int grid, hipStream_t s) {
    if (a.n_items == 0) return hipSuccess;
    return launch_kernel(composite_kernel, dim3(grid), dim3(kTilePixels), s, a);
}

}  // namespace gs
