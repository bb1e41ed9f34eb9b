// gs_composite kernel: per-tile front-to-back alpha compositing.
//
// A persistent grid of 256-thread workgroups pops (view, tile) work items
// from an atomic counter.  Each wave64 owns one 8 x 8 quadrant of the 16 x 16
// tile (one pixel per lane).  The workgroup walks the tile's sorted list in
// batches of 256 entries: every thread gathers one 48-B record into LDS
// (3 x float4) and marks which quadrants the entry can reach (a conservative
// bound of the region where alpha >= alpha_min); then each wave compacts the
// batch to the entries that reach its quadrant with four ballots and
// evaluates only those, in list order.  A pixel stops at the transmittance
// threshold; the workgroup leaves the list once all 256 pixels have stopped.
#include "gs_internal.hpp"

namespace gs {

constexpr int kBatch = 256;

__global__ void __launch_bounds__(kTilePixels) composite_kernel(const CompositeArgs a) {
    __shared__ int64_t s_item;
    __shared__ float4 s_e0[kBatch], s_e1[kBatch], s_e2[kBatch];
    __shared__ uint8_t s_mask[kBatch];
    __shared__ uint8_t s_list[4][kBatch];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int lx, ly;
    tile_pixel(tid, lx, ly);
    while (true) {
        if (tid == 0) s_item = (int64_t)atomicAdd(a.counter, 1u);
        __syncthreads();
        const int64_t item = s_item;
        if (item >= a.n_items) break;
        const int view = (int)(item / a.T);
        const int tile = (int)(item - (int64_t)view * a.T);
        const int tx0 = (tile % a.TX) * kTile, ty0 = (tile / a.TX) * kTile;
        const int px = tx0 + lx, py = ty0 + ly;
        const bool inside = px < a.W && py < a.H;
        const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
        const uint2 range = a.ranges[item];
        float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f, dd = 0.0f;
        uint32_t last = 0;
        bool done = !inside;
        for (uint32_t b0 = range.x; b0 < range.y; b0 += kBatch) {
            const int nb = (int)min((uint32_t)kBatch, range.y - b0);
            if (tid < nb) {
                const uint32_t g = a.vals[b0 + tid];
                const float4 q0 = a.rec[3 * (size_t)g], q1 = a.rec[3 * (size_t)g + 1], q2 = a.rec[3 * (size_t)g + 2];
                const Entry e = make_entry(q0, q1, q2);
                s_e0[tid] = make_float4(e.u, e.v, e.a, e.b);
                s_e1[tid] = make_float4(e.c, e.o, e.z, e.r);
                s_e2[tid] = make_float4(e.g, e.bl, 0.0f, 0.0f);
                s_mask[tid] = (uint8_t)entry_quadrant_mask(q0.x, q0.y, q1.x, q1.y, q1.z, q1.w, a.alpha_min,
                                                           (float)tx0, (float)ty0);
            }
            __syncthreads();
            // this wave's entries of the batch, in list order
            int cnt = 0;
#pragma unroll
            for (int c = 0; c < kBatch / 64; ++c) {
                const int j = c * 64 + lane;
                const bool hit = j < nb && ((s_mask[j] >> wave) & 1u);
                const uint64_t bal = __ballot(hit);
                if (hit) s_list[wave][cnt + __popcll(bal & lt_mask)] = (uint8_t)j;
                cnt += __popcll(bal);
            }
            __builtin_amdgcn_wave_barrier();
            if (!done) {
                for (int q = 0; q < cnt; ++q) {
                    const int k = s_list[wave][q];
                    const float4 e0 = s_e0[k], e1 = s_e1[k];
                    const float dx = fx - e0.x, dy = fy - e0.y;
                    const float p2 = entry_power2(e0.z, e0.w, e1.x, dx, dy);
                    const float al = fminf(a.alpha_max, e1.y * exp2f(p2));
                    if (al < a.alpha_min) continue;
                    const float Tn = T * (1.0f - al);
                    if (Tn < a.t_min) {
                        done = true;
                        break;
                    }
                    const float4 e2 = s_e2[k];
                    const float w = al * T;
                    cr += w * e1.w;
                    cg += w * e2.x;
                    cb += w * e2.y;
                    dd += w * e1.z;
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
