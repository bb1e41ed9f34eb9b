// gs_render_backward kernels.
//
// B1 (per tile, 256 threads = one per pixel, each wave an independent 8 x 8
// quadrant with no workgroup barrier): walks the tile's list back to front
// from the last composited entry of the quadrant, 64 entries at a time,
// recomputing each alpha with exactly the forward's FP32 expression (so every
// skip/stop/clamp decision repeats), recovering the transmittance by
// T_i = T_{i+1} / (1 - alpha_i), and forming the screen-space adjoint of each
// entry (u, v, conic, opacity, colour, depth).  Entries that cannot reach a
// wave's quadrant are dropped by the same conservative bound as the forward;
// per remaining entry the 64 lanes are summed with DPP adds and the last
// lane issues the global float atomics (skipped when no lane contributed).
// With the forward's segment checkpoints a list is cut into segments of
// kSegment entries (a multiple of that for lists longer than kMaxSegments
// segments), popped by a persistent grid, every segment's walk starting from
// the transmittance and the normalised colour still to come that the forward
// recorded at its end; the last segment of a list starts from t_final and
// the background, as the whole list does without them.
//
// B2 (per Gaussian of a segment, scene-major): chains the screen-space
// adjoints of every view that drew the Gaussian through the projection to the
// 3D parameters and writes the dense gradients once (no atomics).  A first
// pass over the segment (B2a) writes zeros plane by plane and lists the
// Gaussians a view of the launch draws; the chain (B2b) then runs over that
// list only.
#include "gs_ewa.hpp"

namespace gs {




// Sum over the wave, complete in lane 63 only, with DPP lane moves fused
// into the adds (no LDS traffic): pairs, quads, half rows, rows (these leave
// every lane of a 16-lane row holding the row sum), then row 0 into row 1
// and row 2 into row 3, then rows 0-1 into row 3.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v) {
    // rows outside ROW_MASK add `old` = 0
    return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

__device__ __forceinline__ float wave_sum_to_last(float v) {
    v = dpp_add<0xB1, 0xF>(v);   // quad_perm [1, 0, 3, 2]
    v = dpp_add<0x4E, 0xF>(v);   // quad_perm [2, 3, 0, 1]
    v = dpp_add<0x141, 0xF>(v);  // row_half_mirror
    v = dpp_add<0x140, 0xF>(v);  // row_mirror
    v = dpp_add<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// zeros for p[0, n) by the whole grid: 16-byte stores on the 16-byte aligned
// stretch, the single floats at its ends by workgroup 0
__device__ __forceinline__ void zero_span_grid(float *p, int64_t n) {
    const uint64_t base = (uint64_t)(uintptr_t)p;  // 4-byte aligned (floats)
    int64_t v0 = 0, v1 = n;
    while (((base + 4u * (uint64_t)v0) & 15u) && v0 < n) ++v0;
    while (((base + 4u * (uint64_t)v1) & 15u) && v1 > v0) --v1;
    if (blockIdx.x == 0) {
        for (int64_t f = threadIdx.x; f < v0; f += blockDim.x) p[f] = 0.0f;
        for (int64_t f = v1 + threadIdx.x; f < n; f += blockDim.x) p[f] = 0.0f;
    }
    float4 *q = reinterpret_cast<float4 *>(p + v0);
    const int64_t m = (v1 - v0) / 4, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += stride)
        q[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// SEG: the work is the listed (tile, segment) pairs (checkpoint mode); else
// one whole list per workgroup, its quadrant sums through LDS (WLDS) or
// added to HBM by each wave.  Bounded to five waves per SIMD (a few
// registers spill): the walk is bound by latency, so one more workgroup in
// flight per CU pays.
template <bool SEG, bool WLDS>
__global__ void __launch_bounds__(kTilePixels, 5) backward_tile_kernel(const BackwardTileArgs a) {
    constexpr bool kLds = SEG || WLDS;
    __shared__ float4 s_e0[4][64], s_e1[4][64], s_e2[4][64], s_q[4][64];
    // 64 list positions: each quadrant wave stores its per-entry sums in its
    // own row, and the workgroup then adds the four rows in FP64 in a fixed
    // order and issues one set of global atomics per entry (instead of one
    // per quadrant)
    __shared__ float s_acc[4][kLds ? kSegment * kG2D : 1];
    __shared__ uint32_t s_gid[kLds ? kSegment : 1];
    __shared__ uint32_t s_top;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    float4 *e0s = s_e0[wave], *e1s = s_e1[wave], *e2s = s_e2[wave], *qs = s_q[wave];
    // work: a (view, tile) list, or with checkpoints one segment of one (the
    // listed pairs, popped by a persistent grid); wave w owns the 8 x 8
    // quadrant w, one pixel per lane
    const uint32_t n_work = a.seg_list ? a.seg_list[0] : (uint32_t)a.n_items;
    if (kLds) {
        for (int i = threadIdx.x; i < 4 * kSegment * kG2D; i += kTilePixels) (&s_acc[0][0])[i] = 0.0f;
        __syncthreads();
    }
    for (uint32_t wk = blockIdx.x; wk < n_work; wk += a.n_groups) {
    const uint32_t entry = a.seg_list ? a.seg_list[1 + wk] : 0u;
    // whole lists with the work order: workgroup wk takes entry wk / 8 of
    // queue wk mod 8 (queue q holds the lists t = q mod 8, longest first, so
    // this maps the workgroups one to one onto the lists)
    const int64_t item = a.seg_list ? (int64_t)(entry >> 6)
                         : a.order  ? (int64_t)a.order[(int64_t)(wk % kOrderQueues) * order_stride(a.n_items) +
                                                       wk / kOrderQueues]
                                    : (int64_t)wk;
    const uint32_t s = a.seg_list ? (entry & 63u) : 0u;
    const int view = (int)(item / a.T);
    const int tile = (int)(item - (int64_t)view * a.T);
    const int qx0 = (tile % a.TX) * kTile + ((wave & 1) << 3);
    const int qy0 = (tile / a.TX) * kTile + ((wave >> 1) << 3);
    const int px = qx0 + (lane & 7), py = qy0 + (lane >> 3);
    const bool inside = px < a.W && py < a.H;
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    const float bx0 = (float)qx0 + 0.5f, by0 = (float)qy0 + 0.5f;
    const uint2 range = a.ranges[item];
    const uint32_t L = range.y - range.x;
    // this segment [seg_lo, seg_lo + seg_len) of list positions: all of them
    // without checkpoints, else segment s of the list's segments (kSegment
    // entries each, or a multiple of that for lists of more than
    // kMaxSegments * kSegment entries)
    static_assert(kSegment == 64 && kMaxSegments <= 64, "six bits name a segment; a chunk is 64 entries");
    const uint32_t seg_len = a.seg_list ? seg_len_of(L) : L;
    const uint32_t seg_lo = a.seg_list ? s * seg_len : 0u;
    const bool last_seg = !a.seg_list || seg_lo + seg_len >= L;
    // A one-chunk middle segment's list values, records and end checkpoint
    // are requested before the pixel state, so that the gather overlaps those
    // loads (requests past what the walk needs are harmless: positions below
    // the list length, slots inside the buffer).
    // A middle segment whose end checkpoint lies past the buffer (sized for a
    // smaller capacity than the binning's) walks from the end of the list,
    // where t_final and the background give the state, and adds only its own
    // entries: the same gradients, slower.
    const uint64_t slot = (range.x + seg_lo + seg_len) / kSegment;
    const bool from_end = !last_seg && slot >= a.ckpt_slots;
    const bool middle = !last_seg && !from_end;
    const bool pre = middle && seg_len == kSegment;
    uint32_t g_pre = 0;
    float4 p0 = make_float4(0.f, 0.f, 0.f, 0.f), p1 = p0, p2 = p0;
    if (pre && seg_lo + lane < L) {
        g_pre = a.vals[range.x + seg_lo + lane];
        p0 = a.rec[3 * (size_t)g_pre];
        p1 = a.rec[3 * (size_t)g_pre + 1];
        p2 = a.rec[3 * (size_t)g_pre + 2];
    }
    const bool ck_ok = middle;
    float ck[kCkptVals] = {1.0f, a.bg0, a.bg1, a.bg2, 0.0f};
    if (ck_ok) {
#pragma unroll
        for (int v = 0; v < kCkptVals; ++v) ck[v] = a.ckpt[ckpt_index(slot, wave, v, lane)];
    }

    float T = 1.0f, Tfin = 1.0f;
    uint32_t last = 0;
    float dR = 0.f, dG = 0.f, dB = 0.f, dD = 0.f, dA = 0.f;
    if (inside) {
        const size_t pix = ((size_t)view * a.H + py) * a.W + px;
        Tfin = a.t_final[pix];
        T = Tfin;
        last = a.n_contrib[pix];
        if (a.d_rgb) {
            dR = a.d_rgb[3 * pix];
            dG = a.d_rgb[3 * pix + 1];
            dB = a.d_rgb[3 * pix + 2];
        }
        if (a.d_depth) dD = a.d_depth[pix];
        if (a.d_alpha) dA = a.d_alpha[pix];
    }
    uint32_t maxlast = last;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) maxlast = max(maxlast, (uint32_t)__shfl_xor((int)maxlast, off, 64));
    maxlast = min(maxlast, L);
    const uint32_t seg_end = (last_seg || from_end) ? maxlast : seg_lo + seg_len;  // state known here
    const uint32_t own_hi = from_end ? seg_lo + seg_len : seg_end;  // entries this walk adds
    const uint32_t seg_hi = seg_end < maxlast ? seg_end : maxlast;
    // Per-entry sums over the four quadrant waves go through LDS, 64 list
    // positions at a time, for segments of at most 64 entries (every middle
    // one, and a last one that short) and, when the launch has many lists,
    // for whole lists: all waves walk the same chunks, from `top` down, and
    // after each chunk the workgroup issues one global atomic per nonzero
    // (entry, value).  Otherwise (a longer last segment, or a few long whole
    // lists, where waves walking in step would wait for each other) each
    // wave adds to HBM directly, with no barrier.  Uniform per workgroup.
    const bool lds_sum = SEG ? (middle || L <= seg_lo + (uint32_t)kSegment) : WLDS;
    if (!lds_sum && seg_lo >= seg_hi) continue;
    uint32_t top = seg_hi;
    if (lds_sum) {
        if (SEG) {
            top = min(seg_lo + seg_len, L);
        } else {  // the longest walk of the four quadrants
            if (threadIdx.x == 0) s_top = 0u;
            __syncthreads();
            if (lane == 0) atomicMax(&s_top, seg_hi);
            __syncthreads();
            top = s_top;
        }
    }
    {
    // suffix colour / depth behind the current entry over its transmittance:
    // the background at the end of the walk, else the checkpoint at seg_end
    float Sr = a.bg0, Sg = a.bg1, Sb = a.bg2, Sd = 0.0f;
    if (seg_end < maxlast && ck_ok) {
        T = ck[0];
        Sr = ck[1];
        Sg = ck[2];
        Sb = ck[3];
        Sd = ck[4];
    }

    // chunks [lo, hi) of list positions, from the back (this wave's entries
    // end at seg_hi)
    for (int64_t hi = (int64_t)top; hi > (int64_t)seg_lo; hi -= 64) {
        const int64_t lo = hi - 64 > (int64_t)seg_lo ? hi - 64 : (int64_t)seg_lo;
        const bool valid = lo + lane < min(hi, (int64_t)seg_hi);
        bool hit = false;
        float4 q0, q1, q2;
        uint32_t g = 0;
        if (valid) {
            if (pre) {  // the one chunk of a middle segment, requested up front
                g = g_pre;
                q0 = p0;
                q1 = p1;
                q2 = p2;
            } else {
                g = a.vals[range.x + (uint32_t)lo + lane];
                q0 = a.rec[3 * (size_t)g];
                q1 = a.rec[3 * (size_t)g + 1];
                q2 = a.rec[3 * (size_t)g + 2];
            }
            hit = entry_reaches_box(q0.x, q0.y, q1.x, q1.y, q1.z, q1.w, a.alpha_min, bx0, by0, bx0 + 7.0f,
                                    by0 + 7.0f);
        }
        const uint64_t bal = __ballot(hit);
        if (hit) {
            const int pos = __popcll(bal & lt_mask);
            const Entry e = make_entry(q0, q1, q2);
            e0s[pos] = make_float4(e.u, e.v, e.a, e.b);
            e1s[pos] = make_float4(e.c, e.o, e.z, e.r);
            e2s[pos] = make_float4(e.g, e.bl, __uint_as_float(g), __uint_as_float((uint32_t)(lo + lane)));
            qs[pos] = make_float4(q1.x, q1.y, q1.z, 0.0f);
        }
        __builtin_amdgcn_wave_barrier();
        const int n = __popcll(bal);
        for (int q = n - 1; q >= 0; --q) {
            const float4 e0 = e0s[q], e1 = e1s[q], e2 = e2s[q];
            const uint32_t pos = __float_as_uint(e2.w);  // list position (< maxlast <= list length)
            float gu = 0.f, gv = 0.f, gA = 0.f, gB = 0.f, gC = 0.f, go = 0.f, gr = 0.f, gg = 0.f, gb = 0.f, gz = 0.f;
            bool contrib = false;
            if (pos < last) {
                const float dx = fx - e0.x, dy = fy - e0.y;
                const float p2 = entry_power2(e0.z, e0.w, e1.x, dx, dy);
                const float G = fast_exp2(p2);
                const float oG = e1.y * G;
                const float al = fminf(a.alpha_max, oG);
                if (!(al < a.alpha_min)) {
                    contrib = true;
                    const float one_m = 1.0f - al;
                    const float r_one_m = __builtin_amdgcn_rcpf(one_m);  // 1 ulp reciprocal (one_m >= 0.01)
                    T = T * r_one_m;  // transmittance in front of this entry
                    const float w = al * T;
                    gr = dR * w;
                    gg = dG * w;
                    gb = dB * w;
                    gz = dD * w;
                    const float dal = T * (dR * (e1.w - Sr) + dG * (e2.x - Sg) + dB * (e2.y - Sb) +
                                           dD * (e1.z - Sd)) +
                                      dA * Tfin * r_one_m;
                    if (!(oG > a.alpha_max)) {
                        const float4 cq = qs[q];
                        go = dal * G;
                        // dL/dP with P the natural-log exponent (dG/dP = G)
                        const float dP = dal * e1.y * G;
                        gu = dP * (cq.x * dx + cq.y * dy);
                        gv = dP * (cq.y * dx + cq.z * dy);
                        gA = -0.5f * dP * dx * dx;
                        gB = -dP * dx * dy;
                        gC = -0.5f * dP * dy * dy;
                    }
                    Sr = al * e1.w + one_m * Sr;
                    Sg = al * e2.x + one_m * Sg;
                    Sb = al * e2.y + one_m * Sb;
                    Sd = al * e1.z + one_m * Sd;
                }
            }
            contrib = contrib && pos < own_hi;  // uniform: a walk from the end passes others' entries
            if (__ballot(contrib) == 0ull) continue;
            gu = wave_sum_to_last(gu);
            gv = wave_sum_to_last(gv);
            gA = wave_sum_to_last(gA);
            gB = wave_sum_to_last(gB);
            gC = wave_sum_to_last(gC);
            go = wave_sum_to_last(go);
            gr = wave_sum_to_last(gr);
            gg = wave_sum_to_last(gg);
            gb = wave_sum_to_last(gb);
            gz = wave_sum_to_last(gz);
            if (kLds && lds_sum) {
                if (lane == 63) {
                    float *acc = s_acc[wave] + (pos - (uint32_t)lo) * kG2D;
                    s_gid[pos - (uint32_t)lo] = __float_as_uint(e2.z);
                    acc[kGU] = gu;
                    acc[kGV] = gv;
                    acc[kGA] = gA;
                    acc[kGB] = gB;
                    acc[kGC] = gC;
                    acc[kGO] = go;
                    acc[kGR] = gr;
                    acc[kGG] = gg;
                    acc[kGBl] = gb;
                    acc[kGZ] = gz;
                }
            } else if (lane == 63) {
                double *dst = a.g2d + (size_t)__float_as_uint(e2.z) * kG2D;
                atomicAdd(dst + kGU, (double)gu);
                atomicAdd(dst + kGV, (double)gv);
                atomicAdd(dst + kGA, (double)gA);
                atomicAdd(dst + kGB, (double)gB);
                atomicAdd(dst + kGC, (double)gC);
                atomicAdd(dst + kGO, (double)go);
                atomicAdd(dst + kGR, (double)gr);
                atomicAdd(dst + kGG, (double)gg);
                atomicAdd(dst + kGBl, (double)gb);
                atomicAdd(dst + kGZ, (double)gz);
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (kLds && lds_sum) {
            // every quadrant has added its sums for this chunk: one global
            // atomic per nonzero (entry, value), and the accumulator is cleared
            __syncthreads();
            for (int i = threadIdx.x; i < kSegment * kG2D; i += kTilePixels) {
                const double v = (((double)s_acc[0][i] + (double)s_acc[1][i]) + (double)s_acc[2][i]) + (double)s_acc[3][i];
                if (v != 0.0) atomicAdd(a.g2d + (size_t)s_gid[i / kG2D] * kG2D + (i % kG2D), v);
#pragma unroll
                for (int q = 0; q < 4; ++q) s_acc[q][i] = 0.0f;
            }
            __syncthreads();
        }
    }
    }  // this wave's walk
    }  // work loop
    // the dense gradient planes, cleared by each workgroup once its walks
    // are done (their stores drain while later workgroups still walk)
    for (int z = 0; z < a.n_zero; ++z) zero_span_grid(a.zero_ptr[z], a.zero_n[z]);
}

// The backward's work list, built by one workgroup of NT threads: for every
// (view, tile) list of L > 0 entries its ceil(L / seg_len_of(L)) <=
// kMaxSegments segments, as (item << 6 | segment) in item order, after their
// count; at most `cap`.
// lists up to which the accumulator clear's first workgroup (256 threads)
// builds the segment list; more get a 1024-thread launch of their own
constexpr int64_t kListInClear = 2048;
template <int NT>
__device__ __forceinline__ void build_segment_list(const uint2 *ranges, int64_t n_items, uint32_t *list,
                                                   uint64_t cap) {
    __shared__ uint32_t s_w[NT / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t per = (n_items + NT - 1) / NT;
    const int64_t t0 = (int64_t)tid * per, t1 = (t0 + per < n_items) ? t0 + per : n_items;
    auto n_seg = [](uint2 r) -> uint32_t {
        const uint32_t L = r.y - r.x;
        return (L + seg_len_of(L) - 1u) / seg_len_of(L);
    };
    uint32_t cnt = 0u;
    for (int64_t t = t0; t < t1; ++t) cnt += n_seg(ranges[t]);
    uint32_t incl = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    uint64_t pos = incl - cnt, total = 0u;
    for (int k = 0; k < NT / 64; ++k) {
        if (k < wave) pos += s_w[k];
        total += s_w[k];
    }
    for (int64_t t = t0; t < t1; ++t) {
        const uint32_t c = n_seg(ranges[t]);
        for (uint32_t q = 0; q < c; ++q, ++pos)
            if (pos < cap) list[1 + pos] = ((uint32_t)t << 6) | q;
    }
    if (tid == 0) list[0] = (uint32_t)(total < cap ? total : cap);
}

// the segment list of a launch with many lists: one 1024-thread workgroup
__global__ void __launch_bounds__(1024) segment_list_kernel(const uint2 *ranges, int64_t n_items, uint32_t *list,
                                                            uint64_t cap) {
    build_segment_list<1024>(ranges, n_items, list, cap);
}

hipError_t launch_backward_tiles(BackwardTileArgs a, int n_cu, hipStream_t s) {
    if (a.n_items == 0) return hipSuccess;
    if (!a.seg_list) {  // one workgroup per list
        a.n_groups = (uint32_t)a.n_items;
        // many lists (more than the GPU holds at once): fewer global atomics
        // pay for the waves of a tile walking in step; few long lists: not
        if (a.n_items >= 2048)
            return launch_kernel(backward_tile_kernel<false, true>, dim3((unsigned)a.n_items), dim3(kTilePixels), s,
                                 a);
        return launch_kernel(backward_tile_kernel<false, false>, dim3((unsigned)a.n_items), dim3(kTilePixels), s, a);
    }
    // the work list: built by the accumulator clear for up to kListInClear
    // lists, else here
    if (a.n_items > kListInClear) {
        const hipError_t e = launch_kernel(segment_list_kernel, dim3(1), dim3(1024), s, a.ranges, a.n_items,
                                           a.seg_list, (uint64_t)(a.ckpt_slots * kListPerSlot));
        if (e != hipSuccess) return e;
    }
    a.n_groups = (uint32_t)(6 * n_cu);  // persistent: about what the CUs hold at once
    return launch_kernel(backward_tile_kernel<true, true>, dim3(a.n_groups), dim3(kTilePixels), s, a);
}

// ---------------------------------------------------------------------------
// B2: screen-space adjoints -> 3D parameters
// ---------------------------------------------------------------------------
// zeros for floats [w * i0, w * i1) of a plane of w floats per Gaussian,
// by the workgroup: 16-byte stores on the 16-byte aligned stretch, single
// floats at the ends
__device__ __forceinline__ void zero_plane(float *p, int w, int64_t i0, int64_t i1) {
    if (!p) return;
    const int64_t f0 = (int64_t)w * i0, f1 = (int64_t)w * i1;
    const uint64_t base = (uint64_t)(uintptr_t)p;  // 4-byte aligned (floats)
    int64_t v0 = f0, v1 = f1;
    while (((base + 4u * (uint64_t)v0) & 15u) && v0 < f1) ++v0;
    while (((base + 4u * (uint64_t)v1) & 15u) && v1 > v0) --v1;
    if (v0 >= v1) {
        for (int64_t f = f0 + threadIdx.x; f < f1; f += blockDim.x) p[f] = 0.0f;
        return;
    }
    for (int64_t f = f0 + threadIdx.x; f < v0; f += blockDim.x) p[f] = 0.0f;
    for (int64_t f = v1 + threadIdx.x; f < f1; f += blockDim.x) p[f] = 0.0f;
    float4 *q = reinterpret_cast<float4 *>(p + v0);
    for (int64_t k = threadIdx.x; k < (v1 - v0) / 4; k += blockDim.x) q[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// B2a: with the first chunk of views, zeros for every gradient the chain
// writes, each workgroup's stretch of every plane written with 16-byte stores
// (the drawn Gaussians are overwritten by B2b; later chunks add to what the
// first wrote); the drawn Gaussians appended to a.list, positions inside the
// workgroup from ballots and one atomic per workgroup (order of arrival: each
// Gaussian is handled on its own).  A workgroup takes kListSpan Gaussians, so
// that few atomics meet on the one counter (they serialise there).
constexpr int kListChunks = 4, kListSpan = 1024 * kListChunks;
__global__ void __launch_bounds__(1024) zero_and_list_kernel(const BackwardProjectArgs a, int sh_floats) {
    __shared__ uint32_t s_cnt[kListChunks][16], s_base;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t g0 = (int64_t)blockIdx.x * kListSpan, g1 = g0 + kListSpan < a.seg.n ? g0 + kListSpan : a.seg.n;
    bool vis[kListChunks];
    uint64_t bal[kListChunks];
#pragma unroll
    for (int c = 0; c < kListChunks; ++c) {
        const int64_t i = g0 + c * 1024 + threadIdx.x;
        vis[c] = false;
        if (i < g1)
            for (int vi = 0; vi < a.nv && !vis[c]; ++vi) vis[c] = a.tiles_touched[a.base[vi] + i] != 0u;
        bal[c] = __ballot(vis[c]);
        if (lane == 0) s_cnt[c][wave] = (uint32_t)__popcll(bal[c]);
    }
    if (a.first && !a.zeroed) {
        const gs_gaussians_grad &G = a.grad;
        zero_plane(G.means, 3, g0, g1);
        zero_plane(G.opacity, 1, g0, g1);
        zero_plane(G.sh, sh_floats, g0, g1);
        if (a.seg.cov6) {
            zero_plane(G.cov6, 6, g0, g1);
        } else {
            zero_plane(G.log_scales, 3, g0, g1);
            zero_plane(G.quats, 4, g0, g1);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t total = 0u;
        for (int c = 0; c < kListChunks; ++c)
            for (int w = 0; w < 16; ++w) {
                const uint32_t k = s_cnt[c][w];
                s_cnt[c][w] = total;
                total += k;
            }
        s_base = total ? atomicAdd(a.count, total) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kListChunks; ++c)
        if (vis[c])
            a.list[s_base + s_cnt[c][wave] + (uint32_t)__popcll(bal[c] & ((1ull << lane) - 1ull))] =
                (uint32_t)(g0 + c * 1024 + threadIdx.x);
}

// B2b: a workgroup of two waves per 64 listed Gaussians.  Wave 0 takes the
// geometry (the FP32 projection repeated for its clamp decisions, then the
// chain in FP64 to the mean and covariance, and the opacity), wave 1 the
// colour (SH coefficients, and the view direction's share of the mean's
// gradient, handed to wave 0 through LDS): two chains of half the length,
// each holding about half the registers.
template <int D>
__global__ void __launch_bounds__(128) backward_project_kernel(const BackwardProjectArgs a) {
    constexpr int K = (D + 1) * (D + 1);
    __shared__ float s_cam[kProjViews * kCamStride];
    __shared__ double s_dmu[3][64];
    const uint32_t count = *a.count;
    if ((int64_t)blockIdx.x * 64 >= (int64_t)count) return;  // uniform per workgroup
    for (int k = threadIdx.x; k < a.nv * 16; k += 128) {
        const int vi = k >> 4, f = k & 15;
        s_cam[vi * kCamStride + f] = reinterpret_cast<const float *>(a.cams + a.view[vi])[f];
    }
    __syncthreads();
    for (int vi = threadIdx.x; vi < a.nv; vi += 128) {
        float *c = s_cam + vi * kCamStride;
#pragma unroll
        for (int j = 0; j < 3; ++j) c[16 + j] = -(c[j] * c[9] + c[3 + j] * c[10] + c[6 + j] * c[11]);
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t li = (int64_t)blockIdx.x * 64 + lane;
    const bool valid = li < (int64_t)count;
    const int64_t i = valid ? (int64_t)a.list[li] : 0;
    const bool use_cov6 = a.seg.cov6 != nullptr;
    const gs_gaussians_grad &G = a.grad;
    const bool first = a.first != 0;
    auto put = [&](float *dst, float v) {
        if (first) *dst = v;
        else *dst += v;
    };
    // FP32 as in the forward where its decisions are repeated (projection,
    // clamps, colour clamp, SH); FP64 along the chain from the conic back to
    // the covariance and the mean, where an elongated Gaussian's adjoints
    // cancel strongly
    float mx = 0.f, my = 0.f, mz = 0.f;
    // the views that draw it, their counts requested together (a listed
    // Gaussian is drawn by one of the launch's views: with one view, by that
    // one); then the drawn views in ascending order
    uint64_t drawn = 0u;
    if (valid) {
        mx = a.seg.means[3 * i + 0];
        my = a.seg.means[3 * i + 1];
        mz = a.seg.means[3 * i + 2];
        drawn = 1u;
        if (a.nv > 1) {
            drawn = 0u;
            for (int v0 = 0; v0 < a.nv; v0 += 16) {
                uint32_t t[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) t[k] = v0 + k < a.nv ? a.tiles_touched[a.base[v0 + k] + i] : 0u;
#pragma unroll
                for (int k = 0; k < 16; ++k) drawn |= (uint64_t)(t[k] != 0u) << (v0 + k);
            }
        }
    }
    if (wave == 1) {
        // ---- colour -> SH coefficients and view direction
        float dsh[3 * K];
#pragma unroll
        for (int k = 0; k < 3 * K; ++k) dsh[k] = 0.f;
        double dmd[3] = {0.0, 0.0, 0.0};
        float sh[3 * K];
#pragma unroll
        for (int k = 0; k < 3 * K; ++k) sh[k] = 0.f;
        if (valid) {
            const float *src = a.seg.sh + (size_t)(3 * K) * i;
#pragma unroll
            for (int k = 0; k < 3 * K; ++k) sh[k] = src[k];
        }
        for (uint64_t m = drawn; m; m &= m - 1u) {
            const int vi = __ffsll((unsigned long long)m) - 1;
            const double *g = a.g2d + (size_t)(a.base[vi] + i) * kG2D;
            float dc[3] = {(float)g[kGR], (float)g[kGG], (float)g[kGBl]};
            const float *cam = s_cam + vi * kCamStride;
            float dx0 = mx - cam[16], dy0 = my - cam[17], dz0 = mz - cam[18];
            const float inv_dist = 1.0f / sqrtf(dx0 * dx0 + dy0 * dy0 + dz0 * dz0);
            const float x = dx0 * inv_dist, y = dy0 * inv_dist, z = dz0 * inv_dist;
            float Y[K];
            float3 dY[K];
            sh_basis<D>(x, y, z, Y);
            sh_basis_grad<D>(x, y, z, dY);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float acc = 0.0f;  // same accumulation order as the forward
#pragma unroll
                for (int k = 0; k < K; ++k) acc += Y[k] * sh[3 * k + ch];
                if (!(acc + 0.5f > 0.0f)) dc[ch] = 0.0f;
            }
            float ddx = 0.f, ddy = 0.f, ddz = 0.f;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float cdot = dc[0] * sh[3 * k] + dc[1] * sh[3 * k + 1] + dc[2] * sh[3 * k + 2];
                ddx += cdot * dY[k].x;
                ddy += cdot * dY[k].y;
                ddz += cdot * dY[k].z;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) dsh[3 * k + ch] += dc[ch] * Y[k];
            }
            const float dd = x * ddx + y * ddy + z * ddz;
            dmd[0] += (double)((ddx - x * dd) * inv_dist);
            dmd[1] += (double)((ddy - y * dd) * inv_dist);
            dmd[2] += (double)((ddz - z * dd) * inv_dist);
        }
        if (valid) {
            float *dst = G.sh + (size_t)(3 * K) * i;
#pragma unroll
            for (int k = 0; k < 3 * K; ++k) put(&dst[k], dsh[k]);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) s_dmu[k][lane] = dmd[k];
    }
    double dmu[3] = {0.0, 0.0, 0.0};
    double dS[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // symmetric adjoint of Sigma (xx, xy, xz, yy, yz, zz)
    float dop = 0.f;
    double scd[3] = {0.0, 0.0, 0.0};
    RotT<double> rotd;
    if (wave == 0 && valid) {
        float S[6];
        double Sd[6];
        if (use_cov6) {
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                S[k] = a.seg.cov6[6 * i + k];
                Sd[k] = (double)S[k];
            }
        } else {
            const float4 q = reinterpret_cast<const float4 *>(a.seg.quats)[i];
            const Rot rot = quat_rot(q.x, q.y, q.z, q.w);
            float sc[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float ls = a.seg.log_scales[3 * i + k];
                sc[k] = expf(ls);
                scd[k] = exp((double)ls);
            }
            cov_from_rot_scale(rot.R, sc, S);
            rotd = quat_rot_t<double>((double)q.x, (double)q.y, (double)q.z, (double)q.w);
            cov_from_rot_scale(rotd.R, scd, Sd);
        }
        for (uint64_t m = drawn; m; m &= m - 1u) {
            const int vi = __ffsll((unsigned long long)m) - 1;
            const double *g = a.g2d + (size_t)(a.base[vi] + i) * kG2D;
            double gl[kG2D];
#pragma unroll
            for (int k = 0; k < kG2D; ++k) gl[k] = g[k];
            const float *cam = s_cam + vi * kCamStride;
            ViewProj p;
            // the same FP32 projection as the forward; the instance is known to
            // be visible (tiles_touched > 0), so every field used below is
            // computed
            const int TX = (a.W + kTile - 1) / kTile, TY = (a.H + kTile - 1) / kTile;
            (void)ewa_project(cam, mx, my, mz, S, a.W, a.H, TX, TY, a.near_plane, a.lowpass, a.sigma_cut, a.fov_clamp,
                              p);
            dop += (float)gl[kGO];
            // ---- the projection in FP64, with the forward's clamp decisions
            double R[9];
    #pragma unroll
            for (int k = 0; k < 9; ++k) R[k] = (double)cam[k];
            const double fxc = (double)cam[12], fyc = (double)cam[13];
            const double tx = R[0] * mx + R[1] * my + R[2] * mz + (double)cam[9];
            const double ty = R[3] * mx + R[4] * my + R[5] * mz + (double)cam[10];
            const double tz = R[6] * mx + R[7] * my + R[8] * mz + (double)cam[11];
            const double iz = 1.0 / tz, iz2 = iz * iz;
            const double limx = (double)a.fov_clamp * (0.5 * (double)a.W / fxc);
            const double limy = (double)a.fov_clamp * (0.5 * (double)a.H / fyc);
            const double xr = p.clx ? (tx * iz < 0.0 ? -limx : limx) : tx * iz;
            const double yr = p.cly ? (ty * iz < 0.0 ? -limy : limy) : ty * iz;
            const double j00 = fxc * iz, j02 = -fxc * xr * iz, j11 = fyc * iz, j12 = -fyc * yr * iz;
            double T0[3], T1[3];
    #pragma unroll
            for (int k = 0; k < 3; ++k) {
                T0[k] = j00 * R[k] + j02 * R[6 + k];
                T1[k] = j11 * R[3 + k] + j12 * R[6 + k];
            }
            double TS0[3], TS1[3];  // T Sigma
            TS0[0] = T0[0] * Sd[0] + T0[1] * Sd[1] + T0[2] * Sd[2];
            TS0[1] = T0[0] * Sd[1] + T0[1] * Sd[3] + T0[2] * Sd[4];
            TS0[2] = T0[0] * Sd[2] + T0[1] * Sd[4] + T0[2] * Sd[5];
            TS1[0] = T1[0] * Sd[0] + T1[1] * Sd[1] + T1[2] * Sd[2];
            TS1[1] = T1[0] * Sd[1] + T1[1] * Sd[3] + T1[2] * Sd[4];
            TS1[2] = T1[0] * Sd[2] + T1[1] * Sd[4] + T1[2] * Sd[5];
            const double lp = (double)a.lowpass;
            const double ca = TS0[0] * T0[0] + TS0[1] * T0[1] + TS0[2] * T0[2] + lp;
            const double cb = TS0[0] * T1[0] + TS0[1] * T1[1] + TS0[2] * T1[2];
            const double cc = TS1[0] * T1[0] + TS1[1] * T1[1] + TS1[2] * T1[2] + lp;
            const double idet = 1.0 / (ca * cc - cb * cb);
            const double qa = cc * idet, qb = -cb * idet, qc = ca * idet;
            // ---- conic -> 2D covariance: dS2 = -Q Gm Q, Gm = [[gA, gB/2], [gB/2, gC]]
            const double ga = gl[kGA], gbh = 0.5 * gl[kGB], gc = gl[kGC];
            const double m00 = qa * ga + qb * gbh, m01 = qa * gbh + qb * gc;
            const double m10 = qb * ga + qc * gbh, m11 = qb * gbh + qc * gc;
            const double s00 = -(m00 * qa + m01 * qb);
            const double s01 = -(m00 * qb + m01 * qc);
            const double s11 = -(m10 * qb + m11 * qc);
            // ---- 2D covariance -> Sigma and T:  S2 = T Sigma T^T + lp I; dSigma += T^T dS2 T
            double U[3][2];
    #pragma unroll
            for (int r = 0; r < 3; ++r) {
                U[r][0] = T0[r] * s00 + T1[r] * s01;
                U[r][1] = T0[r] * s01 + T1[r] * s11;
            }
            dS[0] += U[0][0] * T0[0] + U[0][1] * T1[0];
            dS[1] += U[0][0] * T0[1] + U[0][1] * T1[1];
            dS[2] += U[0][0] * T0[2] + U[0][1] * T1[2];
            dS[3] += U[1][0] * T0[1] + U[1][1] * T1[1];
            dS[4] += U[1][0] * T0[2] + U[1][1] * T1[2];
            dS[5] += U[2][0] * T0[2] + U[2][1] * T1[2];
            // dT = 2 dS2 T Sigma
            double dT0[3], dT1[3];
    #pragma unroll
            for (int c = 0; c < 3; ++c) {
                dT0[c] = 2.0 * (s00 * TS0[c] + s01 * TS1[c]);
                dT1[c] = 2.0 * (s01 * TS0[c] + s11 * TS1[c]);
            }
            // T = J W: dJ = dT W^T;  J00 = fx/z, J02 = -fx xr/z, J11 = fy/z, J12 = -fy yr/z
            const double dJ00 = dT0[0] * R[0] + dT0[1] * R[1] + dT0[2] * R[2];
            const double dJ02 = dT0[0] * R[6] + dT0[1] * R[7] + dT0[2] * R[8];
            const double dJ11 = dT1[0] * R[3] + dT1[1] * R[4] + dT1[2] * R[5];
            const double dJ12 = dT1[0] * R[6] + dT1[1] * R[7] + dT1[2] * R[8];
            double dtx = 0.0, dty = 0.0, dtz = 0.0;
            dtz += -fxc * iz2 * dJ00 - fyc * iz2 * dJ11;
            dtz += dJ02 * fxc * xr * iz2 + dJ12 * fyc * yr * iz2;
            if (!p.clx) {
                dtx += dJ02 * (-fxc * iz) * iz;
                dtz += dJ02 * (-fxc * iz) * (-tx * iz2);
            }
            if (!p.cly) {
                dty += dJ12 * (-fyc * iz) * iz;
                dtz += dJ12 * (-fyc * iz) * (-ty * iz2);
            }
            // ---- projected mean and depth
            dtx += gl[kGU] * fxc * iz;
            dty += gl[kGV] * fyc * iz;
            dtz += -gl[kGU] * fxc * tx * iz2 - gl[kGV] * fyc * ty * iz2 + gl[kGZ];
            dmu[0] += R[0] * dtx + R[3] * dty + R[6] * dtz;
            dmu[1] += R[1] * dtx + R[4] * dty + R[7] * dtz;
            dmu[2] += R[2] * dtx + R[5] * dty + R[8] * dtz;
        }
    }
    __syncthreads();  // the colour wave's share of the mean's gradient is in LDS
    if (wave != 0 || !valid) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) put(&G.means[3 * i + k], (float)(dmu[k] + s_dmu[k][lane]));
    put(&G.opacity[i], dop);
    if (use_cov6) {
        if (G.cov6) {
            // an off-diagonal cov6 entry stands for both symmetric entries
            put(&G.cov6[6 * i + 0], (float)dS[0]);
            put(&G.cov6[6 * i + 1], (float)(2.0 * dS[1]));
            put(&G.cov6[6 * i + 2], (float)(2.0 * dS[2]));
            put(&G.cov6[6 * i + 3], (float)dS[3]);
            put(&G.cov6[6 * i + 4], (float)(2.0 * dS[4]));
            put(&G.cov6[6 * i + 5], (float)dS[5]);
        }
    } else {
        // adjoint of every entry of the full symmetric Sigma
        const double full[9] = {dS[0], dS[1], dS[2], dS[1], dS[3], dS[4], dS[2], dS[4], dS[5]};
        double dls[3], dq[4];
        cov_backward(rotd, scd, full, dls, dq);
        if (G.log_scales) {
#pragma unroll
            for (int k = 0; k < 3; ++k) put(&G.log_scales[3 * i + k], (float)dls[k]);
        }
        if (G.quats) {
#pragma unroll
            for (int k = 0; k < 4; ++k) put(&G.quats[4 * i + k], (float)dq[k]);
        }
    }
}

// The screen-space accumulators of the drawn instances start at zero; B1
// adds only to those and B2 reads only those.  Workgroup 0 also zeroes the
// list counters and, with checkpoints and at most kListInClear lists, builds
// the tile pass's segment list.
__global__ void __launch_bounds__(256) clear_g2d_kernel(const uint32_t *tt, int64_t n, double *g2d,
                                                        uint32_t *counts, int n_counts, const uint2 *ranges,
                                                        int64_t n_items, uint32_t *seg_list, uint64_t seg_cap) {
    static_assert(kG2D % 2 == 0, "two accumulators per 16-B store");
    constexpr uint32_t P = kG2D / 2;  // 16-B pieces per instance
    if (blockIdx.x == 0) {
        for (int k = threadIdx.x; k < n_counts; k += 256) counts[k] = 0u;
        if (seg_list && n_items <= kListInClear) build_segment_list<256>(ranges, n_items, seg_list, seg_cap);
    }
    // a block of 256 instances at a time, its 256 P pieces spread over the
    // threads, so that each store instruction writes consecutive 16-B pieces
    for (int64_t base = (int64_t)blockIdx.x * 256; base < n; base += (int64_t)gridDim.x * 256) {
        double2 *g = reinterpret_cast<double2 *>(g2d + (size_t)base * kG2D);
#pragma unroll
        for (uint32_t r = 0; r < P; ++r) {
            const uint32_t k = r * 256u + threadIdx.x, li = k / P;
            if (base + li < n && tt[base + li]) g[k] = make_double2(0.0, 0.0);
        }
    }
}

hipError_t launch_clear_g2d(const uint32_t *tiles_touched, int64_t n_instances, double *g2d, uint32_t *counts,
                            int n_counts, const uint2 *ranges, int64_t n_items, uint32_t *seg_list, uint64_t seg_cap,
                            hipStream_t s) {
    int64_t grid = (n_instances + 255) / 256;
    if (grid > 8192) grid = 8192;
    if (grid < 1) grid = 1;
    return launch_kernel(clear_g2d_kernel, dim3((unsigned)grid), dim3(256), s, tiles_touched, n_instances, g2d,
                         counts, n_counts, ranges, n_items, seg_list, seg_cap);
}

hipError_t launch_backward_project(const BackwardProjectArgs &a, hipStream_t s) {
    if (a.seg.n == 0) return hipSuccess;
    const int K = (a.seg.sh_degree + 1) * (a.seg.sh_degree + 1);
    hipError_t e;
    if ((e = launch_kernel(zero_and_list_kernel, dim3((unsigned)((a.seg.n + kListSpan - 1) / kListSpan)), dim3(1024), s,
                           a, 3 * K)) != hipSuccess)
        return e;
    if (a.nv == 0) return hipSuccess;
    const unsigned grid = (unsigned)((a.seg.n + 63) / 64);  // 64 listed Gaussians per two-wave workgroup
    switch (a.seg.sh_degree) {
        case 0: return launch_kernel(backward_project_kernel<0>, dim3(grid), dim3(128), s, a);
        case 1: return launch_kernel(backward_project_kernel<1>, dim3(grid), dim3(128), s, a);
        case 2: return launch_kernel(backward_project_kernel<2>, dim3(grid), dim3(128), s, a);
        default: return launch_kernel(backward_project_kernel<3>, dim3(grid), dim3(128), s, a);
    }
}

}  // namespace gs
