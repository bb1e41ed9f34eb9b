// gs_composite kernel: per-tile front-to-back alpha compositing.
//
// Every wave64 is an independent persistent worker: it pops work items from
// an atomic counter, one item per (view, tile, 8 x 8 quadrant), one pixel per
// lane.  A wave walks its tile's sorted list 64 entries at a time: each lane
// gathers one 48-B record, tests whether the entry can reach alpha >=
// alpha_min anywhere in the quadrant (a conservative bound, so culling never
// changes a result), and the entries that can are compacted into the wave's
// LDS slice with a ballot, in list order.  The lanes then evaluate the
// compacted entries front to back.  There are no workgroup barriers: waves
// of different quadrants and tiles interleave on a SIMD and hide each other's
// gather latency.  A wave leaves the list once its 64 pixels have stopped.
//
// Work queues are XCD-aware: queue q holds the (view, tile) items t with
// t mod 8 == q (all four quadrants of each), and a workgroup starts on the
// queue of blockIdx.x mod 8 -- the XCD the dispatcher places it on -- so the
// four quadrant waves of a tile gather its list through one L2, while every
// XCD still gets an even share of the image.  An exhausted queue sends its
// waves on to the other queues (work stealing; a queue seen to be empty by a
// plain load is skipped without an atomic).  Each queue head sits in its own
// 128-B line.  Within a queue the items are popped longest list first (the
// tile work order, a counting sort by list chunks that the binning writes),
// so the waves that bound the kernel's duration start at once and short
// lists fill the gaps at the end.  Placement and order only affect locality
// and timing, never results.  The last workgroup to leave returns the
// counters to zero, so the workspace is ready for the next call without a
// clearing launch.
#include "gs_internal.hpp"

namespace gs {

constexpr int kWavesPerGroup = 4;
constexpr int kQueues = kOrderQueues;  // one per XCD
constexpr int kCounterStride = 32;  // words between queue heads (one 128-B line each)

// wave issue priority 0..3 from the list length (512, 1024, 2048 entries)
__device__ __forceinline__ void set_wave_priority(uint32_t len) {
    if (len >= 2048u) __builtin_amdgcn_s_setprio(3);
    else if (len >= 1024u) __builtin_amdgcn_s_setprio(2);
    else if (len >= 512u) __builtin_amdgcn_s_setprio(1);
}

// The next quadrant item (view * T + tile) * 4 + quadrant, or -1 when every
// queue is exhausted: the home queue first, then the others in turn
// (visited: queues found empty so far, kept by the caller).
__device__ __forceinline__ long long pop_item(const CompositeArgs &a, int home, int &visited) {
    while (visited < kQueues) {
        const int q = (home + visited) % kQueues;
        // queue q: tiles q, q + 8, q + 16, ... -> 4 quadrant items each
        const uint32_t size = a.n_items > q ? (uint32_t)(4 * ((a.n_items - q + kQueues - 1) / kQueues)) : 0u;
        uint32_t *head = a.counter + q * kCounterStride;
        if (visited > 0 && __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= size) {
            ++visited;
            continue;
        }
        const uint32_t k = atomicAdd(head, 1u);
        if (k < size) {
            const uint32_t t = a.order[q * a.qstride + (k >> 2)];
            return t < (uint64_t)a.n_items ? (long long)t * 4 + (k & 3) : -1;  // -1: not an item
        }
        ++visited;
    }
    return -1;
}

// the last workgroup to leave returns the queue heads and its own counter to
// zero (every pop of every wave has happened by then)
__device__ __forceinline__ void leave(const CompositeArgs &a) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t left = atomicAdd(a.counter + kQueues * kCounterStride, 1u);
        if (left == a.n_groups - 1u) {
            for (int q = 0; q <= kQueues; ++q) atomicExch(a.counter + q * kCounterStride, 0u);
        }
    }
}

// One quadrant item walked by one wave (its staging rows e0s, e1s, e2s in
// LDS): gathers, culls and stages the list 64 entries at a time and
// composites the survivors front to back.
__device__ __forceinline__ void walk_one(const CompositeArgs &a, long long item, float4 *e0s, float4 *e1s,
                                         float4 *e2s, int lane, uint64_t lt_mask) {
    const int64_t titem = item >> 2;
    const int quad = (int)(item & 3);
    const int view = (int)(titem / a.T);
    const int tile = (int)(titem - (int64_t)view * a.T);
    const int qx0 = (tile % a.TX) * kTile + ((quad & 1) << 3);
    const int qy0 = (tile / a.TX) * kTile + ((quad >> 1) << 3);
    const int px = qx0 + (lane & 7), py = qy0 + (lane >> 3);
    const bool inside = px < a.W && py < a.H;
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    const float bx0 = (float)qx0 + 0.5f, by0 = (float)qy0 + 0.5f;
    const uint2 range = a.ranges[titem];
    // Waves of long lists get a higher issue priority on their SIMD: the
    // longest lists bound the kernel's duration, and shorter ones fill
    // the issue slots those leave while they wait on memory.
    set_wave_priority(range.y - range.x);
    float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f, dd = 0.0f;
    const float amax = __builtin_canonicalizef(a.alpha_max);  // keeps the clamp's operand out of the loop
    uint32_t last = 0;
    uint32_t done_end = 0;  // list position after the last chunk walked
    bool done = !inside;
    // software pipeline over the list chunks, two deep: the records of
    // chunks c and c + 1 sit in two register sets and the list values of
    // c + 2 and c + 3 are in flight; once chunk c's records have been
    // culled and staged, its set is refilled in place with chunk c + 2
    float4 qa0, qa1, qa2, qb0, qb1, qb2;  // records of this lane's entry in chunks c, c + 1
    uint32_t ga = 0u, gb = 0u;            // list values of its entries in chunks c + 2, c + 3
    // every load is unconditional: a lane past the list's end reads the
    // list's last entry again (a cache hit), so a refill overwrites its
    // whole register set and needs no merge with the old contents
    const uint32_t jl = range.y > range.x ? range.y - 1u : range.x;
    if (range.y > range.x) {
        const uint32_t j0 = range.x + lane;
        const uint32_t g0 = a.vals[min(j0, jl)], g1 = a.vals[min(j0 + 64u, jl)];
        // issued in the order the loop refills them
        qa0 = a.rec[3 * (size_t)g0];
        qa1 = a.rec[3 * (size_t)g0 + 1];
        qa2 = a.rec[3 * (size_t)g0 + 2];
        ga = a.vals[min(j0 + 128u, jl)];
        qb0 = a.rec[3 * (size_t)g1];
        qb1 = a.rec[3 * (size_t)g1 + 1];
        qb2 = a.rec[3 * (size_t)g1 + 2];
        gb = a.vals[min(j0 + 192u, jl)];
    }
    // one chunk of 64 list entries starting at b0 whose records are in
    // (q0, q1, q2); returns true once every pixel of the quadrant stopped
    auto chunk = [&](uint32_t b0, float4 &q0, float4 &q1, float4 &q2, uint32_t &gn) -> bool {
        const uint32_t j = b0 + lane;
        const bool hit = (j < range.y) && entry_reaches_box(q0.x, q0.y, q1.x, q1.y, q1.z, q1.w, a.alpha_min,
                                                           bx0, by0, bx0 + 7.0f, by0 + 7.0f);
        // the whole record set has arrived here on every path, so the
        // in-place refill below never waits on its old loads
        asm volatile("" ::"v"(q0.z), "v"(q0.w), "v"(q2.x), "v"(q2.y), "v"(q2.z));
        const uint64_t bal = __ballot(hit);
        if (hit) {
            const int pos = __popcll(bal & lt_mask);
            const Entry e = make_entry(q0, q1, q2);
            e0s[pos] = make_float4(e.u, e.v, e.a, e.b);
            e1s[pos] = make_float4(e.c, e.o, e.z, e.r);
            e2s[pos] = make_float4(e.g, e.bl, __uint_as_float(b0 - range.x + (uint32_t)lane + 1u), 0.0f);
        }
        // refill: the records of chunk c + 2, the list values of c + 4
        q0 = a.rec[3 * (size_t)gn];
        q1 = a.rec[3 * (size_t)gn + 1];
        q2 = a.rec[3 * (size_t)gn + 2];
        gn = a.vals[min(j + 256u, jl)];
        __builtin_amdgcn_wave_barrier();
        const int n = __popcll(bal);
        // pad the list to a multiple of 4 with entries of zero opacity
        // (alpha 0: always skipped)
        if (lane < ((4 - (n & 3)) & 3)) {
            e0s[n + lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            e1s[n + lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            e2s[n + lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        __builtin_amdgcn_wave_barrier();
        // Uniform trip count, four entries per step (their LDS reads are
        // issued together, ahead of the arithmetic); the per-lane skip /
        // stop / done decisions are predicates, with no divergent exits.
        // T (1 - alpha) is one fused multiply-add, fma(-alpha, T, T): a
        // single rounding of the exact product, where T - (alpha T) would
        // round alpha T first and lose up to alpha / (1 - alpha) ulps
        // (99 at the alpha clamp) -- error the backward's recovery
        // T_i = T_{i+1} / (1 - alpha_i) would carry over whole lists.
        for (int q = 0; q < n; q += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float4 e0 = e0s[q + u], e1 = e1s[q + u], e2 = e2s[q + u];
                const float dx = fx - e0.x, dy = fy - e0.y;
                const float p2 = entry_power2(e0.z, e0.w, e1.x, dx, dy);
                const float al = fminf(amax, e1.y * fast_exp2(p2));
                const float w = al * T;
                const float Tn = fmaf(-al, T, T);
                const bool take = !done && !(al < a.alpha_min);
                const bool stop = take && (Tn < a.t_min);
                const bool use = take && !stop;
                const float ws = use ? w : 0.0f;
                cr = fmaf(ws, e1.w, cr);
                cg = fmaf(ws, e2.x, cg);
                cb = fmaf(ws, e2.y, cb);
                dd = fmaf(ws, e1.z, dd);
                T = use ? Tn : T;
                last = use ? __float_as_uint(e2.z) : last;
                done = done || stop;
            }
        }
        __builtin_amdgcn_wave_barrier();
        // segment checkpoint at the end of this chunk (a multiple of the
        // segment length inside the list): T and the colour so far
        done_end = b0 - range.x + 64u;
        if (a.ckpt && done_end % kSegment == 0u && done_end < range.y - range.x) {
            const uint64_t slot = (range.x + done_end) / kSegment;
            if (slot < a.ckpt_slots) {
                a.ckpt[ckpt_index(slot, quad, 0, lane)] = T;
                a.ckpt[ckpt_index(slot, quad, 1, lane)] = cr;
                a.ckpt[ckpt_index(slot, quad, 2, lane)] = cg;
                a.ckpt[ckpt_index(slot, quad, 3, lane)] = cb;
                a.ckpt[ckpt_index(slot, quad, 4, lane)] = dd;
            }
        }
        return __ballot(!done) == 0ull;
    };
    for (uint32_t b0 = range.x; b0 < range.y; b0 += 128) {
        if (chunk(b0, qa0, qa1, qa2, ga)) break;
        if (b0 + 64 >= range.y) break;
        if (chunk(b0 + 64, qb0, qb1, qb2, gb)) break;
    }
    // the checkpoints crossed become (T_b, what is still to come behind b
    // -- the final colour, background included, minus the colour so far --
    // divided by T_b)
    if (a.ckpt) {
        for (uint32_t b = kSegment; b < done_end && b < range.y - range.x; b += kSegment) {
            const uint64_t slot = (range.x + b) / kSegment;
            if (slot >= a.ckpt_slots) break;
            float *c = a.ckpt;
            const float tb = c[ckpt_index(slot, quad, 0, lane)];
            const float inv = 1.0f / tb;
            c[ckpt_index(slot, quad, 1, lane)] = (cr - c[ckpt_index(slot, quad, 1, lane)] + T * a.bg0) * inv;
            c[ckpt_index(slot, quad, 2, lane)] = (cg - c[ckpt_index(slot, quad, 2, lane)] + T * a.bg1) * inv;
            c[ckpt_index(slot, quad, 3, lane)] = (cb - c[ckpt_index(slot, quad, 3, lane)] + T * a.bg2) * inv;
            c[ckpt_index(slot, quad, 4, lane)] = (dd - c[ckpt_index(slot, quad, 4, lane)]) * inv;
        }
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
    __builtin_amdgcn_s_setprio(0);
}

__global__ void __launch_bounds__(64 * kWavesPerGroup) composite_kernel(const CompositeArgs a) {
    __shared__ float4 s_e0[kWavesPerGroup][64], s_e1[kWavesPerGroup][64], s_e2[kWavesPerGroup][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    float4 *e0s = s_e0[wave], *e1s = s_e1[wave], *e2s = s_e2[wave];
    const int home = (int)(blockIdx.x % kQueues);
    int visited = 0;  // queues found empty so far (meaningful in lane 0)
    while (true) {
        long long item = lane == 0 ? pop_item(a, home, visited) : -1;
        item = __shfl(item, 0, 64);
        if (item < 0) break;
        walk_one(a, item, e0s, e1s, e2s, lane, lt_mask);
    }
    leave(a);
}

// Pair mode, for launches with few quadrant items: the list of one quadrant
// is walked by two waves of a 128-thread workgroup in a pipeline over its
// 64-entry chunks.  The producer wave gathers, culls and stages chunk c (as
// above) and evaluates every staged entry's alpha at its 64 pixels; the
// consumer wave meanwhile runs the front-to-back accumulation over chunk
// c - 1 from those alphas.  Both take exactly the single wave's arithmetic,
// in the same order, so the results are bit-identical; each wave's share of
// the per-entry work is about half, which shortens the longest list's walk
// (the kernel's duration when the items are fewer than the wave slots).
// Chunk buffers alternate between the two waves, one workgroup barrier per
// chunk (step k: chunk k produced, chunk k - 1 consumed); a consumer whose
// pixels have all stopped publishes the item's sequence number in the flag
// of that step's parity, and both waves leave the list after the barrier.
// Two flags, so that the consumer's next step cannot overwrite the one the
// producer is still about to read.
constexpr int kPairChunk = 64;
__global__ void __launch_bounds__(128) composite_pair_kernel(const CompositeArgs a) {
    __shared__ float4 s_e0[kPairChunk];                     // producer only: (u, v, a, b)
    __shared__ float4 s_e1[2][kPairChunk], s_e2[2][kPairChunk];  // (c, o, z, r), (g, b, index + 1, 0)
    __shared__ float4 s_al[2][kPairChunk / 4][64];         // alphas of entries 4 i .. 4 i + 3 at each pixel
    __shared__ uint32_t s_n[2];
    __shared__ long long s_item;
    __shared__ uint32_t s_stop[2];  // by step parity: the item (sequence number) whose pixels have all stopped
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool producer = wave == 0;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int home = (int)(blockIdx.x % kQueues);
    int visited = 0;
    if (threadIdx.x < 2) s_stop[threadIdx.x] = 0u;
    for (uint32_t seq = 1;; ++seq) {
        if (threadIdx.x == 0) s_item = pop_item(a, home, visited);
        __syncthreads();
        const long long item = s_item;
        if (item < 0) break;
        const int64_t titem = item >> 2;
        const int quad = (int)(item & 3);
        const int view = (int)(titem / a.T);
        const int tile = (int)(titem - (int64_t)view * a.T);
        const int qx0 = (tile % a.TX) * kTile + ((quad & 1) << 3);
        const int qy0 = (tile / a.TX) * kTile + ((quad >> 1) << 3);
        const int px = qx0 + (lane & 7), py = qy0 + (lane >> 3);
        const bool inside = px < a.W && py < a.H;
        const uint2 range = a.ranges[titem];
        const uint32_t L = range.y - range.x, nch = (L + kPairChunk - 1) / kPairChunk;
        set_wave_priority(L);
        if (producer) {
            const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
            const float bx0 = (float)qx0 + 0.5f, by0 = (float)qy0 + 0.5f;
            const float amax = __builtin_canonicalizef(a.alpha_max);
            // the same two-deep pipeline of record gathers as the single wave
            float4 qa0, qa1, qa2, qb0, qb1, qb2;
            uint32_t ga = 0u, gb = 0u;
            const uint32_t jl = L > 0u ? range.y - 1u : range.x;
            if (L > 0u) {
                const uint32_t j0 = range.x + lane;
                const uint32_t g0 = a.vals[min(j0, jl)], g1 = a.vals[min(j0 + 64u, jl)];
                qa0 = a.rec[3 * (size_t)g0];
                qa1 = a.rec[3 * (size_t)g0 + 1];
                qa2 = a.rec[3 * (size_t)g0 + 2];
                ga = a.vals[min(j0 + 128u, jl)];
                qb0 = a.rec[3 * (size_t)g1];
                qb1 = a.rec[3 * (size_t)g1 + 1];
                qb2 = a.rec[3 * (size_t)g1 + 2];
                gb = a.vals[min(j0 + 192u, jl)];
            }
            auto produce = [&](uint32_t c, float4 &q0, float4 &q1, float4 &q2, uint32_t &gn) {
                const int buf = (int)(c & 1u);
                const uint32_t b0 = range.x + c * kPairChunk;
                const uint32_t j = b0 + lane;
                const bool hit = (j < range.y) && entry_reaches_box(q0.x, q0.y, q1.x, q1.y, q1.z, q1.w, a.alpha_min,
                                                                   bx0, by0, bx0 + 7.0f, by0 + 7.0f);
                asm volatile("" ::"v"(q0.z), "v"(q0.w), "v"(q2.x), "v"(q2.y), "v"(q2.z));
                const uint64_t bal = __ballot(hit);
                if (hit) {
                    const int pos = __popcll(bal & lt_mask);
                    const Entry e = make_entry(q0, q1, q2);
                    s_e0[pos] = make_float4(e.u, e.v, e.a, e.b);
                    s_e1[buf][pos] = make_float4(e.c, e.o, e.z, e.r);
                    s_e2[buf][pos] = make_float4(e.g, e.bl, __uint_as_float(b0 - range.x + (uint32_t)lane + 1u), 0.0f);
                }
                q0 = a.rec[3 * (size_t)gn];
                q1 = a.rec[3 * (size_t)gn + 1];
                q2 = a.rec[3 * (size_t)gn + 2];
                gn = a.vals[min(j + 256u, jl)];
                __builtin_amdgcn_wave_barrier();
                const int n = __popcll(bal);
                if (lane < ((4 - (n & 3)) & 3)) {  // zero-opacity padding to a multiple of 4
                    s_e0[n + lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    s_e1[buf][n + lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    s_e2[buf][n + lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                }
                __builtin_amdgcn_wave_barrier();
                for (int q = 0; q < n; q += 4) {
                    float al[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const float4 e0 = s_e0[q + u], e1 = s_e1[buf][q + u];
                        const float dx = fx - e0.x, dy = fy - e0.y;
                        const float p2 = entry_power2(e0.z, e0.w, e1.x, dx, dy);
                        al[u] = fminf(amax, e1.y * fast_exp2(p2));
                    }
                    s_al[buf][q >> 2][lane] = make_float4(al[0], al[1], al[2], al[3]);
                }
                if (lane == 0) s_n[buf] = (uint32_t)n;
            };
            // chunk c is produced in step c; the loop mirrors the consumer's
            // barriers exactly
            for (uint32_t c = 0;; c += 2) {
                if (c < nch) produce(c, qa0, qa1, qa2, ga);
                __syncthreads();
                if (s_stop[0] == seq || c >= nch) break;
                if (c + 1 < nch) produce(c + 1, qb0, qb1, qb2, gb);
                __syncthreads();
                if (s_stop[1] == seq || c + 1 >= nch) break;
            }
        } else {
            float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f, dd = 0.0f;
            uint32_t last = 0, done_end = 0;
            bool done = !inside;
            // accumulation over chunk c (step c + 1), then its checkpoint;
            // publishes the item once every pixel has stopped
            auto consume = [&](uint32_t c) {
                const int buf = (int)(c & 1u);
                const int n = (int)s_n[buf];
                for (int q = 0; q < n; q += 4) {
                    const float4 a4 = s_al[buf][q >> 2][lane];
                    const float alv[4] = {a4.x, a4.y, a4.z, a4.w};
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const float4 e1 = s_e1[buf][q + u], e2 = s_e2[buf][q + u];
                        const float al = alv[u];
                        const float w = al * T;
                        const float Tn = fmaf(-al, T, T);
                        const bool take = !done && !(al < a.alpha_min);
                        const bool stop = take && (Tn < a.t_min);
                        const bool use = take && !stop;
                        const float ws = use ? w : 0.0f;
                        cr = fmaf(ws, e1.w, cr);
                        cg = fmaf(ws, e2.x, cg);
                        cb = fmaf(ws, e2.y, cb);
                        dd = fmaf(ws, e1.z, dd);
                        T = use ? Tn : T;
                        last = use ? __float_as_uint(e2.z) : last;
                        done = done || stop;
                    }
                }
                done_end = c * kPairChunk + kPairChunk;
                if (a.ckpt && done_end % kSegment == 0u && done_end < L) {
                    const uint64_t slot = (range.x + done_end) / kSegment;
                    if (slot < a.ckpt_slots) {
                        a.ckpt[ckpt_index(slot, quad, 0, lane)] = T;
                        a.ckpt[ckpt_index(slot, quad, 1, lane)] = cr;
                        a.ckpt[ckpt_index(slot, quad, 2, lane)] = cg;
                        a.ckpt[ckpt_index(slot, quad, 3, lane)] = cb;
                        a.ckpt[ckpt_index(slot, quad, 4, lane)] = dd;
                    }
                }
                if (__ballot(!done) == 0ull && lane == 0) s_stop[(c + 1u) & 1u] = seq;  // step c + 1
            };
            for (uint32_t c = 0;; c += 2) {
                if (c >= 1u) consume(c - 1u);
                __syncthreads();
                if (s_stop[0] == seq || c >= nch) break;
                consume(c);
                __syncthreads();
                if (s_stop[1] == seq || c + 1 >= nch) break;
            }
            if (a.ckpt) {
                for (uint32_t b = kSegment; b < done_end && b < L; b += kSegment) {
                    const uint64_t slot = (range.x + b) / kSegment;
                    if (slot >= a.ckpt_slots) break;
                    float *ck = a.ckpt;
                    const float tb = ck[ckpt_index(slot, quad, 0, lane)];
                    const float inv = 1.0f / tb;
                    ck[ckpt_index(slot, quad, 1, lane)] = (cr - ck[ckpt_index(slot, quad, 1, lane)] + T * a.bg0) * inv;
                    ck[ckpt_index(slot, quad, 2, lane)] = (cg - ck[ckpt_index(slot, quad, 2, lane)] + T * a.bg1) * inv;
                    ck[ckpt_index(slot, quad, 3, lane)] = (cb - ck[ckpt_index(slot, quad, 3, lane)] + T * a.bg2) * inv;
                    ck[ckpt_index(slot, quad, 4, lane)] = (dd - ck[ckpt_index(slot, quad, 4, lane)]) * inv;
                }
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
        }
        __builtin_amdgcn_s_setprio(0);
    }
    leave(a);
}

hipError_t launch_composite(CompositeArgs a, int grid, hipStream_t s) {
    if (a.n_items == 0 || grid <= 0) return hipSuccess;
    a.n_groups = (uint32_t)grid;
    return launch_kernel(composite_kernel, dim3(grid), dim3(64 * kWavesPerGroup), s, a);
}

hipError_t launch_composite_pairs(CompositeArgs a, int grid, hipStream_t s) {
    if (a.n_items == 0 || grid <= 0) return hipSuccess;
    a.n_groups = (uint32_t)grid;
    return launch_kernel(composite_pair_kernel, dim3(grid), dim3(128), s, a);
}

}  // namespace gs
