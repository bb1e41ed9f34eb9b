// gs_capsule_queries kernel: clearance to the nearest avatar capsule and
// swept-step blocking for a batch of agents (Sec. 3.3, Sec. 3.4).
//
// One wave64 per agent: the lanes take the capsules of the agent's avatars
// in turn (capsule j on lane j mod 64), interpolate each in its avatar's
// clip, and keep their smallest gaps; a butterfly of lane exchanges then
// gives the wave minimum (smallest capsule index on ties).  The agent is a
// vertical capsule (axis from its base point up `height`); a step sweeps
// that axis into the parallelogram {p0 + a (p1 - p0) + b height z}.
#include "gs_internal.hpp"

namespace gs {

struct V3 {
    float x, y, z;
};
__device__ __forceinline__ V3 v3(float x, float y, float z) { return {x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ float clamp01(float t) { return fminf(fmaxf(t, 0.0f), 1.0f); }

// squared distance between segments p0 + s u and q0 + t v, s, t in [0, 1]:
// the parameter of one segment is found for the other's, clamped, and the
// first refit to the clamped second (the standard closest-point sequence)
__device__ float seg_seg_dist2(V3 p0, V3 u, V3 q0, V3 v) {
    const V3 w = p0 - q0;
    const float a = dot(u, u), c = dot(v, v), e = dot(v, w);
    float s, t;
    if (a <= 1e-20f && c <= 1e-20f) {
        s = t = 0.0f;
    } else if (a <= 1e-20f) {
        s = 0.0f;
        t = clamp01(e / c);
    } else {
        const float d = dot(u, w);
        if (c <= 1e-20f) {
            t = 0.0f;
            s = clamp01(-d / a);
        } else {
            const float b = dot(u, v);
            const float den = a * c - b * b;
            s = den > 1e-7f * a * c ? clamp01((b * e - c * d) / den) : 0.0f;
            t = (b * s + e) / c;
            if (t < 0.0f) {
                t = 0.0f;
                s = clamp01(-d / a);
            } else if (t > 1.0f) {
                t = 1.0f;
                s = clamp01((b - d) / a);
            }
        }
    }
    const V3 r = (w + s * u) - t * v;
    return dot(r, r);
}

// distance between the segment s0 + l sd (l in [0, 1]) and the
// parallelogram o + a U + b V: zero where the segment crosses it, else the
// least of the segment against the four edges and of the two end points
// against the interior
__device__ float seg_parallelogram_dist(V3 s0, V3 sd, V3 o, V3 U, V3 V) {
    float best = seg_seg_dist2(s0, sd, o, U);
    best = fminf(best, seg_seg_dist2(s0, sd, o + V, U));
    best = fminf(best, seg_seg_dist2(s0, sd, o, V));
    best = fminf(best, seg_seg_dist2(s0, sd, o + U, V));
    best = sqrtf(best);
    const float g11 = dot(U, U), g12 = dot(U, V), g22 = dot(V, V);
    const float gd = g11 * g22 - g12 * g12;
    if (gd > 1e-7f * g11 * g22) {
        const V3 n = cross(U, V);
        const float rn = 1.0f / sqrtf(dot(n, n));
        const V3 ends[2] = {s0, s0 + sd};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const V3 r = ends[k] - o;
            const float ru = dot(r, U), rv = dot(r, V);
            const float a = (g22 * ru - g12 * rv) / gd, b = (g11 * rv - g12 * ru) / gd;
            if (a >= 0.0f && a <= 1.0f && b >= 0.0f && b <= 1.0f) best = fminf(best, fabsf(dot(r, n)) * rn);
        }
        // crossing: s0 + l sd = o + a U + b V, by Cramer's rule on
        // [sd, -U, -V] (l, a, b) = o - s0
        const V3 mu = -1.0f * U, mv = -1.0f * V, rhs = o - s0;
        const float det = dot(sd, cross(mu, mv));
        const float scale = sqrtf(dot(sd, sd) * g11 * g22);
        if (fabsf(det) > 1e-6f * scale) {
            const float l = dot(rhs, cross(mu, mv)) / det;
            const float a = dot(sd, cross(rhs, mv)) / det;
            const float b = dot(sd, cross(mu, rhs)) / det;
            if (l >= 0.0f && l <= 1.0f && a >= 0.0f && a <= 1.0f && b >= 0.0f && b <= 1.0f) best = 0.0f;
        }
    }
    return best;
}

// (gap, index) lexicographic minimum
__device__ __forceinline__ void take_min(float &g, int &i, float g2, int i2) {
    if (g2 < g || (g2 == g && i2 < i)) {
        g = g2;
        i = i2;
    }
}

__global__ void __launch_bounds__(256) capsule_query_kernel(const CapsuleArgs a) {
    const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (e >= a.n_agents) return;  // whole waves leave together
    const V3 p0 = v3(a.agent_pos[3 * e], a.agent_pos[3 * e + 1], a.agent_pos[3 * e + 2]);
    const bool step = a.agent_next != nullptr;
    V3 sd = v3(0.0f, 0.0f, 0.0f);
    if (step) sd = v3(a.agent_next[3 * e], a.agent_next[3 * e + 1], a.agent_next[3 * e + 2]) - p0;
    const V3 up = v3(0.0f, 0.0f, a.height);
    int first = a.agent_avatars[2 * e], count = a.agent_avatars[2 * e + 1];
    const int lo = max(first, 0), hi = min(first + max(count, 0), a.n_avatars);
    const int n = hi > lo ? (hi - lo) * a.n_caps : 0;
    float best = INFINITY, best_step = INFINITY;
    int best_i = -1;
    for (int j = lane; j < n; j += 64) {
        const int av = lo + j / a.n_caps, c = j - (j / a.n_caps) * a.n_caps;
        // the avatar's clip frames around its position (clamped like the skinning clips)
        const int cf = min(max(a.clip_first[av], 0), a.clip_total - 1);
        const int frames = min(max(a.clip_frames[av], 1), a.clip_total - cf);
        const float p = a.frame_pos[av];
        const float pc = p > 0.0f ? fminf(p, (float)(frames - 1)) : 0.0f;
        const int f0 = frames > 1 ? min((int)floorf(pc), frames - 2) : 0;
        const int f1 = frames > 1 ? f0 + 1 : 0;
        const float s = frames > 1 ? pc - (float)f0 : 0.0f;
        const float4 *c0 = reinterpret_cast<const float4 *>(a.caps + ((size_t)(cf + f0) * a.n_caps + c) * 8);
        const float4 *c1 = reinterpret_cast<const float4 *>(a.caps + ((size_t)(cf + f1) * a.n_caps + c) * 8);
        const float4 x0 = c0[0], y0 = c0[1], x1 = c1[0], y1 = c1[1];
        const float t = 1.0f - s;
        const V3 ca = v3(t * x0.x + s * x1.x, t * x0.y + s * x1.y, t * x0.z + s * x1.z);
        const V3 cb = v3(t * y0.x + s * y1.x, t * y0.y + s * y1.y, t * y0.z + s * y1.z);
        const float r = t * x0.w + s * x1.w;
        const V3 cd = cb - ca;
        const float g = sqrtf(seg_seg_dist2(p0, up, ca, cd)) - a.radius - r;
        take_min(best, best_i, g, av * a.n_caps + c);
        if (step) best_step = fminf(best_step, seg_parallelogram_dist(ca, cd, p0, sd, up) - a.radius - r);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const float g2 = __shfl_xor(best, off, 64);
        const int i2 = __shfl_xor(best_i, off, 64);
        take_min(best, best_i, g2, i2);
        best_step = fminf(best_step, __shfl_xor(best_step, off, 64));
    }
    if (lane == 0) {
        a.clearance[e] = best;
        if (a.nearest) a.nearest[e] = best_i;
        if (step) {
            a.step_gap[e] = best_step;
            a.blocked[e] = best_step < 0.0f ? 1 : 0;
        }
    }
}

hipError_t launch_capsule_queries(const CapsuleArgs &a, hipStream_t s) {
    if (a.n_agents <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((a.n_agents + 3) / 4);
    return launch_kernel(capsule_query_kernel, dim3(grid), dim3(256), s, a);
}

}  // namespace gs
