// gs_deform_lbs kernels: linear blend skinning of canonical avatar Gaussians.
//
// One thread per Gaussian.  The blended 3x4 matrix A = sum_k w_k M_{j_k} is
// formed from four joint matrices read through the cache (all avatars'
// matrices are a few KB; in clip mode eight, two frames per joint); the
// Gaussian streams 60 B in and 36 B out, so the kernel is HBM-bound.
#include "gs_internal.hpp"

namespace gs {



// A += wk * M for one row-major 3x4 matrix M
__device__ __forceinline__ void add_matrix(float *A, float wk, const float *Mp) {
    const float4 *M = reinterpret_cast<const float4 *>(Mp);
    const float4 r0 = M[0], r1 = M[1], r2 = M[2];
    A[0] += wk * r0.x;
    A[1] += wk * r0.y;
    A[2] += wk * r0.z;
    A[3] += wk * r0.w;
    A[4] += wk * r1.x;
    A[5] += wk * r1.y;
    A[6] += wk * r1.z;
    A[7] += wk * r1.w;
    A[8] += wk * r2.x;
    A[9] += wk * r2.y;
    A[10] += wk * r2.z;
    A[11] += wk * r2.w;
}

// The blended matrix A = sum_k w_k M_{j_k}.  In clip mode M_j is avatar a's
// joint matrix at its current time: the linear interpolation
// (1 - s) M_j[f] + s M_j[f + 1] of the two clip frames around the
// fractional frame position p (f = floor(p), s = p - f; p clamped to the
// clip, a clip of one frame holds its pose).  Interpolation and blend are
// both linear, so they are fused: A = sum_k w_k (1 - s) M_{j_k}[f] +
// w_k s M_{j_k}[f + 1], eight matrices read through the cache.
template <bool CLIP>
__device__ __forceinline__ void blend_matrix(const LbsArgs &a, int64_t i, float *A) {
    const uchar4 ji = reinterpret_cast<const uchar4 *>(a.joint_idx)[i];
    const float4 w = reinterpret_cast<const float4 *>(a.weights)[i];
    int av = a.avatar_of[i];
    av = av < 0 ? 0 : (av >= a.n_avatars ? a.n_avatars - 1 : av);
    const int j[4] = {min((int)ji.x, a.n_joints - 1), min((int)ji.y, a.n_joints - 1), min((int)ji.z, a.n_joints - 1),
                      min((int)ji.w, a.n_joints - 1)};
    const float wk[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int e = 0; e < 12; ++e) A[e] = 0.0f;
    if (!CLIP) {
        const float *base = a.skin + (size_t)av * a.n_joints * 12;
#pragma unroll
        for (int k = 0; k < 4; ++k) add_matrix(A, wk[k], base + (size_t)j[k] * 12);
        return;
    }
    // the avatar's clip, clamped into the clip array
    const int first = min(max(a.clip_first[av], 0), a.clip_total - 1);
    const int frames = min(max(a.clip_frames[av], 1), a.clip_total - first);
    const float p = a.frame_pos[av];
    const float pc = p > 0.0f ? fminf(p, (float)(frames - 1)) : 0.0f;  // NaN -> 0
    const int f0 = frames > 1 ? min((int)floorf(pc), frames - 2) : 0;
    const int f1 = frames > 1 ? f0 + 1 : 0;
    const float s = frames > 1 ? pc - (float)f0 : 0.0f;
    const float *b0 = a.clip + (size_t)(first + f0) * a.n_joints * 12;
    const float *b1 = a.clip + (size_t)(first + f1) * a.n_joints * 12;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        add_matrix(A, wk[k] * (1.0f - s), b0 + (size_t)j[k] * 12);
        add_matrix(A, wk[k] * s, b1 + (size_t)j[k] * 12);
    }
}

template <bool CLIP>
__global__ void __launch_bounds__(256) lbs_kernel(const LbsArgs a) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    float A[12];
    blend_matrix<CLIP>(a, i, A);
    const float mx = a.means[3 * i], my = a.means[3 * i + 1], mz = a.means[3 * i + 2];
#pragma unroll
    for (int r = 0; r < 3; ++r) a.means_out[3 * i + r] = A[4 * r] * mx + A[4 * r + 1] * my + A[4 * r + 2] * mz + A[4 * r + 3];
    const float4 q = reinterpret_cast<const float4 *>(a.quats)[i];
    const Rot rot = quat_rot(q.x, q.y, q.z, q.w);
    float s[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) s[k] = expf(a.log_scales[3 * i + k]);
    // A3 M with M = R S; Sigma' = (A3 M)(A3 M)^T
    float N[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            N[3 * r + c] = (A[4 * r] * rot.R[c] + A[4 * r + 1] * rot.R[3 + c] + A[4 * r + 2] * rot.R[6 + c]) * s[c];
    float *o = a.cov6_out + 6 * i;
    o[0] = N[0] * N[0] + N[1] * N[1] + N[2] * N[2];
    o[1] = N[0] * N[3] + N[1] * N[4] + N[2] * N[5];
    o[2] = N[0] * N[6] + N[1] * N[7] + N[2] * N[8];
    o[3] = N[3] * N[3] + N[4] * N[4] + N[5] * N[5];
    o[4] = N[3] * N[6] + N[4] * N[7] + N[5] * N[8];
    o[5] = N[6] * N[6] + N[7] * N[7] + N[8] * N[8];
}

template <bool CLIP>
__global__ void __launch_bounds__(256) lbs_backward_kernel(const LbsArgs a) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    float A[12];
    blend_matrix<CLIP>(a, i, A);
    const float gx = a.d_means_out[3 * i], gy = a.d_means_out[3 * i + 1], gz = a.d_means_out[3 * i + 2];
#pragma unroll
    for (int c = 0; c < 3; ++c) a.d_means[3 * i + c] = A[c] * gx + A[4 + c] * gy + A[8 + c] * gz;
    // dSigma = A3^T G A3 with G the full symmetric adjoint of Sigma'
    const float *d = a.d_cov6_out + 6 * i;
    const float G[9] = {d[0], 0.5f * d[1], 0.5f * d[2], 0.5f * d[1], d[3], 0.5f * d[4], 0.5f * d[2], 0.5f * d[4], d[5]};
    float GA[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) GA[3 * r + c] = G[3 * r] * A[c] + G[3 * r + 1] * A[4 + c] + G[3 * r + 2] * A[8 + c];
    float dS[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) dS[3 * r + c] = A[r] * GA[c] + A[4 + r] * GA[3 + c] + A[8 + r] * GA[6 + c];
    const float4 q = reinterpret_cast<const float4 *>(a.quats)[i];
    const Rot rot = quat_rot(q.x, q.y, q.z, q.w);
    float s[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) s[k] = expf(a.log_scales[3 * i + k]);
    float dls[3], dq[4];
    cov_backward(rot, s, dS, dls, dq);
#pragma unroll
    for (int k = 0; k < 3; ++k) a.d_log_scales[3 * i + k] = dls[k];
    reinterpret_cast<float4 *>(a.d_quats)[i] = make_float4(dq[0], dq[1], dq[2], dq[3]);
}

// Adjoint w.r.t. the joint matrices (fixed-matrix mode).  A persistent grid
// walks the Gaussians; each thread forms its Gaussian's 3x4 adjoint dL/dA
// (g mean^T + 2 G A3 Sigma | g) and adds w_k dL/dA to the four joints it
// blends, first into the workgroup's LDS copy of all joint adjoints (when
// they fit, kJointLds floats), then the workgroup adds its nonzero entries to
// the output with float atomics.
constexpr int kJointLds = 4096;

__device__ __forceinline__ void gaussian_matrix_adjoint(const LbsArgs &a, int64_t i, const float *A, float *dA) {
    const float gx = a.d_means_out[3 * i], gy = a.d_means_out[3 * i + 1], gz = a.d_means_out[3 * i + 2];
    const float mx = a.means[3 * i], my = a.means[3 * i + 1], mz = a.means[3 * i + 2];
    const float *d = a.d_cov6_out + 6 * i;
    const float G[9] = {d[0], 0.5f * d[1], 0.5f * d[2], 0.5f * d[1], d[3], 0.5f * d[4], 0.5f * d[2], 0.5f * d[4], d[5]};
    // Sigma = (R S)(R S)^T from the canonical scales and rotation
    const float4 q = reinterpret_cast<const float4 *>(a.quats)[i];
    const Rot rot = quat_rot(q.x, q.y, q.z, q.w);
    float M[9];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float sk = expf(a.log_scales[3 * i + k]);
#pragma unroll
        for (int r = 0; r < 3; ++r) M[3 * r + k] = rot.R[3 * r + k] * sk;
    }
    float S[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) S[3 * r + c] = M[3 * r] * M[3 * c] + M[3 * r + 1] * M[3 * c + 1] + M[3 * r + 2] * M[3 * c + 2];
    // GA = G A3, then dA3 = 2 GA Sigma + g mean^T
    float GA[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) GA[3 * r + c] = G[3 * r] * A[c] + G[3 * r + 1] * A[4 + c] + G[3 * r + 2] * A[8 + c];
    const float g[3] = {gx, gy, gz}, m[3] = {mx, my, mz};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            dA[4 * r + c] = 2.0f * (GA[3 * r] * S[c] + GA[3 * r + 1] * S[3 + c] + GA[3 * r + 2] * S[6 + c]) + g[r] * m[c];
        dA[4 * r + 3] = g[r];
    }
}

__global__ void __launch_bounds__(256) lbs_joint_grad_kernel(const LbsArgs a, float *d_skin) {
    __shared__ float s_acc[kJointLds];
    const int64_t n_mats = (int64_t)a.n_avatars * a.n_joints * 12;
    const bool lds = n_mats <= kJointLds;
    if (lds) {
        for (int k = threadIdx.x; k < n_mats; k += 256) s_acc[k] = 0.0f;
        __syncthreads();
    }
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < a.n; i += stride) {
        float A[12], dA[12];
        blend_matrix<false>(a, i, A);
        gaussian_matrix_adjoint(a, i, A, dA);
        const uchar4 ji = reinterpret_cast<const uchar4 *>(a.joint_idx)[i];
        const float4 w = reinterpret_cast<const float4 *>(a.weights)[i];
        int av = a.avatar_of[i];
        av = av < 0 ? 0 : (av >= a.n_avatars ? a.n_avatars - 1 : av);
        const int j[4] = {min((int)ji.x, a.n_joints - 1), min((int)ji.y, a.n_joints - 1),
                          min((int)ji.z, a.n_joints - 1), min((int)ji.w, a.n_joints - 1)};
        const float wk[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t base = ((int64_t)av * a.n_joints + j[k]) * 12;
#pragma unroll
            for (int e = 0; e < 12; ++e) {
                if (lds) atomicAdd(&s_acc[base + e], wk[k] * dA[e]);
                else atomicAdd(&d_skin[base + e], wk[k] * dA[e]);
            }
        }
    }
    if (lds) {
        __syncthreads();
        for (int k = threadIdx.x; k < n_mats; k += 256)
            if (s_acc[k] != 0.0f) atomicAdd(&d_skin[k], s_acc[k]);
    }
}

hipError_t launch_lbs_joint_grad(const LbsArgs &a, float *d_skin, int n_cu, hipStream_t s) {
    const int64_t n_mats = (int64_t)a.n_avatars * a.n_joints * 12;
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(d_skin), 0u, n_mats, s);
    if (e != hipSuccess || a.n == 0) return e;
    int64_t grid = (a.n + 255) / 256;
    if (grid > (int64_t)n_cu) grid = n_cu;  // one workgroup per CU: few LDS-to-HBM flushes
    return launch_kernel(lbs_joint_grad_kernel, dim3((unsigned)grid), dim3(256), s, a, d_skin);
}

// Forward kinematics: one thread per avatar walks its joints parent first.
// Joint k's world transform G_k = G_parent [R(w_k) | rest_k - rest_parent]
// (the root transform in place of G_parent for a root) is written to the
// output and read back by its children; a second walk turns every G_k into
// the skinning matrix G_k [I | -rest_k].  R(w) = I + a [w]x + b [w]x^2 with
// a = sin t / t and b = (1 - cos t) / t^2 = (sin(t/2) / (t/2))^2 / 2.
__global__ void __launch_bounds__(64) fk_kernel(const FkArgs f) {
    const int a = blockIdx.x * 64 + threadIdx.x;
    if (a >= f.n_avatars) return;
    float *out = f.out + (size_t)a * f.n_joints * 12;
    const float *root = f.root + (size_t)a * 12;
    for (int k = 0; k < f.n_joints; ++k) {
        const float *w = f.pose + ((size_t)a * f.n_joints + k) * 3;
        const float wx = w[0], wy = w[1], wz = w[2];
        const float t = sqrtf(wx * wx + wy * wy + wz * wz);
        float sa = 1.0f, sb = 0.5f;
        if (t > 0.0f) {
            sa = sinf(t) / t;
            const float h = sinf(0.5f * t) / (0.5f * t);
            sb = 0.5f * h * h;
        }
        // [w]x^2 = w w^T - |w|^2 I
        const float R[9] = {1.0f + sb * (wx * wx - t * t), sb * wx * wy - sa * wz, sb * wx * wz + sa * wy,
                            sb * wx * wy + sa * wz, 1.0f + sb * (wy * wy - t * t), sb * wy * wz - sa * wx,
                            sb * wx * wz - sa * wy, sb * wy * wz + sa * wx, 1.0f + sb * (wz * wz - t * t)};
        const int p = f.parents[k];
        float lt[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) lt[c] = f.rest[3 * k + c] - (p >= 0 ? f.rest[3 * p + c] : 0.0f);
        const float *P = p >= 0 ? out + (size_t)p * 12 : root;
        float G[12];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const float p0 = P[4 * r], p1 = P[4 * r + 1], p2 = P[4 * r + 2];
#pragma unroll
            for (int c = 0; c < 3; ++c) G[4 * r + c] = p0 * R[c] + p1 * R[3 + c] + p2 * R[6 + c];
            G[4 * r + 3] = p0 * lt[0] + p1 * lt[1] + p2 * lt[2] + P[4 * r + 3];
        }
#pragma unroll
        for (int e = 0; e < 12; ++e) out[(size_t)k * 12 + e] = G[e];
    }
    for (int k = 0; k < f.n_joints; ++k) {
        float *G = out + (size_t)k * 12;
        const float rx = f.rest[3 * k], ry = f.rest[3 * k + 1], rz = f.rest[3 * k + 2];
#pragma unroll
        for (int r = 0; r < 3; ++r) G[4 * r + 3] -= G[4 * r] * rx + G[4 * r + 1] * ry + G[4 * r + 2] * rz;
    }
}

hipError_t launch_fk(const FkArgs &f, hipStream_t s) {
    if (f.n_avatars <= 0) return hipSuccess;
    return launch_kernel(fk_kernel, dim3((unsigned)((f.n_avatars + 63) / 64)), dim3(64), s, f);
}

hipError_t launch_lbs(const LbsArgs &a, bool backward, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    const unsigned grid = (unsigned)((a.n + 255) / 256);
    if (a.clip) {
        if (backward) return launch_kernel(lbs_backward_kernel<true>, dim3(grid), dim3(256), s, a);
        return launch_kernel(lbs_kernel<true>, dim3(grid), dim3(256), s, a);
    }
    if (backward) return launch_kernel(lbs_backward_kernel<false>, dim3(grid), dim3(256), s, a);
    return launch_kernel(lbs_kernel<false>, dim3(grid), dim3(256), s, a);
}

}  // namespace gs
