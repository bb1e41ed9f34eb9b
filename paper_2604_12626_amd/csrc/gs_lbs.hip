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
