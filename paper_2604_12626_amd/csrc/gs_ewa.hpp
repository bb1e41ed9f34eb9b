// EWA projection of one Gaussian into one view: the arithmetic shared by the
// forward projection kernel and the backward chain kernel (both must take the
// same FP32 decisions).
#pragma once

#include "gs_internal.hpp"

namespace gs {

// Camera staged in LDS: R (9), t (3), fx, fy, cx, cy, camera centre (3), pad.
constexpr int kCamStride = 20;

struct ViewProj {
    float tx, ty, tz;   // camera-space mean
    float u, v;         // projected mean
    float xr, yr;       // t_x/t_z, t_y/t_z after the tangent clamp
    bool clx, cly;      // the clamp was active
    float T0[3], T1[3]; // rows of T = J W
    float a, b, c;      // 2D covariance incl. low-pass
    float A, B, C;      // conic
    float inv_det;
    int radius;
    Rect rect;
};

// Returns false when the instance is culled (near plane, non-positive
// determinant, non-finite values, or an empty tile rect).
__device__ __forceinline__ bool ewa_project(const float *cam, float mx, float my, float mz, const float *S,
                                            int W, int H, int TX, int TY, float near_plane, float lowpass,
                                            float sigma_cut, float fov_clamp, ViewProj &o) {
    const float *R = cam;
    o.tx = R[0] * mx + R[1] * my + R[2] * mz + cam[9];
    o.ty = R[3] * mx + R[4] * my + R[5] * mz + cam[10];
    o.tz = R[6] * mx + R[7] * my + R[8] * mz + cam[11];
    if (!(o.tz > near_plane)) return false;
    const float fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15];
    const float iz = 1.0f / o.tz;
    o.u = fx * o.tx * iz + cx;
    o.v = fy * o.ty * iz + cy;
    const float limx = fov_clamp * (0.5f * (float)W / fx);
    const float limy = fov_clamp * (0.5f * (float)H / fy);
    const float xr0 = o.tx * iz, yr0 = o.ty * iz;
    o.clx = (xr0 < -limx) || (xr0 > limx);
    o.cly = (yr0 < -limy) || (yr0 > limy);
    o.xr = fminf(fmaxf(xr0, -limx), limx);
    o.yr = fminf(fmaxf(yr0, -limy), limy);
    // J = [[fx/z, 0, -fx xr/z], [0, fy/z, -fy yr/z]];  T = J W
    const float j00 = fx * iz, j02 = -fx * o.xr * iz, j11 = fy * iz, j12 = -fy * o.yr * iz;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        o.T0[k] = j00 * R[k] + j02 * R[6 + k];
        o.T1[k] = j11 * R[3 + k] + j12 * R[6 + k];
    }
    // Sigma as (xx, xy, xz, yy, yz, zz)
    const float s00 = S[0], s01 = S[1], s02 = S[2], s11 = S[3], s12 = S[4], s22 = S[5];
    const float m0x = s00 * o.T0[0] + s01 * o.T0[1] + s02 * o.T0[2];
    const float m0y = s01 * o.T0[0] + s11 * o.T0[1] + s12 * o.T0[2];
    const float m0z = s02 * o.T0[0] + s12 * o.T0[1] + s22 * o.T0[2];
    const float m1x = s00 * o.T1[0] + s01 * o.T1[1] + s02 * o.T1[2];
    const float m1y = s01 * o.T1[0] + s11 * o.T1[1] + s12 * o.T1[2];
    const float m1z = s02 * o.T1[0] + s12 * o.T1[1] + s22 * o.T1[2];
    o.a = o.T0[0] * m0x + o.T0[1] * m0y + o.T0[2] * m0z + lowpass;
    o.b = o.T1[0] * m0x + o.T1[1] * m0y + o.T1[2] * m0z;
    o.c = o.T1[0] * m1x + o.T1[1] * m1y + o.T1[2] * m1z + lowpass;
    // det = a c - b^2 with the rounding error of b^2 recovered by an FMA
    const float bb = o.b * o.b;
    const float bb_err = fmaf(o.b, o.b, -bb);
    const float det = fmaf(o.a, o.c, -bb) - bb_err;
    if (!(det > 0.0f)) return false;
    o.inv_det = 1.0f / det;
    o.A = o.c * o.inv_det;
    o.B = -o.b * o.inv_det;
    o.C = o.a * o.inv_det;
    // major eigenvalue with the 0.1 floor under the root; (m^2 - det) written
    // as ((a - c)/2)^2 + b^2, which has no cancellation
    const float m = 0.5f * (o.a + o.c);
    const float h = 0.5f * (o.a - o.c);
    const float disc = fmaxf(fmaf(h, h, bb), 0.1f);
    const float lam = m + sqrtf(disc);
    float rr = ceilf(sigma_cut * sqrtf(lam));
    if (!(rr == rr) || !isfinite(o.u) || !isfinite(o.v)) return false;
    rr = fminf(rr, kRadiusCap);
    o.radius = (int)rr;
    o.rect = tile_rect(o.u, o.v, o.radius, TX, TY);
    return o.rect.x0 < o.rect.x1 && o.rect.y0 < o.rect.y1;
}

}  // namespace gs
