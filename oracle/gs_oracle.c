/*
 * gs_oracle.c -- plain, slow FP64 CPU oracle for the 3D Gaussian Splatting
 * sensor-rendering path of Habitat-GS (arXiv 2604.12626).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP implementation; neither
 * side includes or links the other.
 *
 * What it follows (the paper gives the system, the 3DGS lineage it cites
 * gives the arithmetic):
 *   - Sec. 2.2 "Neural Rendering": scenes are explicit anisotropic 3D
 *     Gaussians rendered by tile-based rasterization.
 *   - Sec. 3.1 "System Overview": per-Gaussian attributes are positions, SH
 *     coefficients, opacities, scales, rotations (and LBS weights for avatars);
 *     the render engine produces colour and depth.
 *   - Sec. 3.2 "3DGS Scene Rendering Integration": CUDA tile-based rendering;
 *     all avatars' deformed Gaussians rasterized in a single pass together
 *     with the scene (read here as one union index space).
 *   - Sec. 3.3 "Dynamic Gaussian Avatar Module": canonical Gaussians deformed
 *     by linear blend skinning with per-frame joint matrices.
 * Where the paper is silent the readings are the numbered ones of the design
 * document (camera axes, pixel centres, near plane, low-pass, 3-sigma radius,
 * rect rule, SH convention, thresholds as FP32 values, stop-before-composite,
 * z-depth output, union of avatars and scene).
 *
 * Every floating-point step is in double precision.  Inputs are the same FP32
 * arrays the GPU path consumes, promoted exactly.  The three compositing
 * thresholds are the FP32 values fl32(0.99), fl32(1/255), fl32(1e-4) promoted
 * to double (the caller passes them).
 *
 * Where a discrete decision (visibility at the near plane, the integer radius,
 * the floor of the projected mean, the alpha skip, the transmittance stop, the
 * depth order) lies within a stated relative margin of its threshold, the
 * oracle reports it, and for the two compositing decisions it enumerates both
 * outcomes (bounded depth): any of the enumerated results is a correct image
 * for an FP32 implementation of the same definition.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXL 8
#define OR_MAXK ((OR_MAXL + 1) * (OR_MAXL + 1))
#define OR_PROJ_STRIDE 40
#define OR_MAXC 8 /* candidate results per pixel */
#define OR_CAND_STRIDE 10

/* ------------------------------------------------------------------------ */
/* parameters and camera                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int W, H, tile;
    double near_plane, lowpass, sigma_cut, fov_clamp;
    double alpha_max, alpha_min, t_min;
    double bg[3];
    double d_skip, d_stop; /* relative margins of the two compositing decisions */
    double d_near, d_int;  /* margins of the near-plane test and integer decisions */
    double d_tie;          /* relative depth margin for order ties */
    int max_flips;
    double img_tol;        /* image tolerance a branch must meet to be taken as an implementation's */
} oprm;

/* prm layout: 0 W, 1 H, 2 near, 3 lowpass, 4 sigma_cut, 5 fov_clamp,
 * 6 alpha_max, 7 alpha_min, 8 t_min, 9..11 bg, 12 tile, 13 d_skip, 14 d_stop,
 * 15 d_near, 16 d_int, 17 d_tie, 18 max_flips, 19 img_tol */
static oprm unpack_prm(const double *p)
{
    oprm o;
    o.W = (int)p[0];
    o.H = (int)p[1];
    o.near_plane = p[2];
    o.lowpass = p[3];
    o.sigma_cut = p[4];
    o.fov_clamp = p[5];
    o.alpha_max = p[6];
    o.alpha_min = p[7];
    o.t_min = p[8];
    o.bg[0] = p[9];
    o.bg[1] = p[10];
    o.bg[2] = p[11];
    o.tile = (int)p[12];
    o.d_skip = p[13];
    o.d_stop = p[14];
    o.d_near = p[15];
    o.d_int = p[16];
    o.d_tie = p[17];
    o.max_flips = (int)p[18];
    o.img_tol = p[19];
    return o;
}

typedef struct {
    double R[9], t[3], fx, fy, cx, cy;
} ocam;

/* cam layout: R row-major (world -> camera, OpenCV axes), t, fx, fy, cx, cy */
static ocam unpack_cam(const double *c)
{
    ocam o;
    for (int i = 0; i < 9; ++i) o.R[i] = c[i];
    for (int i = 0; i < 3; ++i) o.t[i] = c[9 + i];
    o.fx = c[12];
    o.fy = c[13];
    o.cx = c[14];
    o.cy = c[15];
    return o;
}

/* ------------------------------------------------------------------------ */
/* real spherical harmonics (Condon-Shortley phase), l-major, m = -l..l       */
/* ------------------------------------------------------------------------ */
static double factorial(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

/* Legendre polynomial coefficients by Bonnet's recursion:
 * (l+1) P_{l+1}(z) = (2l+1) z P_l(z) - l P_{l-1}(z). */
static void legendre_coeffs(int L, double P[OR_MAXL + 1][OR_MAXL + 1])
{
    memset(P, 0, sizeof(double) * (OR_MAXL + 1) * (OR_MAXL + 1));
    P[0][0] = 1.0;
    if (L >= 1) P[1][1] = 1.0;
    for (int l = 1; l < L; ++l) {
        for (int k = 0; k <= l + 1; ++k) {
            double a = (k > 0) ? (2.0 * l + 1.0) * P[l][k - 1] : 0.0;
            double b = (k <= l - 1) ? l * P[l - 1][k] : 0.0;
            P[l + 1][k] = (a - b) / (l + 1.0);
        }
    }
}

static double poly_eval(const double *c, int deg, double z)
{
    double r = 0.0;
    for (int k = deg; k >= 0; --k) r = r * z + c[k];
    return r;
}

/* Y_lm(d) and its gradient w.r.t. d (as a polynomial in x, y, z; any smooth
 * extension off the unit sphere gives the same derivative once projected onto
 * the tangent plane).  On the unit sphere:
 *   m > 0 : sqrt2 K_l^m Re((x+iy)^m) Q_l^m(z)
 *   m < 0 : sqrt2 K_l^|m| Im((x+iy)^|m|) Q_l^|m|(z)
 *   m = 0 : K_l^0 P_l(z)
 * with Q_l^m(z) = (-1)^m d^m P_l / dz^m (the Condon-Shortley phase), so that
 * P_l^m(cos t) = Q_l^m(cos t) sin^m t, and
 * K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!). */
void or_sh_basis(int D, const double *d, double *Y, double *dY)
{
    double P[OR_MAXL + 1][OR_MAXL + 1];
    legendre_coeffs(D, P);
    const double x = d[0], y = d[1], z = d[2];
    for (int l = 0; l <= D; ++l) {
        double q[OR_MAXL + 1];
        memcpy(q, P[l], sizeof(q));
        int deg = l;
        double complex w = 1.0, wm1 = 0.0; /* (x+iy)^m and (x+iy)^(m-1) */
        for (int m = 0; m <= l; ++m) {
            if (m > 0) {
                for (int k = 0; k < deg; ++k) q[k] = (k + 1) * q[k + 1];
                q[deg] = 0.0;
                deg -= 1;
                wm1 = w;
                w = w * (x + I * y);
            }
            const double sgn = (m & 1) ? -1.0 : 1.0;
            const double Qv = sgn * poly_eval(q, deg, z);
            double dq[OR_MAXL + 1] = {0};
            for (int k = 0; k < deg; ++k) dq[k] = (k + 1) * q[k + 1];
            const double Qd = (deg > 0) ? sgn * poly_eval(dq, deg - 1, z) : 0.0;
            const double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - m) / factorial(l + m));
            if (m == 0) {
                const int k = l * l + l;
                Y[k] = K * Qv;
                if (dY) {
                    dY[3 * k + 0] = 0.0;
                    dY[3 * k + 1] = 0.0;
                    dY[3 * k + 2] = K * Qd;
                }
            } else {
                const double c = sqrt(2.0) * K;
                const double re = creal(w), im = cimag(w);
                /* d/dx (x+iy)^m = m (x+iy)^(m-1);  d/dy = i m (x+iy)^(m-1) */
                const double dre_dx = m * creal(wm1), dre_dy = -m * cimag(wm1);
                const double dim_dx = m * cimag(wm1), dim_dy = m * creal(wm1);
                const int kp = l * l + l + m, kn = l * l + l - m;
                Y[kp] = c * re * Qv;
                Y[kn] = c * im * Qv;
                if (dY) {
                    dY[3 * kp + 0] = c * dre_dx * Qv;
                    dY[3 * kp + 1] = c * dre_dy * Qv;
                    dY[3 * kp + 2] = c * re * Qd;
                    dY[3 * kn + 0] = c * dim_dx * Qv;
                    dY[3 * kn + 1] = c * dim_dy * Qv;
                    dY[3 * kn + 2] = c * im * Qd;
                }
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* small linear algebra                                                      */
/* ------------------------------------------------------------------------ */
/* unit quaternion (w, x, y, z) -> rotation matrix, row-major */
static void quat_to_rot(const double *q, double *R)
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* partial derivatives dR_ij / d(w, x, y, z) of quat_to_rot */
static void quat_to_rot_grad(const double *q, double dR[9][4])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    const double g[9][4] = {
        {0, 0, -4 * y, -4 * z},
        {-2 * z, 2 * y, 2 * x, -2 * w},
        {2 * y, 2 * z, 2 * w, 2 * x},
        {2 * z, 2 * y, 2 * x, 2 * w},
        {0, -4 * x, 0, -4 * z},
        {-2 * x, -2 * w, 2 * z, 2 * y},
        {-2 * y, 2 * z, -2 * w, 2 * x},
        {2 * x, 2 * w, 2 * z, 2 * y},
        {0, -4 * x, -4 * y, 0},
    };
    memcpy(dR, g, sizeof(g));
}

/* C = A (m x k) * B (k x n), row-major */
static void matmul(const double *A, const double *B, double *C, int m, int k, int n)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int l = 0; l < k; ++l) s += A[i * k + l] * B[l * n + j];
            C[i * n + j] = s;
        }
}

static void transpose(const double *A, double *AT, int m, int n)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) AT[j * m + i] = A[i * n + j];
}

/* ------------------------------------------------------------------------ */
/* projection of one Gaussian into one camera                                */
/* ------------------------------------------------------------------------ */

typedef struct {
    int vis, amb;
    double qn, q[4], R[9], s[3], Sig[9];
    int use_cov6;
    double tc[3], u, v, xr, yr;
    int clx, cly;
    double J[6], T[6], S2[3], det, conic[3], lam;
    int radius, rect[4], arect[4], irect[4];
    double dir[3], dist, raw[3], rgb[3], opacity;
    double m_near, m_rad, m_u, m_v;
} oproj;

static int64_t fdiv(int64_t a, int64_t b) /* floor division, b > 0 */
{
    return (a >= 0) ? a / b : -((-a + b - 1) / b);
}

/* Tiles whose pixel extent [tile*t, tile*t+tile) meets the closed square
 * [u-r, u+r] x [v-r, v+r]; with ix = floor(u), iy = floor(v) and an integer r
 * this is exactly x in [fdiv(ix-r, tile), fdiv(ix+r, tile)] clipped to the
 * grid (and likewise in y). */
static void rect_of(int64_t ix, int64_t iy, int64_t r, int TX, int TY, int tile, int *rect)
{
    int64_t x0 = fdiv(ix - r, tile), x1 = fdiv(ix + r, tile) + 1;
    int64_t y0 = fdiv(iy - r, tile), y1 = fdiv(iy + r, tile) + 1;
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    if (x1 > TX) x1 = TX;
    if (y1 > TY) y1 = TY;
    rect[0] = (int)x0;
    rect[1] = (int)x1;
    rect[2] = (int)y0;
    rect[3] = (int)y1;
}

static int rect_empty(const int *r) { return r[0] >= r[1] || r[2] >= r[3]; }

#define OR_COORD_CLAMP 1048576.0 /* 2^20: projected means are clamped before floor */
#define OR_RADIUS_CAP 16777216   /* 2^24: larger radii cover every tile anyway */

static int64_t radius_of(double x)
{
    double c = ceil(x);
    if (c > OR_RADIUS_CAP) c = OR_RADIUS_CAP;
    return (int64_t)c;
}

/* One Gaussian's parameters in double precision (FP32 inputs are promoted
 * exactly; the finite-difference checks perturb them below FP32 resolution). */
typedef struct {
    int D, use_cov6;
    double mean[3], lsc[3], q[4], cov6[6], opac;
    double sh[3 * OR_MAXK];
} oin;

static void load_in(int D, const float *mean, const float *lsc, const float *quat, const float *cov6, float opac,
                    const float *sh, oin *g)
{
    memset(g, 0, sizeof(*g));
    g->D = D;
    for (int k = 0; k < 3; ++k) g->mean[k] = mean[k];
    if (cov6) {
        g->use_cov6 = 1;
        for (int k = 0; k < 6; ++k) g->cov6[k] = cov6[k];
    } else {
        for (int k = 0; k < 3; ++k) g->lsc[k] = lsc[k];
        for (int k = 0; k < 4; ++k) g->q[k] = quat[k];
    }
    g->opac = opac;
    for (int k = 0; k < 3 * (D + 1) * (D + 1); ++k) g->sh[k] = sh[k];
}

static void project_one(const oprm *p, const ocam *cam, const oin *g, oproj *o)
{
    const int D = g->D;
    memset(o, 0, sizeof(*o));
    o->opacity = g->opac;
    const double mu[3] = {g->mean[0], g->mean[1], g->mean[2]};
    if (!isfinite(o->opacity)) return; /* non-finite input is culled (vis = 0) */
    /* O1/O2: covariance */
    if (g->use_cov6) {
        const double *cov6 = g->cov6;
        o->use_cov6 = 1;
        o->Sig[0] = cov6[0];
        o->Sig[1] = o->Sig[3] = cov6[1];
        o->Sig[2] = o->Sig[6] = cov6[2];
        o->Sig[4] = cov6[3];
        o->Sig[5] = o->Sig[7] = cov6[4];
        o->Sig[8] = cov6[5];
    } else {
        double q[4] = {g->q[0], g->q[1], g->q[2], g->q[3]};
        double n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
        if (!(n2 >= 1e-24)) {
            o->qn = 0.0;
            o->q[0] = 1.0;
            o->q[1] = o->q[2] = o->q[3] = 0.0;
        } else {
            o->qn = sqrt(n2);
            for (int i = 0; i < 4; ++i) o->q[i] = q[i] / o->qn;
        }
        quat_to_rot(o->q, o->R);
        for (int i = 0; i < 3; ++i) o->s[i] = exp(g->lsc[i]);
        double M[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) M[3 * i + j] = o->R[3 * i + j] * o->s[j];
        double MT[9];
        transpose(M, MT, 3, 3);
        matmul(M, MT, o->Sig, 3, 3, 3);
    }
    /* O3: camera-space mean and near-plane cull */
    const double *W = cam->R;
    double mag = fabs(cam->t[2]);
    for (int i = 0; i < 3; ++i) {
        o->tc[i] = cam->t[i];
        for (int j = 0; j < 3; ++j) o->tc[i] += W[3 * i + j] * mu[j];
    }
    for (int j = 0; j < 3; ++j) mag += fabs(W[6 + j] * mu[j]);
    const double tx = o->tc[0], ty = o->tc[1], tz = o->tc[2];
    o->m_near = (tz - p->near_plane) / (mag > 1.0 ? mag : 1.0);
    if (!(tz > p->near_plane)) {
        o->vis = 0;
        o->amb = fabs(o->m_near) <= p->d_near;
        return;
    }
    /* O4: projected mean; pixel (x, y) samples (x + 1/2, y + 1/2) */
    o->u = cam->fx * tx / tz + cam->cx;
    o->v = cam->fy * ty / tz + cam->cy;
    /* O5: Jacobian with the tangent clamp */
    const double limx = p->fov_clamp * (0.5 * p->W / cam->fx);
    const double limy = p->fov_clamp * (0.5 * p->H / cam->fy);
    double xr = tx / tz, yr = ty / tz;
    o->clx = (xr < -limx) || (xr > limx);
    o->cly = (yr < -limy) || (yr > limy);
    if (xr < -limx) xr = -limx;
    if (xr > limx) xr = limx;
    if (yr < -limy) yr = -limy;
    if (yr > limy) yr = limy;
    o->xr = xr;
    o->yr = yr;
    o->J[0] = cam->fx / tz;
    o->J[1] = 0.0;
    o->J[2] = -cam->fx * xr / tz;
    o->J[3] = 0.0;
    o->J[4] = cam->fy / tz;
    o->J[5] = -cam->fy * yr / tz;
    /* O6: 2D covariance with the low-pass, conic */
    matmul(o->J, W, o->T, 2, 3, 3);
    double TS[6], TT[6], S2m[4];
    matmul(o->T, o->Sig, TS, 2, 3, 3);
    transpose(o->T, TT, 2, 3);
    matmul(TS, TT, S2m, 2, 3, 2);
    const double a = S2m[0] + p->lowpass, b = 0.5 * (S2m[1] + S2m[2]), c = S2m[3] + p->lowpass;
    o->S2[0] = a;
    o->S2[1] = b;
    o->S2[2] = c;
    o->det = a * c - b * b;
    if (!(o->det > 0.0)) {
        o->vis = 0;
        return;
    }
    o->conic[0] = c / o->det;
    o->conic[1] = -b / o->det;
    o->conic[2] = a / o->det;
    /* O7: radius from the major eigenvalue */
    const double m = 0.5 * (a + c);
    double disc = m * m - o->det;
    if (disc < 0.1) disc = 0.1;
    o->lam = m + sqrt(disc);
    const double rr = p->sigma_cut * sqrt(o->lam);
    if (!isfinite(rr) || !isfinite(o->u) || !isfinite(o->v)) {
        o->vis = 0;
        return;
    }
    const int64_t r = radius_of(rr);
    o->radius = (int)r;
    o->m_rad = fabs(rr - nearbyint(rr)) / (rr > 1.0 ? rr : 1.0);
    /* O8: tile rect */
    double uc = o->u, vc = o->v;
    if (uc < -OR_COORD_CLAMP) uc = -OR_COORD_CLAMP;
    if (uc > OR_COORD_CLAMP) uc = OR_COORD_CLAMP;
    if (vc < -OR_COORD_CLAMP) vc = -OR_COORD_CLAMP;
    if (vc > OR_COORD_CLAMP) vc = OR_COORD_CLAMP;
    const int64_t ix = (int64_t)floor(uc), iy = (int64_t)floor(vc);
    o->m_u = fabs(uc - nearbyint(uc)) / (fabs(uc) > 1.0 ? fabs(uc) : 1.0);
    o->m_v = fabs(vc - nearbyint(vc)) / (fabs(vc) > 1.0 ? fabs(vc) : 1.0);
    const int TX = (p->W + p->tile - 1) / p->tile, TY = (p->H + p->tile - 1) / p->tile;
    rect_of(ix, iy, r, TX, TY, p->tile, o->rect);
    /* alternatives within the integer-decision margins */
    int64_t ixs[2] = {ix, ix}, iys[2] = {iy, iy}, rs[2] = {r, r};
    if (o->m_u <= p->d_int) {
        ixs[0] = (int64_t)nearbyint(uc) - 1;
        ixs[1] = (int64_t)nearbyint(uc);
    }
    if (o->m_v <= p->d_int) {
        iys[0] = (int64_t)nearbyint(vc) - 1;
        iys[1] = (int64_t)nearbyint(vc);
    }
    if (o->m_rad <= p->d_int) {
        rs[0] = radius_of(nearbyint(rr));
        rs[1] = radius_of(nearbyint(rr) + 0.5);
    }
    memcpy(o->arect, o->rect, sizeof(o->rect));
    memcpy(o->irect, o->rect, sizeof(o->rect));
    int any_empty = rect_empty(o->rect), all_empty = rect_empty(o->rect);
    for (int a0 = 0; a0 < 2; ++a0)
        for (int a1 = 0; a1 < 2; ++a1)
            for (int a2 = 0; a2 < 2; ++a2) {
                int rc[4];
                rect_of(ixs[a0], iys[a1], rs[a2], TX, TY, p->tile, rc);
                if (memcmp(rc, o->rect, sizeof(rc)) != 0) o->amb = 1;
                if (rc[0] > o->irect[0]) o->irect[0] = rc[0];
                if (rc[1] < o->irect[1]) o->irect[1] = rc[1];
                if (rc[2] > o->irect[2]) o->irect[2] = rc[2];
                if (rc[3] < o->irect[3]) o->irect[3] = rc[3];
                if (!rect_empty(rc)) {
                    if (all_empty) {
                        memcpy(o->arect, rc, sizeof(rc));
                        all_empty = 0;
                    } else {
                        if (rc[0] < o->arect[0]) o->arect[0] = rc[0];
                        if (rc[1] > o->arect[1]) o->arect[1] = rc[1];
                        if (rc[2] < o->arect[2]) o->arect[2] = rc[2];
                        if (rc[3] > o->arect[3]) o->arect[3] = rc[3];
                    }
                } else {
                    any_empty = 1;
                }
            }
    (void)any_empty;
    if (fabs(o->m_near) <= p->d_near) {
        o->amb = 1;
        memset(o->irect, 0, sizeof(o->irect)); /* the alternative is "not visible" */
    }
    if (rect_empty(o->rect)) {
        o->vis = 0;
        return;
    }
    o->vis = 1;
    /* O9: view-dependent colour from SH, world-space direction from the camera centre */
    double cpos[3];
    for (int j = 0; j < 3; ++j) cpos[j] = -(W[0 + j] * cam->t[0] + W[3 + j] * cam->t[1] + W[6 + j] * cam->t[2]);
    double dv[3] = {mu[0] - cpos[0], mu[1] - cpos[1], mu[2] - cpos[2]};
    o->dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    for (int j = 0; j < 3; ++j) o->dir[j] = dv[j] / o->dist;
    double Y[OR_MAXK];
    or_sh_basis(D, o->dir, Y, NULL);
    const int K = (D + 1) * (D + 1);
    for (int ch = 0; ch < 3; ++ch) {
        double s = 0.0;
        for (int k = 0; k < K; ++k) s += Y[k] * g->sh[3 * k + ch];
        o->raw[ch] = s + 0.5;
        o->rgb[ch] = o->raw[ch] > 0.0 ? o->raw[ch] : 0.0;
    }
}

/* O1/O2 alone: 3D covariance (xx, xy, xz, yy, yz, zz) from log-scales and
 * quaternions, for the pins of the rotation and covariance steps. */
void or_cov3d(int64_t n, const float *lsc, const float *quats, double *cov6)
{
    for (int64_t i = 0; i < n; ++i) {
        oproj o;
        oprm p;
        ocam c;
        memset(&p, 0, sizeof(p));
        memset(&c, 0, sizeof(c));
        const float zero3[3] = {0, 0, 0}, sh0[3] = {0, 0, 0};
        p.near_plane = 1e300; /* cull right after the covariance step */
        oin g;
        load_in(0, zero3, lsc + 3 * i, quats + 4 * i, NULL, 0.5f, sh0, &g);
        project_one(&p, &c, &g, &o);
        cov6[6 * i + 0] = o.Sig[0];
        cov6[6 * i + 1] = o.Sig[1];
        cov6[6 * i + 2] = o.Sig[2];
        cov6[6 * i + 3] = o.Sig[4];
        cov6[6 * i + 4] = o.Sig[5];
        cov6[6 * i + 5] = o.Sig[8];
    }
}

/* Per-Gaussian projection for one camera.  out: [n][OR_PROJ_STRIDE]
 *  0 vis, 1 u, 2 v, 3 depth, 4 A, 5 B, 6 C, 7 opacity, 8..10 rgb, 11 radius,
 *  12..15 rect x0 x1 y0 y1, 16 lambda, 17 near margin, 18 radius margin,
 *  19 u margin, 20 v margin, 21 ambiguous, 22..25 union rect, 26..28 a b c,
 *  29..31 raw colour before the clamp, 32..35 intersection of the rects over
 *  the ambiguous alternatives (empty if an alternative is "culled"). */
void or_project(int64_t n, int D, const float *means, const float *lsc, const float *quats, const float *cov6,
                const uint8_t *use_cov6, const float *opacity, const float *sh, const double *camp,
                const double *prm, double *out)
{
    const oprm p = unpack_prm(prm);
    const ocam cam = unpack_cam(camp);
    const int K = (D + 1) * (D + 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        oproj o;
        const float *c6 = (cov6 && (!use_cov6 || use_cov6[i])) ? cov6 + 6 * i : NULL;
        oin g;
        load_in(D, means + 3 * i, lsc ? lsc + 3 * i : NULL, quats ? quats + 4 * i : NULL, c6, opacity[i],
                sh + (size_t)3 * K * i, &g);
        project_one(&p, &cam, &g, &o);
        double *r = out + OR_PROJ_STRIDE * i;
        memset(r, 0, sizeof(double) * OR_PROJ_STRIDE);
        r[0] = o.vis;
        r[1] = o.u;
        r[2] = o.v;
        r[3] = o.tc[2];
        r[4] = o.conic[0];
        r[5] = o.conic[1];
        r[6] = o.conic[2];
        r[7] = o.opacity;
        r[8] = o.rgb[0];
        r[9] = o.rgb[1];
        r[10] = o.rgb[2];
        r[11] = o.radius;
        for (int k = 0; k < 4; ++k) r[12 + k] = o.rect[k];
        r[16] = o.lam;
        r[17] = o.m_near;
        r[18] = o.m_rad;
        r[19] = o.m_u;
        r[20] = o.m_v;
        r[21] = o.amb;
        for (int k = 0; k < 4; ++k) r[22 + k] = o.arect[k];
        r[26] = o.S2[0];
        r[27] = o.S2[1];
        r[28] = o.S2[2];
        r[29] = o.raw[0];
        r[30] = o.raw[1];
        r[31] = o.raw[2];
        for (int k = 0; k < 4; ++k) r[32 + k] = o.irect[k];
    }
}

/* ------------------------------------------------------------------------ */
/* binning: (tile, depth) keys from FP32 records, stable order               */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t key;
    uint32_t val;
} okv;

static int cmp_kv(const void *a, const void *b)
{
    const okv *x = (const okv *)a, *y = (const okv *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->val != y->val) return x->val < y->val ? -1 : 1;
    return 0;
}

static uint32_t f32_bits(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

/* Record layout read here (the GPU path's projected record, 12 floats):
 *   0 u, 1 v, 2 depth, 3 radius (int32 bits), ..., 11 view (int32 bits).
 * For every instance with visible[i] != 0: rect from (floor(u), floor(v), r),
 * tiles_touched[i] = rect area, and one key per covered tile in row-major
 * order: key = ((view * T + ty * TX + tx) << 32) | bits(fp32 depth), value = i.
 * The keys are then sorted ascending with ties broken by the value (the order
 * a stable sort of index-ordered emission gives).  ranges[t] = [first, last+1)
 * of tile t's run (0, 0 when empty).  Writes at most `capacity` pairs; returns
 * the total number K. */
int64_t or_bin(int64_t m, const float *rec, const uint8_t *visible, int W, int H, int tile, int n_views,
               uint32_t *tiles_touched, uint64_t *keys, uint32_t *vals, int64_t capacity, uint32_t *ranges)
{
    const int TX = (W + tile - 1) / tile, TY = (H + tile - 1) / tile, T = TX * TY;
    int64_t K = 0;
    for (int64_t i = 0; i < m; ++i) {
        tiles_touched[i] = 0;
        if (!visible[i]) continue;
        const float *r = rec + 12 * i;
        int32_t rad, view;
        memcpy(&rad, r + 3, 4);
        memcpy(&view, r + 11, 4);
        double uc = r[0], vc = r[1];
        if (uc < -OR_COORD_CLAMP) uc = -OR_COORD_CLAMP;
        if (uc > OR_COORD_CLAMP) uc = OR_COORD_CLAMP;
        if (vc < -OR_COORD_CLAMP) vc = -OR_COORD_CLAMP;
        if (vc > OR_COORD_CLAMP) vc = OR_COORD_CLAMP;
        int rc[4];
        rect_of((int64_t)floor(uc), (int64_t)floor(vc), rad, TX, TY, tile, rc);
        if (rect_empty(rc)) continue;
        tiles_touched[i] = (uint32_t)((rc[1] - rc[0]) * (rc[3] - rc[2]));
        K += tiles_touched[i];
    }
    okv *kv = (okv *)malloc(sizeof(okv) * (K > 0 ? K : 1));
    int64_t k = 0;
    for (int64_t i = 0; i < m; ++i) {
        if (!tiles_touched[i]) continue;
        const float *r = rec + 12 * i;
        int32_t rad, view;
        memcpy(&rad, r + 3, 4);
        memcpy(&view, r + 11, 4);
        double uc = r[0], vc = r[1];
        if (uc < -OR_COORD_CLAMP) uc = -OR_COORD_CLAMP;
        if (uc > OR_COORD_CLAMP) uc = OR_COORD_CLAMP;
        if (vc < -OR_COORD_CLAMP) vc = -OR_COORD_CLAMP;
        if (vc > OR_COORD_CLAMP) vc = OR_COORD_CLAMP;
        int rc[4];
        rect_of((int64_t)floor(uc), (int64_t)floor(vc), rad, TX, TY, tile, rc);
        for (int ty = rc[2]; ty < rc[3]; ++ty)
            for (int tx = rc[0]; tx < rc[1]; ++tx) {
                const uint64_t tg = (uint64_t)view * T + (uint64_t)ty * TX + tx;
                kv[k].key = (tg << 32) | f32_bits(r[2]);
                kv[k].val = (uint32_t)i;
                ++k;
            }
    }
    qsort(kv, K, sizeof(okv), cmp_kv);
    for (int64_t t = 0; t < (int64_t)n_views * T; ++t) ranges[2 * t] = ranges[2 * t + 1] = 0;
    for (int64_t j = 0; j < K; ++j) {
        if (j < capacity) {
            keys[j] = kv[j].key;
            vals[j] = kv[j].val;
        }
        const uint64_t tg = kv[j].key >> 32;
        if (j == 0 || (kv[j - 1].key >> 32) != tg) ranges[2 * tg] = (uint32_t)j;
        if (j == K - 1 || (kv[j + 1].key >> 32) != tg) ranges[2 * tg + 1] = (uint32_t)(j + 1);
    }
    free(kv);
    return K;
}

/* ------------------------------------------------------------------------ */
/* compositing with enumeration of near-threshold decisions                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    const double *u, *v, *A, *B, *C, *o, *z, *rgb; /* per-entry (gathered) */
    const int *idx;
    int len;
    double px, py;
    const oprm *p;
} octx;

typedef struct {
    double c[3], d, T;
    double eT; /* bound on the relative error of an FP32 evaluation of T */
    int n;
    int ncomp;    /* number of composited entries */
    uint32_t sig; /* signature of the composited index set */
} ostate;

typedef struct {
    int n;
    /* r, g, b, depth, alpha, T, n_contrib, flips used, composited count, set signature */
    double r[OR_MAXC][OR_CAND_STRIDE];
    int truncated;
    int saw_amb; /* some decision on the explored paths lay inside its margin */
} ocands;

enum { OUT_SKIP = 0, OUT_STOP = 1, OUT_COMP = 2 };

/* Bound on the error of log(alpha) as an FP32 implementation evaluates it
 * from the same record at the same pixel.  The exponent is a sum of terms of
 * total magnitude S = |A| dx^2 / 2 + |C| dy^2 / 2 + |B dx dy|; the pixel
 * offsets, the products and the sum each round to 2^-24 of a partial sum
 * (plus a rescaling of the conic for a base-2 exponential), so its absolute
 * error is a few units of 2^-24 S; the exponential, the opacity product and
 * the clamp add a few units of 2^-24.  For a needle-shaped Gaussian far along
 * its axis S exceeds |P| by orders of magnitude, and so does this bound the
 * fixed window d_skip.  Windows are therefore taken on log(alpha):
 * |log(alpha / alpha_min)| <= log(1 + d_skip) + this bound. */
#define OR_FP32_ROUNDINGS 16.0
static double fp32_alpha_err(double S) { return OR_FP32_ROUNDINGS * 0x1p-24 * (S + 1.0); }

/* the skip window of an entry on log(alpha), and whether alpha lies in it */
static double skip_window(const oprm *p, double err) { return log1p(p->d_skip) + err; }
static int in_skip_window(double a, double amin, double w) { return a > 0.0 && fabs(log(a / amin)) <= w; }

static double exponent_terms(double A, double B, double C, double dx, double dy)
{
    return 0.5 * fabs(A) * dx * dx + 0.5 * fabs(C) * dy * dy + fabs(B * dx * dy);
}

/* relative error bound of T (1 - alpha) given those of T and of alpha */
static double next_eT(double eT, double a, double ea) { return eT + a / (1.0 - a) * (ea + 0x1p-24) + 0x1p-24; }

static void entry_alpha(const octx *cx, int j, double *alpha, double *err, double *G, int *clamped, double *dx,
                        double *dy)
{
    const double ddx = cx->px - cx->u[j], ddy = cx->py - cx->v[j];
    double P = -0.5 * (cx->A[j] * ddx * ddx + cx->C[j] * ddy * ddy) - cx->B[j] * ddx * ddy;
    if (err) *err = fp32_alpha_err(exponent_terms(cx->A[j], cx->B[j], cx->C[j], ddx, ddy));
    if (P > 0.0) P = 0.0;
    const double g = exp(P);
    double a = cx->o[j] * g;
    int cl = 0;
    if (a > cx->p->alpha_max) {
        /* clamped on both sides: the FP32 value is the clamp constant itself */
        if (err && a >= cx->p->alpha_max * exp(*err)) *err = 0.0;
        a = cx->p->alpha_max;
        cl = 1;
    }
    *alpha = a;
    if (G) *G = g;
    if (clamped) *clamped = cl;
    if (dx) *dx = ddx;
    if (dy) *dy = ddy;
}

static void push_cand(ocands *cb, const ostate *s, const oprm *p, int flips_used)
{
    if (cb->n >= OR_MAXC) {
        cb->truncated = 1;
        return;
    }
    double *r = cb->r[cb->n++];
    for (int ch = 0; ch < 3; ++ch) r[ch] = s->c[ch] + s->T * p->bg[ch];
    r[3] = s->d;
    r[4] = 1.0 - s->T;
    r[5] = s->T;
    r[6] = s->n;
    r[7] = flips_used;
    r[8] = s->ncomp;
    r[9] = s->sig;
}

static void apply_comp(const octx *cx, int j, double a, double ea, ostate *s)
{
    for (int ch = 0; ch < 3; ++ch) s->c[ch] += cx->rgb[3 * j + ch] * a * s->T;
    s->d += cx->z[j] * a * s->T;
    s->T = s->T * (1.0 - a);
    s->eT = next_eT(s->eT, a, ea);
    s->n = j + 1;
    s->ncomp += 1;
    s->sig = s->sig * 1000003u + (uint32_t)(j + 1);
}

/* O11: front-to-back over the entry list; every decision within its window
 * (the fixed d_skip / d_stop plus the FP32 rounding bound of that entry's
 * alpha and of the transmittance so far) is explored both ways while flips
 * remain. */
static void comp_rec(const octx *cx, int j, ostate s, int flips, int used, ocands *cb)
{
    const oprm *p = cx->p;
    for (; j < cx->len; ++j) {
        double a, ea;
        entry_alpha(cx, j, &a, &ea, NULL, NULL, NULL, NULL);
        const double Tn = s.T * (1.0 - a);
        const int skip = a < p->alpha_min;
        const int stop = Tn < p->t_min;
        const int primary = skip ? OUT_SKIP : (stop ? OUT_STOP : OUT_COMP);
        const int amb_skip = in_skip_window(a, p->alpha_min, skip_window(p, ea));
        const int amb_stop = fabs(Tn - p->t_min) <= (p->d_stop + next_eT(s.eT, a, ea)) * p->t_min;
        if (amb_skip || (amb_stop && !skip)) cb->saw_amb = 1;
        if (flips > 0) {
            int alts[3] = {0, 0, 0};
            if (amb_skip) {
                alts[OUT_SKIP] = 1;
                alts[stop ? OUT_STOP : OUT_COMP] = 1;
            }
            if (amb_stop && (!skip || amb_skip)) {
                alts[OUT_STOP] = 1;
                alts[OUT_COMP] = 1;
            }
            for (int alt = 0; alt < 3; ++alt) {
                if (!alts[alt] || alt == primary) continue;
                ostate s2 = s;
                if (alt == OUT_STOP) {
                    push_cand(cb, &s2, p, used + 1);
                } else if (alt == OUT_SKIP) {
                    comp_rec(cx, j + 1, s2, flips - 1, used + 1, cb);
                } else {
                    apply_comp(cx, j, a, ea, &s2);
                    comp_rec(cx, j + 1, s2, flips - 1, used + 1, cb);
                }
            }
        }
        if (primary == OUT_SKIP) continue;
        if (primary == OUT_STOP) {
            push_cand(cb, &s, p, used);
            return;
        }
        apply_comp(cx, j, a, ea, &s);
    }
    push_cand(cb, &s, p, used);
}

/* Composite one pixel: fills cands (candidate 0 is the unperturbed result). */
static void composite_pixel(const octx *cx, ocands *cb)
{
    ostate s;
    memset(&s, 0, sizeof(s));
    s.T = 1.0;
    cb->n = 0;
    cb->truncated = 0;
    cb->saw_amb = 0;
    /* the primary path must be candidate 0: run it first with no flips */
    comp_rec(cx, 0, s, 0, 0, cb);
    if (cx->p->max_flips > 0 && cb->saw_amb) {
        ocands alt;
        alt.n = 0;
        alt.truncated = 0;
        alt.saw_amb = 0;
        comp_rec(cx, 0, s, cx->p->max_flips, 0, &alt);
        for (int k = 0; k < alt.n; ++k) {
            if (alt.r[k][7] == 0) continue; /* the primary path again */
            if (cb->n >= OR_MAXC) {
                cb->truncated = 1;
                break;
            }
            memcpy(cb->r[cb->n++], alt.r[k], sizeof(alt.r[k]));
        }
        cb->truncated |= alt.truncated;
    }
}

typedef struct {
    double u, v, A, B, C, o, z, rgb[3];
} oentry;

/* composite every pixel of one tile from gathered entries */
static void composite_tile(const oprm *p, const oentry *ents, int len, int tx, int ty, double *img /*[H][W][10]*/,
                           int32_t *ncand, double *cands /*[H][W][MAXC][8] nullable*/)
{
    double *u = malloc(sizeof(double) * (len + 1) * 10);
    double *v = u + (len + 1), *A = v + (len + 1), *B = A + (len + 1), *C = B + (len + 1), *o = C + (len + 1),
           *z = o + (len + 1), *rgb = z + (len + 1);
    for (int j = 0; j < len; ++j) {
        u[j] = ents[j].u;
        v[j] = ents[j].v;
        A[j] = ents[j].A;
        B[j] = ents[j].B;
        C[j] = ents[j].C;
        o[j] = ents[j].o;
        z[j] = ents[j].z;
        rgb[3 * j + 0] = ents[j].rgb[0];
        rgb[3 * j + 1] = ents[j].rgb[1];
        rgb[3 * j + 2] = ents[j].rgb[2];
    }
    octx cx = {u, v, A, B, C, o, z, rgb, NULL, len, 0, 0, p};
    for (int py = ty * p->tile; py < (ty + 1) * p->tile && py < p->H; ++py)
        for (int px = tx * p->tile; px < (tx + 1) * p->tile && px < p->W; ++px) {
            cx.px = px + 0.5;
            cx.py = py + 0.5;
            ocands cb;
            composite_pixel(&cx, &cb);
            double *out = img + OR_CAND_STRIDE * ((size_t)py * p->W + px);
            for (int k = 0; k < OR_CAND_STRIDE; ++k) out[k] = cb.r[0][k];
            ncand[(size_t)py * p->W + px] = cb.truncated ? -cb.n : cb.n;
            if (cands) {
                double *cc = cands + (size_t)OR_MAXC * OR_CAND_STRIDE * ((size_t)py * p->W + px);
                for (int c = 0; c < OR_MAXC; ++c)
                    for (int k = 0; k < OR_CAND_STRIDE; ++k) cc[c * OR_CAND_STRIDE + k] = c < cb.n ? cb.r[c][k] : NAN;
            }
        }
    free(u);
}

/* Composite from FP32 records and sorted per-tile lists (O11), one view at a
 * time.  rec: [m][12] (0 u, 1 v, 2 depth, 3 radius bits, 4 A, 5 B, 6 C,
 * 7 opacity, 8..10 rgb, 11 view bits); vals/ranges as produced by or_bin.
 * img: [V][H][W][10] = r, g, b, depth, alpha, T, n_contrib, flips (0),
 * composited count, composited-set signature; ncand
 * [V][H][W] (negative when the candidate list was truncated); cands optional. */
void or_composite(int n_views, const float *rec, const uint32_t *vals, const uint32_t *ranges, const double *prm,
                  double *img, int32_t *ncand, double *cands)
{
    const oprm p = unpack_prm(prm);
    const int TX = (p.W + p.tile - 1) / p.tile, TY = (p.H + p.tile - 1) / p.tile, T = TX * TY;
    const size_t HW = (size_t)p.H * p.W;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < (int64_t)n_views * T; ++t) {
        const int view = (int)(t / T), tt = (int)(t % T);
        const uint32_t b = ranges[2 * t], e = ranges[2 * t + 1];
        const int len = (int)(e - b);
        oentry *ents = malloc(sizeof(oentry) * (len + 1));
        for (int j = 0; j < len; ++j) {
            const float *r = rec + 12 * (size_t)vals[b + j];
            ents[j].u = r[0];
            ents[j].v = r[1];
            ents[j].z = r[2];
            ents[j].A = r[4];
            ents[j].B = r[5];
            ents[j].C = r[6];
            ents[j].o = r[7];
            ents[j].rgb[0] = r[8];
            ents[j].rgb[1] = r[9];
            ents[j].rgb[2] = r[10];
        }
        composite_tile(&p, ents, len, tt % TX, tt / TX, img + OR_CAND_STRIDE * HW * view, ncand + HW * view,
                       cands ? cands + (size_t)OR_MAXC * OR_CAND_STRIDE * HW * view : NULL);
        free(ents);
    }
}

/* ------------------------------------------------------------------------ */
/* fully independent FP64 render of one view                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    double z;
    int64_t i;
} ozi;

static int cmp_zi(const void *a, const void *b)
{
    const ozi *x = (const ozi *)a, *y = (const ozi *)b;
    if (x->z != y->z) return x->z < y->z ? -1 : 1;
    if (x->i != y->i) return x->i < y->i ? -1 : 1;
    return 0;
}

/* Builds the per-tile depth-ordered lists of the oracle's own projection.
 * list_ptr [T+1], list_idx [sum] (caller frees *list_idx). */
static void build_lists(const oprm *p, int64_t n, const double *proj, int64_t **list_ptr, int64_t **list_idx)
{
    const int TX = (p->W + p->tile - 1) / p->tile, TY = (p->H + p->tile - 1) / p->tile, T = TX * TY;
    int64_t *cnt = calloc((size_t)(T > 0 ? T : 0) + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        const double *r = proj + OR_PROJ_STRIDE * i;
        if (r[0] == 0.0) continue;
        for (int ty = (int)r[14]; ty < (int)r[15]; ++ty)
            for (int tx = (int)r[12]; tx < (int)r[13]; ++tx) cnt[ty * TX + tx + 1]++;
    }
    for (int t = 0; t < T; ++t) cnt[t + 1] += cnt[t];
    int64_t *idx = malloc(sizeof(int64_t) * (cnt[T] + 1));
    int64_t *fill = calloc((size_t)(T > 0 ? T : 1), sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        const double *r = proj + OR_PROJ_STRIDE * i;
        if (r[0] == 0.0) continue;
        for (int ty = (int)r[14]; ty < (int)r[15]; ++ty)
            for (int tx = (int)r[12]; tx < (int)r[13]; ++tx) {
                const int t = ty * TX + tx;
                idx[cnt[t] + fill[t]++] = i;
            }
    }
    free(fill);
    for (int t = 0; t < T; ++t) {
        const int64_t len = cnt[t + 1] - cnt[t];
        ozi *zi = malloc(sizeof(ozi) * (len + 1));
        for (int64_t j = 0; j < len; ++j) {
            zi[j].i = idx[cnt[t] + j];
            zi[j].z = proj[OR_PROJ_STRIDE * zi[j].i + 3];
        }
        qsort(zi, len, sizeof(ozi), cmp_zi);
        for (int64_t j = 0; j < len; ++j) idx[cnt[t] + j] = zi[j].i;
        free(zi);
    }
    *list_ptr = cnt;
    *list_idx = idx;
}

/* Pixels where a Gaussian with an ambiguous rect or visibility reaches the
 * skip threshold (within its margin) in a tile that only some of its
 * alternative rects cover: bit 0 of flags. */
static void rect_flags(const oprm *pp, int64_t n, const double *proj, uint8_t *flags)
{
    const oprm p = *pp;
    for (int64_t i = 0; i < n; ++i) {
        const double *r = proj + OR_PROJ_STRIDE * i;
        if (r[21] == 0.0) continue;
        int x0 = (int)r[22], x1 = (int)r[23], y0 = (int)r[24], y1 = (int)r[25];
        if (r[0] != 0.0) {
            if (r[12] < x0) x0 = (int)r[12];
            if (r[13] > x1) x1 = (int)r[13];
            if (r[14] < y0) y0 = (int)r[14];
            if (r[15] > y1) y1 = (int)r[15];
        }
        if (r[1] != r[1] || r[6] != r[6]) continue; /* no 2D footprint (culled at the near plane) */
        for (int ty = y0; ty < y1; ++ty)
            for (int tx = x0; tx < x1; ++tx) {
                const int core = tx >= (int)r[32] && tx < (int)r[33] && ty >= (int)r[34] && ty < (int)r[35];
                if (core) continue;
                for (int py = ty * p.tile; py < (ty + 1) * p.tile && py < p.H; ++py)
                    for (int px = tx * p.tile; px < (tx + 1) * p.tile && px < p.W; ++px) {
                        const double ddx = px + 0.5 - r[1], ddy = py + 0.5 - r[2];
                        double P = -0.5 * (r[4] * ddx * ddx + r[6] * ddy * ddy) - r[5] * ddx * ddy;
                        if (P > 0.0) P = 0.0;
                        const double win = skip_window(&p, fp32_alpha_err(exponent_terms(r[4], r[5], r[6], ddx, ddy)));
                        if (r[7] * exp(P) >= p.alpha_min * exp(-win)) flags[(size_t)py * p.W + px] |= 1;
                    }
            }
    }
}

/* Full FP64 forward render of one view from the oracle's own projection
 * (proj: the output of or_project for the same view).  Also flags pixels
 * whose result depends on a decision inside its margin that the compositing
 * enumeration does not cover: a Gaussian whose rect or visibility is
 * ambiguous and whose alpha at the pixel reaches the skip threshold in a
 * tile that only some alternatives cover (bit 0), or two entries of the
 * pixel's list with depths within the tie margin that both reach the skip
 * threshold before the pixel stops (bit 1).
 * img [H][W][10]; ncand [H][W]; flags [H][W]; cands optional [H][W][MAXC][10];
 * pairs_out (nullable): number of (pixel, entry) evaluations of the primary
 * path before its stop. */
void or_render_view(int64_t n, const double *proj, const double *prm, double *img, int32_t *ncand, uint8_t *flags,
                    double *cands, int64_t *pairs_out)
{
    const oprm p = unpack_prm(prm);
    const int TX = (p.W + p.tile - 1) / p.tile, TY = (p.H + p.tile - 1) / p.tile, T = TX * TY;
    int64_t *lp, *li;
    build_lists(&p, n, proj, &lp, &li);
    memset(flags, 0, (size_t)p.H * p.W);
    rect_flags(&p, n, proj, flags);
    int64_t pairs = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : pairs)
    for (int t = 0; t < T; ++t) {
        const int len = (int)(lp[t + 1] - lp[t]);
        oentry *ents = malloc(sizeof(oentry) * (len + 1));
        for (int j = 0; j < len; ++j) {
            const double *r = proj + OR_PROJ_STRIDE * li[lp[t] + j];
            ents[j].u = r[1];
            ents[j].v = r[2];
            ents[j].z = r[3];
            ents[j].A = r[4];
            ents[j].B = r[5];
            ents[j].C = r[6];
            ents[j].o = r[7];
            ents[j].rgb[0] = r[8];
            ents[j].rgb[1] = r[9];
            ents[j].rgb[2] = r[10];
        }
        const int tx = t % TX, ty = t / TX;
        composite_tile(&p, ents, len, tx, ty, img, ncand, cands);
        /* primary-path evaluation count, and depth near-ties between two
         * entries that both reach the skip threshold at the pixel before it
         * stops (their order decides the result) */
        for (int py = ty * p.tile; py < (ty + 1) * p.tile && py < p.H; ++py)
            for (int px = tx * p.tile; px < (tx + 1) * p.tile && px < p.W; ++px) {
                double T_ = 1.0, zlast = -1.0, alast = 0.0, Tlast = 1.0;
                const double *clast = NULL;
                int j = 0, tie = 0;
                for (; j < len; ++j) {
                    const double ddx = px + 0.5 - ents[j].u, ddy = py + 0.5 - ents[j].v;
                    double P = -0.5 * (ents[j].A * ddx * ddx + ents[j].C * ddy * ddy) - ents[j].B * ddx * ddy;
                    if (P > 0.0) P = 0.0;
                    double a = ents[j].o * exp(P);
                    if (a > p.alpha_max) a = p.alpha_max;
                    const double win =
                        skip_window(&p, fp32_alpha_err(exponent_terms(ents[j].A, ents[j].B, ents[j].C, ddx, ddy)));
                    if (a < p.alpha_min * exp(-win)) continue;
                    if (zlast > 0.0 && fabs(ents[j].z - zlast) <= p.d_tie * (ents[j].z > zlast ? ents[j].z : zlast)) {
                        /* swapping two adjacent entries changes the colour by exactly
                         * T a1 a2 (c1 - c2) (the depth likewise), and leaves the
                         * transmittance after both unchanged; it matters when that
                         * can reach a tenth of the tolerance, or when the first of
                         * the two may stop the pixel */
                        double dc = fabs(ents[j].z - zlast);
                        for (int ch = 0; ch < 3; ++ch) dc = fmax(dc, fabs(ents[j].rgb[ch] - clast[ch]));
                        const double effect = Tlast * alast * a * dc;
                        const int near_stop = Tlast * (1.0 - fmax(a, alast)) < p.t_min * 1.01;
                        if (effect > 0.1 * p.img_tol || near_stop) tie = 1;
                    }
                    zlast = ents[j].z;
                    alast = a;
                    clast = ents[j].rgb;
                    Tlast = T_;
                    if (a < p.alpha_min) continue;
                    const double Tn = T_ * (1.0 - a);
                    if (Tn < p.t_min) {
                        ++j;
                        break;
                    }
                    T_ = Tn;
                }
                pairs += j;
                if (tie) flags[(size_t)py * p.W + px] |= 2;
            }
        free(ents);
    }
    if (pairs_out) *pairs_out = pairs;
    free(lp);
    free(li);
}

/* ------------------------------------------------------------------------ */
/* adjoint (O12)                                                             */
/* ------------------------------------------------------------------------ */
/* 2D gradient slots per Gaussian */
enum { G_U = 0, G_V, G_A, G_B, G_C, G_O, G_R, G_G, G_BL, G_Z, G_N };

static void atomic_add(double *p, double v)
{
#pragma omp atomic
    *p += v;
}

/* The per-pixel adjoint of O12 along one fixed branch: the composited
 * entries cj[0..nc) (positions in the list `ent`, front to back) with their
 * alpha, transmittance before them, Gaussian value and pixel offset; T_end
 * is the final transmittance.  Accumulates into g2d. */
typedef struct {
    int j, clamped;
    double a, T, G, dx, dy;
    double err; /* bound on the FP32 rounding error of log(alpha) */
    double win; /* window of its skip decision on log(alpha) */
} ocomp;

static void adjoint_pixel(const oprm *p, const double *proj, const int64_t *ent, const ocomp *cc, int nc,
                          double T_end, const double dC[3], double dD, double dA, double *g2d)
{
    double S[3] = {p->bg[0], p->bg[1], p->bg[2]}, SD = 0.0;
    for (int k = nc - 1; k >= 0; --k) {
        const int64_t gi = ent[cc[k].j];
        const double *r = proj + OR_PROJ_STRIDE * gi;
        const double a = cc[k].a, Ti = cc[k].T;
        double dalpha = 0.0;
        for (int ch = 0; ch < 3; ++ch) dalpha += dC[ch] * (r[8 + ch] - S[ch]);
        dalpha += dD * (r[3] - SD);
        dalpha *= Ti;
        dalpha += dA * T_end / (1.0 - a);
        double *g = g2d + G_N * gi;
        for (int ch = 0; ch < 3; ++ch) atomic_add(&g[G_R + ch], dC[ch] * a * Ti);
        atomic_add(&g[G_Z], dD * a * Ti);
        if (!cc[k].clamped) {
            const double dG = dalpha * r[7];
            atomic_add(&g[G_O], dalpha * cc[k].G);
            const double dP = dG * cc[k].G;
            const double dx = cc[k].dx, dy = cc[k].dy;
            atomic_add(&g[G_U], dP * (r[4] * dx + r[5] * dy));
            atomic_add(&g[G_V], dP * (r[5] * dx + r[6] * dy));
            atomic_add(&g[G_A], dP * (-0.5 * dx * dx));
            atomic_add(&g[G_B], dP * (-dx * dy));
            atomic_add(&g[G_C], dP * (-0.5 * dy * dy));
        }
        for (int ch = 0; ch < 3; ++ch) S[ch] = a * r[8 + ch] + (1.0 - a) * S[ch];
        SD = a * r[3] + (1.0 - a) * SD;
    }
}

/* alpha of list entry gi at pixel centre (cx, cy) from the FP64 projection
 * (0 for a Gaussian the FP64 projection culls) */
static void pixel_alpha(const oprm *p, const double *proj, int64_t gi, double cx, double cy, ocomp *e)
{
    const double *r = proj + OR_PROJ_STRIDE * gi;
    e->a = e->G = e->dx = e->dy = 0.0;
    e->clamped = 0;
    e->err = 0.0;
    e->win = skip_window(p, 0.0);
    if (r[0] == 0.0) return;
    e->dx = cx - r[1];
    e->dy = cy - r[2];
    e->err = fp32_alpha_err(exponent_terms(r[4], r[5], r[6], e->dx, e->dy));
    e->win = skip_window(p, e->err);
    double P = -0.5 * (r[4] * e->dx * e->dx + r[6] * e->dy * e->dy) - r[5] * e->dx * e->dy;
    if (P > 0.0) P = 0.0;
    e->G = exp(P);
    e->a = r[7] * e->G;
    if (e->a > p->alpha_max) {
        if (e->a >= p->alpha_max * exp(e->err)) { /* the clamp constant on both sides */
            e->err = 0.0;
            e->win = skip_window(p, 0.0);
        }
        e->a = p->alpha_max;
        e->clamped = 1;
    }
}

#define OR_MAX_ENUM 4 /* skip decisions enumerated per pixel in the implementation's-branch mode */

/* Implementation's-branch mode, one pixel: entries ent[0..len) in the
 * implementation's list order, nc its n_contrib, img its (r, g, b, depth,
 * alpha).  Picks the skip decisions (see or_backward_2d), writes the
 * composited entries into cc and returns their count; *T_end the final
 * transmittance; *stat the pixel status. */
static int branch_from_image(const oprm *p, const double *proj, const int64_t *ent, int len, int nc, double cx,
                             double cy, const float *img, ocomp *all, ocomp *cc, double *T_end, int *stat)
{
    const double amin = p->alpha_min, tmin = p->t_min;
    int st = 0;
    if (nc > len) {
        st = 2;
        nc = len;
    }
    /* FP64 alphas of the entries up to the implementation's last composited one */
    int amb[OR_MAX_ENUM], namb = 0;
    for (int j = 0; j < nc; ++j) {
        pixel_alpha(p, proj, ent[j], cx, cy, &all[j]);
        all[j].j = j;
    }
    /* skip decisions inside the window, nearest the threshold first */
    for (int j = 0; j + 1 < nc; ++j) {
        if (!in_skip_window(all[j].a, amin, all[j].win)) continue;
        const double m = fabs(log(all[j].a / amin));
        if (namb < OR_MAX_ENUM) {
            amb[namb++] = j;
        } else {
            int far = 0;
            for (int k = 1; k < namb; ++k)
                if (fabs(log(all[amb[k]].a / amin)) > fabs(log(all[amb[far]].a / amin))) far = k;
            if (m < fabs(log(all[amb[far]].a / amin))) amb[far] = j;
        }
    }
    if (nc > 0 && all[nc - 1].a < amin) /* the implementation composited it: its FP64 alpha must be in the window */
        if (!in_skip_window(all[nc - 1].a, amin, all[nc - 1].win)) st = 2;
    /* every combination of the ambiguous decisions; the FP64 one first */
    double best = INFINITY;
    int best_combo = 0;
    const int ncombo = 1 << namb;
    int primary = 0;
    for (int k = 0; k < namb; ++k)
        if (!(all[amb[k]].a < amin)) primary |= 1 << k;
    for (int t = 0; t < ncombo; ++t) {
        const int combo = t == 0 ? primary : (t == primary ? 0 : t);
        double T = 1.0, C[3] = {0, 0, 0}, D = 0.0;
        for (int j = 0; j < nc; ++j) {
            int take = !(all[j].a < amin) || j == nc - 1;
            for (int k = 0; k < namb; ++k)
                if (amb[k] == j) take = (combo >> k) & 1;
            if (!take) continue;
            const double *r = proj + OR_PROJ_STRIDE * ent[j];
            for (int ch = 0; ch < 3; ++ch) C[ch] += r[8 + ch] * all[j].a * T;
            D += r[3] * all[j].a * T;
            T *= 1.0 - all[j].a;
        }
        double d = 0.0;
        for (int ch = 0; ch < 3; ++ch) d = fmax(d, fabs(C[ch] + T * p->bg[ch] - img[ch]) / p->img_tol);
        d = fmax(d, fabs(D - img[3]) / (p->img_tol * fmax(1.0, fabs(D))));
        d = fmax(d, fabs(1.0 - T - img[4]) / p->img_tol);
        if (d < best) {
            best = d;
            best_combo = combo;
        }
    }
    if (best > 1.0) st = 2;
    if (best_combo != primary && st == 0) st = 1;
    if (nc > 0 && all[nc - 1].a < amin && st == 0) st = 1;
    /* the chosen branch, with its stop decisions checked against the FP64 values */
    double T = 1.0, eT = 0.0;
    int n = 0;
    for (int j = 0; j < nc; ++j) {
        int take = !(all[j].a < amin) || j == nc - 1;
        for (int k = 0; k < namb; ++k)
            if (amb[k] == j) take = (best_combo >> k) & 1;
        if (!take) continue;
        all[j].T = T;
        cc[n++] = all[j];
        const double Tn = T * (1.0 - all[j].a);
        eT = next_eT(eT, all[j].a, all[j].err);
        if (Tn < tmin) { /* the FP64 path stops here, the implementation composited it */
            if (fabs(Tn - tmin) > (p->d_stop + eT) * tmin) st = 2;
            else if (st == 0) st = 1;
        }
        T = Tn;
    }
    /* after the last composited entry the implementation stops, or its list ends: the first entry it may take
     * (FP64 alpha not clearly below the threshold) must stop it */
    int resolved = 0;
    for (int j = nc; j < len && !resolved; ++j) {
        ocomp e;
        pixel_alpha(p, proj, ent[j], cx, cy, &e);
        if (e.a < amin * exp(-e.win)) continue; /* skipped on both sides */
        const double Tn = T * (1.0 - e.a);
        if (Tn < tmin) {
            if (e.a < amin && st == 0) st = 1; /* taken (and stopping) only inside the skip window */
            resolved = 1;
        } else if (fabs(Tn - tmin) <= (p->d_stop + next_eT(eT, e.a, e.err)) * tmin) {
            if (st == 0) st = 1;
            resolved = 1;
        } else if (e.a < amin * exp(e.win)) {
            if (st == 0) st = 1; /* the implementation skipped it inside the window; go on */
        } else {
            st = 2; /* the FP64 path would composite it */
            resolved = 1;
        }
    }
    *T_end = T;
    *stat = st;
    return n;
}

/* Backward of one view (O12): per-Gaussian screen-space adjoints g2d [n][10]
 * (u, v, A, B, C, opacity, r, g, b, z), accumulated, with the discrete
 * decisions (list membership and order, skips, the stop) held fixed.
 * proj: the oracle's own FP64 projection of the view.
 *
 * lvals == NULL: the decisions are the oracle's own FP64 ones on its own
 * lists.
 *
 * Otherwise an implementation's decisions are given and the adjoint
 * differentiates the branch it took, evaluated at the FP64 values:
 * membership and order from its per-tile lists (lvals / lranges as produced
 * by the binning; a value minus val_base indexes proj), the stop from its
 * n_contrib (the list position after the last composited entry), and each
 * skip decision from the FP64 alpha, except those within d_skip of the
 * threshold (relative), which are set to the combination whose forward
 * result is nearest the implementation's image gimg [H][W][5] (r, g, b,
 * depth, alpha).  pstat [H][W] (nullable): 0 the given decisions are the
 * FP64 ones and the image is reproduced within img_tol (depth: img_tol
 * max(1, |D|)); 1 they differ only in decisions inside their windows (d_skip,
 * d_stop) and the image is reproduced; 2 otherwise. */
void or_backward_2d(int64_t n, const double *proj, const double *prm, const float *d_rgb, const float *d_depth,
                    const float *d_alpha, double *g2d, const uint32_t *lvals, const uint32_t *lranges,
                    int64_t val_base, const int32_t *ncontrib, const float *gimg, uint8_t *pstat)
{
    const oprm p = unpack_prm(prm);
    const int TX = (p.W + p.tile - 1) / p.tile, TY = (p.H + p.tile - 1) / p.tile, T = TX * TY;
    int64_t *lp = NULL, *li = NULL;
    if (!lvals) build_lists(&p, n, proj, &lp, &li);
#pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < T; ++t) {
        const int tx = t % TX, ty = t / TX;
        int len;
        int64_t *ent;
        int bad_val = 0;
        if (lvals) {
            const uint32_t b = lranges[2 * t], e = lranges[2 * t + 1];
            len = e > b ? (int)(e - b) : 0;
            ent = malloc(sizeof(int64_t) * (len + 1));
            for (int j = 0; j < len; ++j) {
                ent[j] = (int64_t)lvals[b + j] - val_base;
                if (ent[j] < 0 || ent[j] >= n) {
                    bad_val = 1;
                    ent[j] = 0;
                }
            }
        } else {
            len = (int)(lp[t + 1] - lp[t]);
            ent = malloc(sizeof(int64_t) * (len + 1));
            for (int j = 0; j < len; ++j) ent[j] = li[lp[t] + j];
        }
        ocomp *all = malloc(sizeof(ocomp) * (len + 1));
        ocomp *cc = malloc(sizeof(ocomp) * (len + 1));
        for (int py = ty * p.tile; py < (ty + 1) * p.tile && py < p.H; ++py)
            for (int px = tx * p.tile; px < (tx + 1) * p.tile && px < p.W; ++px) {
                const size_t pix = (size_t)py * p.W + px;
                const double cx = px + 0.5, cy = py + 0.5;
                int nc = 0, st = 0;
                double Tcur = 1.0;
                if (lvals) {
                    nc = branch_from_image(&p, proj, ent, len, ncontrib[pix] < 0 ? 0 : ncontrib[pix], cx, cy,
                                           gimg + 5 * pix, all, cc, &Tcur, &st);
                    if (bad_val) st = 2;
                } else {
                    /* O11 on the oracle's own list with its FP64 decisions */
                    for (int j = 0; j < len; ++j) {
                        ocomp e;
                        pixel_alpha(&p, proj, ent[j], cx, cy, &e);
                        e.j = j;
                        if (e.a < p.alpha_min) continue;
                        const double Tn = Tcur * (1.0 - e.a);
                        if (Tn < p.t_min) break;
                        e.T = Tcur;
                        cc[nc++] = e;
                        Tcur = Tn;
                    }
                }
                if (pstat) pstat[pix] = (uint8_t)st;
                const double dC[3] = {d_rgb[3 * pix], d_rgb[3 * pix + 1], d_rgb[3 * pix + 2]};
                adjoint_pixel(&p, proj, ent, cc, nc, Tcur, dC, d_depth[pix], d_alpha[pix], g2d);
            }
        free(ent);
        free(all);
        free(cc);
    }
    free(lp);
    free(li);
}

/* Chain the 2D gradients of one view to the 3D parameters (adds into the
 * gradient buffers).  Gradient layouts mirror the inputs: d_means [n][3],
 * d_lsc [n][3], d_quats [n][4], d_opacity [n], d_sh [n][K][3], d_cov6 [n][6]. */
void or_backward_3d(int64_t n, int D, const float *means, const float *lsc, const float *quats, const float *cov6,
                    const uint8_t *use_cov6, const float *opacity, const float *sh, const double *camp,
                    const double *prm, const double *g2d, double *d_means, double *d_lsc, double *d_quats,
                    double *d_opacity, double *d_sh, double *d_cov6)
{
    const oprm p = unpack_prm(prm);
    const ocam cam = unpack_cam(camp);
    const int K = (D + 1) * (D + 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double *g = g2d + G_N * i;
        int nz = 0;
        for (int k = 0; k < G_N; ++k) nz |= g[k] != 0.0;
        if (!nz) continue;
        oproj o;
        const int c6 = cov6 && (!use_cov6 || use_cov6[i]);
        oin gi;
        load_in(D, means + 3 * i, lsc ? lsc + 3 * i : NULL, quats ? quats + 4 * i : NULL, c6 ? cov6 + 6 * i : NULL,
                opacity[i], sh + (size_t)3 * K * i, &gi);
        project_one(&p, &cam, &gi, &o);
        if (!o.vis) continue;
        const double *W = cam.R;
        double dmu[3] = {0, 0, 0};
        d_opacity[i] += g[G_O];
        /* colour -> SH coefficients and view direction */
        double Y[OR_MAXK], dY[3 * OR_MAXK];
        or_sh_basis(D, o.dir, Y, dY);
        double dc[3];
        for (int ch = 0; ch < 3; ++ch) dc[ch] = (o.raw[ch] > 0.0) ? g[G_R + ch] : 0.0;
        double ddir[3] = {0, 0, 0};
        const float *shi = sh + (size_t)3 * K * i;
        for (int k = 0; k < K; ++k)
            for (int ch = 0; ch < 3; ++ch) {
                d_sh[(size_t)3 * K * i + 3 * k + ch] += dc[ch] * Y[k];
                for (int j = 0; j < 3; ++j) ddir[j] += dc[ch] * shi[3 * k + ch] * dY[3 * k + j];
            }
        const double dd = o.dir[0] * ddir[0] + o.dir[1] * ddir[1] + o.dir[2] * ddir[2];
        for (int j = 0; j < 3; ++j) dmu[j] += (ddir[j] - o.dir[j] * dd) / o.dist;
        /* conic -> 2D covariance:  dS2 = -Q G Q, G the symmetric adjoint of Q */
        const double Q[4] = {o.conic[0], o.conic[1], o.conic[1], o.conic[2]};
        const double Gm[4] = {g[G_A], 0.5 * g[G_B], 0.5 * g[G_B], g[G_C]};
        double QG[4], dS2[4];
        matmul(Q, Gm, QG, 2, 2, 2);
        matmul(QG, Q, dS2, 2, 2, 2);
        for (int k = 0; k < 4; ++k) dS2[k] = -dS2[k];
        /* S2 = T Sig T^T + lp I,  T = J W */
        double TT[6], tmp[6], dSig[9], dT[6], TSig[6];
        transpose(o.T, TT, 2, 3);
        matmul(TT, dS2, tmp, 3, 2, 2);
        matmul(tmp, o.T, dSig, 3, 2, 3);
        matmul(o.T, o.Sig, TSig, 2, 3, 3);
        matmul(dS2, TSig, dT, 2, 2, 3);
        for (int k = 0; k < 6; ++k) dT[k] *= 2.0;
        double WT[9], dJ[6];
        transpose(W, WT, 3, 3);
        matmul(dT, WT, dJ, 2, 3, 3);
        /* J entries -> camera-space mean */
        const double tx = o.tc[0], ty = o.tc[1], tz = o.tc[2];
        double dt[3] = {0, 0, 0};
        dt[2] += -cam.fx / (tz * tz) * dJ[0] - cam.fy / (tz * tz) * dJ[4];
        /* J02 = -fx * xr / tz, xr = tx/tz unless clamped */
        dt[2] += dJ[2] * cam.fx * o.xr / (tz * tz);
        dt[2] += dJ[5] * cam.fy * o.yr / (tz * tz);
        if (!o.clx) {
            dt[0] += dJ[2] * (-cam.fx / tz) * (1.0 / tz);
            dt[2] += dJ[2] * (-cam.fx / tz) * (-tx / (tz * tz));
        }
        if (!o.cly) {
            dt[1] += dJ[5] * (-cam.fy / tz) * (1.0 / tz);
            dt[2] += dJ[5] * (-cam.fy / tz) * (-ty / (tz * tz));
        }
        /* projected mean and depth */
        dt[0] += g[G_U] * cam.fx / tz;
        dt[1] += g[G_V] * cam.fy / tz;
        dt[2] += -g[G_U] * cam.fx * tx / (tz * tz) - g[G_V] * cam.fy * ty / (tz * tz) + g[G_Z];
        for (int j = 0; j < 3; ++j) dmu[j] += W[0 + j] * dt[0] + W[3 + j] * dt[1] + W[6 + j] * dt[2];
        for (int j = 0; j < 3; ++j) d_means[3 * i + j] += dmu[j];
        /* 3D covariance -> parameters */
        if (c6) {
            d_cov6[6 * i + 0] += dSig[0];
            d_cov6[6 * i + 1] += dSig[1] + dSig[3];
            d_cov6[6 * i + 2] += dSig[2] + dSig[6];
            d_cov6[6 * i + 3] += dSig[4];
            d_cov6[6 * i + 4] += dSig[5] + dSig[7];
            d_cov6[6 * i + 5] += dSig[8];
        } else {
            /* Sig = M M^T, M = R S:  dM = (dSig + dSig^T) M */
            double M[9], dSs[9], dM[9];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    M[3 * a + b] = o.R[3 * a + b] * o.s[b];
                    dSs[3 * a + b] = dSig[3 * a + b] + dSig[3 * b + a];
                }
            matmul(dSs, M, dM, 3, 3, 3);
            for (int k = 0; k < 3; ++k) {
                double rtdm = 0.0; /* (R^T dM)_kk */
                for (int a = 0; a < 3; ++a) rtdm += o.R[3 * a + k] * dM[3 * a + k];
                d_lsc[3 * i + k] += rtdm * o.s[k];
            }
            if (o.qn > 0.0) {
                double dR[9];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) dR[3 * a + b] = dM[3 * a + b] * o.s[b];
                double gR[9][4];
                quat_to_rot_grad(o.q, gR);
                double dqh[4] = {0, 0, 0, 0};
                for (int e = 0; e < 9; ++e)
                    for (int c = 0; c < 4; ++c) dqh[c] += dR[e] * gR[e][c];
                const double qd = o.q[0] * dqh[0] + o.q[1] * dqh[1] + o.q[2] * dqh[2] + o.q[3] * dqh[3];
                for (int c = 0; c < 4; ++c) d_quats[4 * i + c] += (dqh[c] - o.q[c] * qd) / o.qn;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* central finite differences of an image loss (pins of the adjoint)          */
/* ------------------------------------------------------------------------ */
/* Per-pixel loss l = sum_k lin[k] y_k + quad[k] (y_k - tgt[k])^2 over
 * y = (r, g, b, depth, alpha); the loss is summed over the view's pixels. */
typedef struct {
    double T, C[3], D;
    uint64_t sig; /* hash of the composited Gaussians in order */
    int stopped;
} opix;

static void pix_entry(const oprm *p, double cx, double cy, int64_t gi, double u, double v, double A, double B,
                      double Cc, double o, double z, const double *rgb, opix *s)
{
    if (s->stopped) return;
    const double dx = cx - u, dy = cy - v;
    double P = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy;
    if (P > 0.0) P = 0.0;
    double a = o * exp(P);
    if (a > p->alpha_max) a = p->alpha_max;
    if (a < p->alpha_min) return;
    const double Tn = s->T * (1.0 - a);
    if (Tn < p->t_min) {
        s->stopped = 1;
        return;
    }
    for (int ch = 0; ch < 3; ++ch) s->C[ch] += rgb[ch] * a * s->T;
    s->D += z * a * s->T;
    s->T = Tn;
    s->sig = s->sig * 1000003u + (uint64_t)gi + 1u;
}

static void pix_entry_proj(const oprm *p, const double *proj, int64_t gi, double cx, double cy, opix *s)
{
    const double *r = proj + OR_PROJ_STRIDE * gi;
    pix_entry(p, cx, cy, gi, r[1], r[2], r[4], r[5], r[6], r[7], r[3], r + 8, s);
}

/* param index k of the flat per-Gaussian vector: 0..2 mean, 3..5 log-scale,
 * 6..9 quaternion, 10 opacity, 11..11+3K-1 SH (k, channel), then 6 cov6 */
static double *param_ptr(oin *g, int k)
{
    const int K = (g->D + 1) * (g->D + 1);
    if (k < 3) return &g->mean[k];
    if (k < 6) return &g->lsc[k - 3];
    if (k < 10) return &g->q[k - 6];
    if (k == 10) return &g->opac;
    if (k < 11 + 3 * K) return &g->sh[k - 11];
    if (k < 17 + 3 * K) return &g->cov6[k - 11 - 3 * K];
    return NULL;
}

/* FD gradient of the loss w.r.t. parameter param[s] of Gaussian gauss[s],
 * step h[s] (double, central).  The view is re-rendered only where Gaussian
 * gauss[s] can change it (the tiles of its rects at theta and theta +- h),
 * with the other Gaussians' FP64 projection and the oracle's lists at theta.
 * flag[s] = 1 when a discrete decision (composited set, list order or
 * membership) differs between theta - h, theta and theta + h: the sample is
 * then not a derivative and fd[s] is left 0. */
void or_fd_loss(int64_t n, int D, const float *means, const float *lsc, const float *quats, const float *cov6,
                const uint8_t *use_cov6, const float *opacity, const float *sh, const double *camp, const double *prm,
                const double *proj, const double *lin, const double *quad, const double *tgt, int64_t n_samples,
                const int64_t *gauss, const int32_t *param, const double *h, double *fd, int32_t *flag)
{
    const oprm p = unpack_prm(prm);
    const ocam cam = unpack_cam(camp);
    const int K = (D + 1) * (D + 1);
    const int TX = (p.W + p.tile - 1) / p.tile, TY = (p.H + p.tile - 1) / p.tile;
    int64_t *lp, *li;
    build_lists(&p, n, proj, &lp, &li);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < n_samples; ++s) {
        const int64_t i = gauss[s];
        fd[s] = 0.0;
        flag[s] = 0;
        const int c6 = cov6 && (!use_cov6 || use_cov6[i]);
        oin g0;
        load_in(D, means + 3 * i, lsc ? lsc + 3 * i : NULL, quats ? quats + 4 * i : NULL, c6 ? cov6 + 6 * i : NULL,
                opacity[i], sh + (size_t)3 * K * i, &g0);
        oin gv[3] = {g0, g0, g0}; /* theta - h, theta, theta + h */
        double *pm = param_ptr(&gv[0], param[s]), *pp = param_ptr(&gv[2], param[s]);
        if (!pm || !pp) {
            flag[s] = 2;
            continue;
        }
        *pm -= h[s];
        *pp += h[s];
        oproj o[3];
        for (int k = 0; k < 3; ++k) project_one(&p, &cam, &gv[k], &o[k]);
        /* tiles any variant covers */
        int x0 = TX, x1 = 0, y0 = TY, y1 = 0;
        for (int k = 0; k < 3; ++k) {
            if (!o[k].vis) continue;
            if (o[k].rect[0] < x0) x0 = o[k].rect[0];
            if (o[k].rect[1] > x1) x1 = o[k].rect[1];
            if (o[k].rect[2] < y0) y0 = o[k].rect[2];
            if (o[k].rect[3] > y1) y1 = o[k].rect[3];
        }
        double dL = 0.0;
        for (int ty = y0; ty < y1 && !flag[s]; ++ty)
            for (int tx = x0; tx < x1 && !flag[s]; ++tx) {
                const int t = ty * TX + tx;
                const int64_t b = lp[t], e = lp[t + 1];
                /* the position of i among the other entries of the list, per variant (sorted by depth, then index) */
                int64_t pos[3];
                int mem[3];
                for (int k = 0; k < 3; ++k) {
                    mem[k] = o[k].vis && tx >= o[k].rect[0] && tx < o[k].rect[1] && ty >= o[k].rect[2] &&
                             ty < o[k].rect[3];
                    int64_t c = 0;
                    for (int64_t j = b; j < e; ++j) {
                        const int64_t gj = li[j];
                        if (gj == i) continue;
                        const double zj = proj[OR_PROJ_STRIDE * gj + 3];
                        if (zj < o[k].tc[2] || (zj == o[k].tc[2] && gj < i)) ++c;
                    }
                    pos[k] = c;
                }
                int64_t pos0 = -1;
                for (int k = 0; k < 3; ++k) {
                    if (!mem[k]) continue;
                    if (pos0 >= 0 && pos[k] != pos0) flag[s] = 1; /* the list order changes */
                    pos0 = pos[k];
                }
                if (flag[s]) break;
                if (pos0 < 0) continue; /* no variant covers this tile */
                for (int py = ty * p.tile; py < (ty + 1) * p.tile && py < p.H; ++py)
                    for (int px = tx * p.tile; px < (tx + 1) * p.tile && px < p.W; ++px) {
                        const double cx = px + 0.5, cy = py + 0.5;
                        opix pre = {1.0, {0, 0, 0}, 0.0, 0u, 0};
                        int64_t j = b, c = 0;
                        for (; j < e && c < pos0; ++j) {
                            if (li[j] == i) continue;
                            pix_entry_proj(&p, proj, li[j], cx, cy, &pre);
                            ++c;
                        }
                        if (pre.stopped) continue;
                        opix st[3];
                        for (int k = 0; k < 3; ++k) {
                            st[k] = pre;
                            if (mem[k])
                                pix_entry(&p, cx, cy, i, o[k].u, o[k].v, o[k].conic[0], o[k].conic[1], o[k].conic[2],
                                          o[k].opacity, o[k].tc[2], o[k].rgb, &st[k]);
                            for (int64_t jj = j; jj < e && !st[k].stopped; ++jj)
                                if (li[jj] != i) pix_entry_proj(&p, proj, li[jj], cx, cy, &st[k]);
                        }
                        if (st[0].sig != st[1].sig || st[2].sig != st[1].sig) {
                            flag[s] = 1;
                            break;
                        }
                        const size_t pix = (size_t)py * p.W + px;
                        double yp[5], ym[5];
                        for (int ch = 0; ch < 3; ++ch) {
                            yp[ch] = st[2].C[ch] + st[2].T * p.bg[ch];
                            ym[ch] = st[0].C[ch] + st[0].T * p.bg[ch];
                        }
                        yp[3] = st[2].D;
                        ym[3] = st[0].D;
                        yp[4] = 1.0 - st[2].T;
                        ym[4] = 1.0 - st[0].T;
                        for (int k = 0; k < 5; ++k) {
                            const double dy = yp[k] - ym[k];
                            dL += lin[5 * pix + k] * dy + quad[k] * dy * (yp[k] + ym[k] - 2.0 * tgt[5 * pix + k]);
                        }
                    }
            }
        if (!flag[s]) fd[s] = dL / (2.0 * h[s]);
    }
    free(lp);
    free(li);
}

/* ------------------------------------------------------------------------ */
/* linear blend skinning (dense weights)                                     */
/* ------------------------------------------------------------------------ */
/* Blended 3x4 matrix A = sum_j w_ij * skin[avatar_i][j]; mean' = A3 mean + a;
 * Sig' = A3 Sig A3^T with Sig = R(q) diag(exp(2s)) R(q)^T.  w: dense [n][J];
 * skin [A][J][12] row-major 3x4.  Outputs are double. */
void or_lbs(int64_t n, const float *means, const float *lsc, const float *quats, const double *w,
            const int32_t *avatar_of, const float *skin, int J, double *means_out, double *cov6_out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double Am[12] = {0};
        for (int j = 0; j < J; ++j) {
            const double wj = w[(size_t)J * i + j];
            const float *M = skin + ((size_t)avatar_of[i] * J + j) * 12;
            for (int k = 0; k < 12; ++k) Am[k] += wj * M[k];
        }
        for (int a = 0; a < 3; ++a)
            means_out[3 * i + a] =
                Am[4 * a + 0] * means[3 * i] + Am[4 * a + 1] * means[3 * i + 1] + Am[4 * a + 2] * means[3 * i + 2] +
                Am[4 * a + 3];
        double q[4] = {quats[4 * i], quats[4 * i + 1], quats[4 * i + 2], quats[4 * i + 3]};
        double n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3], R[9];
        if (!(n2 >= 1e-24)) {
            q[0] = 1;
            q[1] = q[2] = q[3] = 0;
        } else {
            const double qn = sqrt(n2);
            for (int c = 0; c < 4; ++c) q[c] /= qn;
        }
        quat_to_rot(q, R);
        double M[9], MT[9], Sig[9], A3[9], A3T[9], t1[9], S2[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) M[3 * a + b] = R[3 * a + b] * exp((double)lsc[3 * i + b]);
        transpose(M, MT, 3, 3);
        matmul(M, MT, Sig, 3, 3, 3);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) A3[3 * a + b] = Am[4 * a + b];
        transpose(A3, A3T, 3, 3);
        matmul(A3, Sig, t1, 3, 3, 3);
        matmul(t1, A3T, S2, 3, 3, 3);
        cov6_out[6 * i + 0] = S2[0];
        cov6_out[6 * i + 1] = S2[1];
        cov6_out[6 * i + 2] = S2[2];
        cov6_out[6 * i + 3] = S2[4];
        cov6_out[6 * i + 4] = S2[5];
        cov6_out[6 * i + 5] = S2[8];
    }
}

/* Adjoint of or_lbs w.r.t. the canonical means, log-scales and quaternions
 * (the blend weights and joint matrices are held fixed). */
void or_lbs_backward(int64_t n, const float *means, const float *lsc, const float *quats, const double *w,
                     const int32_t *avatar_of, const float *skin, int J, const float *d_means_out,
                     const float *d_cov6_out, double *d_means, double *d_lsc, double *d_quats)
{
    (void)means;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double Am[12] = {0};
        for (int j = 0; j < J; ++j) {
            const double wj = w[(size_t)J * i + j];
            const float *M = skin + ((size_t)avatar_of[i] * J + j) * 12;
            for (int k = 0; k < 12; ++k) Am[k] += wj * M[k];
        }
        double A3[9], A3T[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) A3[3 * a + b] = Am[4 * a + b];
        transpose(A3, A3T, 3, 3);
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int a = 0; a < 3; ++a) s += A3[3 * a + b] * d_means_out[3 * i + a];
            d_means[3 * i + b] = s;
        }
        const float *dc = d_cov6_out + 6 * i;
        const double G[9] = {dc[0],       0.5 * dc[1], 0.5 * dc[2], 0.5 * dc[1], dc[3],
                             0.5 * dc[4], 0.5 * dc[2], 0.5 * dc[4], dc[5]};
        double t1[9], dSig[9];
        matmul(A3T, G, t1, 3, 3, 3);
        matmul(t1, A3, dSig, 3, 3, 3);
        double q[4] = {quats[4 * i], quats[4 * i + 1], quats[4 * i + 2], quats[4 * i + 3]};
        double n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3], R[9], qn = 0.0;
        if (!(n2 >= 1e-24)) {
            q[0] = 1;
            q[1] = q[2] = q[3] = 0;
        } else {
            qn = sqrt(n2);
            for (int c = 0; c < 4; ++c) q[c] /= qn;
        }
        quat_to_rot(q, R);
        double s[3], M[9], dSs[9], dM[9];
        for (int k = 0; k < 3; ++k) s[k] = exp((double)lsc[3 * i + k]);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                M[3 * a + b] = R[3 * a + b] * s[b];
                dSs[3 * a + b] = dSig[3 * a + b] + dSig[3 * b + a];
            }
        matmul(dSs, M, dM, 3, 3, 3);
        for (int k = 0; k < 3; ++k) {
            double rtdm = 0.0;
            for (int a = 0; a < 3; ++a) rtdm += R[3 * a + k] * dM[3 * a + k];
            d_lsc[3 * i + k] = rtdm * s[k];
        }
        for (int c = 0; c < 4; ++c) d_quats[4 * i + c] = 0.0;
        if (qn > 0.0) {
            double dR[9], gR[9][4], dqh[4] = {0, 0, 0, 0};
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) dR[3 * a + b] = dM[3 * a + b] * s[b];
            quat_to_rot_grad(q, gR);
            for (int e = 0; e < 9; ++e)
                for (int c = 0; c < 4; ++c) dqh[c] += dR[e] * gR[e][c];
            const double qd = q[0] * dqh[0] + q[1] * dqh[1] + q[2] * dqh[2] + q[3] * dqh[3];
            for (int c = 0; c < 4; ++c) d_quats[4 * i + c] = (dqh[c] - q[c] * qd) / qn;
        }
    }
}

int or_version(void) { return 1; }

/* Thread count of the oracle's OpenMP loops (the benchmark's CPU baseline
 * times it on one thread and on all of them). */
#include <omp.h>
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int or_get_threads(void) { return omp_get_max_threads(); }
