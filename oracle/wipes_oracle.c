/*
 * WIPES reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately unoptimised CPU model of what the wavelet
 * rasterizer computes, written from the paper (arXiv 2508.12615, "WIPES:
 * Wavelet-based Visual Primitives").  It is used by tests/, by the smoke
 * check and by the CPU-baseline leg of the benchmark, and by nothing else.
 * It shares no code, header, table or constant with the HIP library, and it
 * is never called on the product path.
 *
 * Arithmetic is FP64, except where a result is *defined* in FP32:
 *   - the depth key that orders primitives for alpha compositing, and
 *   - the tile binning rule (pixel box -> tile rectangle -> keys -> ranges),
 * both of which are written out here in C float with -ffp-contract=off and
 * with explicit fmaf() wherever the definition fuses a multiply-add.
 *
 * What the paper fixes, and where:
 *   - Gaussian envelope G(x) = exp(-1/2 (x-mu)^T Sigma^-1 (x-mu))      Sec. 3.1, Eq. 1
 *   - 3D covariance Sigma = R S S^T R^T                               Sec. 3.1
 *   - EWA projection Sigma_hat = J W Sigma W^T J^T, Sigma' = 2x2 block Sec. 3.1, Eq. 2
 *   - front-to-back alpha blending over depth-sorted primitives       Sec. 3.1, Eq. 3
 *   - additive (weighted-sum) blending for 2D images                  Sec. 3.2, Eq. 4
 *   - wavelet W = 1/2 [cos(f.(x-mu)) + 1] G(x)                        Sec. 4.1, Eq. 6
 *   - screen-space wavelet W'(x'; mu', f', Sigma')                     Sec. 4.1, Eq. 7
 *   - f transformed by the same ray-space map (W, J) as Sigma          Sec. 4.1 (text after Fig. 4)
 *   - 2D covariance by Cholesky or rotation-scale (as GaussianImage)   Sec. 5.1
 * Everything else (support truncation, alpha clamp, termination, pixel
 * centres, guard band, low-pass dilation, key layout) is a reading of a
 * silent paper; each reading is named where it is used below.
 *
 * Parity pins live in tests/test_oracle_*.py (closed forms, finite
 * differences, library routines, brute force, quadrature).  Every function
 * has one: projection (closed form on the axis, numerical Jacobian off it),
 * W' and both blends (Poisson-summation sums, pointwise identities, scipy's
 * Gaussian, compositing closed forms), the backward (central differences,
 * closed-form sum gradients), the covector transform (closed forms, phase
 * invariance, finite differences), the carrier phase (closed forms, finite
 * differences), SH colour (scipy's spherical harmonics, quadrature,
 * degree-0 reduction, finite differences), O-bin (pixel enumeration, scipy
 * minimisation, numpy's stable sort) and the support counts (a numpy brute
 * force).  tests/test_oracle_mutations.py plants plausible mistakes and
 * checks that these pins fail.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Parameters                                                               */
/* ------------------------------------------------------------------------ */

enum { OR_MODE_ADD2D = 0, OR_MODE_ALPHA3D = 1 };
enum { OR_COV_CHOLESKY = 0, OR_COV_RS = 1, OR_COV_QUAT_SCALE = 2 };
enum { OR_FREQ_VECTOR = 0, OR_FREQ_COVECTOR = 1 };

typedef struct {
    int32_t mode;        /* OR_MODE_* */
    int32_t cov;         /* OR_COV_* */
    int32_t freq_xform;  /* OR_FREQ_* */
    int32_t sh_degree;   /* < 0: colour is the direct RGB input; 0..3: spherical-harmonic colour */
    double alpha_min;    /* skip a pair whose o*W' is below this (alpha mode) */
    double alpha_max;    /* clamp of o*W' (alpha mode) */
    double T_min;        /* stop once transmittance falls below this */
    double q_add;        /* additive support: include iff q <= q_add */
    double blur_eps;     /* Sigma' += eps * I */
    double near_plane;   /* cull if camera z <= near */
    double fov_guard;    /* clamp of x/z, y/z inside J, in units of half-fov */
    double bg[3];        /* background colour (alpha mode) */
} or_params;

typedef struct {
    int32_t width, height;
    double fx, fy, cx, cy;
    double viewmat[16];  /* world -> camera, row-major 4x4, OpenCV axes */
    double time;         /* tau for mu(tau) = mu0 + v tau */
} or_camera;

/* FP64 screen record, one row of 16 doubles per primitive. */
enum {
    SR_MX = 0, SR_MY, SR_CA, SR_CB, SR_CC, SR_FX, SR_FY, SR_OP,
    SR_R, SR_G, SR_B, SR_DEPTH, SR_RX, SR_RY, SR_Q, SR_VALID, SR_PH, SR_N
};
/* Screen-space gradient row: d/d(mu'x, mu'y, a, b, c, f'x, f'y, o, r, g, b, phase). */
enum { SG_MX = 0, SG_MY, SG_CA, SG_CB, SG_CC, SG_FX, SG_FY, SG_OP, SG_R, SG_G, SG_B, SG_PH, SG_N };

/* Per-pixel tie flags (decisions within a stated margin of their threshold).
 * With every flag the renders also accumulate a bound on how far the pixel's
 * value (jump[0], max over channels) and final transmittance (jump[1]) move
 * if that decision goes the other way, with cmax = the largest |colour| or
 * |bg| of the scene:
 *   support (additive)  o W' max|c|            -- the pair's whole contribution
 *   skip / cull (alpha) 2 cmax (T a + T_min)   -- the pair's contribution, plus
 *                                                  the tail a moved stop decision drops
 *   stop                2 cmax T               -- the tail after the stopping pair
 *   clamp               0                      -- the value is continuous there
 *   near-plane cull     2 cmax                 -- anything
 */
enum {
    TIE_SUPPORT = 1,   /* |q - q_add| < dq + 1e-7 q_add (q_err below)   (additive support) */
    TIE_SKIP = 2,      /* |o W' - alpha_min| < 1e-5 alpha_min + da      (alpha skip)       */
    TIE_STOP = 4,      /* |T_after - T_min| < (1e-4 + dT) T_min         (termination)      */
    TIE_CLAMP = 8,     /* |o W' - alpha_max| < 1e-5 alpha_max + da      (clamp kink)       */
    TIE_CULL = 16      /* primitive-level cull decision near its threshold                  */
};

/*
 * Reading of the tie bands: a decision counts as a tie when the rendered
 * quantity lies within the error with which an FP32 evaluation (the
 * renderer's arithmetic, with hardware exp2 and cos) can place it.  For
 * o W' = o kappa e that error is absolute in the carrier kappa, not relative
 * to alpha_min: a pair near the skip threshold with a small kappa (close to a
 * trough of the cosine) and a large phase can be decided differently by any
 * FP32 evaluation.  Bound used, per pair (phi in radians):
 *   phase error     dphi  = 4e-7 |phi| + 4e-6 |f'| + 1e-6
 *                           (rounding of the phase sum, of the mean to ~1e-6 px
 *                            times |f'|, and of the argument reduction)
 *   carrier error   dkap  = |sin phi| dphi / 2 + 2e-6   (cos approximation)
 *   envelope error  de/e  = 1e-6 + 2e-7 q               (exp2 and the quadratic)
 *   da = o (e dkap + kappa e de/e)
 * and the transmittance carries the accumulated relative error
 * dT = sum of da / (1 - alpha) over the pixel's contributing pairs
 * (a_err below).
 */

/* ------------------------------------------------------------------------ */
/* Small FP64 linear algebra                                                */
/* ------------------------------------------------------------------------ */

/* Rotation matrix of a unit quaternion (w, x, y, z), row-major. */
static void quat_to_rot(const double q[4], double R[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* dR/dq_k for a unit quaternion, k = 0..3 over (w, x, y, z). */
static void quat_rot_deriv(const double q[4], int k, double D[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    switch (k) {
    case 0: /* d/dw */
        D[0] = 0;        D[1] = -2 * z;  D[2] = 2 * y;
        D[3] = 2 * z;    D[4] = 0;       D[5] = -2 * x;
        D[6] = -2 * y;   D[7] = 2 * x;   D[8] = 0;
        break;
    case 1: /* d/dx */
        D[0] = 0;        D[1] = 2 * y;   D[2] = 2 * z;
        D[3] = 2 * y;    D[4] = -4 * x;  D[5] = -2 * w;
        D[6] = 2 * z;    D[7] = 2 * w;   D[8] = -4 * x;
        break;
    case 2: /* d/dy */
        D[0] = -4 * y;   D[1] = 2 * x;   D[2] = 2 * w;
        D[3] = 2 * x;    D[4] = 0;       D[5] = 2 * z;
        D[6] = -2 * w;   D[7] = 2 * z;   D[8] = -4 * y;
        break;
    default: /* d/dz */
        D[0] = -4 * z;   D[1] = -2 * w;  D[2] = 2 * x;
        D[3] = 2 * w;    D[4] = -4 * z;  D[5] = 2 * y;
        D[6] = 2 * x;    D[7] = 2 * y;   D[8] = 0;
        break;
    }
}

/* ------------------------------------------------------------------------ */
/* Spherical-harmonic colour                                                */
/* ------------------------------------------------------------------------ */

/*
 * 3DGS stores view-dependent colour as spherical-harmonic coefficients
 * (Sec. 3.1).  Reading: the real spherical harmonics with the Condon-Shortley
 * phase, Y_{l,m} = sqrt(2) Re Y_l^m (m > 0), sqrt(2) Im Y_l^|m| (m < 0),
 * Y_l^0 (m = 0), where Y_l^m is the complex harmonic, of degree l <= 3,
 * indexed k = l^2 + l + m, evaluated at the unit direction from the camera
 * centre to the (time-shifted) mean; colour_c = sum_k Y_k sh[k][c], with no
 * offset and no clamp.  The degree-<=3 harmonics are written out as their
 * Cartesian polynomials in (x, y, z) on the unit sphere; G (may be NULL)
 * receives the gradient of each polynomial in R^3 (3 values per k).
 */
static int sh_count(int deg) { return (deg + 1) * (deg + 1); }

static void sh_basis(int deg, double x, double y, double z, double* Y, double* G)
{
    const double pi = 3.14159265358979323846;
    const double c0 = 0.5 * sqrt(1.0 / pi), c1 = sqrt(3.0 / (4.0 * pi));
    const double c2a = 0.5 * sqrt(15.0 / pi), c2b = 0.25 * sqrt(5.0 / pi), c2c = 0.25 * sqrt(15.0 / pi);
    const double c3a = 0.25 * sqrt(35.0 / (2.0 * pi)), c3b = 0.5 * sqrt(105.0 / pi);
    const double c3c = 0.25 * sqrt(21.0 / (2.0 * pi)), c3d = 0.25 * sqrt(7.0 / pi), c3e = 0.25 * sqrt(105.0 / pi);
    double g[16][3];
    double v[16];
    memset(g, 0, sizeof(g));
    v[0] = c0;
    if (deg >= 1) {
        v[1] = -c1 * y;  g[1][1] = -c1;
        v[2] = c1 * z;   g[2][2] = c1;
        v[3] = -c1 * x;  g[3][0] = -c1;
    }
    if (deg >= 2) {
        v[4] = c2a * x * y;                        g[4][0] = c2a * y;  g[4][1] = c2a * x;
        v[5] = -c2a * y * z;                       g[5][1] = -c2a * z; g[5][2] = -c2a * y;
        v[6] = c2b * (2 * z * z - x * x - y * y);  g[6][0] = -2 * c2b * x; g[6][1] = -2 * c2b * y; g[6][2] = 4 * c2b * z;
        v[7] = -c2a * x * z;                       g[7][0] = -c2a * z; g[7][2] = -c2a * x;
        v[8] = c2c * (x * x - y * y);              g[8][0] = 2 * c2c * x; g[8][1] = -2 * c2c * y;
    }
    if (deg >= 3) {
        v[9] = -c3a * y * (3 * x * x - y * y);
        g[9][0] = -c3a * 6 * x * y; g[9][1] = -c3a * (3 * x * x - 3 * y * y);
        v[10] = c3b * x * y * z;
        g[10][0] = c3b * y * z; g[10][1] = c3b * x * z; g[10][2] = c3b * x * y;
        v[11] = -c3c * y * (4 * z * z - x * x - y * y);
        g[11][0] = c3c * 2 * x * y; g[11][1] = -c3c * (4 * z * z - x * x - 3 * y * y); g[11][2] = -c3c * 8 * y * z;
        v[12] = c3d * z * (2 * z * z - 3 * x * x - 3 * y * y);
        g[12][0] = -c3d * 6 * x * z; g[12][1] = -c3d * 6 * y * z; g[12][2] = c3d * (6 * z * z - 3 * x * x - 3 * y * y);
        v[13] = -c3c * x * (4 * z * z - x * x - y * y);
        g[13][0] = -c3c * (4 * z * z - 3 * x * x - y * y); g[13][1] = c3c * 2 * x * y; g[13][2] = -c3c * 8 * x * z;
        v[14] = c3e * z * (x * x - y * y);
        g[14][0] = c3e * 2 * x * z; g[14][1] = -c3e * 2 * y * z; g[14][2] = c3e * (x * x - y * y);
        v[15] = -c3a * x * (x * x - 3 * y * y);
        g[15][0] = -c3a * (3 * x * x - 3 * y * y); g[15][1] = c3a * 6 * x * y;
    }
    int K = sh_count(deg);
    for (int k = 0; k < K; ++k) {
        Y[k] = v[k];
        if (G) for (int a = 0; a < 3; ++a) G[3 * k + a] = g[k][a];
    }
}

/* Real SH basis of n unit directions (for the pins): Y[n][(deg+1)^2]. */
void or_sh_basis(int32_t deg, int64_t n, const double* dirs, double* Y, double* G)
{
    for (int64_t i = 0; i < n; ++i)
        sh_basis(deg, dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2], Y + (size_t)sh_count(deg) * i,
                 G ? G + (size_t)3 * sh_count(deg) * i : NULL);
}

/* World position of the camera centre: -W^T w for the world->camera map [W | w]. */
static void camera_centre(const or_camera* cam, double C[3])
{
    const double* V = cam->viewmat;
    for (int k = 0; k < 3; ++k) C[k] = -(V[k] * V[3] + V[4 + k] * V[7] + V[8 + k] * V[11]);
}

/* ------------------------------------------------------------------------ */
/* Depth key (defined in FP32)                                              */
/* ------------------------------------------------------------------------ */

/*
 * Alpha compositing visits primitives in ascending camera depth (Eq. 3 sums
 * over "sorted" primitives).  Reading: the sort key is the FP32 camera z of
 * the (time-shifted) mean, evaluated as
 *     m_k = fma(v_k, tau, mu_k)                        (k = x, y, z; m = mu if no velocity)
 *     z   = fma(W20, m_x, fma(W21, m_y, fma(W22, m_z, W23)))
 * with W the world->camera matrix rounded to FP32; equal keys go by index.
 */
float or_depth_key(const float mean[3], const float* vel, float tau, const float W[16])
{
    float mx = mean[0], my = mean[1], mz = mean[2];
    if (vel) {
        mx = fmaf(vel[0], tau, mx);
        my = fmaf(vel[1], tau, my);
        mz = fmaf(vel[2], tau, mz);
    }
    return fmaf(W[8], mx, fmaf(W[9], my, fmaf(W[10], mz, W[11])));
}

static uint32_t float_bits(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

/* Depth keys of n primitives as FP32 bit patterns (vel may be NULL). */
void or_depth_keys(int64_t n, const float* mean, const float* vel, float tau, const float W[16], uint32_t* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = float_bits(or_depth_key(mean + 3 * i, vel ? vel + 3 * i : NULL, tau, W));
}

/* ------------------------------------------------------------------------ */
/* Projection (FP64)                                                        */
/* ------------------------------------------------------------------------ */

/*
 * 2D primitive (Sec. 5.1; Eq. 4 with W' of Eq. 7): the primitive already
 * lives on the image plane, so mu' = mu and f' = f.  Sigma from
 *   Cholesky: L = [[l11, 0], [l21, l22]], Sigma = L L^T
 *   RS:       Sigma = R(theta) diag(s1^2, s2^2) R(theta)^T
 * Reading: Sigma' = Sigma + eps I, conic A = Sigma'^-1, additive support
 * q = d^T A d <= q_add, whose exact bounding box has half-extents
 * sqrt(q_add Sigma'_xx), sqrt(q_add Sigma'_yy).
 */
static void project_2d(const or_params* P, int64_t i, const double* mean, const double* covp,
                       const double* freq, const double* color, const double* opac, const double* phase, double* s)
{
    double Sxx, Sxy, Syy;
    if (P->cov == OR_COV_CHOLESKY) {
        double l11 = covp[3 * i], l21 = covp[3 * i + 1], l22 = covp[3 * i + 2];
        Sxx = l11 * l11;
        Sxy = l11 * l21;
        Syy = l21 * l21 + l22 * l22;
    } else {
        double s1 = covp[3 * i], s2 = covp[3 * i + 1], th = covp[3 * i + 2];
        double c = cos(th), sn = sin(th);
        Sxx = c * c * s1 * s1 + sn * sn * s2 * s2;
        Sxy = c * sn * (s1 * s1 - s2 * s2);
        Syy = sn * sn * s1 * s1 + c * c * s2 * s2;
    }
    Sxx += P->blur_eps;
    Syy += P->blur_eps;
    double det = Sxx * Syy - Sxy * Sxy;
    s[SR_MX] = mean[2 * i];
    s[SR_MY] = mean[2 * i + 1];
    s[SR_FX] = freq[2 * i];
    s[SR_FY] = freq[2 * i + 1];
    s[SR_OP] = opac[i];
    s[SR_R] = color[3 * i];
    s[SR_G] = color[3 * i + 1];
    s[SR_B] = color[3 * i + 2];
    s[SR_DEPTH] = 0.0;
    s[SR_PH] = phase ? phase[i] : 0.0;
    if (!(det > 0.0)) {
        s[SR_VALID] = 0.0;
        return;
    }
    s[SR_CA] = Syy / det;
    s[SR_CB] = -Sxy / det;
    s[SR_CC] = Sxx / det;
    s[SR_Q] = P->q_add;
    s[SR_RX] = sqrt(P->q_add * Sxx);
    s[SR_RY] = sqrt(P->q_add * Syy);
    s[SR_VALID] = 1.0;
}

/* Everything the 3D projection derives from one primitive, kept for the backward. */
typedef struct {
    double m[3], t[3];       /* world mean at time tau, camera-space mean */
    double Rw[9];            /* world->camera rotation */
    double J[6], M[6];       /* 2x3 Jacobian and M = J Rw */
    int clampx, clampy;      /* x/z or y/z hit the guard band */
    double qn[4], qnorm;     /* normalised quaternion and the norm it had */
    double Rq[9], sc[3];     /* primitive rotation and scales */
    double S3[9];            /* world covariance */
    double Sp[3];            /* Sigma' (xx, xy, yy) including eps */
    double f3[3];            /* world frequency */
    double Jfull[9];         /* 3x3 ray-space Jacobian (covector variant only) */
} proj3;

/*
 * 3D primitive (Sec. 3.1 Eq. 2; Sec. 4.1 Eq. 6-7 and the f transform):
 *   t   = W mu(tau) + w,  mu(tau) = mu0 + v tau  (reading: linear-in-time offset)
 *   mu' = (fx t_x / t_z + cx, fy t_y / t_z + cy)
 *   J   = [[fx/t_z, 0, -fx u/t_z], [0, fy/t_z, -fy v/t_z]], u, v = t_x/t_z, t_y/t_z
 *         clamped to +-guard * half-fov (reading, gsplat lineage)
 *   Sigma' = (J W) Sigma (J W)^T + eps I,   Sigma = R(q) diag(s^2) R(q)^T
 *   f'  = (J W) f     (f goes through the same ray-space map as Sigma)
 * Reading for alpha mode: cull if o < alpha_min, support bound
 * q <= 2 ln(o / alpha_min) (W' <= G' makes o W' < alpha_min outside it).
 */
static int project_3d_core(const or_params* P, const or_camera* cam, int64_t i, const double* mean,
                           const double* quat, const double* scale, const double* freq, const double* vel,
                           proj3* pj)
{
    const double* V = cam->viewmat;
    for (int k = 0; k < 3; ++k) {
        pj->m[k] = (double)mean[3 * i + k] + (vel ? (double)vel[3 * i + k] * cam->time : 0.0);
        pj->f3[k] = freq[3 * i + k];
        pj->sc[k] = scale[3 * i + k];
    }
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) pj->Rw[3 * r + c] = V[4 * r + c];
        pj->t[r] = V[4 * r] * pj->m[0] + V[4 * r + 1] * pj->m[1] + V[4 * r + 2] * pj->m[2] + V[4 * r + 3];
    }
    double tz = pj->t[2];
    double u = pj->t[0] / tz, v = pj->t[1] / tz;
    double limx = P->fov_guard * 0.5 * cam->width / cam->fx;
    double limy = P->fov_guard * 0.5 * cam->height / cam->fy;
    pj->clampx = (u < -limx || u > limx);
    pj->clampy = (v < -limy || v > limy);
    double uc = u < -limx ? -limx : (u > limx ? limx : u);
    double vc = v < -limy ? -limy : (v > limy ? limy : v);
    pj->J[0] = cam->fx / tz; pj->J[1] = 0.0;          pj->J[2] = -cam->fx * uc / tz;
    pj->J[3] = 0.0;          pj->J[4] = cam->fy / tz; pj->J[5] = -cam->fy * vc / tz;
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            pj->M[3 * r + c] = pj->J[3 * r] * pj->Rw[c] + pj->J[3 * r + 1] * pj->Rw[3 + c] +
                               pj->J[3 * r + 2] * pj->Rw[6 + c];
    double qq[4] = {quat[4 * i], quat[4 * i + 1], quat[4 * i + 2], quat[4 * i + 3]};
    pj->qnorm = sqrt(qq[0] * qq[0] + qq[1] * qq[1] + qq[2] * qq[2] + qq[3] * qq[3]);
    if (!(pj->qnorm > 0.0)) return 0;
    for (int k = 0; k < 4; ++k) pj->qn[k] = qq[k] / pj->qnorm;
    quat_to_rot(pj->qn, pj->Rq);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += pj->Rq[3 * r + k] * pj->sc[k] * pj->sc[k] * pj->Rq[3 * c + k];
            pj->S3[3 * r + c] = acc;
        }
    double MS[6];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += pj->M[3 * r + k] * pj->S3[3 * k + c];
            MS[3 * r + c] = acc;
        }
    double sxx = 0, sxy = 0, syy = 0;
    for (int k = 0; k < 3; ++k) {
        sxx += MS[k] * pj->M[k];
        sxy += MS[k] * pj->M[3 + k];
        syy += MS[3 + k] * pj->M[3 + k];
    }
    pj->Sp[0] = sxx + P->blur_eps;
    pj->Sp[1] = sxy;
    pj->Sp[2] = syy + P->blur_eps;
    /* 3x3 ray-space Jacobian (third row: d|t|/dt ~ t/|t|), used by the covector variant. */
    double tl = sqrt(pj->t[0] * pj->t[0] + pj->t[1] * pj->t[1] + tz * tz);
    for (int k = 0; k < 6; ++k) pj->Jfull[k] = pj->J[k];
    pj->Jfull[6] = pj->t[0] / tl;
    pj->Jfull[7] = pj->t[1] / tl;
    pj->Jfull[8] = tz / tl;
    return 1;
}

static int inv3(const double A[9], double B[9])
{
    double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                 A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (det == 0.0) return 0;
    B[0] = (A[4] * A[8] - A[5] * A[7]) / det;
    B[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    B[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    B[3] = (A[5] * A[6] - A[3] * A[8]) / det;
    B[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    B[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    B[6] = (A[3] * A[7] - A[4] * A[6]) / det;
    B[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    B[8] = (A[0] * A[4] - A[1] * A[3]) / det;
    return 1;
}

static void project_3d(const or_params* P, const or_camera* cam, int64_t i, const double* mean,
                       const double* quat, const double* scale, const double* freq, const double* color,
                       const double* opac, const double* vel, const double* phase, const double* sh, double* s)
{
    proj3 pj;
    s[SR_OP] = opac[i];
    if (P->sh_degree < 0) {
        s[SR_R] = color[3 * i];
        s[SR_G] = color[3 * i + 1];
        s[SR_B] = color[3 * i + 2];
    }
    s[SR_PH] = phase ? phase[i] : 0.0;
    s[SR_VALID] = 0.0;
    double o = opac[i];
    if (!project_3d_core(P, cam, i, mean, quat, scale, freq, vel, &pj)) return;
    if (P->sh_degree >= 0) {
        /* view-dependent colour from the direction camera centre -> mean */
        double Cc[3], d[3], Y[16];
        camera_centre(cam, Cc);
        for (int k = 0; k < 3; ++k) d[k] = pj.m[k] - Cc[k];
        double dl = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        sh_basis(P->sh_degree, d[0] / dl, d[1] / dl, d[2] / dl, Y, NULL);
        int K = sh_count(P->sh_degree);
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < K; ++k) acc += Y[k] * sh[((size_t)i * K + k) * 3 + c];
            s[SR_R + c] = acc;
        }
    }
    double tz = pj.t[2];
    s[SR_DEPTH] = tz;
    if (!(tz > P->near_plane)) return;
    if (!(o >= P->alpha_min)) return;
    s[SR_MX] = cam->fx * pj.t[0] / tz + cam->cx;
    s[SR_MY] = cam->fy * pj.t[1] / tz + cam->cy;
    double det = pj.Sp[0] * pj.Sp[2] - pj.Sp[1] * pj.Sp[1];
    if (!(det > 0.0)) return;
    s[SR_CA] = pj.Sp[2] / det;
    s[SR_CB] = -pj.Sp[1] / det;
    s[SR_CC] = pj.Sp[0] / det;
    if (P->freq_xform == OR_FREQ_VECTOR) {
        s[SR_FX] = pj.M[0] * pj.f3[0] + pj.M[1] * pj.f3[1] + pj.M[2] * pj.f3[2];
        s[SR_FY] = pj.M[3] * pj.f3[0] + pj.M[4] * pj.f3[1] + pj.M[5] * pj.f3[2];
    } else {
        /* phase-preserving alternative: f' = first two rows of (Jfull Rw)^-T f */
        double A[9], Ai[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                A[3 * r + c] = pj.Jfull[3 * r] * pj.Rw[c] + pj.Jfull[3 * r + 1] * pj.Rw[3 + c] +
                               pj.Jfull[3 * r + 2] * pj.Rw[6 + c];
        if (!inv3(A, Ai)) return;
        /* (A^-T f)_r = sum_c Ai[c][r] f_c */
        s[SR_FX] = Ai[0] * pj.f3[0] + Ai[3] * pj.f3[1] + Ai[6] * pj.f3[2];
        s[SR_FY] = Ai[1] * pj.f3[0] + Ai[4] * pj.f3[1] + Ai[7] * pj.f3[2];
    }
    double Q = 2.0 * log(o / P->alpha_min);
    s[SR_Q] = Q;
    s[SR_RX] = sqrt(Q * pj.Sp[0]);
    s[SR_RY] = sqrt(Q * pj.Sp[2]);
    s[SR_VALID] = 1.0;
}

void or_project(const or_params* P, const or_camera* cam, int64_t n, const double* mean, const double* covp,
                const double* quat, const double* scale, const double* freq, const double* color,
                const double* opac, const double* vel, const double* phase, const double* sh, double* screen)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double* s = screen + SR_N * i;
        memset(s, 0, sizeof(double) * SR_N);
        if (P->mode == OR_MODE_ADD2D)
            project_2d(P, i, mean, covp, freq, color, opac, phase, s);
        else
            project_3d(P, cam, i, mean, quat, scale, freq, color, opac, vel, phase, sh, s);
    }
}

/* ------------------------------------------------------------------------ */
/* Per-pixel rule (FP64)                                                    */
/* ------------------------------------------------------------------------ */

/*
 * Evaluation of one (pixel, primitive) pair.  Reading: the centre of pixel
 * (x, y) is (x + 1/2, y + 1/2).  Then d = p - mu', q = d^T A d,
 * phi = f'.d + phi0 (radians), e = exp(-q/2), kappa = (1 + cos phi)/2 and
 * W' = kappa e (Eq. 6-7).  phi0 is an optional per-primitive carrier phase
 * (Eq. 6 has none, so phi0 = 0 gives the paper's primitive; a phase is the
 * primitive variant in which the carrier is cos(f.(x - mu) + phi0)).
 */
typedef struct {
    double dx, dy, q, phi, e, kappa, w;
} pair_eval;

static void eval_pair(const double* s, double px, double py, pair_eval* pe)
{
    pe->dx = px - s[SR_MX];
    pe->dy = py - s[SR_MY];
    pe->q = s[SR_CA] * pe->dx * pe->dx + 2.0 * s[SR_CB] * pe->dx * pe->dy + s[SR_CC] * pe->dy * pe->dy;
    pe->phi = s[SR_FX] * pe->dx + s[SR_FY] * pe->dy + s[SR_PH];
    pe->e = exp(-0.5 * pe->q);
    pe->kappa = 0.5 * (1.0 + cos(pe->phi));
    pe->w = pe->kappa * pe->e;
}

/* FP32 evaluation error bound of q = d^T A d (the additive support band):
 * the conic enters rounded to FP32 and pre-scaled (two roundings, 1.2e-7
 * relative per coefficient), the quadratic form is summed in three rounded
 * operations (1.8e-7 relative to the sum of the magnitudes of its terms,
 * which exceeds q when the cross term cancels, up to twice the condition
 * number of A), the threshold itself is rounded once, and the offset d
 * carries the FP32 rounding of the block-relative mean (at most 2e-6 px,
 * zero for 2D means that are FP32 inputs).  Bound:
 *   dq = 4e-7 (|a| dx^2 + 2 |b dx dy| + |c| dy^2) + 4e-6 (|a dx + b dy| + |b dx + c dy|). */
static double q_err(const double* s, const pair_eval* pe)
{
    const double a = s[SR_CA], b = s[SR_CB], c = s[SR_CC], dx = pe->dx, dy = pe->dy;
    return 4e-7 * (fabs(a) * dx * dx + 2.0 * fabs(b * dx * dy) + fabs(c) * dy * dy) +
           4e-6 * (fabs(a * dx + b * dy) + fabs(b * dx + c * dy));
}

/* FP32 evaluation error bound da of a = o W' (the tie bands above). */
static double a_err(const double* s, const pair_eval* pe)
{
    const double fn = sqrt(s[SR_FX] * s[SR_FX] + s[SR_FY] * s[SR_FY]);
    const double dphi = 4e-7 * fabs(pe->phi) + 4e-6 * fn + 1e-6;
    const double dkap = 0.5 * fabs(sin(pe->phi)) * dphi + 2e-6;
    return s[SR_OP] * (pe->e * dkap + pe->w * (1e-6 + 2e-7 * pe->q));
}

/* Candidate test: a padded box around the exact support box.  Outside the
 * exact box the rule rejects the pair in exact arithmetic, so the padding only
 * widens the set in which ties are looked for. */
static int in_padded_box(const double* s, double px, double py)
{
    if (s[SR_VALID] == 0.0) return 0;
    double padx = 0.01 + 1e-5 * s[SR_RX], pady = 0.01 + 1e-5 * s[SR_RY];
    return fabs(px - s[SR_MX]) <= s[SR_RX] + padx && fabs(py - s[SR_MY]) <= s[SR_RY] + pady;
}

/* Accumulate the screen-space gradient of one pair, given dL/dW' (Appendix
 * of the derivation: dW'/dq = -W'/2, dW'/dphi = -sin(phi) e / 2,
 * dq/dmu' = -2 A d, dq/d(a,b,c) = (dx^2, 2 dx dy, dy^2), dphi/dmu' = -f',
 * dphi/df' = d). */
static void pair_grad_w(const double* s, const pair_eval* pe, double dLdw, double* g)
{
    double dq = dLdw * (-0.5 * pe->w);
    double dphi = dLdw * (-0.5 * sin(pe->phi) * pe->e);
    double Adx = s[SR_CA] * pe->dx + s[SR_CB] * pe->dy;
    double Ady = s[SR_CB] * pe->dx + s[SR_CC] * pe->dy;
    g[SG_MX] += dq * (-2.0 * Adx) + dphi * (-s[SR_FX]);
    g[SG_MY] += dq * (-2.0 * Ady) + dphi * (-s[SR_FY]);
    g[SG_CA] += dq * pe->dx * pe->dx;
    g[SG_CB] += dq * 2.0 * pe->dx * pe->dy;
    g[SG_CC] += dq * pe->dy * pe->dy;
    g[SG_FX] += dphi * pe->dx;
    g[SG_FY] += dphi * pe->dy;
    g[SG_PH] += dphi;
}

typedef struct {
    int64_t id;
    uint32_t key;
} order_ent;

static int cmp_order(const void* a, const void* b)
{
    const order_ent* x = (const order_ent*)a;
    const order_ent* y = (const order_ent*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);
}

/* One contributing pair in a pixel's front-to-back list. */
typedef struct {
    int64_t id;
    pair_eval pe;
    double a, alpha, T_before;
    int clamped;
} contrib;

/*
 * Front-to-back alpha compositing of one pixel (Eq. 3 with W'), reading:
 *   a = o W'; skip the pair if a < alpha_min; alpha = min(a, alpha_max);
 *   C += T alpha c; T *= (1 - alpha); stop after a pair that leaves T < T_min;
 *   finally C += T bg.
 * cand[] holds the candidates already in (depth key, index) order.
 * Returns the number of contributing pairs written to out[] (may be NULL).
 */
static int64_t composite_pixel(const or_params* P, const double* screen, const order_ent* cand, int64_t ncand,
                               double px, double py, double C[3], double* T_out, int* tie, contrib* out,
                               double cmax, double* jump)
{
    double T = 1.0, dT = 0.0;
    int64_t nc = 0;
    C[0] = C[1] = C[2] = 0.0;
    for (int64_t k = 0; k < ncand; ++k) {
        const double* s = screen + SR_N * cand[k].id;
        pair_eval pe;
        eval_pair(s, px, py, &pe);
        double a = s[SR_OP] * pe.w;
        const double da = a_err(s, &pe);
        if (fabs(a - P->alpha_min) < 1e-5 * P->alpha_min + da) {
            *tie |= TIE_SKIP;
            if (jump) { jump[0] += 2.0 * cmax * (T * a + P->T_min); jump[1] += T * a + P->T_min; }
        }
        if (a < P->alpha_min) continue;
        if (fabs(a - P->alpha_max) < 1e-5 * P->alpha_max + da) *tie |= TIE_CLAMP;
        int clamped = a > P->alpha_max;
        double alpha = clamped ? P->alpha_max : a;
        if (out) {
            out[nc].id = cand[k].id;
            out[nc].pe = pe;
            out[nc].a = a;
            out[nc].alpha = alpha;
            out[nc].T_before = T;
            out[nc].clamped = clamped;
        }
        ++nc;
        C[0] += T * alpha * s[SR_R];
        C[1] += T * alpha * s[SR_G];
        C[2] += T * alpha * s[SR_B];
        T *= (1.0 - alpha);
        dT += da / (1.0 - alpha);
        if (fabs(T - P->T_min) < (1e-4 + dT) * P->T_min) {
            *tie |= TIE_STOP;
            if (jump) { jump[0] += 2.0 * cmax * T; jump[1] += T; }
        }
        if (T < P->T_min) break;
    }
    C[0] += T * P->bg[0];
    C[1] += T * P->bg[1];
    C[2] += T * P->bg[2];
    *T_out = T;
    return nc;
}

static int cull_tie(const or_params* P, const double* s)
{
    /* a primitive whose cull decision (near plane, opacity floor) sits on its
     * threshold: 2 = near plane (any jump), 1 = opacity floor */
    if (P->mode != OR_MODE_ALPHA3D) return 0;
    if (fabs(s[SR_DEPTH] - P->near_plane) < 1e-6 * (1.0 + P->near_plane)) return 2;
    return fabs(s[SR_OP] - P->alpha_min) < 1e-5 * P->alpha_min ? 1 : 0;
}

/* Jump bound of a cull tie of kind k (cull_tie) at transmittance T. */
static void cull_jump(const or_params* P, int k, double T, double cmax, double* jump)
{
    if (!jump) return;
    if (k == 2) { jump[0] += 2.0 * cmax; jump[1] += 1.0; }
    else { jump[0] += 2.0 * cmax * (T * P->alpha_min + P->T_min); jump[1] += T * P->alpha_min + P->T_min; }
}

/* Largest |colour| of the valid primitives and |bg| (the scale of every jump bound). */
static double colour_max(const or_params* P, const double* screen, int64_t n)
{
    double m = 0.0;
    for (int k = 0; k < 3; ++k) m = fmax(m, fabs(P->bg[k]));
    for (int64_t i = 0; i < n; ++i) {
        const double* s = screen + SR_N * i;
        if (s[SR_VALID] == 0.0) continue;
        for (int k = 0; k < 3; ++k) m = fmax(m, fabs(s[SR_R + k]));
    }
    return m;
}

/*
 * Depth order used by alpha compositing: key[i] is the FP32 camera depth key
 * (or_depth_key) supplied by the caller; ties go by index.
 */
static order_ent* make_order(const double* screen, int64_t n, const uint32_t* key, int64_t* nvalid)
{
    order_ent* ord = (order_ent*)malloc(sizeof(order_ent) * (size_t)(n > 0 ? n : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (screen[SR_N * i + SR_VALID] != 0.0) {
            ord[m].id = i;
            ord[m].key = key ? key[i] : 0u;
            ++m;
        }
    qsort(ord, (size_t)m, sizeof(order_ent), cmp_order);
    *nvalid = m;
    return ord;
}

/* ------------------------------------------------------------------------ */
/* O1: brute force, pixel by pixel over every primitive                     */
/* ------------------------------------------------------------------------ */

static int64_t pix_of(const int64_t* pix, int64_t k) { return pix ? pix[k] : k; }

/*
 * Forward render of the listed pixels (pix == NULL: all W*H pixels, row-major).
 * depth_key: FP32 depth keys as uint32 bit patterns (alpha mode), else NULL.
 * Outputs per listed pixel: image[3], T_final, n_contrib, tie flags.
 */
void or_render_o1(const or_params* P, int32_t W, int32_t H, int64_t n, const double* screen,
                  const uint32_t* depth_key, int64_t npix, const int64_t* pix, double* image, double* T_final,
                  int32_t* n_contrib, uint8_t* tie, double* jump)
{
    (void)H;
    int64_t nvalid = 0;
    order_ent* ord = make_order(screen, n, P->mode == OR_MODE_ALPHA3D ? depth_key : NULL, &nvalid);
    uint8_t* ptie = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
    for (int64_t i = 0; i < n; ++i) ptie[i] = (uint8_t)cull_tie(P, screen + SR_N * i);
    const double cmax = colour_max(P, screen, n);
#pragma omp parallel
    {
        order_ent* cand = (order_ent*)malloc(sizeof(order_ent) * (size_t)(nvalid > 0 ? nvalid : 1));
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < npix; ++k) {
            int64_t p = pix_of(pix, k);
            double px = (double)(p % W) + 0.5, py = (double)(p / W) + 0.5;
            int t = 0;
            int64_t nc = 0;
            double jb[2] = {0.0, 0.0};
            for (int64_t j = 0; j < nvalid; ++j) {
                const double* s = screen + SR_N * ord[j].id;
                if (in_padded_box(s, px, py)) {
                    cand[nc++] = ord[j];
                    if (ptie[ord[j].id]) {
                        t |= TIE_CULL;
                        cull_jump(P, ptie[ord[j].id], 1.0, cmax, jb);
                    }
                }
            }
            double* C = image + 3 * k;
            if (P->mode == OR_MODE_ADD2D) {
                int32_t cnt = 0;
                C[0] = C[1] = C[2] = 0.0;
                for (int64_t j = 0; j < nc; ++j) {
                    const double* s = screen + SR_N * cand[j].id;
                    pair_eval pe;
                    eval_pair(s, px, py, &pe);
                    if (fabs(pe.q - s[SR_Q]) < q_err(s, &pe) + 1e-7 * s[SR_Q]) {
                        t |= TIE_SUPPORT;
                        jb[0] += fabs(s[SR_OP] * pe.w) *
                                 fmax(fabs(s[SR_R]), fmax(fabs(s[SR_G]), fabs(s[SR_B])));
                    }
                    if (!(pe.q <= s[SR_Q])) continue;
                    double cw = s[SR_OP] * pe.w;
                    C[0] += s[SR_R] * cw;
                    C[1] += s[SR_G] * cw;
                    C[2] += s[SR_B] * cw;
                    ++cnt;
                }
                if (T_final) T_final[k] = 1.0;
                if (n_contrib) n_contrib[k] = cnt;
            } else {
                double T;
                int64_t cnt = composite_pixel(P, screen, cand, nc, px, py, C, &T, &t, NULL, cmax, jb);
                if (T_final) T_final[k] = T;
                if (n_contrib) n_contrib[k] = (int32_t)cnt;
            }
            if (tie) tie[k] = (uint8_t)t;
            if (jump) { jump[2 * k] = jb[0]; jump[2 * k + 1] = jb[1]; }
        }
        free(cand);
    }
    free(ptie);
    free(ord);
}

/*
 * Backward of or_render_o1 for the listed pixels: given dL/dC at each listed
 * pixel (dLdC[3k..3k+2]), accumulate screen-space gradients into
 * dscreen[n][SG_N] (overwritten).  Decisions (support, skip, stop, clamp) are
 * held fixed; the clamp has derivative zero.  Alpha mode walks each pixel's
 * contributing list back to front with S (colour behind) starting at bg:
 *   dL/dalpha_k = T_k (c_k - S_k) . g,   S_{k-1} = alpha_k c_k + (1 - alpha_k) S_k.
 * Pixel contributions are summed in pixel order, so the result is
 * deterministic for a given thread count.
 */
void or_render_bwd_o1(const or_params* P, int32_t W, int32_t H, int64_t n, const double* screen,
                      const uint32_t* depth_key, int64_t npix, const int64_t* pix, const double* dLdC,
                      double* dscreen, int32_t max_threads)
{
    (void)H;
    int64_t nvalid = 0;
    order_ent* ord = make_order(screen, n, P->mode == OR_MODE_ALPHA3D ? depth_key : NULL, &nvalid);
    memset(dscreen, 0, sizeof(double) * SG_N * (size_t)n);
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    /* bound the per-thread dense accumulators to about 1 GB in total */
    int64_t per = (int64_t)SG_N * 8 * (n > 0 ? n : 1);
    int64_t cap = (int64_t)(1ll << 30) / per;
    if (cap < 1) cap = 1;
    if (nthr > cap) nthr = (int)cap;
    if (max_threads > 0 && nthr > max_threads) nthr = max_threads;
    double* acc = (double*)calloc((size_t)nthr * (size_t)SG_N * (size_t)(n > 0 ? n : 1), sizeof(double));
#pragma omp parallel num_threads(nthr)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* g_all = acc + (size_t)tid * SG_N * (size_t)(n > 0 ? n : 1);
        order_ent* cand = (order_ent*)malloc(sizeof(order_ent) * (size_t)(nvalid > 0 ? nvalid : 1));
        contrib* list = (contrib*)malloc(sizeof(contrib) * (size_t)(nvalid > 0 ? nvalid : 1));
        int64_t chunk = (npix + nthr - 1) / nthr;
        int64_t k0 = (int64_t)tid * chunk, k1 = k0 + chunk < npix ? k0 + chunk : npix;
        for (int64_t k = k0; k < k1; ++k) {
            int64_t p = pix_of(pix, k);
            double px = (double)(p % W) + 0.5, py = (double)(p / W) + 0.5;
            const double* g = dLdC + 3 * k;
            if (g[0] == 0.0 && g[1] == 0.0 && g[2] == 0.0) continue;
            int64_t nc = 0;
            for (int64_t j = 0; j < nvalid; ++j)
                if (in_padded_box(screen + SR_N * ord[j].id, px, py)) cand[nc++] = ord[j];
            if (P->mode == OR_MODE_ADD2D) {
                for (int64_t j = 0; j < nc; ++j) {
                    const double* s = screen + SR_N * cand[j].id;
                    pair_eval pe;
                    eval_pair(s, px, py, &pe);
                    if (!(pe.q <= s[SR_Q])) continue;
                    double* gi = g_all + SG_N * cand[j].id;
                    double cg = s[SR_R] * g[0] + s[SR_G] * g[1] + s[SR_B] * g[2];
                    double ow = s[SR_OP] * pe.w;
                    gi[SG_R] += ow * g[0];
                    gi[SG_G] += ow * g[1];
                    gi[SG_B] += ow * g[2];
                    gi[SG_OP] += pe.w * cg;
                    pair_grad_w(s, &pe, s[SR_OP] * cg, gi);
                }
            } else {
                double C[3], T;
                int t = 0;
                int64_t m = composite_pixel(P, screen, cand, nc, px, py, C, &T, &t, list, 0.0, NULL);
                double S[3] = {P->bg[0], P->bg[1], P->bg[2]};
                for (int64_t j = m - 1; j >= 0; --j) {
                    const contrib* cb = &list[j];
                    const double* s = screen + SR_N * cb->id;
                    double* gi = g_all + SG_N * cb->id;
                    double c[3] = {s[SR_R], s[SR_G], s[SR_B]};
                    double dalpha = cb->T_before * ((c[0] - S[0]) * g[0] + (c[1] - S[1]) * g[1] + (c[2] - S[2]) * g[2]);
                    for (int ch = 0; ch < 3; ++ch) {
                        gi[SG_R + ch] += cb->T_before * cb->alpha * g[ch];
                        S[ch] = cb->alpha * c[ch] + (1.0 - cb->alpha) * S[ch];
                    }
                    if (!cb->clamped) {
                        gi[SG_OP] += cb->pe.w * dalpha;
                        pair_grad_w(s, &cb->pe, s[SR_OP] * dalpha, gi);
                    }
                }
            }
        }
        free(cand);
        free(list);
    }
    for (int t = 0; t < nthr; ++t) {
        const double* g_all = acc + (size_t)t * SG_N * (size_t)(n > 0 ? n : 1);
        for (int64_t i = 0; i < SG_N * n; ++i) dscreen[i] += g_all[i];
    }
    free(acc);
    free(ord);
}

/* ------------------------------------------------------------------------ */
/* O2: support scatter over the whole image                                 */
/* ------------------------------------------------------------------------ */

/*
 * Same per-pixel rule as O1, organised the other way round: primitives are
 * visited once in the compositing order (index order for additive, (depth key,
 * index) for alpha) and each updates the pixels of its padded support box.
 * Every pixel therefore sees its candidates in exactly the order O1 uses.
 * Rows are split between threads; a thread owns whole rows, so no pixel is
 * shared.  Outputs cover all W*H pixels, row-major.
 */
void or_render_o2(const or_params* P, int32_t W, int32_t H, int64_t n, const double* screen,
                  const uint32_t* depth_key, double* image, double* T_final, int32_t* last_id, uint8_t* tie,
                  double* jump)
{
    int64_t nvalid = 0;
    order_ent* ord = make_order(screen, n, P->mode == OR_MODE_ALPHA3D ? depth_key : NULL, &nvalid);
    const double cmax = colour_max(P, screen, n);
    int64_t npx = (int64_t)W * H;
    double* T = (double*)malloc(sizeof(double) * (size_t)(npx > 0 ? npx : 1));
    double* dT = (double*)calloc((size_t)(npx > 0 ? npx : 1), sizeof(double));
    uint8_t* done = (uint8_t*)calloc((size_t)(npx > 0 ? npx : 1), 1);
    for (int64_t p = 0; p < npx; ++p) {
        T[p] = 1.0;
        image[3 * p] = image[3 * p + 1] = image[3 * p + 2] = 0.0;
        if (tie) tie[p] = 0;
        if (jump) jump[2 * p] = jump[2 * p + 1] = 0.0;
        if (last_id) last_id[p] = -1;
    }
#pragma omp parallel for schedule(static, 1)
    for (int32_t band = 0; band < (H + 7) / 8; ++band) {
        int32_t ya = band * 8, yb = ya + 8 < H ? ya + 8 : H;
        for (int64_t j = 0; j < nvalid; ++j) {
            const double* s = screen + SR_N * ord[j].id;
            double padx = 0.01 + 1e-5 * s[SR_RX], pady = 0.01 + 1e-5 * s[SR_RY];
            double fx0 = ceil(s[SR_MX] - s[SR_RX] - padx - 0.5), fx1 = floor(s[SR_MX] + s[SR_RX] + padx - 0.5);
            double fy0 = ceil(s[SR_MY] - s[SR_RY] - pady - 0.5), fy1 = floor(s[SR_MY] + s[SR_RY] + pady - 0.5);
            if (fx0 < 0) fx0 = 0;
            if (fy0 < ya) fy0 = ya;
            if (fx1 > W - 1) fx1 = W - 1;
            if (fy1 > yb - 1) fy1 = yb - 1;
            if (!(fx0 <= fx1 && fy0 <= fy1)) continue;
            int ct = cull_tie(P, s);
            for (int32_t y = (int32_t)fy0; y <= (int32_t)fy1; ++y)
                for (int32_t x = (int32_t)fx0; x <= (int32_t)fx1; ++x) {
                    int64_t p = (int64_t)y * W + x;
                    double px = x + 0.5, py = y + 0.5;
                    if (!in_padded_box(s, px, py)) continue;
                    double* jb = jump ? jump + 2 * p : NULL;
                    if (ct && tie && !done[p]) {
                        tie[p] |= TIE_CULL;
                        cull_jump(P, ct, T[p], cmax, jb);
                    }
                    pair_eval pe;
                    eval_pair(s, px, py, &pe);
                    double* C = image + 3 * p;
                    if (P->mode == OR_MODE_ADD2D) {
                        if (tie && fabs(pe.q - s[SR_Q]) < q_err(s, &pe) + 1e-7 * s[SR_Q]) {
                            tie[p] |= TIE_SUPPORT;
                            if (jb)
                                jb[0] += fabs(s[SR_OP] * pe.w) *
                                         fmax(fabs(s[SR_R]), fmax(fabs(s[SR_G]), fabs(s[SR_B])));
                        }
                        if (!(pe.q <= s[SR_Q])) continue;
                        double cw = s[SR_OP] * pe.w;
                        C[0] += s[SR_R] * cw;
                        C[1] += s[SR_G] * cw;
                        C[2] += s[SR_B] * cw;
                        if (last_id) last_id[p] = (int32_t)ord[j].id;
                    } else {
                        if (done[p]) continue;
                        double a = s[SR_OP] * pe.w;
                        const double da = tie ? a_err(s, &pe) : 0.0;
                        if (tie && fabs(a - P->alpha_min) < 1e-5 * P->alpha_min + da) {
                            tie[p] |= TIE_SKIP;
                            if (jb) { jb[0] += 2.0 * cmax * (T[p] * a + P->T_min); jb[1] += T[p] * a + P->T_min; }
                        }
                        if (a < P->alpha_min) continue;
                        if (tie && fabs(a - P->alpha_max) < 1e-5 * P->alpha_max + da) tie[p] |= TIE_CLAMP;
                        double alpha = a > P->alpha_max ? P->alpha_max : a;
                        C[0] += T[p] * alpha * s[SR_R];
                        C[1] += T[p] * alpha * s[SR_G];
                        C[2] += T[p] * alpha * s[SR_B];
                        T[p] *= (1.0 - alpha);
                        dT[p] += da / (1.0 - alpha);
                        if (last_id) last_id[p] = (int32_t)ord[j].id;
                        if (tie && fabs(T[p] - P->T_min) < (1e-4 + dT[p]) * P->T_min) {
                            tie[p] |= TIE_STOP;
                            if (jb) { jb[0] += 2.0 * cmax * T[p]; jb[1] += T[p]; }
                        }
                        if (T[p] < P->T_min) done[p] = 1;
                    }
                }
        }
    }
    for (int64_t p = 0; p < npx; ++p) {
        if (P->mode == OR_MODE_ALPHA3D) {
            image[3 * p] += T[p] * P->bg[0];
            image[3 * p + 1] += T[p] * P->bg[1];
            image[3 * p + 2] += T[p] * P->bg[2];
            if (T_final) T_final[p] = T[p];
        } else if (T_final) {
            T_final[p] = 1.0;
        }
    }
    free(T);
    free(dT);
    free(done);
    free(ord);
}

/*
 * Backward of O2 over the whole image (dLdC[3p..3p+2] for every pixel).
 * Alpha mode walks the compositing order back to front; each pixel starts at
 * its final transmittance and its last contributing primitive (from the
 * forward) and recovers T before each contribution as T_after / (1 - alpha).
 * Per-band dense accumulators, summed in band order (deterministic).
 */
void or_render_bwd_o2(const or_params* P, int32_t W, int32_t H, int64_t n, const double* screen,
                      const uint32_t* depth_key, const double* T_final, const int32_t* last_id,
                      const double* dLdC, double* dscreen, int32_t max_threads)
{
    int64_t nvalid = 0;
    order_ent* ord = make_order(screen, n, P->mode == OR_MODE_ALPHA3D ? depth_key : NULL, &nvalid);
    int64_t* rank = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) rank[i] = -1;
    for (int64_t j = 0; j < nvalid; ++j) rank[ord[j].id] = j;
    int64_t npx = (int64_t)W * H;
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    int64_t per = (int64_t)SG_N * 8 * (n > 0 ? n : 1);
    int64_t cap = (int64_t)(1ll << 30) / per;
    if (cap < 1) cap = 1;
    if (nthr > cap) nthr = (int)cap;
    if (max_threads > 0 && nthr > max_threads) nthr = max_threads;
    int32_t nband = (H + 7) / 8;
    if (nthr > nband) nthr = nband > 0 ? nband : 1;
    double* acc = (double*)calloc((size_t)nthr * SG_N * (size_t)(n > 0 ? n : 1), sizeof(double));
    double* T = (double*)malloc(sizeof(double) * (size_t)(npx > 0 ? npx : 1));
    double* S = (double*)malloc(sizeof(double) * 3 * (size_t)(npx > 0 ? npx : 1));
    for (int64_t p = 0; p < npx; ++p) {
        T[p] = T_final ? T_final[p] : 1.0;
        S[3 * p] = P->bg[0];
        S[3 * p + 1] = P->bg[1];
        S[3 * p + 2] = P->bg[2];
    }
#pragma omp parallel num_threads(nthr)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* g_all = acc + (size_t)tid * SG_N * (size_t)(n > 0 ? n : 1);
        for (int32_t band = tid; band < nband; band += nthr) {
            int32_t ya = band * 8, yb = ya + 8 < H ? ya + 8 : H;
            for (int64_t jj = nvalid - 1; jj >= 0; --jj) {
                const double* s = screen + SR_N * ord[jj].id;
                double padx = 0.01 + 1e-5 * s[SR_RX], pady = 0.01 + 1e-5 * s[SR_RY];
                double fx0 = ceil(s[SR_MX] - s[SR_RX] - padx - 0.5), fx1 = floor(s[SR_MX] + s[SR_RX] + padx - 0.5);
                double fy0 = ceil(s[SR_MY] - s[SR_RY] - pady - 0.5), fy1 = floor(s[SR_MY] + s[SR_RY] + pady - 0.5);
                if (fx0 < 0) fx0 = 0;
                if (fy0 < ya) fy0 = ya;
                if (fx1 > W - 1) fx1 = W - 1;
                if (fy1 > yb - 1) fy1 = yb - 1;
                if (!(fx0 <= fx1 && fy0 <= fy1)) continue;
                double* gi = g_all + SG_N * ord[jj].id;
                for (int32_t y = (int32_t)fy0; y <= (int32_t)fy1; ++y)
                    for (int32_t x = (int32_t)fx0; x <= (int32_t)fx1; ++x) {
                        int64_t p = (int64_t)y * W + x;
                        const double* g = dLdC + 3 * p;
                        double px = x + 0.5, py = y + 0.5;
                        if (!in_padded_box(s, px, py)) continue;
                        pair_eval pe;
                        eval_pair(s, px, py, &pe);
                        if (P->mode == OR_MODE_ADD2D) {
                            if (!(pe.q <= s[SR_Q])) continue;
                            double cg = s[SR_R] * g[0] + s[SR_G] * g[1] + s[SR_B] * g[2];
                            double ow = s[SR_OP] * pe.w;
                            gi[SG_R] += ow * g[0];
                            gi[SG_G] += ow * g[1];
                            gi[SG_B] += ow * g[2];
                            gi[SG_OP] += pe.w * cg;
                            pair_grad_w(s, &pe, s[SR_OP] * cg, gi);
                        } else {
                            if (last_id[p] < 0 || rank[last_id[p]] < jj) continue;
                            double a = s[SR_OP] * pe.w;
                            if (a < P->alpha_min) continue;
                            int clamped = a > P->alpha_max;
                            double alpha = clamped ? P->alpha_max : a;
                            double Tb = T[p] / (1.0 - alpha);
                            double* Sp = S + 3 * p;
                            double c[3] = {s[SR_R], s[SR_G], s[SR_B]};
                            double dalpha = Tb * ((c[0] - Sp[0]) * g[0] + (c[1] - Sp[1]) * g[1] + (c[2] - Sp[2]) * g[2]);
                            for (int ch = 0; ch < 3; ++ch) {
                                gi[SG_R + ch] += Tb * alpha * g[ch];
                                Sp[ch] = alpha * c[ch] + (1.0 - alpha) * Sp[ch];
                            }
                            T[p] = Tb;
                            if (!clamped) {
                                gi[SG_OP] += pe.w * dalpha;
                                pair_grad_w(s, &pe, s[SR_OP] * dalpha, gi);
                            }
                        }
                    }
            }
        }
    }
    memset(dscreen, 0, sizeof(double) * SG_N * (size_t)n);
    for (int t = 0; t < nthr; ++t) {
        const double* g_all = acc + (size_t)t * SG_N * (size_t)(n > 0 ? n : 1);
        for (int64_t i = 0; i < SG_N * n; ++i) dscreen[i] += g_all[i];
    }
    free(acc);
    free(T);
    free(S);
    free(rank);
    free(ord);
}

/* ------------------------------------------------------------------------ */
/* Projection backward (FP64 chain rule)                                    */
/* ------------------------------------------------------------------------ */

/*
 * From screen-space gradients (dscreen[n][SG_N]) to parameter gradients.
 * Conic: A = Sigma'^-1, so dL/dSigma' = -A (dL/dA) A with the symmetric
 * dL/dA = [[ga, gb/2], [gb/2, gc]].
 * Covector frequency transform: f3' = A3^-T f with A3 = Jfull W (3x3) and
 * f' its first two entries, so dL/df = A3^-1 g3 (g3 = (dL/df', 0)) and
 * dL/dA3 = -f3' (dL/df)^T, which reaches t through the two rows of J and the
 * third row t/|t| (derivative (I - t t^T/|t|^2)/|t|).
 * SH colour: dL/dsh[k] = Y_k dL/dc, and the view direction carries
 * dL/dmean += (I - u u^T)/|d| sum_k grad Y_k (sh[k] . dL/dc), u = d/|d|.
 * Output arrays (any may be NULL): dmean[n*D], dcov[n*3] (2D), dquat[n*4],
 * dscale[n*3], dfreq[n*D], dcolor[n*3] (direct RGB only), dopac[n], dvel[n*3],
 * dphase[n], dsh[n*(deg+1)^2*3].
 * Invalid (culled) primitives get zero gradients.
 */
void or_project_bwd(const or_params* P, const or_camera* cam, int64_t n, const double* mean, const double* covp,
                    const double* quat, const double* scale, const double* freq, const double* opac, const double* vel,
                    const double* sh, const double* screen, const double* dscreen, double* dmean, double* dcov,
                    double* dquat, double* dscale, double* dfreq, double* dcolor, double* dopac, double* dvel,
                    double* dphase, double* dsh)
{
    int D = P->mode == OR_MODE_ADD2D ? 2 : 3;
    (void)opac;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double* s = screen + SR_N * i;
        const double* g = dscreen + SG_N * i;
        if (dmean) for (int k = 0; k < D; ++k) dmean[D * i + k] = 0.0;
        if (dfreq) for (int k = 0; k < D; ++k) dfreq[D * i + k] = 0.0;
        if (dcov) for (int k = 0; k < 3; ++k) dcov[3 * i + k] = 0.0;
        if (dquat) for (int k = 0; k < 4; ++k) dquat[4 * i + k] = 0.0;
        if (dscale) for (int k = 0; k < 3; ++k) dscale[3 * i + k] = 0.0;
        if (dvel) for (int k = 0; k < 3; ++k) dvel[3 * i + k] = 0.0;
        if (dcolor) for (int k = 0; k < 3; ++k) dcolor[3 * i + k] = 0.0;
        if (dopac) dopac[i] = 0.0;
        if (dphase) dphase[i] = 0.0;
        const int KSH = P->sh_degree >= 0 ? sh_count(P->sh_degree) : 0;
        if (dsh) for (int k = 0; k < 3 * KSH; ++k) dsh[(size_t)3 * KSH * i + k] = 0.0;
        if (s[SR_VALID] == 0.0) continue;
        if (dcolor && KSH == 0) for (int k = 0; k < 3; ++k) dcolor[3 * i + k] = g[SG_R + k];
        if (dopac) dopac[i] = g[SG_OP];
        if (dphase) dphase[i] = g[SG_PH];
        /* dL/dSigma' (symmetric 2x2) */
        double a = s[SR_CA], b = s[SR_CB], c = s[SR_CC];
        double GA[4] = {g[SG_CA], 0.5 * g[SG_CB], 0.5 * g[SG_CB], g[SG_CC]};
        double A[4] = {a, b, b, c};
        double T1[4], GS[4];
        for (int r = 0; r < 2; ++r)
            for (int cc = 0; cc < 2; ++cc) T1[2 * r + cc] = A[2 * r] * GA[cc] + A[2 * r + 1] * GA[2 + cc];
        for (int r = 0; r < 2; ++r)
            for (int cc = 0; cc < 2; ++cc) GS[2 * r + cc] = -(T1[2 * r] * A[cc] + T1[2 * r + 1] * A[2 + cc]);
        if (P->mode == OR_MODE_ADD2D) {
            if (dmean) { dmean[2 * i] = g[SG_MX]; dmean[2 * i + 1] = g[SG_MY]; }
            if (dfreq) { dfreq[2 * i] = g[SG_FX]; dfreq[2 * i + 1] = g[SG_FY]; }
            if (!dcov) continue;
            if (P->cov == OR_COV_CHOLESKY) {
                double l11 = covp[3 * i], l21 = covp[3 * i + 1], l22 = covp[3 * i + 2];
                /* Sigma = L L^T: dL = 2 G L (lower triangle) */
                dcov[3 * i] = 2.0 * (GS[0] * l11 + GS[1] * l21);
                dcov[3 * i + 1] = 2.0 * (GS[2] * l11 + GS[3] * l21);
                dcov[3 * i + 2] = 2.0 * GS[3] * l22;
            } else {
                double s1 = covp[3 * i], s2 = covp[3 * i + 1], th = covp[3 * i + 2];
                double cs = cos(th), sn = sin(th);
                double R[4] = {cs, -sn, sn, cs};
                double Rd[4] = {-sn, -cs, cs, -sn};
                double Dg[2] = {s1 * s1, s2 * s2};
                /* dL/dD_kk = (R^T G R)_kk */
                double dD[2];
                for (int k = 0; k < 2; ++k) {
                    double acc = 0.0;
                    for (int r = 0; r < 2; ++r)
                        for (int cc = 0; cc < 2; ++cc) acc += R[2 * r + k] * GS[2 * r + cc] * R[2 * cc + k];
                    dD[k] = acc;
                }
                dcov[3 * i] = 2.0 * s1 * dD[0];
                dcov[3 * i + 1] = 2.0 * s2 * dD[1];
                /* dSigma/dtheta = Rd D R^T + R D Rd^T */
                double acc = 0.0;
                for (int r = 0; r < 2; ++r)
                    for (int cc = 0; cc < 2; ++cc) {
                        double dS = 0.0;
                        for (int k = 0; k < 2; ++k)
                            dS += Rd[2 * r + k] * Dg[k] * R[2 * cc + k] + R[2 * r + k] * Dg[k] * Rd[2 * cc + k];
                        acc += GS[2 * r + cc] * dS;
                    }
                dcov[3 * i + 2] = acc;
            }
            continue;
        }
        /* ---- 3D ---- */
        proj3 pj;
        project_3d_core(P, cam, i, mean, quat, scale, freq, vel, &pj);
        double tx = pj.t[0], ty = pj.t[1], tz = pj.t[2];
        double fxc = cam->fx, fyc = cam->fy;
        double M[6];
        memcpy(M, pj.M, sizeof(M));
        /* dL/dM = 2 G M Sigma3 (+ dL/df' f^T for the vector transform) */
        double dM[6] = {0, 0, 0, 0, 0, 0};
        for (int r = 0; r < 2; ++r)
            for (int cc = 0; cc < 3; ++cc) {
                double acc = 0.0;
                for (int k = 0; k < 2; ++k)
                    for (int l = 0; l < 3; ++l) acc += GS[2 * r + k] * M[3 * k + l] * pj.S3[3 * l + cc];
                dM[3 * r + cc] = 2.0 * acc;
            }
        double dfw[3] = {0, 0, 0};
        double dJ3[3] = {0, 0, 0};   /* dL/d(third row of Jfull) (covector only) */
        double dJc[6] = {0, 0, 0, 0, 0, 0};   /* dL/d(rows 0-1 of Jfull) from the covector */
        if (P->freq_xform == OR_FREQ_VECTOR) {
            for (int cc = 0; cc < 3; ++cc) {
                dM[cc] += g[SG_FX] * pj.f3[cc];
                dM[3 + cc] += g[SG_FY] * pj.f3[cc];
                dfw[cc] = M[cc] * g[SG_FX] + M[3 + cc] * g[SG_FY];
            }
        } else {
            double A3[9], Ai[9];
            for (int r = 0; r < 3; ++r)
                for (int cc = 0; cc < 3; ++cc)
                    A3[3 * r + cc] = pj.Jfull[3 * r] * pj.Rw[cc] + pj.Jfull[3 * r + 1] * pj.Rw[3 + cc] +
                                     pj.Jfull[3 * r + 2] * pj.Rw[6 + cc];
            inv3(A3, Ai);
            double f3p[3], g3[3] = {g[SG_FX], g[SG_FY], 0.0};
            for (int r = 0; r < 3; ++r) f3p[r] = Ai[r] * pj.f3[0] + Ai[3 + r] * pj.f3[1] + Ai[6 + r] * pj.f3[2];
            for (int r = 0; r < 3; ++r) dfw[r] = Ai[3 * r] * g3[0] + Ai[3 * r + 1] * g3[1] + Ai[3 * r + 2] * g3[2];
            /* dL/dA3 = -f3' dfw^T, then dL/dJfull = dL/dA3 W^T */
            for (int r = 0; r < 3; ++r)
                for (int cc = 0; cc < 3; ++cc) {
                    double acc = 0.0;
                    for (int k = 0; k < 3; ++k) acc += -f3p[r] * dfw[k] * pj.Rw[3 * cc + k];
                    if (r < 2) dJc[3 * r + cc] = acc; else dJ3[cc] = acc;
                }
        }
        /* dL/dSigma3 = M^T G M */
        double dS3[9];
        for (int r = 0; r < 3; ++r)
            for (int cc = 0; cc < 3; ++cc) {
                double acc = 0.0;
                for (int k = 0; k < 2; ++k)
                    for (int l = 0; l < 2; ++l) acc += M[3 * k + r] * GS[2 * k + l] * M[3 * l + cc];
                dS3[3 * r + cc] = acc;
            }
        /* dL/dJ = dM Rw^T (+ the covector's direct term) */
        double dJ[6];
        for (int r = 0; r < 2; ++r)
            for (int cc = 0; cc < 3; ++cc) {
                double acc = dJc[3 * r + cc];
                for (int k = 0; k < 3; ++k) acc += dM[3 * r + k] * pj.Rw[3 * cc + k];
                dJ[3 * r + cc] = acc;
            }
        /* J entries as functions of t:  J00 = fx/tz, J02 = -fx u/tz, J11 = fy/tz, J12 = -fy v/tz */
        double dt[3] = {0, 0, 0};
        dt[2] += dJ[0] * (-fxc / (tz * tz)) + dJ[4] * (-fyc / (tz * tz));
        if (!pj.clampx) {
            /* J02 = -fx tx / tz^2 */
            dt[0] += dJ[2] * (-fxc / (tz * tz));
            dt[2] += dJ[2] * (2.0 * fxc * tx / (tz * tz * tz));
        } else {
            double uc = -pj.J[2] * tz / fxc;
            dt[2] += dJ[2] * (fxc * uc / (tz * tz));
        }
        if (!pj.clampy) {
            dt[1] += dJ[5] * (-fyc / (tz * tz));
            dt[2] += dJ[5] * (2.0 * fyc * ty / (tz * tz * tz));
        } else {
            double vc = -pj.J[5] * tz / fyc;
            dt[2] += dJ[5] * (fyc * vc / (tz * tz));
        }
        /* third row of Jfull = t / |t| (covector only) */
        {
            double tl = sqrt(tx * tx + ty * ty + tz * tz), th[3] = {tx / tl, ty / tl, tz / tl};
            double dot = th[0] * dJ3[0] + th[1] * dJ3[1] + th[2] * dJ3[2];
            for (int k = 0; k < 3; ++k) dt[k] += (dJ3[k] - th[k] * dot) / tl;
        }
        /* mu' = (fx tx/tz + cx, fy ty/tz + cy) */
        dt[0] += g[SG_MX] * fxc / tz;
        dt[1] += g[SG_MY] * fyc / tz;
        dt[2] += g[SG_MX] * (-fxc * tx / (tz * tz)) + g[SG_MY] * (-fyc * ty / (tz * tz));
        /* t = Rw m + w  ->  dL/dm = Rw^T dL/dt */
        double dm[3];
        for (int k = 0; k < 3; ++k) dm[k] = pj.Rw[k] * dt[0] + pj.Rw[3 + k] * dt[1] + pj.Rw[6 + k] * dt[2];
        if (KSH > 0) {
            /* colour = sum_k Y_k(u) sh[k], u = (m - C)/|m - C| */
            double Cc[3], d[3], Y[16], G[48];
            camera_centre(cam, Cc);
            for (int k = 0; k < 3; ++k) d[k] = pj.m[k] - Cc[k];
            double dl = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double u[3] = {d[0] / dl, d[1] / dl, d[2] / dl};
            sh_basis(P->sh_degree, u[0], u[1], u[2], Y, G);
            double du[3] = {0, 0, 0};
            for (int k = 0; k < KSH; ++k) {
                const double* c = sh + ((size_t)i * KSH + k) * 3;
                double w = c[0] * g[SG_R] + c[1] * g[SG_G] + c[2] * g[SG_B];
                for (int a = 0; a < 3; ++a) du[a] += G[3 * k + a] * w;
                if (dsh)
                    for (int cc = 0; cc < 3; ++cc) dsh[((size_t)i * KSH + k) * 3 + cc] = Y[k] * g[SG_R + cc];
            }
            double dot = u[0] * du[0] + u[1] * du[1] + u[2] * du[2];
            for (int a = 0; a < 3; ++a) dm[a] += (du[a] - u[a] * dot) / dl;
        }
        if (dmean) for (int k = 0; k < 3; ++k) dmean[3 * i + k] = dm[k];
        if (dvel && vel) for (int k = 0; k < 3; ++k) dvel[3 * i + k] = dm[k] * cam->time;
        if (dfreq) for (int k = 0; k < 3; ++k) dfreq[3 * i + k] = dfw[k];
        /* Sigma3 = Rq diag(s^2) Rq^T */
        if (dscale) {
            for (int k = 0; k < 3; ++k) {
                double acc = 0.0;
                for (int r = 0; r < 3; ++r)
                    for (int cc = 0; cc < 3; ++cc) acc += dS3[3 * r + cc] * pj.Rq[3 * r + k] * pj.Rq[3 * cc + k];
                dscale[3 * i + k] = 2.0 * pj.sc[k] * acc;
            }
        }
        if (dquat) {
            double dqn[4];
            for (int k = 0; k < 4; ++k) {
                double Dr[9];
                quat_rot_deriv(pj.qn, k, Dr);
                /* dSigma3 = Dr S2 Rq^T + Rq S2 Dr^T */
                double acc = 0.0;
                for (int r = 0; r < 3; ++r)
                    for (int cc = 0; cc < 3; ++cc) {
                        double dS = 0.0;
                        for (int l = 0; l < 3; ++l) {
                            double s2 = pj.sc[l] * pj.sc[l];
                            dS += Dr[3 * r + l] * s2 * pj.Rq[3 * cc + l] + pj.Rq[3 * r + l] * s2 * Dr[3 * cc + l];
                        }
                        acc += dS3[3 * r + cc] * dS;
                    }
                dqn[k] = acc;
            }
            /* through q_hat = q / |q| */
            double dot = 0.0;
            for (int k = 0; k < 4; ++k) dot += pj.qn[k] * dqn[k];
            for (int k = 0; k < 4; ++k) dquat[4 * i + k] = (dqn[k] - pj.qn[k] * dot) / pj.qnorm;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* O-bin: the tile binning rule, defined in FP32                            */
/* ------------------------------------------------------------------------ */

/*
 * Reading of the 3DGS-like pipeline of Sec. 4.1: every primitive is
 * duplicated once per screen tile its support box touches; the duplicates are
 * keyed by (tile, depth) and stably sorted, and each tile's run of the sorted
 * list is its range.  The rule, in FP32 with exactly these operations:
 *   culled unless rx >= 0, ry >= 0 and |mx|, |my| < 1e30
 *   x0 = max(ceil((mx - rx) - 0.5), 0),  x1 = min(floor((mx + rx) - 0.5), W - 1)   (same for y)
 *   empty unless x0 <= x1 and y0 <= y1           -- pixel box of covered centres
 *   tile rect = [x0 / tw, x1 / tw] x [y0 / th, y1 / th]  (integer division)
 *   tile id = ty * ceil(W / tw) + tx;  key = tile << 32 | float bits(depth)  (alpha)
 *                                      key = tile                            (additive)
 *   instances are emitted in primitive order, tiles of one primitive row-major,
 *   and sorted stably by key; range of tile t = [first, last + 1), empty = (0, 0).
 * box[4*i..] receives (x0, y0, x1, y1) or (1, 1, 0, 0) when empty.
 * Call once with keys == NULL to learn K (*K_out), then again with arrays of
 * at least K entries.
 */
typedef struct {
    uint64_t key;
    uint32_t val;
    uint32_t seq;
} bin_ent;

static int cmp_bin(const void* a, const void* b)
{
    const bin_ent* x = (const bin_ent*)a;
    const bin_ent* y = (const bin_ent*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->seq < y->seq ? -1 : (x->seq > y->seq ? 1 : 0);
}

/*
 * Ellipse part of the binning rule (a reading; Sec. 4.1 bins like 3DGS): a
 * tile of a primitive's tile rectangle gets an instance only if the padded
 * support ellipse q(x) <= Qs, q = ca dx^2 + 2 cb dx dy + cc dy^2, reaches the
 * rectangle of pixel centres of (tile intersected with the pixel box).  The
 * minimum of the convex q over that rectangle is 0 if the mean lies inside,
 * else it lies on an edge, where it is a clamped one-dimensional minimum.
 * FP32 in exactly this sequence (explicit fmaf, IEEE division).  Rectangles
 * of more than 64 tiles keep every tile.
 */
static float or_q32(float ca, float cb, float cc, float dx, float dy)
{
    return fmaf(ca * dx, dx, fmaf(2.0f * cb * dx, dy, cc * dy * dy));
}

static float or_clamp32(float v, float lo, float hi) { return fminf(fmaxf(v, lo), hi); }

static int or_ellipse_meets(float mx, float my, float ca, float cb, float cc, float Qs, int32_t x0, int32_t y0,
                            int32_t x1, int32_t y1)
{
    const float fx0 = (float)x0 + 0.5f, fx1 = (float)x1 + 0.5f, fy0 = (float)y0 + 0.5f, fy1 = (float)y1 + 0.5f;
    if (mx >= fx0 && mx <= fx1 && my >= fy0 && my <= fy1) return 1;
    const float sy = -cb / cc, sx = -cb / ca;
    const float dxa = fx0 - mx, dxb = fx1 - mx, dya = fy0 - my, dyb = fy1 - my;
    float m = or_q32(ca, cb, cc, dxa, or_clamp32(sy * dxa, dya, dyb));
    m = fminf(m, or_q32(ca, cb, cc, dxb, or_clamp32(sy * dxb, dya, dyb)));
    m = fminf(m, or_q32(ca, cb, cc, or_clamp32(sx * dya, dxa, dxb), dya));
    m = fminf(m, or_q32(ca, cb, cc, or_clamp32(sx * dyb, dxa, dxb), dyb));
    return m <= Qs;
}

#define OR_BIN_CULL_MAX_TILES 64

/* Whether tile (tx, ty) of primitive i's rectangle is kept. */
static int or_bin_keep(const int32_t* b, int32_t tw, int32_t th, int32_t tx, int32_t ty, int32_t nt, float mx,
                       float my, float ca, float cb, float cc, float Qs)
{
    if (nt > OR_BIN_CULL_MAX_TILES) return 1;
    const int32_t x0 = tx * tw > b[0] ? tx * tw : b[0], y0 = ty * th > b[1] ? ty * th : b[1];
    const int32_t x1 = tx * tw + tw - 1 < b[2] ? tx * tw + tw - 1 : b[2];
    const int32_t y1 = ty * th + th - 1 < b[3] ? ty * th + th - 1 : b[3];
    return or_ellipse_meets(mx, my, ca, cb, cc, Qs, x0, y0, x1, y1);
}

void or_bin(int32_t W, int32_t H, int32_t tw, int32_t th, int32_t mode, int64_t n, const float* mx, const float* my,
            const float* rx, const float* ry, const float* depth, const float* ca, const float* cb, const float* cc,
            const float* Qs, int32_t* box, int32_t* count, int64_t* K_out, uint64_t* keys, uint32_t* vals,
            uint32_t* ranges)
{
    int32_t tiles_x = (W + tw - 1) / tw, tiles_y = (H + th - 1) / th;
    int64_t K = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t* b = box + 4 * i;
        b[0] = 1; b[1] = 1; b[2] = 0; b[3] = 0;
        count[i] = 0;
        float x = mx[i], y = my[i], ex = rx[i], ey = ry[i];
        if (!(ex >= 0.0f && ey >= 0.0f && fabsf(x) < 1e30f && fabsf(y) < 1e30f)) continue;
        float x0 = ceilf((x - ex) - 0.5f), x1 = floorf((x + ex) - 0.5f);
        float y0 = ceilf((y - ey) - 0.5f), y1 = floorf((y + ey) - 0.5f);
        if (x0 < 0.0f) x0 = 0.0f;
        if (y0 < 0.0f) y0 = 0.0f;
        if (x1 > (float)(W - 1)) x1 = (float)(W - 1);
        if (y1 > (float)(H - 1)) y1 = (float)(H - 1);
        if (!(x0 <= x1 && y0 <= y1)) continue;
        b[0] = (int32_t)x0; b[1] = (int32_t)y0; b[2] = (int32_t)x1; b[3] = (int32_t)y1;
        int32_t tx0 = b[0] / tw, tx1 = b[2] / tw, ty0 = b[1] / th, ty1 = b[3] / th;
        const int32_t nt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
        int32_t c = 0;
        for (int32_t ty = ty0; ty <= ty1; ++ty)
            for (int32_t tx = tx0; tx <= tx1; ++tx)
                c += or_bin_keep(b, tw, th, tx, ty, nt, x, y, ca[i], cb[i], cc[i], Qs[i]);
        count[i] = c;
        K += count[i];
    }
    *K_out = K;
    if (!keys) return;
    bin_ent* e = (bin_ent*)malloc(sizeof(bin_ent) * (size_t)(K > 0 ? K : 1));
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (count[i] == 0) continue;
        const int32_t* b = box + 4 * i;
        const int32_t nt = (b[2] / tw - b[0] / tw + 1) * (b[3] / th - b[1] / th + 1);
        for (int32_t ty = b[1] / th; ty <= b[3] / th; ++ty)
            for (int32_t tx = b[0] / tw; tx <= b[2] / tw; ++tx) {
                if (!or_bin_keep(b, tw, th, tx, ty, nt, mx[i], my[i], ca[i], cb[i], cc[i], Qs[i])) continue;
                uint64_t tile = (uint64_t)ty * (uint64_t)tiles_x + (uint64_t)tx;
                e[k].key = mode == OR_MODE_ALPHA3D ? (tile << 32) | float_bits(depth[i]) : tile;
                e[k].val = (uint32_t)i;
                e[k].seq = (uint32_t)k;
                ++k;
            }
    }
    qsort(e, (size_t)K, sizeof(bin_ent), cmp_bin);
    int64_t ntiles = (int64_t)tiles_x * tiles_y;
    for (int64_t t = 0; t < 2 * ntiles; ++t) ranges[t] = 0;
    for (int64_t j = 0; j < K; ++j) {
        keys[j] = e[j].key;
        vals[j] = e[j].val;
        uint64_t tile = mode == OR_MODE_ALPHA3D ? e[j].key >> 32 : e[j].key;
        if (j == 0 || (mode == OR_MODE_ALPHA3D ? e[j - 1].key >> 32 : e[j - 1].key) != tile)
            ranges[2 * tile] = (uint32_t)j;
        ranges[2 * tile + 1] = (uint32_t)(j + 1);
    }
    free(e);
}

/* ------------------------------------------------------------------------ */
/* Work counts                                                              */
/* ------------------------------------------------------------------------ */

/*
 * Support pairs per listed pixel: pairs whose pixel lies inside the
 * primitive's support ellipse q <= Q (Q = q_add, or 2 ln(o / alpha_min) in
 * alpha mode), counted
 *   fwd[k]: over the pairs the per-pixel rule evaluates (alpha: up to and
 *           including the stopping pair);
 *   bwd[k]: alpha: up to and including the last contributing pair; additive:
 *           equal to fwd.
 */
void or_support_counts(const or_params* P, int32_t W, int32_t H, int64_t n, const double* screen,
                       const uint32_t* depth_key, int64_t npix, const int64_t* pix, int64_t* fwd, int64_t* bwd)
{
    (void)H;
    int64_t nvalid = 0;
    order_ent* ord = make_order(screen, n, P->mode == OR_MODE_ALPHA3D ? depth_key : NULL, &nvalid);
#pragma omp parallel
    {
        order_ent* cand = (order_ent*)malloc(sizeof(order_ent) * (size_t)(nvalid > 0 ? nvalid : 1));
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < npix; ++k) {
            int64_t p = pix_of(pix, k);
            double px = (double)(p % W) + 0.5, py = (double)(p / W) + 0.5;
            int64_t nc = 0;
            for (int64_t j = 0; j < nvalid; ++j)
                if (in_padded_box(screen + SR_N * ord[j].id, px, py)) cand[nc++] = ord[j];
            int64_t cf = 0, cb = 0, pending = 0;
            double T = 1.0;
            for (int64_t j = 0; j < nc; ++j) {
                const double* s = screen + SR_N * cand[j].id;
                pair_eval pe;
                eval_pair(s, px, py, &pe);
                int in = pe.q <= s[SR_Q];
                cf += in;
                if (P->mode == OR_MODE_ADD2D) continue;
                pending += in;
                double a = s[SR_OP] * pe.w;
                if (a < P->alpha_min) continue;
                cb += pending;          /* support pairs up to this contributing pair */
                pending = 0;
                double alpha = a > P->alpha_max ? P->alpha_max : a;
                T *= (1.0 - alpha);
                if (T < P->T_min) break;
            }
            fwd[k] = cf;
            bwd[k] = P->mode == OR_MODE_ADD2D ? cf : cb;
        }
        free(cand);
    }
    free(ord);
}
