// Projection of 2D and 3D wavelet primitives to 64-byte screen records.
//
// 2D (Sec. 5.1, Eq. 4 with W'): the primitive lives on the image plane, so
// mu' = mu and f' = f; Sigma comes from a Cholesky factor or a rotation and
// two scales.  3D (Sec. 3.1 Eq. 2, Sec. 4.1 Eq. 7): EWA splatting,
// Sigma' = M Sigma M^T + eps I with M = J W (J the local affine Jacobian of
// the perspective map, W the camera rotation), and the frequency goes
// through the same map, f' = M f.
//
// One thread per primitive.  The arithmetic runs in FP64 (about a hundred
// flops per primitive, invisible next to the record traffic) because the
// records feed a carrier of up to half a cycle per pixel: an FP32 mean at
// x ~ 1000 px is off by up to 3e-5 px, i.e. ~1e-4 rad of phase.  The mean is
// stored as an FP32 pair (hi, lo) so the blend can rebuild it exactly.
// The depth key is the one exception: it is defined as an FP32 evaluation
// (fused multiply-adds in a fixed order) so that the compositing order is
// reproducible bit for bit.
#include <cstring>

#include "common.hpp"

namespace wipes {

// Carrier phase phi0 (radians; none = 0) as the record stores it: in
// revolutions, reduced to [0, 1) in FP64 so that the blend's phase sum stays
// exact however large phi0 is.
__device__ __forceinline__ float phase_rev(const float* __restrict__ phase, int32_t j)
{
    if (!phase) return 0.0f;
    const double r = (double)phase[j] * 0.15915494309189533577;
    return (float)(r - floor(r));
}

__device__ __forceinline__ void store_record(Rec* __restrict__ recs, int32_t i, double mx, double my, double ca,
                                             double cb, double cc, float fx, float fy, float op, float r, float g,
                                             float b, float ph)
{
    float mxh = (float)mx, myh = (float)my;
    float mxl = (float)(mx - (double)mxh), myl = (float)(my - (double)myh);
    float4* o = reinterpret_cast<float4*>(recs + i);
    o[0] = make_float4(mxh, myh, (float)ca, (float)cb);
    o[1] = make_float4((float)cc, fx, fy, op);
    o[2] = make_float4(r, g, b, mxl);
    o[3] = make_float4(myl, ph, 0.0f, 0.0f);
}

__device__ __forceinline__ void store_culled(Rec* __restrict__ recs, Aux* __restrict__ aux, int32_t i, float depth)
{
    float4* o = reinterpret_cast<float4*>(recs + i);
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    o[0] = z; o[1] = z; o[2] = z; o[3] = z;
    aux[i] = Aux{-1.0f, -1.0f, depth, 0.0f};
}

// Half-extents of the support box q <= Q of Sigma', padded so that the FP32
// per-pixel test can never accept a pixel outside it.
__device__ __forceinline__ void support_box(double sxx, double syy, double Q, float* rx, float* ry)
{
    *rx = (float)(sqrt(Q * sxx) * 1.0001 + 1e-3);
    *ry = (float)(sqrt(Q * syy) * 1.0001 + 1e-3);
}

// The same support, as a threshold on q for the binning's ellipse test, with
// the same kind of margin (0.1 % + 1e-3).
__device__ __forceinline__ float support_threshold(double Q) { return (float)(Q * 1.001 + 1e-3); }

__global__ void __launch_bounds__(256) k_project_2d(const ImgDesc* __restrict__ descs_mem, int B, int32_t n_total,
                                                     KParams kp, Rec* __restrict__ recs, Aux* __restrict__ aux, DescArgs da, int nda, ImgDesc* __restrict__ tab)
{
    // a table that came as the argument is read from there, and stored for
    // the kernels after this one
    const ImgDesc* __restrict__ descs = nda ? da.d : descs_mem;
    if (nda && blockIdx.x == 0) {
        const uint32_t words = (uint32_t)nda * (uint32_t)(sizeof(ImgDesc) / 4);
        for (uint32_t k = threadIdx.x; k < words; k += 256u)
            reinterpret_cast<uint32_t*>(tab)[k] = reinterpret_cast<const uint32_t*>(da.d)[k];
    }
    const int32_t i = (int32_t)(blockIdx.x * 256u + threadIdx.x);
    if (i >= n_total) return;
    const ImgDesc& d = descs[image_of_prim(descs, B, i)];
    const int32_t j = i - d.prim_begin;
    const double c0 = d.cov[3 * j], c1 = d.cov[3 * j + 1], c2 = d.cov[3 * j + 2];
    double sxx, sxy, syy;
    if (kp.cov == WIPES_COV_CHOLESKY) {          // L = [[c0, 0], [c1, c2]]
        sxx = c0 * c0;
        sxy = c0 * c1;
        syy = c1 * c1 + c2 * c2;
    } else {                                     // (s1, s2, theta)
        double sn, cs;
        sincos(c2, &sn, &cs);
        const double a = c0 * c0, e = c1 * c1;
        sxx = cs * cs * a + sn * sn * e;
        sxy = cs * sn * (a - e);
        syy = sn * sn * a + cs * cs * e;
    }
    sxx += kp.blur_eps;
    syy += kp.blur_eps;
    const double det = sxx * syy - sxy * sxy;
    if (!(det > 0.0)) {
        store_culled(recs, aux, i, 0.0f);
        return;
    }
    const double inv = 1.0 / det;
    const float2 mu = reinterpret_cast<const float2*>(d.mean)[j];
    const float2 f = reinterpret_cast<const float2*>(d.freq)[j];
    store_record(recs, i, mu.x, mu.y, syy * inv, -sxy * inv, sxx * inv, f.x, f.y, d.opac[j], d.color[3 * j],
                 d.color[3 * j + 1], d.color[3 * j + 2], phase_rev(d.phase, j));
    float rx, ry;
    support_box(sxx, syy, kp.q_add, &rx, &ry);
    aux[i] = Aux{rx, ry, 0.0f, support_threshold(kp.q_add)};
}

// View-dependent colour (Sec. 3.1: 3DGS keeps colour as spherical-harmonic
// coefficients): colour_c = sum_k Y_k(u) sh[k][c] over the real harmonics of
// degree <= deg (Condon-Shortley phase, k = l^2 + l + m) at the unit
// direction u from the camera centre to the mean.  Each Y_k is its
// Cartesian polynomial on the unit sphere, built band by band from the
// products of (x, y, z).
__device__ __forceinline__ void sh_colour(int deg, const float* __restrict__ c, double x, double y, double z,
                                          double out[3])
{
    const double kPi = 3.14159265358979323846;
    double Y[16];
    Y[0] = 0.5 / sqrt(kPi);
    int K = 1;
    if (deg >= 1) {
        const double a = sqrt(3.0 / (4.0 * kPi));
        Y[1] = -a * y;
        Y[2] = a * z;
        Y[3] = -a * x;
        K = 4;
    }
    if (deg >= 2) {
        const double xx = x * x, yy = y * y, zz = z * z;
        const double a = 0.5 * sqrt(15.0 / kPi), b = 0.25 * sqrt(5.0 / kPi), h = 0.25 * sqrt(15.0 / kPi);
        Y[4] = a * x * y;
        Y[5] = -a * y * z;
        Y[6] = b * (2.0 * zz - xx - yy);
        Y[7] = -a * x * z;
        Y[8] = h * (xx - yy);
        K = 9;
    }
    if (deg >= 3) {
        const double xx = x * x, yy = y * y, zz = z * z;
        const double a = 0.25 * sqrt(35.0 / (2.0 * kPi)), b = 0.5 * sqrt(105.0 / kPi);
        const double e = 0.25 * sqrt(21.0 / (2.0 * kPi)), g = 0.25 * sqrt(7.0 / kPi), h = 0.25 * sqrt(105.0 / kPi);
        const double t = 4.0 * zz - xx - yy;
        Y[9] = -a * y * (3.0 * xx - yy);
        Y[10] = b * x * y * z;
        Y[11] = -e * y * t;
        Y[12] = g * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
        Y[13] = -e * x * t;
        Y[14] = h * z * (xx - yy);
        Y[15] = -a * x * (xx - 3.0 * yy);
        K = 16;
    }
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.0;
        for (int k = 0; k < K; ++k) acc += Y[k] * (double)c[3 * k + ch];
        out[ch] = acc;
    }
}

// FP32 depth key: z = fma(V20, m_x, fma(V21, m_y, fma(V22, m_z, V23))), m = fma(v, tau, mu).
__device__ __forceinline__ float depth_key(const float* __restrict__ V, float mx, float my, float mz)
{
    return fmaf(V[8], mx, fmaf(V[9], my, fmaf(V[10], mz, V[11])));
}

__global__ void __launch_bounds__(256) k_project_3d(const ImgDesc* __restrict__ descs_mem, int B, int32_t n_total,
                                                     KParams kp, Rec* __restrict__ recs, Aux* __restrict__ aux, DescArgs da, int nda, ImgDesc* __restrict__ tab)
{
    // a table that came as the argument is read from there, and stored for
    // the kernels after this one
    const ImgDesc* __restrict__ descs = nda ? da.d : descs_mem;
    if (nda && blockIdx.x == 0) {
        const uint32_t words = (uint32_t)nda * (uint32_t)(sizeof(ImgDesc) / 4);
        for (uint32_t k = threadIdx.x; k < words; k += 256u)
            reinterpret_cast<uint32_t*>(tab)[k] = reinterpret_cast<const uint32_t*>(da.d)[k];
    }
    const int32_t i = (int32_t)(blockIdx.x * 256u + threadIdx.x);
    if (i >= n_total) return;
    const ImgDesc& d = descs[image_of_prim(descs, B, i)];
    const int32_t j = i - d.prim_begin;
    float m32[3] = {d.mean[3 * j], d.mean[3 * j + 1], d.mean[3 * j + 2]};
    if (d.vel) {
        for (int k = 0; k < 3; ++k) m32[k] = fmaf(d.vel[3 * j + k], d.time, m32[k]);
    }
    const float zkey = depth_key(d.view, m32[0], m32[1], m32[2]);
    const float op = d.opac[j];
    // camera-space mean in FP64
    double m[3];
    for (int k = 0; k < 3; ++k)
        m[k] = (double)d.mean[3 * j + k] + (d.vel ? (double)d.vel[3 * j + k] * (double)d.time : 0.0);
    double t[3];
    for (int r = 0; r < 3; ++r)
        t[r] = (double)d.view[4 * r] * m[0] + (double)d.view[4 * r + 1] * m[1] + (double)d.view[4 * r + 2] * m[2] +
               (double)d.view[4 * r + 3];
    if (!(zkey > kp.near_plane) || !(op >= kp.alpha_min)) {
        store_culled(recs, aux, i, zkey);
        return;
    }
    const double tz = t[2], iz = 1.0 / tz;
    double u = t[0] * iz, v = t[1] * iz;
    const double lx = d.limx, ly = d.limy;
    u = u < -lx ? -lx : (u > lx ? lx : u);
    v = v < -ly ? -ly : (v > ly ? ly : v);
    const double fxc = d.fx, fyc = d.fy;
    const double J00 = fxc * iz, J02 = -fxc * u * iz, J11 = fyc * iz, J12 = -fyc * v * iz;
    // M = J W (2x3); W rows are view[0..2], view[4..6], view[8..10]
    double M[2][3];
    for (int c = 0; c < 3; ++c) {
        M[0][c] = J00 * d.view[c] + J02 * d.view[8 + c];
        M[1][c] = J11 * d.view[4 + c] + J12 * d.view[8 + c];
    }
    double q0 = d.quat[4 * j], q1 = d.quat[4 * j + 1], q2 = d.quat[4 * j + 2], q3 = d.quat[4 * j + 3];
    const double qq = q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3;
    if (!(qq > 0.0)) {
        store_culled(recs, aux, i, zkey);
        return;
    }
    const double qi = 1.0 / sqrt(qq);
    q0 *= qi; q1 *= qi; q2 *= qi; q3 *= qi;
    const double Rq[3][3] = {
        {1.0 - 2.0 * (q2 * q2 + q3 * q3), 2.0 * (q1 * q2 - q0 * q3), 2.0 * (q1 * q3 + q0 * q2)},
        {2.0 * (q1 * q2 + q0 * q3), 1.0 - 2.0 * (q1 * q1 + q3 * q3), 2.0 * (q2 * q3 - q0 * q1)},
        {2.0 * (q1 * q3 - q0 * q2), 2.0 * (q2 * q3 + q0 * q1), 1.0 - 2.0 * (q1 * q1 + q2 * q2)}};
    const double s[3] = {d.scale[3 * j], d.scale[3 * j + 1], d.scale[3 * j + 2]};
    // T = M Rq diag(s): Sigma' = T T^T + eps I
    double T[2][3];
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k) T[r][k] = (M[r][0] * Rq[0][k] + M[r][1] * Rq[1][k] + M[r][2] * Rq[2][k]) * s[k];
    const double sxx = T[0][0] * T[0][0] + T[0][1] * T[0][1] + T[0][2] * T[0][2] + kp.blur_eps;
    const double sxy = T[0][0] * T[1][0] + T[0][1] * T[1][1] + T[0][2] * T[1][2];
    const double syy = T[1][0] * T[1][0] + T[1][1] * T[1][1] + T[1][2] * T[1][2] + kp.blur_eps;
    const double det = sxx * syy - sxy * sxy;
    if (!(det > 0.0)) {
        store_culled(recs, aux, i, zkey);
        return;
    }
    const double inv = 1.0 / det;
    const double f0 = d.freq[3 * j], f1 = d.freq[3 * j + 1], f2 = d.freq[3 * j + 2];
    float fx, fy;
    if (kp.freq_xform == WIPES_FREQ_VECTOR) {   // f' = M f
        fx = (float)(M[0][0] * f0 + M[0][1] * f1 + M[0][2] * f2);
        fy = (float)(M[1][0] * f0 + M[1][1] * f1 + M[1][2] * f2);
    } else {
        // covector: f' = rows 0-1 of (J3 W)^-T f = J3^-T (W f) (W a rotation),
        // J3 = J with the third row t/|t|; J3^-T g = adj(J3)^T g / det J3
        const double tl = sqrt(t[0] * t[0] + t[1] * t[1] + tz * tz);
        const double J3[3][3] = {{J00, 0.0, J02}, {0.0, J11, J12}, {t[0] / tl, t[1] / tl, tz / tl}};
        double g[3];
        for (int r = 0; r < 3; ++r) g[r] = d.view[4 * r] * f0 + d.view[4 * r + 1] * f1 + d.view[4 * r + 2] * f2;
        // cofactors C[r][c] of J3: (J3^-T g)_r = sum_c C[r][c] g_c / det
        const double C00 = J3[1][1] * J3[2][2] - J3[1][2] * J3[2][1], C01 = J3[1][2] * J3[2][0] - J3[1][0] * J3[2][2];
        const double C02 = J3[1][0] * J3[2][1] - J3[1][1] * J3[2][0];
        const double C10 = J3[0][2] * J3[2][1] - J3[0][1] * J3[2][2], C11 = J3[0][0] * J3[2][2] - J3[0][2] * J3[2][0];
        const double C12 = J3[0][1] * J3[2][0] - J3[0][0] * J3[2][1];
        const double dj = J3[0][0] * C00 + J3[0][1] * C01 + J3[0][2] * C02;
        if (!(dj != 0.0)) {
            store_culled(recs, aux, i, zkey);
            return;
        }
        fx = (float)((C00 * g[0] + C01 * g[1] + C02 * g[2]) / dj);
        fy = (float)((C10 * g[0] + C11 * g[1] + C12 * g[2]) / dj);
    }
    float cr, cg, cb;
    if (kp.sh_degree >= 0) {   // colour from the view direction camera centre -> mean(tau)
        const double dx = m[0] - (double)d.cam_c[0], dy = m[1] - (double)d.cam_c[1], dz = m[2] - (double)d.cam_c[2];
        const double il = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
        const int K = (kp.sh_degree + 1) * (kp.sh_degree + 1);
        double col[3];
        sh_colour(kp.sh_degree, d.sh + (size_t)j * K * 3, dx * il, dy * il, dz * il, col);
        cr = (float)col[0];
        cg = (float)col[1];
        cb = (float)col[2];
    } else {
        cr = d.color[3 * j];
        cg = d.color[3 * j + 1];
        cb = d.color[3 * j + 2];
    }
    const double mx = fxc * t[0] * iz + d.cx, my = fyc * t[1] * iz + d.cy;
    store_record(recs, i, mx, my, syy * inv, -sxy * inv, sxx * inv, fx, fy, op, cr, cg, cb, phase_rev(d.phase, j));
    float rx, ry;
    const double Q = 2.0 * log((double)op / (double)kp.alpha_min);
    support_box(sxx, syy, Q, &rx, &ry);
    aux[i] = Aux{rx, ry, zkey, support_threshold(Q)};
}

}  // namespace wipes

namespace wipes {

hipError_t launch_project(const ImgDesc* descs, int B, int32_t n_total, const KParams& kp, Rec* recs, Aux* aux,
                          hipStream_t s, const DescArgs* da, int nda)
{
    if (n_total <= 0) return hipGetLastError();
    const dim3 grid(((uint32_t)n_total + 255u) / 256u);
    DescArgs a;
    if (da) a = *da;
    else memset(&a, 0, sizeof(a));
    if (!da) nda = 0;
    ImgDesc* tab = const_cast<ImgDesc*>(descs);
    if (kp.mode == WIPES_2D_ADDITIVE)
        hipLaunchKernelGGL(k_project_2d, grid, dim3(256), 0, s, descs, B, n_total, kp, recs, aux, a, nda, tab);
    else
        hipLaunchKernelGGL(k_project_3d, grid, dim3(256), 0, s, descs, B, n_total, kp, recs, aux, a, nda, tab);
    return hipGetLastError();
}

}  // namespace wipes
