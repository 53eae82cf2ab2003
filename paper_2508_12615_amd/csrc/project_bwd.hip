// Projection backward: per primitive, sum the gradient slots of its instances
// -- stored contiguously at [off_id, off_id + count) in the order of its tile
// rectangle, so the sum reads one run of memory and does not depend on launch
// order or on the batch -- and apply the chain rule back to the primitive's
// parameters.
//
// Screen-space gradient -> parameters:
//   conic A = Sigma'^-1:  dL/dSigma' = -A (dL/dA) A, dL/dA = [[da, db/2], [db/2, dc]]
//   2D (Sec. 5.1): Cholesky  dL/dL = 2 G L (lower triangle);
//                  RS        dL/ds_k = 2 s_k (R^T G R)_kk,
//                            dL/dtheta = 2 (s1^2 - s2^2) r0^T G r1  (r_k columns of R)
//   3D (Sec. 3.1 Eq. 2, Sec. 4.1): Sigma' = M Sigma M^T + eps I, f' = M f,
//                  M = J W;  dL/dM = 2 G M Sigma + (dL/df') f^T,
//                  dL/dSigma = M^T G M, dL/df = M^T dL/df', then J(t), mu'(t),
//                  t = W mu + w and Sigma = V V^T with V = R(q) diag(s),
//                  q normalised inside.
//   Covector frequency f' = rows 0-1 of A^-T f, A = J3 W (J3 = J over the
//                  row t/|t|): dL/df = A^-1 g (g = (dL/df', 0)) and
//                  dL/dA = -(A^-T f) (dL/df)^T, whose rows 0-1 join dL/dM and
//                  whose row 2 reaches t through t/|t|.
//   Carrier phase: dL/dphi0 is the slot sum of dL/dphi itself.
//   Spherical-harmonic colour c = sum_k Y_k(u) sh_k, u = d/|d|, d = mu - C:
//                  dL/dsh_k = Y_k dL/dc, dL/dmu += (I - u u^T)/|d| sum_k
//                  grad Y_k (sh_k . dL/dc).
// The arithmetic is FP32: the inputs (screen record, slot sums, parameters)
// are FP32 and the gradients are compared at 1e-3 relative, so FP64 would only
// cost time (the forward projection is FP64 for the mean's sub-pixel phase).
#include <cstring>

#include "common.hpp"

// Multiply-adds within one expression fuse into FMAs here (the rest of the
// library builds with contraction off): the chain rule is FP32 and compared
// at a relative tolerance, so only its rounding changes.
#pragma clang fp contract(on)

namespace wipes {

constexpr int kSlotB = 12;
using real = float;

// Value and gradient in R^3 of a polynomial in (x, y, z), carried through
// products and sums (forward-mode derivatives), so each spherical harmonic's
// gradient comes from the same expression as its value.
struct Poly3 {
    float v, gx, gy, gz;
};
__device__ __forceinline__ Poly3 operator*(Poly3 a, Poly3 b)
{
    return {a.v * b.v, a.gx * b.v + a.v * b.gx, a.gy * b.v + a.v * b.gy, a.gz * b.v + a.v * b.gz};
}
__device__ __forceinline__ Poly3 operator*(float s, Poly3 a) { return {s * a.v, s * a.gx, s * a.gy, s * a.gz}; }
__device__ __forceinline__ Poly3 operator+(Poly3 a, Poly3 b) { return {a.v + b.v, a.gx + b.gx, a.gy + b.gy, a.gz + b.gz}; }
__device__ __forceinline__ Poly3 operator-(Poly3 a, Poly3 b) { return {a.v - b.v, a.gx - b.gx, a.gy - b.gy, a.gz - b.gz}; }

// Real spherical harmonics of degree <= deg (Condon-Shortley phase, index
// l^2 + l + m) at (x, y, z) as polynomials; returns the count (deg + 1)^2.
__device__ __forceinline__ int sh_poly(int deg, float ux, float uy, float uz, Poly3 Y[16])
{
    const float kPi = 3.14159265358979f;
    const Poly3 x{ux, 1.f, 0.f, 0.f}, y{uy, 0.f, 1.f, 0.f}, z{uz, 0.f, 0.f, 1.f};
    Y[0] = {0.5f / sqrtf(kPi), 0.f, 0.f, 0.f};
    if (deg < 1) return 1;
    const float a1 = sqrtf(3.0f / (4.0f * kPi));
    Y[1] = (-a1) * y;
    Y[2] = a1 * z;
    Y[3] = (-a1) * x;
    if (deg < 2) return 4;
    const Poly3 xx = x * x, yy = y * y, zz = z * z;
    const float a2 = 0.5f * sqrtf(15.0f / kPi), b2 = 0.25f * sqrtf(5.0f / kPi), h2 = 0.25f * sqrtf(15.0f / kPi);
    Y[4] = a2 * (x * y);
    Y[5] = (-a2) * (y * z);
    Y[6] = b2 * (2.0f * zz - xx - yy);
    Y[7] = (-a2) * (x * z);
    Y[8] = h2 * (xx - yy);
    if (deg < 3) return 9;
    const float a3 = 0.25f * sqrtf(35.0f / (2.0f * kPi)), b3 = 0.5f * sqrtf(105.0f / kPi);
    const float e3 = 0.25f * sqrtf(21.0f / (2.0f * kPi)), g3 = 0.25f * sqrtf(7.0f / kPi);
    const float h3 = 0.25f * sqrtf(105.0f / kPi);
    const Poly3 t = 4.0f * zz - xx - yy;
    Y[9] = (-a3) * (y * (3.0f * xx - yy));
    Y[10] = b3 * (x * y * z);
    Y[11] = (-e3) * (y * t);
    Y[12] = g3 * (z * (2.0f * zz - 3.0f * xx - 3.0f * yy));
    Y[13] = (-e3) * (x * t);
    Y[14] = h3 * (z * (xx - yy));
    Y[15] = (-a3) * (x * (xx - 3.0f * yy));
    return 16;
}

// Five waves per SIMD (at most 96 registers; left free the compiler takes
// 101 and four fit): the kernel streams slots, parameters and gradients, and
// the fifth wave hides more of that memory latency than the few registers it
// costs (six waves spill and are slower).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) k_project_bwd(const ImgDesc* __restrict__ descs_mem, int B, int32_t n_total,
                                                      KParams kp, const Rec* __restrict__ recs,
                                                      const uint32_t* __restrict__ count,
                                                      const uint32_t* __restrict__ off_id,
                                                      const float* __restrict__ slots,
                                                      const uint32_t* __restrict__ valid,
                                                      const uint32_t* __restrict__ overflow,
                                                      float* __restrict__ dscreen, DescArgs da, int nda)
{
    // a table that came as the argument (the gradient pointers of this call)
    // is read from there, and stored for later calls
    const ImgDesc* __restrict__ descs = nda ? da.d : descs_mem;
    if (nda && blockIdx.x == 0) {
        const uint32_t words = (uint32_t)nda * (uint32_t)(sizeof(ImgDesc) / 4);
        for (uint32_t k = threadIdx.x; k < words; k += 256u)
            reinterpret_cast<uint32_t*>(const_cast<ImgDesc*>(descs_mem))[k] = reinterpret_cast<const uint32_t*>(da.d)[k];
    }
    // slots per lane staged per chunk: a chunk of 128 slots lets a lane add
    // more of its primitive's slots per pass (the wave pays, per chunk, for
    // the lane with the most slots in it)
    constexpr int SPL = 2;
    constexpr uint32_t CH = (uint32_t)kWave * SPL;
    __shared__ float4 s_slot[4][CH][3];
    const int wv = (int)(threadIdx.x >> 6), l = lane_id();
    const int32_t i0 = (int32_t)(blockIdx.x * 256u + (uint32_t)wv * kWave);
    if (i0 >= n_total || *overflow) return;   // wave-uniform
    const int32_t i = i0 + l;
    const bool inr = i < n_total;
    // The slots of the wave's 64 primitives form one contiguous run (they are
    // numbered in primitive order).  The wave streams the run through LDS CH
    // slots at a time with coalesced loads, and each lane adds up its own
    // primitive's slots in ascending order (the same order at any batch size).
    // The next chunk is loaded while the current one is added; the slots'
    // written-bits come from a window of 64 words (2048 slots) that lane j
    // holds word wbase + j of, refilled when a chunk runs past it.
    const uint32_t c = inr ? count[i] : 0u;
    const uint32_t base = inr ? off_id[i] : 0u;
    const uint32_t first = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);   // lane 0 is in range
    const uint32_t total = wave_sum_u32(c);
    const uint32_t my0 = base - first, my1 = my0 + c;
    float acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = 0.0f;
    const uint32_t wlast = total ? (first + total - 1u) >> 5 : 0u;
    uint32_t wbase = first >> 5;
    uint32_t vword = (total && wbase + (uint32_t)l <= wlast) ? valid[wbase + (uint32_t)l] : 0u;
    // a slot the backward did not write (no pixel of its tile reached it) is
    // zero: it is neither loaded nor added (vm: the written slots of the chunk)
    auto fetch = [&](uint32_t k0, float4 (&sl)[SPL][3], uint64_t (&vm)[SPL]) {
        const uint32_t lastw = (first + min(k0 + CH, total) - 1u) >> 5;
        if (lastw - wbase >= (uint32_t)kWave) {   // uniform: the window moves on
            wbase = (first + k0) >> 5;
            vword = wbase + (uint32_t)l <= wlast ? valid[wbase + (uint32_t)l] : 0u;
        }
#pragma unroll
        for (int q = 0; q < SPL; ++q) {
            const uint32_t kk = k0 + (uint32_t)(q * kWave + l), e = first + kk;
            const uint32_t word = (uint32_t)__shfl((int)vword, (int)(((e >> 5) - wbase) & 63u), kWave);
            sl[q][0] = sl[q][1] = sl[q][2] = make_float4(0.f, 0.f, 0.f, 0.f);
            const bool w = kk < total && ((word >> (e & 31u)) & 1u);
            vm[q] = __ballot(w);
            if (w) {
                const float4* src = reinterpret_cast<const float4*>(slots + (size_t)e * kSlotB);
                sl[q][0] = src[0];
                sl[q][1] = src[1];
                sl[q][2] = src[2];
            }
        }
    };
    float4 cur[SPL][3];
    uint64_t cm[SPL] = {};
    if (total) fetch(0, cur, cm);
    for (uint32_t k0 = 0; k0 < total; k0 += CH) {
        float4 b[SPL][3];
        uint64_t bm[SPL] = {};
        if (k0 + CH < total) fetch(k0 + CH, b, bm);
#pragma unroll
        for (int q = 0; q < SPL; ++q) {
            if (k0 + (uint32_t)(q * kWave + l) < total) {
                s_slot[wv][q * kWave + l][0] = cur[q][0];
                s_slot[wv][q * kWave + l][1] = cur[q][1];
                s_slot[wv][q * kWave + l][2] = cur[q][2];
            }
        }
        wave_lds_sync();
        // this lane's written slots of the chunk, in ascending order
        const uint32_t lo = max(my0, k0), hi = min(my1, k0 + CH);
        const uint32_t r0 = lo < hi ? lo - k0 : 0u, r1 = lo < hi ? hi - k0 : 0u;   // chunk-relative [r0, r1)
#pragma unroll
        for (int q = 0; q < SPL; ++q) {
            const uint32_t a = max(r0, (uint32_t)(q * kWave)), z = min(r1, (uint32_t)(q * kWave + kWave));
            uint64_t m = 0ull;
            if (a < z) {
                const uint32_t a1 = a - (uint32_t)(q * kWave), z1 = z - (uint32_t)(q * kWave);
                const uint64_t upto = z1 >= 64u ? ~0ull : ((1ull << z1) - 1ull);
                m = cm[q] & upto & ~((1ull << a1) - 1ull);
            }
            while (m) {
                const uint32_t t = (uint32_t)__builtin_ctzll(m) + (uint32_t)(q * kWave);
                m &= m - 1ull;
                const float4 x0 = s_slot[wv][t][0], x1 = s_slot[wv][t][1], x2 = s_slot[wv][t][2];
                acc[0] += x0.x; acc[1] += x0.y; acc[2] += x0.z; acc[3] += x0.w;
                acc[4] += x1.x; acc[5] += x1.y; acc[6] += x1.z; acc[7] += x1.w;
                acc[8] += x2.x; acc[9] += x2.y; acc[10] += x2.z; acc[11] += x2.w;
            }
        }
        wave_lds_sync();   // the stage is rewritten next
#pragma unroll
        for (int q = 0; q < SPL; ++q) {
            cur[q][0] = b[q][0];
            cur[q][1] = b[q][1];
            cur[q][2] = b[q][2];
            cm[q] = bm[q];
        }
    }
    if (!inr) return;
    // The slots hold sums of (dq dx, dq dy, dq dx^2, dq dx dy, dq dy^2,
    // dphi dx, dphi dy, opacity, colour, dphi) over the primitive's pixels,
    // the dq terms without their factor -o/2 and the dphi terms without -o
    // (the blend builds them from half the Gaussian factor), applied here:
    // with its conic and f' they give d/d(mu', conic, f') (q = ca dx^2 +
    // 2 cb dx dy + cc dy^2 and phi = f' . (x - mu')).  A primitive with no
    // instance keeps all-zero sums (its record need not be finite).
    if (c) {
        const Rec& R0 = recs[i];
        const float hop = -0.5f * R0.op, mop = -R0.op;
#pragma unroll
        for (int k = 0; k < 5; ++k) acc[k] *= hop;
        acc[5] *= mop;
        acc[6] *= mop;
        acc[11] *= mop;
        const float sqx = acc[0], sqy = acc[1], sph = acc[11];
        acc[0] = -2.0f * (R0.ca * sqx + R0.cb * sqy) - R0.fx * sph;
        acc[1] = -2.0f * (R0.cb * sqx + R0.cc * sqy) - R0.fy * sph;
        acc[3] = 2.0f * acc[3];
    }
    const ImgDesc& d = descs[image_of_prim(descs, B, i)];
    const int32_t j = i - d.prim_begin;
    if (dscreen) {
#pragma unroll
        for (int k = 0; k < 12; ++k) dscreen[(size_t)i * 12 + k] = acc[k];
    }
    const int D = kp.mode == WIPES_2D_ADDITIVE ? 2 : 3;
    const bool sh = kp.sh_degree >= 0;
    if (d.g_color && !sh)
        for (int k = 0; k < 3; ++k) d.g_color[3 * j + k] = acc[8 + k];
    if (d.g_opac) d.g_opac[j] = acc[7];
    if (d.g_phase) d.g_phase[j] = acc[11];
    if (c == 0) {
        if (d.g_sh) {
            const int K3 = 3 * (kp.sh_degree + 1) * (kp.sh_degree + 1);
            for (int k = 0; k < K3; ++k) d.g_sh[(size_t)K3 * j + k] = 0.0f;
        }
        // culled or off-screen: zero gradients
        if (d.g_mean) for (int k = 0; k < D; ++k) d.g_mean[D * j + k] = 0.0f;
        if (d.g_freq) for (int k = 0; k < D; ++k) d.g_freq[D * j + k] = 0.0f;
        if (d.g_cov) for (int k = 0; k < 3; ++k) d.g_cov[3 * j + k] = 0.0f;
        if (d.g_quat) for (int k = 0; k < 4; ++k) d.g_quat[4 * j + k] = 0.0f;
        if (d.g_scale) for (int k = 0; k < 3; ++k) d.g_scale[3 * j + k] = 0.0f;
        if (d.g_vel) for (int k = 0; k < 3; ++k) d.g_vel[3 * j + k] = 0.0f;
        return;
    }
    // dL/dSigma' = -A GA A
    const Rec& R = recs[i];
    const real a = R.ca, b = R.cb, cc = R.cc;
    const real ga = acc[2], gb = 0.5f * (real)acc[3], gc = acc[4];
    const real P00 = a * ga + b * gb, P01 = a * gb + b * gc, P10 = b * ga + cc * gb, P11 = b * gb + cc * gc;
    const real G00 = -(P00 * a + P01 * b), G01 = -(P00 * b + P01 * cc), G11 = -(P10 * b + P11 * cc);

    if (kp.mode == WIPES_2D_ADDITIVE) {
        if (d.g_mean) { d.g_mean[2 * j] = acc[0]; d.g_mean[2 * j + 1] = acc[1]; }
        if (d.g_freq) { d.g_freq[2 * j] = acc[5]; d.g_freq[2 * j + 1] = acc[6]; }
        if (!d.g_cov) return;
        const real c0 = d.cov[3 * j], c1 = d.cov[3 * j + 1], c2 = d.cov[3 * j + 2];
        if (kp.cov == WIPES_COV_CHOLESKY) {
            d.g_cov[3 * j] = (float)(2.0f * (G00 * c0 + G01 * c1));
            d.g_cov[3 * j + 1] = (float)(2.0f * (G01 * c0 + G11 * c1));
            d.g_cov[3 * j + 2] = (float)(2.0f * G11 * c2);
        } else {
            real sn, cs;
            sincosf(c2, &sn, &cs);
            // r0 = (cs, sn), r1 = (-sn, cs)
            const real q00 = cs * (G00 * cs + G01 * sn) + sn * (G01 * cs + G11 * sn);
            const real q11 = -sn * (-G00 * sn + G01 * cs) + cs * (-G01 * sn + G11 * cs);
            const real q01 = cs * (-G00 * sn + G01 * cs) + sn * (-G01 * sn + G11 * cs);
            d.g_cov[3 * j] = (float)(2.0f * c0 * q00);
            d.g_cov[3 * j + 1] = (float)(2.0f * c1 * q11);
            d.g_cov[3 * j + 2] = (float)(2.0f * (c0 * c0 - c1 * c1) * q01);
        }
        return;
    }

    // ---- 3D: recompute the forward quantities
    real m[3];
    for (int k = 0; k < 3; ++k)
        m[k] = (real)d.mean[3 * j + k] + (d.vel ? (real)d.vel[3 * j + k] * (real)d.time : 0.0f);
    real t[3];
    for (int r = 0; r < 3; ++r)
        t[r] = (real)d.view[4 * r] * m[0] + (real)d.view[4 * r + 1] * m[1] + (real)d.view[4 * r + 2] * m[2] +
               (real)d.view[4 * r + 3];
    const real tz = t[2], iz = 1.0f / tz;
    const real ur = t[0] * iz, vr = t[1] * iz;
    const real lx = d.limx, ly = d.limy;
    const bool clx = ur < -lx || ur > lx, cly = vr < -ly || vr > ly;
    const real u = clx ? (ur < 0 ? -lx : lx) : ur;
    const real v = cly ? (vr < 0 ? -ly : ly) : vr;
    const real fxc = d.fx, fyc = d.fy;
    const real J00 = fxc * iz, J02 = -fxc * u * iz, J11 = fyc * iz, J12 = -fyc * v * iz;
    real Rw[3][3];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) Rw[r][k] = d.view[4 * r + k];
    real M[2][3];
    for (int k = 0; k < 3; ++k) {
        M[0][k] = J00 * Rw[0][k] + J02 * Rw[2][k];
        M[1][k] = J11 * Rw[1][k] + J12 * Rw[2][k];
    }
    const real q0r = d.quat[4 * j], q1r = d.quat[4 * j + 1], q2r = d.quat[4 * j + 2], q3r = d.quat[4 * j + 3];
    // one reciprocal of |q| serves the normalisation and its derivative (a
    // division costs about ten instructions, a multiply one)
    const real iqn = 1.0f / sqrtf(q0r * q0r + q1r * q1r + q2r * q2r + q3r * q3r);
    const real w = q0r * iqn, x = q1r * iqn, y = q2r * iqn, z = q3r * iqn;
    const real Rq[3][3] = {{1.0f - 2.0f * (y * y + z * z), 2.0f * (x * y - w * z), 2.0f * (x * z + w * y)},
                             {2.0f * (x * y + w * z), 1.0f - 2.0f * (x * x + z * z), 2.0f * (y * z - w * x)},
                             {2.0f * (x * z - w * y), 2.0f * (y * z + w * x), 1.0f - 2.0f * (x * x + y * y)}};
    const real s[3] = {d.scale[3 * j], d.scale[3 * j + 1], d.scale[3 * j + 2]};
    real V[3][3];   // Rq diag(s)
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) V[r][k] = Rq[r][k] * s[k];
    real T[2][3];   // M V
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k) T[r][k] = M[r][0] * V[0][k] + M[r][1] * V[1][k] + M[r][2] * V[2][k];
    const real f3[3] = {d.freq[3 * j], d.freq[3 * j + 1], d.freq[3 * j + 2]};
    const real dfp[2] = {acc[5], acc[6]};
    const real G[2][2] = {{G00, G01}, {G01, G11}};
    // dM = 2 G (M Sigma) + dfp f^T,  M Sigma = T V^T
    real MS[2][3];
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k) MS[r][k] = T[r][0] * V[k][0] + T[r][1] * V[k][1] + T[r][2] * V[k][2];
    real dM[2][3];
    const bool cov_f = kp.freq_xform == WIPES_FREQ_COVECTOR;
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k)
            dM[r][k] = 2.0f * (G[r][0] * MS[0][k] + G[r][1] * MS[1][k]) + (cov_f ? 0.0f : dfp[r] * f3[k]);
    // covector frequency: A = J3 W, f'3 = A^-T f, dL/df = A^-1 (dfp, 0),
    // dL/dA = -f'3 (dL/df)^T (rows 0-1 into dM; row 2 through t/|t| below)
    real dfw[3] = {0.0f, 0.0f, 0.0f}, dA2[3] = {0.0f, 0.0f, 0.0f};
    const real tl = cov_f ? sqrtf(t[0] * t[0] + t[1] * t[1] + tz * tz) : 1.0f;   // |t|, covector path only
    if (cov_f) {
        real A[3][3];
        for (int k = 0; k < 3; ++k) {
            A[0][k] = M[0][k];
            A[1][k] = M[1][k];
            A[2][k] = (t[0] * Rw[0][k] + t[1] * Rw[1][k] + tz * Rw[2][k]) / tl;
        }
        // inverse by cofactors: Ai[r][c] = Cof[c][r] / det
        real Cf[3][3];
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < 3; ++k) {
                const int r1 = (r + 1) % 3, r2 = (r + 2) % 3, k1 = (k + 1) % 3, k2 = (k + 2) % 3;
                Cf[r][k] = A[r1][k1] * A[r2][k2] - A[r1][k2] * A[r2][k1];
            }
        const real det = A[0][0] * Cf[0][0] + A[0][1] * Cf[0][1] + A[0][2] * Cf[0][2];
        const real id = 1.0f / det;
        real f3p[3];
        for (int r = 0; r < 3; ++r)   // (A^-T f)_r = sum_c Ai[c][r] f_c = sum_c Cf[r][c] f_c / det
            f3p[r] = (Cf[r][0] * f3[0] + Cf[r][1] * f3[1] + Cf[r][2] * f3[2]) * id;
        for (int k = 0; k < 3; ++k)   // (A^-1 g)_k = sum_r Cf[r][k] g_r / det
            dfw[k] = (Cf[0][k] * dfp[0] + Cf[1][k] * dfp[1]) * id;
        for (int k = 0; k < 3; ++k) {
            dM[0][k] -= f3p[0] * dfw[k];
            dM[1][k] -= f3p[1] * dfw[k];
            dA2[k] = -f3p[2] * dfw[k];
        }
    }
    // dSigma = M^T G M
    real GM[2][3];
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k) GM[r][k] = G[r][0] * M[0][k] + G[r][1] * M[1][k];
    real dS[3][3];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) dS[r][k] = M[0][r] * GM[0][k] + M[1][r] * GM[1][k];
    // Sigma = V V^T: dV = 2 dS V
    real dV[3][3];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) dV[r][k] = 2.0f * (dS[r][0] * V[0][k] + dS[r][1] * V[1][k] + dS[r][2] * V[2][k]);
    if (d.g_scale)
        for (int k = 0; k < 3; ++k)
            d.g_scale[3 * j + k] = (float)(dV[0][k] * Rq[0][k] + dV[1][k] * Rq[1][k] + dV[2][k] * Rq[2][k]);
    if (d.g_quat) {
        real dR[3][3];
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < 3; ++k) dR[r][k] = dV[r][k] * s[k];
        const real dw = 2.0f * (-z * dR[0][1] + y * dR[0][2] + z * dR[1][0] - x * dR[1][2] - y * dR[2][0] +
                                 x * dR[2][1]);
        const real dx = 2.0f * (y * dR[0][1] + z * dR[0][2] + y * dR[1][0] - 2.0f * x * dR[1][1] - w * dR[1][2] +
                                 z * dR[2][0] + w * dR[2][1] - 2.0f * x * dR[2][2]);
        const real dy = 2.0f * (-2.0f * y * dR[0][0] + x * dR[0][1] + w * dR[0][2] + x * dR[1][0] + z * dR[1][2] -
                                 w * dR[2][0] + z * dR[2][1] - 2.0f * y * dR[2][2]);
        const real dz = 2.0f * (-2.0f * z * dR[0][0] - w * dR[0][1] + x * dR[0][2] + w * dR[1][0] -
                                 2.0f * z * dR[1][1] + y * dR[1][2] + x * dR[2][0] + y * dR[2][1]);
        const real dot = w * dw + x * dx + y * dy + z * dz;
        d.g_quat[4 * j] = (float)((dw - w * dot) * iqn);
        d.g_quat[4 * j + 1] = (float)((dx - x * dot) * iqn);
        d.g_quat[4 * j + 2] = (float)((dy - y * dot) * iqn);
        d.g_quat[4 * j + 3] = (float)((dz - z * dot) * iqn);
    }
    if (d.g_freq)
        for (int k = 0; k < 3; ++k) d.g_freq[3 * j + k] = cov_f ? dfw[k] : (float)(M[0][k] * dfp[0] + M[1][k] * dfp[1]);
    // dJ = dM W^T
    real dJ[2][3];
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k) dJ[r][k] = dM[r][0] * Rw[k][0] + dM[r][1] * Rw[k][1] + dM[r][2] * Rw[k][2];
    real dt[3] = {0.0f, 0.0f, 0.0f};
    const real iz2 = iz * iz;
    dt[2] += -fxc * iz2 * dJ[0][0] - fyc * iz2 * dJ[1][1];
    if (!clx) {
        dt[0] += -fxc * iz2 * dJ[0][2];
        dt[2] += 2.0f * fxc * t[0] * iz2 * iz * dJ[0][2];
    } else {
        dt[2] += fxc * u * iz2 * dJ[0][2];
    }
    if (!cly) {
        dt[1] += -fyc * iz2 * dJ[1][2];
        dt[2] += 2.0f * fyc * t[1] * iz2 * iz * dJ[1][2];
    } else {
        dt[2] += fyc * v * iz2 * dJ[1][2];
    }
    if (cov_f) {   // row 2 of A is (t/|t|)^T W: dL/dt += (I - th th^T)/|t| (W dA2)
        real gth[3], th[3];
        for (int r = 0; r < 3; ++r) {
            gth[r] = Rw[r][0] * dA2[0] + Rw[r][1] * dA2[1] + Rw[r][2] * dA2[2];
            th[r] = (r == 0 ? t[0] : r == 1 ? t[1] : tz) / tl;
        }
        const real dot = th[0] * gth[0] + th[1] * gth[1] + th[2] * gth[2];
        for (int r = 0; r < 3; ++r) dt[r] += (gth[r] - th[r] * dot) / tl;
    }
    dt[0] += fxc * iz * acc[0];
    dt[1] += fyc * iz * acc[1];
    dt[2] += -fxc * t[0] * iz2 * acc[0] - fyc * t[1] * iz2 * acc[1];
    real dm[3];
    for (int k = 0; k < 3; ++k) dm[k] = Rw[0][k] * dt[0] + Rw[1][k] * dt[1] + Rw[2][k] * dt[2];
    if (sh) {   // colour from the view direction u = (mu - C)/|mu - C|
        const real dx = m[0] - d.cam_c[0], dy = m[1] - d.cam_c[1], dz = m[2] - d.cam_c[2];
        const real dl = sqrtf(dx * dx + dy * dy + dz * dz), il = 1.0f / dl;
        const real ux = dx * il, uy = dy * il, uz = dz * il;
        Poly3 Y[16];
        const int K = sh_poly(kp.sh_degree, ux, uy, uz, Y);
        const float* shc = d.sh + (size_t)j * K * 3;
        const real gr = acc[8], gg = acc[9], gb = acc[10];
        real du[3] = {0.0f, 0.0f, 0.0f};
        for (int k = 0; k < K; ++k) {
            const real w = shc[3 * k] * gr + shc[3 * k + 1] * gg + shc[3 * k + 2] * gb;
            du[0] += Y[k].gx * w;
            du[1] += Y[k].gy * w;
            du[2] += Y[k].gz * w;
            if (d.g_sh) {
                float* o = d.g_sh + ((size_t)j * K + k) * 3;
                o[0] = Y[k].v * gr;
                o[1] = Y[k].v * gg;
                o[2] = Y[k].v * gb;
            }
        }
        const real dot = ux * du[0] + uy * du[1] + uz * du[2];
        dm[0] += (du[0] - ux * dot) * il;
        dm[1] += (du[1] - uy * dot) * il;
        dm[2] += (du[2] - uz * dot) * il;
    }
    if (d.g_mean)
        for (int k = 0; k < 3; ++k) d.g_mean[3 * j + k] = (float)dm[k];
    if (d.g_vel)
        for (int k = 0; k < 3; ++k) d.g_vel[3 * j + k] = d.vel ? (float)(dm[k] * (real)d.time) : 0.0f;
}

hipError_t launch_project_bwd(const ImgDesc* descs, int B, int32_t n_total, const KParams& kp, const Rec* recs,
                              const uint32_t* count, const uint32_t* off_id, const float* slots,
                              const uint32_t* valid, const uint32_t* overflow, float* dscreen, hipStream_t s,
                              const DescArgs* da, int nda)
{
    DescArgs a;
    if (da) a = *da;
    else memset(&a, 0, sizeof(a));
    if (!da) nda = 0;
    if (n_total > 0)
        hipLaunchKernelGGL(k_project_bwd, dim3(((uint32_t)n_total + 255u) / 256u), dim3(256), 0, s, descs, B, n_total,
                           kp, recs, count, off_id, slots, valid, overflow, dscreen, a, nda);
    return hipGetLastError();
}

}  // namespace wipes
