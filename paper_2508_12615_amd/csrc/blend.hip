// Per-tile blending of wavelet primitives, forward and backward, for gfx950.
//
// Work decomposition (CDNA4-first, no workgroup barriers):
//  * one 64-lane wave owns one TW x TH tile; the tile is split into 8 x 8
//    sub-blocks and lane l owns pixel (l & 7, l >> 3) of every sub-block, so
//    a lane carries TW*TH/64 pixels;
//  * the wave walks the tile's sorted primitive list with wave-uniform
//    indices, so the list entries and the 64-byte records arrive through the
//    scalar data cache straight into SGPRs -- no record is staged in LDS (a
//    small per-wave LDS buffer only repacks live pixels, see "pixel rows");
//  * before touching pixels the wave intersects the primitive's pixel box with
//    each sub-block (scalar integer compares) and skips sub-blocks it misses;
//  * alpha mode keeps a uniform mask of sub-blocks that still have live
//    pixels (ballots) and leaves the list when none is left;
//  * coordinates are made tile-relative once per primitive with the record's
//    (hi, lo) mean, so d = p - mu' costs one subtraction per pixel and stays
//    exact to FP32 rounding of d itself;
//  * the backward reduces the eleven per-pair gradients of a primitive over
//    the wave with a halving butterfly (each step exchanges half the values),
//    and writes them, without atomics, to the instance's slot -- slots are
//    numbered in primitive order (the sort carries each instance's slot index),
//    so the projection backward sums a primitive's slots from one contiguous
//    run in a fixed order: gradients are deterministic and independent of the
//    batch a primitive is rendered in.
//
// Per-pair rule (shared by forward and backward through eval_pair so their
// FP32 decisions agree bit for bit):
//   e2 = -q/2 log2(e) from the pre-scaled conic, E = exp2(e2),
//   phase in revolutions ph = (f'/2pi).d, K = (1 + cos 2pi ph)/2, W' = K E.
// Paper: W' of Eq. 7 (Sec. 4.1), blended by Eq. 4 (additive) or Eq. 3 (alpha).
#include "common.hpp"

namespace wipes {

constexpr int kWpb = 4;   // waves (tiles) per workgroup

struct PrimU {            // per-primitive, wave-uniform values
    float mrx, mry;       // mean relative to the tile origin
    float ca2, cb2, cc2;  // conic scaled by -log2(e)/2 (cb2 includes the factor 2)
    float fxr, fyr;       // frequency in revolutions per pixel
    float op, r, g, b;
    float ca, cb, cc, fx, fy;   // raw values for the backward
};

__device__ __forceinline__ PrimU load_prim(const Rec* __restrict__ recs, uint32_t prim, int ox, int oy,
                                           uint32_t* box0, uint32_t* box1)
{
    const Rec R = recs[prim];
    PrimU u;
    u.mrx = (R.mx - (float)ox) + R.mxl;
    u.mry = (R.my - (float)oy) + R.myl;
    const float k = -0.5f * kLog2e;
    u.ca2 = R.ca * k;
    u.cb2 = R.cb * (2.0f * k);
    u.cc2 = R.cc * k;
    u.fxr = R.fx * kInv2Pi;
    u.fyr = R.fy * kInv2Pi;
    u.op = R.op;
    u.r = R.r; u.g = R.g; u.b = R.b;
    u.ca = R.ca; u.cb = R.cb; u.cc = R.cc; u.fx = R.fx; u.fy = R.fy;
    *box0 = R.box0;
    *box1 = R.box1;
    return u;
}

struct PairEval {
    float dx, dy, e2, E, ph, K, W;
};

__device__ __forceinline__ PairEval eval_pair(const PrimU& u, float lx, float ly)
{
    PairEval p;
    p.dx = lx - u.mrx;
    p.dy = ly - u.mry;
    const float t = fmaf(u.ca2, p.dx, u.cb2 * p.dy);
    p.e2 = fmaf(t, p.dx, (u.cc2 * p.dy) * p.dy);
    p.ph = fmaf(u.fxr, p.dx, u.fyr * p.dy);
    p.E = __builtin_amdgcn_exp2f(p.e2);
    p.K = fmaf(0.5f, __builtin_amdgcn_cosf(__builtin_amdgcn_fractf(p.ph)), 0.5f);
    p.W = p.K * p.E;
    return p;
}

// Sub-blocks (8 x 8) of a TW x TH tile hit by the pixel box, as a bit mask.
template <int TW, int TH>
__device__ __forceinline__ uint32_t subblock_mask(uint32_t box0, uint32_t box1, int ox, int oy)
{
    constexpr int SBX = TW / 8, NSB = (TW / 8) * (TH / 8);
    const int x0 = lo16(box0) - ox, y0 = hi16(box0) - oy, x1 = lo16(box1) - ox, y1 = hi16(box1) - oy;
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < NSB; ++k) {
        const int sx = (k % SBX) * 8, sy = (k / SBX) * 8;
        const bool hit = x0 <= sx + 7 && x1 >= sx && y0 <= sy + 7 && y1 >= sy;
        m |= hit ? (1u << k) : 0u;
    }
    return m;
}

// Map a wave to its tile.  Grid mode remaps workgroups so that each of the 8
// XCDs (which receive workgroups round-robin) walks a contiguous band of
// tiles and its L2 sees the primitives of neighbouring tiles.
__device__ __forceinline__ uint32_t grid_tile_of_wave()
{
    const uint32_t nb = gridDim.x, b = blockIdx.x;
    const uint32_t xcd = b & 7u, idx = b >> 3, per = nb >> 3, rem = nb & 7u;
    const uint32_t nbk = xcd * per + min(xcd, rem) + idx;
    // wave-uniform by construction; readfirstlane tells the compiler so, which
    // turns every list and record fetch derived from it into a scalar load
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)(nbk * kWpb + (threadIdx.x >> 6)));
}

struct TileGeo {
    int b;             // image
    int ox, oy;        // tile origin (pixels)
    uint32_t start, end;
};

__device__ __forceinline__ TileGeo tile_geo(const ImgDesc* __restrict__ descs, int B, const uint2* __restrict__ ranges,
                                            uint32_t t, int TW, int TH)
{
    TileGeo g;
    g.b = image_of_tile(descs, B, (int32_t)t);
    const ImgDesc& d = descs[g.b];
    const int lt = (int)t - d.tile_begin;
    const int ty = lt / d.tiles_x, tx = lt - ty * d.tiles_x;
    g.ox = tx * TW;
    g.oy = ty * TH;
    const uint2 r = ranges[t];
    g.start = r.x;
    g.end = r.y;
    return g;
}

// ------------------------------------------------------------ pixel rows
//
// Alpha mode keeps the tile's live pixels in "rows": row r, lane l holds one
// pixel (packed local coordinates x | y << 8) or nothing (-1).  A row is only
// evaluated against a primitive whose pixel box meets the row's bounding box
// (wave-uniform, recomputed whenever rows are rebuilt).  Rows are rebuilt
// through a per-wave LDS buffer of one word per tile pixel.

__device__ __forceinline__ int32_t wave_min_i32(int32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
    return v;
}

struct RowBox {
    int x0, y0, x1, y1;
};

// Bounding box of the occupied slots of one row (uniform); empty rows get an
// inverted box that no primitive meets.
__device__ __forceinline__ RowBox row_box(int32_t pk)
{
    const bool on = pk >= 0;
    const int x = pk & 255, y = pk >> 8;
    RowBox b;
    b.x0 = __builtin_amdgcn_readfirstlane(wave_min_i32(on ? x : 1 << 20));
    b.y0 = __builtin_amdgcn_readfirstlane(wave_min_i32(on ? y : 1 << 20));
    b.x1 = __builtin_amdgcn_readfirstlane(wave_max_i32(on ? x : -(1 << 20)));
    b.y1 = __builtin_amdgcn_readfirstlane(wave_max_i32(on ? y : -(1 << 20)));
    return b;
}

__device__ __forceinline__ bool box_meets(const RowBox& r, int x0, int y0, int x1, int y1)
{
    return x0 <= r.x1 && x1 >= r.x0 && y0 <= r.y1 && y1 >= r.y0;
}

// Move one per-slot value of the occupied slots (dst index idx[r]) to the
// compacted layout: slot j = r * 64 + l of the first `rows_out` rows receives
// the value with idx == j (j < count), or `fill`.
template <int NR>
__device__ __forceinline__ void route(uint32_t* lds, const bool on[NR], const uint32_t idx[NR], uint32_t v[NR],
                                      int rows_in, int rows_out, uint32_t count, uint32_t fill)
{
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if (r < rows_in && on[r]) lds[idx[r]] = v[r];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint32_t l = (uint32_t)lane_id();
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const uint32_t j = (uint32_t)r * kWave + l;
        v[r] = (r < rows_out && j < count) ? lds[j] : fill;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------ forward

template <int MODE, int TW, int TH>
__device__ __forceinline__ void fwd_tile(const ImgDesc* __restrict__ descs, int B, const KParams& kp,
                                         const Rec* __restrict__ recs, const uint32_t* __restrict__ vals,
                                         const uint2* __restrict__ ranges, uint32_t t, float* __restrict__ image,
                                         float* __restrict__ T_final, int32_t* __restrict__ last)
{
    constexpr int SBX = TW / 8, NSB = (TW / 8) * (TH / 8);
    const TileGeo G = tile_geo(descs, B, ranges, t, TW, TH);
    const ImgDesc& d = descs[G.b];
    const int l = lane_id();
    float lx[NSB], ly[NSB];
    bool valid[NSB];
    float C[NSB][3], T[NSB];
    int32_t lst[NSB];
    bool alive[NSB];
#pragma unroll
    for (int k = 0; k < NSB; ++k) {
        const int px = (k % SBX) * 8 + (l & 7), py = (k / SBX) * 8 + (l >> 3);
        lx[k] = (float)px + 0.5f;
        ly[k] = (float)py + 0.5f;
        valid[k] = (G.ox + px) < d.W && (G.oy + py) < d.H;
        C[k][0] = C[k][1] = C[k][2] = 0.0f;
        T[k] = 1.0f;
        lst[k] = -1;
        alive[k] = valid[k];
    }
    uint32_t live = 0;
#pragma unroll
    for (int k = 0; k < NSB; ++k) live |= __ballot(alive[k]) ? (1u << k) : 0u;
    const float thr2 = kp.q_add * (-0.5f * kLog2e);

    for (uint32_t s = G.start; s < G.end; ++s) {
        if (MODE == WIPES_3D_ALPHA && live == 0u) break;
        const uint32_t prim = vals[s];
        uint32_t b0, b1;
        const PrimU u = load_prim(recs, prim, G.ox, G.oy, &b0, &b1);
        uint32_t m = subblock_mask<TW, TH>(b0, b1, G.ox, G.oy);
        if (MODE == WIPES_3D_ALPHA) m &= live;
        if (m == 0u) continue;
        if (MODE == WIPES_2D_ADDITIVE) {
            const float cr = u.r * u.op, cg = u.g * u.op, cb = u.b * u.op;
#pragma unroll
            for (int k = 0; k < NSB; ++k) {
                if (!(m & (1u << k))) continue;
                const PairEval p = eval_pair(u, lx[k], ly[k]);
                const float w = p.e2 >= thr2 ? p.W : 0.0f;
                C[k][0] = fmaf(cr, w, C[k][0]);
                C[k][1] = fmaf(cg, w, C[k][1]);
                C[k][2] = fmaf(cb, w, C[k][2]);
            }
        } else {
            bool changed = false;
#pragma unroll
            for (int k = 0; k < NSB; ++k) {
                if (!(m & (1u << k))) continue;
                const PairEval p = eval_pair(u, lx[k], ly[k]);
                const float a = u.op * p.W;
                if (alive[k] && a >= kp.alpha_min) {
                    const float al = fminf(a, kp.alpha_max);
                    const float wt = T[k] * al;
                    C[k][0] = fmaf(wt, u.r, C[k][0]);
                    C[k][1] = fmaf(wt, u.g, C[k][1]);
                    C[k][2] = fmaf(wt, u.b, C[k][2]);
                    T[k] = T[k] * (1.0f - al);
                    lst[k] = (int32_t)s;
                    if (T[k] < kp.T_min) {
                        alive[k] = false;
                        changed = true;
                    }
                }
            }
            if (__ballot(changed)) {
                live = 0;
#pragma unroll
                for (int k = 0; k < NSB; ++k) live |= __ballot(alive[k]) ? (1u << k) : 0u;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NSB; ++k) {
        if (!valid[k]) continue;
        const int px = G.ox + (k % SBX) * 8 + (l & 7), py = G.oy + (k / SBX) * 8 + (l >> 3);
        const uint32_t pix = (uint32_t)d.pix_begin + (uint32_t)(py * d.W + px);
        float c0 = C[k][0], c1 = C[k][1], c2 = C[k][2];
        if (MODE == WIPES_3D_ALPHA) {
            c0 = fmaf(T[k], kp.bg[0], c0);
            c1 = fmaf(T[k], kp.bg[1], c1);
            c2 = fmaf(T[k], kp.bg[2], c2);
            if (T_final) T_final[pix] = T[k];
            if (last) last[pix] = lst[k];
        }
        float* o = d.out_image ? d.out_image + 3 * (pix - (uint32_t)d.pix_begin) : image + 3 * pix;
        o[0] = c0;
        o[1] = c1;
        o[2] = c2;
    }
}

// Alpha forward with live-pixel compaction.  A pixel writes its outputs the
// moment it terminates and leaves its row; whenever the live pixels fit in
// fewer rows the wave repacks them (row-major order, so rows stay spatially
// coherent) and recomputes the row boxes.  The wave leaves the list as soon as
// no pixel is live.
template <int TW, int TH>
__device__ __forceinline__ void fwd_tile_alpha(const ImgDesc* __restrict__ descs, int B, const KParams& kp,
                                               const Rec* __restrict__ recs, const uint32_t* __restrict__ vals,
                                               const uint2* __restrict__ ranges, uint32_t t,
                                               float* __restrict__ image, float* __restrict__ T_final,
                                               int32_t* __restrict__ last, uint32_t* lds)
{
    constexpr int SBX = TW / 8, NR = (TW / 8) * (TH / 8);
    const TileGeo G = tile_geo(descs, B, ranges, t, TW, TH);
    const ImgDesc& d = descs[G.b];
    const int l = lane_id();
    const uint64_t lt_mask = (l == 0) ? 0ull : (~0ull >> (64 - l));
    uint32_t pk[NR], c0[NR], c1[NR], c2[NR], tt[NR], ls[NR];   // FP32 values travel as bits
    RowBox rb[NR];
    uint32_t A = 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int px = (r % SBX) * 8 + (l & 7), py = (r / SBX) * 8 + (l >> 3);
        const bool valid = (G.ox + px) < d.W && (G.oy + py) < d.H;
        pk[r] = valid ? (uint32_t)(px | (py << 8)) : 0xffffffffu;
        c0[r] = c1[r] = c2[r] = __float_as_uint(0.0f);
        tt[r] = __float_as_uint(1.0f);
        ls[r] = 0xffffffffu;
        rb[r] = row_box((int32_t)pk[r]);
        A += (uint32_t)__popcll(__ballot(valid));
    }
    int nrows = NR;

    auto emit = [&](int r) {
        const int px = (int)(pk[r] & 255u), py = (int)(pk[r] >> 8);
        const uint32_t pix = (uint32_t)d.pix_begin + (uint32_t)((G.oy + py) * d.W + (G.ox + px));
        const float T = __uint_as_float(tt[r]);
        float* o = d.out_image ? d.out_image + 3 * (pix - (uint32_t)d.pix_begin) : image + 3 * pix;
        o[0] = fmaf(T, kp.bg[0], __uint_as_float(c0[r]));
        o[1] = fmaf(T, kp.bg[1], __uint_as_float(c1[r]));
        o[2] = fmaf(T, kp.bg[2], __uint_as_float(c2[r]));
        T_final[pix] = T;
        last[pix] = (int32_t)ls[r];
    };

    for (uint32_t s = G.start; s < G.end && A > 0u; ++s) {
        const uint32_t prim = vals[s];
        uint32_t b0, b1;
        const PrimU u = load_prim(recs, prim, G.ox, G.oy, &b0, &b1);
        const int x0 = lo16(b0) - G.ox, y0 = hi16(b0) - G.oy, x1 = lo16(b1) - G.ox, y1 = hi16(b1) - G.oy;
        bool died = false;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (r >= nrows) break;
            if (!box_meets(rb[r], x0, y0, x1, y1)) continue;
            if ((int32_t)pk[r] < 0) continue;
            const float lx = (float)(pk[r] & 255u) + 0.5f, ly = (float)(pk[r] >> 8) + 0.5f;
            const PairEval p = eval_pair(u, lx, ly);
            const float a = u.op * p.W;
            if (a >= kp.alpha_min) {
                const float al = fminf(a, kp.alpha_max);
                const float T = __uint_as_float(tt[r]);
                const float wt = T * al;
                c0[r] = __float_as_uint(fmaf(wt, u.r, __uint_as_float(c0[r])));
                c1[r] = __float_as_uint(fmaf(wt, u.g, __uint_as_float(c1[r])));
                c2[r] = __float_as_uint(fmaf(wt, u.b, __uint_as_float(c2[r])));
                const float Tn = T * (1.0f - al);
                tt[r] = __float_as_uint(Tn);
                ls[r] = s;
                if (Tn < kp.T_min) {
                    emit(r);
                    pk[r] = 0xffffffffu;
                    died = true;
                }
            }
        }
        if (!__ballot(died)) continue;
        // live count per row; repack when fewer rows suffice
        uint32_t idx[NR];
        bool on[NR];
        uint32_t base = 0;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            on[r] = r < nrows && (int32_t)pk[r] >= 0;
            const uint64_t m = __ballot(on[r]);
            idx[r] = base + (uint32_t)__popcll(m & lt_mask);
            base += (uint32_t)__popcll(m);
        }
        A = base;
        const int want = (int)((A + kWave - 1) / kWave);
        if (want < nrows) {
            route<NR>(lds, on, idx, pk, nrows, want, A, 0xffffffffu);
            route<NR>(lds, on, idx, c0, nrows, want, A, 0u);
            route<NR>(lds, on, idx, c1, nrows, want, A, 0u);
            route<NR>(lds, on, idx, c2, nrows, want, A, 0u);
            route<NR>(lds, on, idx, tt, nrows, want, A, 0u);
            route<NR>(lds, on, idx, ls, nrows, want, A, 0u);
            nrows = want;
#pragma unroll
            for (int r = 0; r < NR; ++r)
                if (r < nrows) rb[r] = row_box((int32_t)pk[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if (r < nrows && (int32_t)pk[r] >= 0) emit(r);
}

template <int MODE, int TW, int TH>
__global__ void __launch_bounds__(kWave * kWpb) k_blend_fwd(const ImgDesc* __restrict__ descs, int B, KParams kp,
                                                            const Rec* __restrict__ recs,
                                                            const uint32_t* __restrict__ vals,
                                                            const uint2* __restrict__ ranges,
                                                            const uint32_t* __restrict__ ovf, uint32_t n_tiles,
                                                            float* __restrict__ image, float* __restrict__ T_final,
                                                            int32_t* __restrict__ last)
{
    __shared__ __attribute__((aligned(16))) uint32_t lds[kWpb][TW * TH];
    if (*ovf) return;   // instance overflow: the sort produced nothing usable
    const uint32_t t = grid_tile_of_wave();
    if (t >= n_tiles) return;
    if (MODE == WIPES_3D_ALPHA)
        fwd_tile_alpha<TW, TH>(descs, B, kp, recs, vals, ranges, t, image, T_final, last, lds[threadIdx.x >> 6]);
    else
        fwd_tile<MODE, TW, TH>(descs, B, kp, recs, vals, ranges, t, image, T_final, last);
}

// Persistent variant: a grid sized to the machine pulls tiles from a queue
// (longest list first when `order` is given) until it is empty.
template <int MODE, int TW, int TH>
__global__ void __launch_bounds__(kWave * kWpb) k_blend_fwd_q(const ImgDesc* __restrict__ descs, int B, KParams kp,
                                                              const Rec* __restrict__ recs,
                                                              const uint32_t* __restrict__ vals,
                                                              const uint2* __restrict__ ranges,
                                                              const uint32_t* __restrict__ ovf, uint32_t n_tiles,
                                                              const uint32_t* __restrict__ order,
                                                              uint32_t* __restrict__ queue, float* __restrict__ image,
                                                              float* __restrict__ T_final, int32_t* __restrict__ last)
{
    __shared__ __attribute__((aligned(16))) uint32_t lds[kWpb][TW * TH];
    if (*ovf) return;
    for (;;) {
        uint32_t idx = 0;
        if (lane_id() == 0) idx = atomicAdd(queue, 1u);
        idx = (uint32_t)__builtin_amdgcn_readfirstlane((int)idx);
        if (idx >= n_tiles) break;
        const uint32_t t = order ? order[idx] : idx;
        if (MODE == WIPES_3D_ALPHA)
            fwd_tile_alpha<TW, TH>(descs, B, kp, recs, vals, ranges, t, image, T_final, last, lds[threadIdx.x >> 6]);
        else
            fwd_tile<MODE, TW, TH>(descs, B, kp, recs, vals, ranges, t, image, T_final, last);
    }
}

// ------------------------------------------------------------ backward

// Sum 16 per-lane values over the wave.  Each step pairs lanes across one
// bit, keeps half the values and adds the partner's copy of that half, so 16
// values cost 8+4+2+1 exchanges instead of 16*6.  On return lane l holds, in
// v[0], the wave total of value (l >> 2) & 15.
__device__ __forceinline__ void wave_reduce16(float v[16])
{
    const int l = lane_id();
    {
        const bool h = (l & 32) != 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float send = h ? v[j] : v[j + 8];
            const float keep = h ? v[j + 8] : v[j];
            v[j] = keep + __shfl_xor(send, 32, kWave);
        }
    }
    {
        const bool h = (l & 16) != 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float send = h ? v[j] : v[j + 4];
            const float keep = h ? v[j + 4] : v[j];
            v[j] = keep + __shfl_xor(send, 16, kWave);
        }
    }
    {
        const bool h = (l & 8) != 0;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const float send = h ? v[j] : v[j + 2];
            const float keep = h ? v[j + 2] : v[j];
            v[j] = keep + __shfl_xor(send, 8, kWave);
        }
    }
    {
        const bool h = (l & 4) != 0;
        const float send = h ? v[0] : v[1];
        const float keep = h ? v[1] : v[0];
        v[0] = keep + __shfl_xor(send, 4, kWave);
    }
    v[0] += __shfl_xor(v[0], 2, kWave);
    v[0] += __shfl_xor(v[0], 1, kWave);
}

// The same reduction on VALU cross-lane paths only (no LDS): gfx950's
// permlane32/permlane16 swaps exchange the two halves / row pairs of two
// registers in one instruction, and DPP row_mirror, row_half_mirror and
// quad_perm pair lanes inside a 16-lane row.  Pairing lanes by a mirror flips
// several low bits at once, which is still a valid butterfly as long as the
// kept half is chosen by the bit the pairing flips last; the final layout is
// the same as wave_reduce16's (lane l holds value (l >> 2) & 15).
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

__device__ __forceinline__ void wave_reduce16_valu(float v[16])
{
    const int l = lane_id();
#pragma unroll
    for (int j = 0; j < 8; ++j) {   // lanes 0-31 keep v[j], lanes 32-63 keep v[j + 8]
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(v[j]), __float_as_int(v[j + 8]), false, false);
        v[j] = __int_as_float(r[0]) + __int_as_float(r[1]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {   // even rows keep v[j], odd rows keep v[j + 4]
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(v[j]), __float_as_int(v[j + 4]), false, false);
        v[j] = __int_as_float(r[0]) + __int_as_float(r[1]);
    }
    {
        const bool h = (l & 8) != 0;   // row_mirror pairs i with 15 - i
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const float a = v[j] + dpp_mov<0x140>(v[j]);
            const float b = v[j + 2] + dpp_mov<0x140>(v[j + 2]);
            v[j] = h ? b : a;
        }
    }
    {
        const bool h = (l & 4) != 0;   // row_half_mirror pairs i with 7 - i inside each half row
        const float a = v[0] + dpp_mov<0x141>(v[0]);
        const float b = v[1] + dpp_mov<0x141>(v[1]);
        v[0] = h ? b : a;
    }
    v[0] += dpp_mov<0x4e>(v[0]);      // quad_perm [2, 3, 0, 1]
    v[0] += dpp_mov<0xb1>(v[0]);      // quad_perm [1, 0, 3, 2]
}

// Gradient slot layout per instance: 12 floats, the first 11 used, in the
// order d/d(mu'x, mu'y, ca, cb, cc, f'x, f'y, opacity, r, g, b).
constexpr int kSlot = 12;

template <int MODE, int TW, int TH>
__device__ __forceinline__ void bwd_tile(const ImgDesc* __restrict__ descs, int B, const KParams& kp,
                                         const Rec* __restrict__ recs, const uint32_t* __restrict__ vals,
                                         const uint32_t* __restrict__ eidx, const uint2* __restrict__ ranges,
                                         uint32_t t,
                                         const float* __restrict__ T_final, const int32_t* __restrict__ last,
                                         const float* __restrict__ dLdC, float* __restrict__ slots)
{
    constexpr int SBX = TW / 8, NSB = (TW / 8) * (TH / 8);
    const TileGeo G = tile_geo(descs, B, ranges, t, TW, TH);
    const ImgDesc& d = descs[G.b];
    const int l = lane_id();
    float lx[NSB], ly[NSB], g[NSB][3], T[NSB], Sg[NSB];
    int32_t lst[NSB];
    int32_t smax = -1;
    uint32_t sb_valid = 0;
#pragma unroll
    for (int k = 0; k < NSB; ++k) {
        const int px = (k % SBX) * 8 + (l & 7), py = (k / SBX) * 8 + (l >> 3);
        lx[k] = (float)px + 0.5f;
        ly[k] = (float)py + 0.5f;
        const bool ok = (G.ox + px) < d.W && (G.oy + py) < d.H;
        const uint32_t pix = (uint32_t)d.pix_begin + (uint32_t)((G.oy + py) * d.W + (G.ox + px));
        g[k][0] = ok ? dLdC[3 * pix] : 0.0f;
        g[k][1] = ok ? dLdC[3 * pix + 1] : 0.0f;
        g[k][2] = ok ? dLdC[3 * pix + 2] : 0.0f;
        if (MODE == WIPES_3D_ALPHA) {
            T[k] = ok ? T_final[pix] : 1.0f;
            lst[k] = ok ? last[pix] : -1;
            Sg[k] = kp.bg[0] * g[k][0] + kp.bg[1] * g[k][1] + kp.bg[2] * g[k][2];
            smax = max(smax, lst[k]);
        } else {
            T[k] = 1.0f;
            lst[k] = ok ? 0x7fffffff : -1;
            Sg[k] = 0.0f;
        }
        sb_valid |= __ballot(ok) ? (1u << k) : 0u;
    }
    uint32_t s_hi;   // one past the last list position any pixel of the tile used
    if (MODE == WIPES_3D_ALPHA) {
        smax = __builtin_amdgcn_readfirstlane(wave_max_i32(smax));
        // clamped to the tile's range, so a `last` from a mismatched forward
        // can only give wrong gradients, never an access outside the list
        s_hi = smax < (int32_t)G.start ? G.start : min((uint32_t)smax + 1u, G.end);
    } else {
        s_hi = G.end;
    }
    // positions no pixel reached get zero gradient slots
    for (uint32_t s = s_hi + (uint32_t)l; s < G.end; s += kWave) {
        float4* o = reinterpret_cast<float4*>(slots + (size_t)eidx[s] * kSlot);
        o[0] = make_float4(0.f, 0.f, 0.f, 0.f);
        o[1] = make_float4(0.f, 0.f, 0.f, 0.f);
        o[2] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    const float thr2 = kp.q_add * (-0.5f * kLog2e);
    for (uint32_t s = s_hi; s-- > G.start;) {
        const uint32_t prim = vals[s];
        uint32_t b0, b1;
        const PrimU u = load_prim(recs, prim, G.ox, G.oy, &b0, &b1);
        const uint32_t m = subblock_mask<TW, TH>(b0, b1, G.ox, G.oy) & sb_valid;
        float v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = 0.0f;
        bool any = false;
#pragma unroll
        for (int k = 0; k < NSB; ++k) {
            if (!(m & (1u << k))) continue;
            if ((int32_t)s > lst[k]) continue;
            const PairEval p = eval_pair(u, lx[k], ly[k]);
            float dW;   // dL/dW'
            if (MODE == WIPES_2D_ADDITIVE) {
                if (!(p.e2 >= thr2)) continue;
                const float cg = u.r * g[k][0] + u.g * g[k][1] + u.b * g[k][2];
                const float ow = u.op * p.W;
                v[8] = fmaf(ow, g[k][0], v[8]);
                v[9] = fmaf(ow, g[k][1], v[9]);
                v[10] = fmaf(ow, g[k][2], v[10]);
                v[7] = fmaf(p.W, cg, v[7]);
                dW = u.op * cg;
            } else {
                const float a = u.op * p.W;
                if (!(a >= kp.alpha_min)) continue;
                const float al = fminf(a, kp.alpha_max);
                const float Tb = T[k] / (1.0f - al);
                const float cg = u.r * g[k][0] + u.g * g[k][1] + u.b * g[k][2];
                const float dal = Tb * (cg - Sg[k]);
                const float wt = Tb * al;
                v[8] = fmaf(wt, g[k][0], v[8]);
                v[9] = fmaf(wt, g[k][1], v[9]);
                v[10] = fmaf(wt, g[k][2], v[10]);
                Sg[k] = fmaf(al, cg - Sg[k], Sg[k]);
                T[k] = Tb;
                const float da = a <= kp.alpha_max ? dal : 0.0f;
                v[7] = fmaf(p.W, da, v[7]);
                dW = u.op * da;
            }
            any = true;
            const float sn = __builtin_amdgcn_sinf(__builtin_amdgcn_fractf(p.ph));
            const float dq = dW * (-0.5f * p.W);             // dL/dq
            const float dph = dW * (-0.5f * p.E * sn);       // dL/dphi (radians)
            const float Adx = fmaf(u.ca, p.dx, u.cb * p.dy), Ady = fmaf(u.cb, p.dx, u.cc * p.dy);
            v[0] = fmaf(-2.0f * dq, Adx, fmaf(-dph, u.fx, v[0]));
            v[1] = fmaf(-2.0f * dq, Ady, fmaf(-dph, u.fy, v[1]));
            v[2] = fmaf(dq * p.dx, p.dx, v[2]);
            v[3] = fmaf(2.0f * dq * p.dx, p.dy, v[3]);
            v[4] = fmaf(dq * p.dy, p.dy, v[4]);
            v[5] = fmaf(dph, p.dx, v[5]);
            v[6] = fmaf(dph, p.dy, v[6]);
        }
        float* o = slots + (size_t)eidx[s] * kSlot;
        if (__ballot(any)) {
            wave_reduce16_valu(v);
            const int idx = l >> 2;
            if ((l & 3) == 0 && idx < kSlot) o[idx] = v[0];
        } else if (l < kSlot) {
            o[l] = 0.0f;
        }
    }
}

// Alpha backward with pixels ranked by `last`.  A pixel only takes part in
// list positions s <= last (it walks back to front from its last contributing
// pair), so the tile's pixels are ranked by descending last (ties by pixel
// order) and dealt to rows in that order: at position s exactly the rows whose
// first pixel has last >= s are active, and they form a prefix.  Pixels that
// never contributed take no part at all.
template <int TW, int TH>
__device__ __forceinline__ void bwd_tile_alpha(const ImgDesc* __restrict__ descs, int B, const KParams& kp,
                                               const Rec* __restrict__ recs, const uint32_t* __restrict__ vals,
                                               const uint32_t* __restrict__ eidx,
                                               const uint2* __restrict__ ranges, uint32_t t,
                                               const float* __restrict__ T_final, const int32_t* __restrict__ last,
                                               const float* __restrict__ dLdC, float* __restrict__ slots,
                                               uint32_t* lds)
{
    constexpr int SBX = TW / 8, NR = (TW / 8) * (TH / 8), P = TW * TH;
    const TileGeo G = tile_geo(descs, B, ranges, t, TW, TH);
    const ImgDesc& d = descs[G.b];
    const int l = lane_id();
    uint32_t pk[NR], ls[NR], tt[NR], g0[NR], g1[NR], g2[NR];
    bool on[NR];
    uint32_t A = 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int px = (r % SBX) * 8 + (l & 7), py = (r / SBX) * 8 + (l >> 3);
        const bool valid = (G.ox + px) < d.W && (G.oy + py) < d.H;
        const uint32_t pix = (uint32_t)d.pix_begin + (uint32_t)((G.oy + py) * d.W + (G.ox + px));
        const int32_t lv = valid ? last[pix] : -1;
        on[r] = lv >= 0;
        pk[r] = (uint32_t)(px | (py << 8));
        ls[r] = (uint32_t)lv;
        tt[r] = on[r] ? __float_as_uint(T_final[pix]) : 0u;
        g0[r] = on[r] ? __float_as_uint(dLdC[3 * pix]) : 0u;
        g1[r] = on[r] ? __float_as_uint(dLdC[3 * pix + 1]) : 0u;
        g2[r] = on[r] ? __float_as_uint(dLdC[3 * pix + 2]) : 0u;
        A += (uint32_t)__popcll(__ballot(on[r]));
    }
    // rank: number of pixels with larger last, or equal last and smaller slot
#pragma unroll
    for (int r = 0; r < NR; ++r) lds[r * kWave + l] = ls[r];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint32_t idx[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) idx[r] = 0;
    for (int q = 0; q < P; q += 4) {
        const uint4 v4 = *reinterpret_cast<const uint4*>(lds + q);
        const int32_t lq[4] = {(int32_t)v4.x, (int32_t)v4.y, (int32_t)v4.z, (int32_t)v4.w};
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int self = r * kWave + l;
            const int32_t lv = (int32_t)ls[r];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                idx[r] += (lq[k] > lv || (lq[k] == lv && q + k < self)) ? 1u : 0u;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int nrows = (int)((A + kWave - 1) / kWave);
    route<NR>(lds, on, idx, pk, NR, nrows, A, 0xffffffffu);
    route<NR>(lds, on, idx, ls, NR, nrows, A, 0xffffffffu);
    route<NR>(lds, on, idx, tt, NR, nrows, A, 0u);
    route<NR>(lds, on, idx, g0, NR, nrows, A, 0u);
    route<NR>(lds, on, idx, g1, NR, nrows, A, 0u);
    route<NR>(lds, on, idx, g2, NR, nrows, A, 0u);
    RowBox rb[NR];
    int32_t rowmax[NR];
    float Sg[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        rb[r] = row_box(r < nrows ? (int32_t)pk[r] : -1);
        rowmax[r] = r < nrows ? __builtin_amdgcn_readfirstlane((int32_t)ls[r]) : -1;
        Sg[r] = kp.bg[0] * __uint_as_float(g0[r]) + kp.bg[1] * __uint_as_float(g1[r]) +
                kp.bg[2] * __uint_as_float(g2[r]);
    }
    // clamped to the tile's range (a `last` from a mismatched forward gives
    // wrong gradients, never an access outside the list)
    const uint32_t s_hi = (A > 0u && rowmax[0] >= (int32_t)G.start) ? min((uint32_t)rowmax[0] + 1u, G.end) : G.start;
    for (uint32_t s = s_hi + (uint32_t)l; s < G.end; s += kWave) {
        float4* o = reinterpret_cast<float4*>(slots + (size_t)eidx[s] * kSlot);
        o[0] = make_float4(0.f, 0.f, 0.f, 0.f);
        o[1] = make_float4(0.f, 0.f, 0.f, 0.f);
        o[2] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    int nact = 0;
    for (uint32_t s = s_hi; s-- > G.start;) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if (nact == r && r < nrows && rowmax[r] >= (int32_t)s) nact = r + 1;
        const uint32_t prim = vals[s];
        uint32_t b0, b1;
        const PrimU u = load_prim(recs, prim, G.ox, G.oy, &b0, &b1);
        const int x0 = lo16(b0) - G.ox, y0 = hi16(b0) - G.oy, x1 = lo16(b1) - G.ox, y1 = hi16(b1) - G.oy;
        float v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = 0.0f;
        bool any = false;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (r >= nact) break;
            if (!box_meets(rb[r], x0, y0, x1, y1)) continue;
            if ((int32_t)ls[r] < (int32_t)s) continue;      // not reached yet (or empty slot)
            const float lx = (float)(pk[r] & 255u) + 0.5f, ly = (float)(pk[r] >> 8) + 0.5f;
            const PairEval p = eval_pair(u, lx, ly);
            const float a = u.op * p.W;
            if (!(a >= kp.alpha_min)) continue;
            const float gr = __uint_as_float(g0[r]), gg = __uint_as_float(g1[r]), gb = __uint_as_float(g2[r]);
            const float al = fminf(a, kp.alpha_max);
            const float Tb = __uint_as_float(tt[r]) / (1.0f - al);
            const float cg = u.r * gr + u.g * gg + u.b * gb;
            const float dal = Tb * (cg - Sg[r]);
            const float wt = Tb * al;
            v[8] = fmaf(wt, gr, v[8]);
            v[9] = fmaf(wt, gg, v[9]);
            v[10] = fmaf(wt, gb, v[10]);
            Sg[r] = fmaf(al, cg - Sg[r], Sg[r]);
            tt[r] = __float_as_uint(Tb);
            const float da = a <= kp.alpha_max ? dal : 0.0f;
            v[7] = fmaf(p.W, da, v[7]);
            const float dW = u.op * da;
            any = true;
            const float sn = __builtin_amdgcn_sinf(__builtin_amdgcn_fractf(p.ph));
            const float dq = dW * (-0.5f * p.W);
            const float dph = dW * (-0.5f * p.E * sn);
            const float Adx = fmaf(u.ca, p.dx, u.cb * p.dy), Ady = fmaf(u.cb, p.dx, u.cc * p.dy);
            v[0] = fmaf(-2.0f * dq, Adx, fmaf(-dph, u.fx, v[0]));
            v[1] = fmaf(-2.0f * dq, Ady, fmaf(-dph, u.fy, v[1]));
            v[2] = fmaf(dq * p.dx, p.dx, v[2]);
            v[3] = fmaf(2.0f * dq * p.dx, p.dy, v[3]);
            v[4] = fmaf(dq * p.dy, p.dy, v[4]);
            v[5] = fmaf(dph, p.dx, v[5]);
            v[6] = fmaf(dph, p.dy, v[6]);
        }
        float* o = slots + (size_t)eidx[s] * kSlot;
        if (__ballot(any)) {
            wave_reduce16_valu(v);
            const int id = l >> 2;
            if ((l & 3) == 0 && id < kSlot) o[id] = v[0];
        } else if (l < kSlot) {
            o[l] = 0.0f;
        }
    }
}

template <int MODE, int TW, int TH>
__global__ void __launch_bounds__(kWave * kWpb) k_blend_bwd(const ImgDesc* __restrict__ descs, int B, KParams kp,
                                                            const Rec* __restrict__ recs,
                                                            const uint32_t* __restrict__ vals,
                                                            const uint32_t* __restrict__ eidx,
                                                            const uint2* __restrict__ ranges,
                                                            const uint32_t* __restrict__ ovf, uint32_t n_tiles,
                                                            const float* __restrict__ T_final,
                                                            const int32_t* __restrict__ last,
                                                            const float* __restrict__ dLdC,
                                                            float* __restrict__ slots)
{
    __shared__ __attribute__((aligned(16))) uint32_t lds[kWpb][TW * TH];
    if (*ovf) return;
    const uint32_t t = grid_tile_of_wave();
    if (t >= n_tiles) return;
    if (MODE == WIPES_3D_ALPHA)
        bwd_tile_alpha<TW, TH>(descs, B, kp, recs, vals, eidx, ranges, t, T_final, last, dLdC, slots,
                               lds[threadIdx.x >> 6]);
    else
        bwd_tile<MODE, TW, TH>(descs, B, kp, recs, vals, eidx, ranges, t, T_final, last, dLdC, slots);
}

template <int MODE, int TW, int TH>
__global__ void __launch_bounds__(kWave * kWpb) k_blend_bwd_q(const ImgDesc* __restrict__ descs, int B, KParams kp,
                                                              const Rec* __restrict__ recs,
                                                              const uint32_t* __restrict__ vals,
                                                              const uint32_t* __restrict__ eidx,
                                                              const uint2* __restrict__ ranges,
                                                              const uint32_t* __restrict__ ovf, uint32_t n_tiles,
                                                              const uint32_t* __restrict__ order,
                                                              uint32_t* __restrict__ queue,
                                                              const float* __restrict__ T_final,
                                                              const int32_t* __restrict__ last,
                                                              const float* __restrict__ dLdC,
                                                              float* __restrict__ slots)
{
    __shared__ __attribute__((aligned(16))) uint32_t lds[kWpb][TW * TH];
    if (*ovf) return;
    for (;;) {
        uint32_t idx = 0;
        if (lane_id() == 0) idx = atomicAdd(queue, 1u);
        idx = (uint32_t)__builtin_amdgcn_readfirstlane((int)idx);
        if (idx >= n_tiles) break;
        const uint32_t t = order ? order[idx] : idx;
        if (MODE == WIPES_3D_ALPHA)
            bwd_tile_alpha<TW, TH>(descs, B, kp, recs, vals, eidx, ranges, t, T_final, last, dLdC, slots,
                                   lds[threadIdx.x >> 6]);
        else
            bwd_tile<MODE, TW, TH>(descs, B, kp, recs, vals, eidx, ranges, t, T_final, last, dLdC, slots);
    }
}

// ------------------------------------------------------------ work counts

// Support pairs (forward / backward), tile pairs and sub-block pairs of one
// tile, summed over the grid into out[0..3].  Support: q <= q_add (additive),
// q <= 2 ln(o / alpha_min) (alpha: outside it o W' < alpha_min).
template <int MODE, int TW, int TH>
__global__ void __launch_bounds__(kWave * kWpb) k_pair_stats(const ImgDesc* __restrict__ descs, int B, KParams kp,
                                                             const Rec* __restrict__ recs,
                                                             const uint32_t* __restrict__ vals,
                                                             const uint2* __restrict__ ranges,
                                                             const uint32_t* __restrict__ ovf, uint32_t n_tiles,
                                                             const float* __restrict__ T_final,
                                                             const int32_t* __restrict__ last,
                                                             unsigned long long* __restrict__ out)
{
    constexpr int SBX = TW / 8, NSB = (TW / 8) * (TH / 8);
    if (*ovf) return;
    const uint32_t t = grid_tile_of_wave();
    if (t >= n_tiles) return;
    const TileGeo G = tile_geo(descs, B, ranges, t, TW, TH);
    const ImgDesc& d = descs[G.b];
    const int l = lane_id();
    float lx[NSB], ly[NSB];
    bool ok[NSB];
    int32_t lst[NSB];
    bool stopped[NSB];
    uint32_t npix = 0;
#pragma unroll
    for (int k = 0; k < NSB; ++k) {
        const int px = (k % SBX) * 8 + (l & 7), py = (k / SBX) * 8 + (l >> 3);
        lx[k] = (float)px + 0.5f;
        ly[k] = (float)py + 0.5f;
        ok[k] = (G.ox + px) < d.W && (G.oy + py) < d.H;
        const uint32_t pix = (uint32_t)d.pix_begin + (uint32_t)((G.oy + py) * d.W + (G.ox + px));
        lst[k] = (MODE == WIPES_3D_ALPHA && ok[k]) ? last[pix] : 0x7fffffff;
        stopped[k] = MODE == WIPES_3D_ALPHA && ok[k] && T_final[pix] < kp.T_min;
        npix += ok[k] ? 1u : 0u;
    }
    unsigned long long cf = 0, cb = 0, csub = 0;
    const float kq = -0.5f * kLog2e;
    for (uint32_t s = G.start; s < G.end; ++s) {
        const uint32_t prim = vals[s];
        uint32_t b0, b1;
        const PrimU u = load_prim(recs, prim, G.ox, G.oy, &b0, &b1);
        const uint32_t m = subblock_mask<TW, TH>(b0, b1, G.ox, G.oy);
        const float thr = kq * (MODE == WIPES_2D_ADDITIVE ? kp.q_add : 2.0f * logf(u.op / kp.alpha_min));
#pragma unroll
        for (int k = 0; k < NSB; ++k) {
            if (!(m & (1u << k))) continue;
            csub += 1;
            if (!ok[k]) continue;
            const PairEval p = eval_pair(u, lx[k], ly[k]);
            if (!(p.e2 >= thr)) continue;
            const bool fwd = !(stopped[k] && (int32_t)s > lst[k]);
            cf += fwd ? 1u : 0u;
            cb += ((int32_t)s <= lst[k]) ? 1u : 0u;
        }
    }
    // wave sums (every lane participates)
    for (int o = 32; o > 0; o >>= 1) {
        cf += __shfl_xor(cf, o, kWave);
        cb += __shfl_xor(cb, o, kWave);
        npix += (uint32_t)__shfl_xor((int)npix, o, kWave);
    }
    if (l == 0) {
        atomicAdd(&out[0], cf);
        atomicAdd(&out[1], cb);
        atomicAdd(&out[2], (unsigned long long)npix * (unsigned long long)(G.end - G.start));
        atomicAdd(&out[3], csub * (unsigned long long)kWave);
    }
}

// ------------------------------------------------------------- host side

template <int MODE, int TW, int TH>
static void launch_fwd_t(const ImgDesc* descs, int B, const KParams& kp, const Rec* recs, const uint32_t* vals,
                         const uint2* ranges, const uint32_t* ovf, uint32_t n_tiles, const uint32_t* order,
                         uint32_t* queue, uint32_t persistent_blocks, float* image, float* T_final, int32_t* last,
                         hipStream_t s)
{
    if (queue) {
        if (persistent_blocks == 0) return;
        hipLaunchKernelGGL((k_blend_fwd_q<MODE, TW, TH>), dim3(persistent_blocks), dim3(kWave * kWpb), 0, s, descs, B,
                           kp, recs, vals, ranges, ovf, n_tiles, order, queue, image, T_final, last);
        return;
    }
    const uint32_t nb = (n_tiles + kWpb - 1) / kWpb;
    if (nb == 0) return;
    hipLaunchKernelGGL((k_blend_fwd<MODE, TW, TH>), dim3(nb), dim3(kWave * kWpb), 0, s, descs, B, kp, recs, vals,
                       ranges, ovf, n_tiles, image, T_final, last);
}

template <int MODE, int TW, int TH>
static void launch_bwd_t(const ImgDesc* descs, int B, const KParams& kp, const Rec* recs, const uint32_t* vals,
                         const uint32_t* eidx, const uint2* ranges, const uint32_t* ovf, uint32_t n_tiles,
                         const uint32_t* order, uint32_t* queue, uint32_t persistent_blocks, const float* T_final,
                         const int32_t* last, const float* dLdC, float* slots, hipStream_t s)
{
    if (queue) {
        if (persistent_blocks == 0) return;
        hipLaunchKernelGGL((k_blend_bwd_q<MODE, TW, TH>), dim3(persistent_blocks), dim3(kWave * kWpb), 0, s, descs, B,
                           kp, recs, vals, eidx, ranges, ovf, n_tiles, order, queue, T_final, last, dLdC, slots);
        return;
    }
    const uint32_t nb = (n_tiles + kWpb - 1) / kWpb;
    if (nb == 0) return;
    hipLaunchKernelGGL((k_blend_bwd<MODE, TW, TH>), dim3(nb), dim3(kWave * kWpb), 0, s, descs, B, kp, recs, vals,
                       eidx, ranges, ovf, n_tiles, T_final, last, dLdC, slots);
}

#define WIPES_TILE_DISPATCH(FN, MODE, ...)                                          \
    do {                                                                            \
        if (kp.tile_w == 8 && kp.tile_h == 8) FN<MODE, 8, 8>(__VA_ARGS__);          \
        else if (kp.tile_w == 16 && kp.tile_h == 8) FN<MODE, 16, 8>(__VA_ARGS__);   \
        else if (kp.tile_w == 16 && kp.tile_h == 16) FN<MODE, 16, 16>(__VA_ARGS__); \
        else if (kp.tile_w == 32 && kp.tile_h == 8) FN<MODE, 32, 8>(__VA_ARGS__);   \
        else if (kp.tile_w == 8 && kp.tile_h == 16) FN<MODE, 8, 16>(__VA_ARGS__);   \
        else FN<MODE, 32, 16>(__VA_ARGS__);                                         \
    } while (0)

template <int MODE, int TW, int TH>
static void launch_stats_t(const ImgDesc* descs, int B, const KParams& kp, const Rec* recs, const uint32_t* vals,
                           const uint2* ranges, const uint32_t* ovf, uint32_t n_tiles, const float* T_final,
                           const int32_t* last, unsigned long long* out, hipStream_t s)
{
    const uint32_t nb = (n_tiles + kWpb - 1) / kWpb;
    if (nb == 0) return;
    hipLaunchKernelGGL((k_pair_stats<MODE, TW, TH>), dim3(nb), dim3(kWave * kWpb), 0, s, descs, B, kp, recs, vals,
                       ranges, ovf, n_tiles, T_final, last, out);
}

hipError_t launch_pair_stats(const ImgDesc* descs, int B, const KParams& kp, const Rec* recs, const uint32_t* vals,
                             const uint2* ranges, const uint32_t* ovf, uint32_t n_tiles, const float* T_final,
                             const int32_t* last, unsigned long long* out, hipStream_t s)
{
    if (kp.mode == WIPES_2D_ADDITIVE)
        WIPES_TILE_DISPATCH(launch_stats_t, WIPES_2D_ADDITIVE, descs, B, kp, recs, vals, ranges, ovf, n_tiles, T_final,
                            last, out, s);
    else
        WIPES_TILE_DISPATCH(launch_stats_t, WIPES_3D_ALPHA, descs, B, kp, recs, vals, ranges, ovf, n_tiles, T_final,
                            last, out, s);
    return hipGetLastError();
}

hipError_t launch_blend_fwd(const ImgDesc* descs, int B, const KParams& kp, const Rec* recs, const uint32_t* vals,
                            const uint2* ranges, const uint32_t* ovf, uint32_t n_tiles, const uint32_t* order,
                            uint32_t* queue, uint32_t persistent_blocks, float* image, float* T_final, int32_t* last,
                            hipStream_t s)
{
    if (kp.mode == WIPES_2D_ADDITIVE)
        WIPES_TILE_DISPATCH(launch_fwd_t, WIPES_2D_ADDITIVE, descs, B, kp, recs, vals, ranges, ovf, n_tiles, order,
                            queue, persistent_blocks, image, T_final, last, s);
    else
        WIPES_TILE_DISPATCH(launch_fwd_t, WIPES_3D_ALPHA, descs, B, kp, recs, vals, ranges, ovf, n_tiles, order,
                            queue, persistent_blocks, image, T_final, last, s);
    return hipGetLastError();
}

hipError_t launch_blend_bwd(const ImgDesc* descs, int B, const KParams& kp, const Rec* recs, const uint32_t* vals,
                            const uint32_t* eidx, const uint2* ranges, const uint32_t* ovf, uint32_t n_tiles,
                            const uint32_t* order, uint32_t* queue, uint32_t persistent_blocks, const float* T_final,
                            const int32_t* last, const float* dLdC, float* slots, hipStream_t s)
{
    if (kp.mode == WIPES_2D_ADDITIVE)
        WIPES_TILE_DISPATCH(launch_bwd_t, WIPES_2D_ADDITIVE, descs, B, kp, recs, vals, eidx, ranges, ovf, n_tiles,
                            order, queue, persistent_blocks, T_final, last, dLdC, slots, s);
    else
        WIPES_TILE_DISPATCH(launch_bwd_t, WIPES_3D_ALPHA, descs, B, kp, recs, vals, eidx, ranges, ovf, n_tiles, order,
                            queue, persistent_blocks, T_final, last, dLdC, slots, s);
    return hipGetLastError();
}

}  // namespace wipes
