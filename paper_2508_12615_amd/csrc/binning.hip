// Tile binning: pixel boxes, per-primitive tile counts, instance emission and
// per-tile ranges.
//
// The binning rule (a reading of the 3DGS-style pipeline the paper follows,
// Sec. 4.1), in FP32 with exactly these operations so that it is reproducible:
//   x0 = max(ceil((mx - rx) - 1/2), 0), x1 = min(floor((mx + rx) - 1/2), W - 1)
//   (same for y); empty unless x0 <= x1 and y0 <= y1; tile rect = box / tile size;
//   a rectangle of at most 64 tiles keeps only the tiles whose part of the box
//   the padded support ellipse reaches (ellipse_reaches below).
// (mx, rx) are the FP32 record mean and padded support half-extent, so the box
// holds every pixel whose centre can pass the per-pixel test.
//
// Emission order defines the order of equal keys after the stable sort:
//   additive: primitive index order, key = global tile;
//   alpha:    ascending (depth key, index) order (primitives pre-sorted by
//             depth), key = global tile.  The stable tile sort then leaves
//             every tile's list in (depth key, index) order -- the same list a
//             single sort on (tile << 32 | depth bits) would give.
#include "common.hpp"

namespace wipes {

constexpr uint32_t kEmptyBox0 = 0x0000ffffu;   // x0 = 65535 > x1 = 0
constexpr uint32_t kEmptyBox1 = 0u;

// Ellipse part of the binning rule: whether the padded support ellipse
// q(x) <= Qs, q = ca dx^2 + 2 cb dx dy + cc dy^2, reaches the rectangle of
// pixel centres [x0 + 1/2, x1 + 1/2] x [y0 + 1/2, y1 + 1/2].  The minimum of
// the convex q over the rectangle is 0 if the mean lies inside, else it lies
// on an edge, where it is a clamped one-dimensional minimum.  FP32 in exactly
// this sequence (explicit fma, IEEE division).
__device__ __forceinline__ float q32(float ca, float cb, float cc, float dx, float dy)
{
    return fmaf(ca * dx, dx, fmaf(2.0f * cb * dx, dy, cc * dy * dy));
}

__device__ __forceinline__ float clamp32(float v, float lo, float hi) { return fminf(fmaxf(v, lo), hi); }

// sy = -cb / cc and sx = -cb / ca (the slopes of the clamped minima) depend
// on the primitive only and are passed in, divided once per primitive.
__device__ __forceinline__ bool ellipse_reaches(float mx, float my, float ca, float cb, float cc, float sy, float sx,
                                                float Qs, int32_t x0, int32_t y0, int32_t x1, int32_t y1)
{
    const float fx0 = (float)x0 + 0.5f, fx1 = (float)x1 + 0.5f, fy0 = (float)y0 + 0.5f, fy1 = (float)y1 + 0.5f;
    if (mx >= fx0 && mx <= fx1 && my >= fy0 && my <= fy1) return true;
    const float dxa = fx0 - mx, dxb = fx1 - mx, dya = fy0 - my, dyb = fy1 - my;
    float m = q32(ca, cb, cc, dxa, clamp32(sy * dxa, dya, dyb));
    m = fminf(m, q32(ca, cb, cc, dxb, clamp32(sy * dxb, dya, dyb)));
    m = fminf(m, q32(ca, cb, cc, clamp32(sx * dya, dxa, dxb), dya));
    m = fminf(m, q32(ca, cb, cc, clamp32(sx * dyb, dxa, dxb), dyb));
    return m <= Qs;
}

constexpr int32_t kCullMaxTiles = 64;   // larger tile rectangles keep every tile

// count[i] = tiles of the pixel box's tile rectangle that the support ellipse
// reaches; writes the pixel box into the record and the PrimPack (count, box,
// kept-tile mask) into pk[i].  Alpha mode also emits (depth key, index) pairs
// for the depth sort, with culled or off-screen primitives keyed to the end.
__global__ void __launch_bounds__(256) k_bin_count(const ImgDesc* __restrict__ descs, int B, int32_t n_total,
                                                    KParams kp, Rec* __restrict__ recs,
                                                    const Aux* __restrict__ aux, uint32_t* __restrict__ count,
                                                    PrimPack* __restrict__ pk, uint32_t* __restrict__ dkey,
                                                    uint32_t* __restrict__ dval, uint32_t* __restrict__ wsum,
                                                    Clear2 clr)
{
    // zero what the later stages of this bin_sort expect cleared
    {
        const uint32_t g = blockIdx.x * 256u + threadIdx.x, gs = gridDim.x * 256u;
        for (uint32_t k = g; k < clr.n0; k += gs) clr.p0[k] = 0u;
        for (uint32_t k = g; k < clr.n1; k += gs) clr.p1[k] = 0u;
    }
    // per lane of each wave: the ellipse and rectangle its primitive's tile
    // tests need, the offset of those tests in the wave's list, the kept mask
    __shared__ float4 s_pa[4][kWave];             // mx, my, ca, cb
    __shared__ float4 s_pb[4][kWave];             // cc, sy, sx, Qs
    __shared__ uint4 s_pc[4][kWave];              // box0, box1, first tile (x | y << 16), tiles per row
    __shared__ uint32_t s_off[4][kWave];
    __shared__ unsigned long long s_mask[4][kWave];
    const int w = (int)(threadIdx.x >> 6), l = lane_id();
    if ((int32_t)(blockIdx.x * 256u + (uint32_t)w * kWave) >= n_total) return;   // wave-uniform
    const int32_t i = (int32_t)(blockIdx.x * 256u + threadIdx.x);
    const bool inr = i < n_total;
    uint32_t c = 0, b0 = kEmptyBox0, b1 = kEmptyBox1, full = 1, ncull = 0;
    Aux a{};
    float mx = 0.0f, my = 0.0f, ca = 0.0f, cb = 0.0f, cc = 0.0f, sy = 0.0f, sx = 0.0f;
    int32_t tx0 = 0, ty0 = 0, ntx = 1;
    if (inr) {
        const ImgDesc& d = descs[image_of_prim(descs, B, i)];
        a = aux[i];
        mx = recs[i].mx;
        my = recs[i].my;
        if (a.rx >= 0.0f && a.ry >= 0.0f && fabsf(mx) < 1e30f && fabsf(my) < 1e30f) {
            float x0 = ceilf((mx - a.rx) - 0.5f), x1 = floorf((mx + a.rx) - 0.5f);
            float y0 = ceilf((my - a.ry) - 0.5f), y1 = floorf((my + a.ry) - 0.5f);
            x0 = fmaxf(x0, 0.0f);
            y0 = fmaxf(y0, 0.0f);
            x1 = fminf(x1, (float)(d.W - 1));
            y1 = fminf(y1, (float)(d.H - 1));
            if (x0 <= x1 && y0 <= y1) {
                const int32_t ix0 = (int32_t)x0, iy0 = (int32_t)y0, ix1 = (int32_t)x1, iy1 = (int32_t)y1;
                b0 = pack16(ix0, iy0);
                b1 = pack16(ix1, iy1);
                tx0 = ix0 >> kp.log2_tw;
                ty0 = iy0 >> kp.log2_th;
                const int32_t tx1 = ix1 >> kp.log2_tw, ty1 = iy1 >> kp.log2_th;
                ntx = tx1 - tx0 + 1;
                const int32_t nt = ntx * (ty1 - ty0 + 1);
                if (nt > kCullMaxTiles) {
                    c = (uint32_t)nt;
                } else {
                    full = 0;
                    ncull = (uint32_t)nt;
                    ca = recs[i].ca;
                    cb = recs[i].cb;
                    cc = recs[i].cc;
                    sy = -cb / cc;
                    sx = -cb / ca;
                }
            }
        }
    }
    // The wave shares the tile tests of its primitives' rectangles over its
    // lanes (test k of a primitive is tile k of its rectangle, row-major), so
    // it takes ceil(sum / 64) rounds instead of as many as its largest
    // rectangle has tiles.  Each test is the same FP32 rule as per primitive.
    uint32_t tot;
    const uint32_t off = wave_excl_scan_u32(ncull, &tot);
    uint64_t mask = 0;
    if (tot) {   // wave-uniform
        s_pa[w][l] = make_float4(mx, my, ca, cb);
        s_pb[w][l] = make_float4(cc, sy, sx, a.Qs);
        s_pc[w][l] = make_uint4(b0, b1, (uint32_t)tx0 | ((uint32_t)ty0 << 16), (uint32_t)ntx);
        s_off[w][l] = off;
        s_mask[w][l] = 0ull;
        wave_lds_sync();
        for (uint32_t j0 = 0; j0 < tot; j0 += kWave) {
            const uint32_t j = j0 + (uint32_t)l;
            if (j < tot) {
                // owner: the last lane whose first test is at or before j
                int o = 0;
#pragma unroll
                for (int step = kWave / 2; step > 0; step >>= 1)
                    if (s_off[w][o + step] <= j) o += step;
                const uint32_t k = j - s_off[w][o];
                const float4 pa = s_pa[w][o], pb = s_pb[w][o];
                const uint4 pc = s_pc[w][o];
                // k < 64 and the row length <= 64: the float quotient of
                // k + 1/2 is at least 1/128 from an integer, so its floor is exact
                const uint32_t ky = (uint32_t)(((float)k + 0.5f) * __builtin_amdgcn_rcpf((float)pc.w));
                const int32_t tx = (int32_t)lo16(pc.z) + (int32_t)(k - ky * pc.w), ty = (int32_t)hi16(pc.z) + (int32_t)ky;
                const int32_t rx0 = max(tx * kp.tile_w, (int32_t)lo16(pc.x)), ry0 = max(ty * kp.tile_h, (int32_t)hi16(pc.x));
                const int32_t rx1 = min(tx * kp.tile_w + kp.tile_w - 1, (int32_t)lo16(pc.y));
                const int32_t ry1 = min(ty * kp.tile_h + kp.tile_h - 1, (int32_t)hi16(pc.y));
                if (ellipse_reaches(pa.x, pa.y, pa.z, pa.w, pb.x, pb.y, pb.z, pb.w, rx0, ry0, rx1, ry1))
                    atomicOr(&s_mask[w][o], 1ull << k);
            }
        }
        wave_lds_sync();
        mask = s_mask[w][l];
        if (ncull) c = (uint32_t)__popcll(mask);
    }
    {   // the wave's count sum, for the offset scan
        const uint32_t ws = wave_sum_u32(c);
        if (l == 0) wsum[(blockIdx.x * 256u + (uint32_t)w * kWave) >> 6] = ws;
    }
    if (!inr) return;
    recs[i].box0 = b0;
    recs[i].box1 = b1;
    count[i] = c;
    PrimPack q;
    q.count = c;
    q.box0 = b0;
    q.box1 = b1;
    q.base = 0;
    q.mlo = (uint32_t)mask;
    q.mhi = (uint32_t)(mask >> 32);
    q.full = full;
    q.pad = 0;
    pk[i] = q;
    if (dkey) {
        dkey[i] = c ? __float_as_uint(a.depth) : 0xffffffffu;
        dval[i] = (uint32_t)i;
    }
}

// Position of the k-th (0-based) set bit of m (k < popcount(m)).
__device__ __forceinline__ uint32_t nth_set_bit(uint64_t m, uint32_t k)
{
    uint32_t pos = 0, v = (uint32_t)m, c = (uint32_t)__popc(v);
    if (k >= c) {
        k -= c;
        pos = 32;
        v = (uint32_t)(m >> 32);
    }
#pragma unroll
    for (int w = 16; w >= 1; w >>= 1) {
        c = (uint32_t)__popc(v & ((1u << w) - 1u));
        if (k >= c) {
            k -= c;
            pos += (uint32_t)w;
            v >>= w;
        }
    }
    return pos;
}

// Instance offsets by primitive: off_id[i] = pk[i].base = exclusive prefix
// of count, from the scanned wave sums woff (one per 64 primitives) and the
// prefix within the wave.
__device__ __forceinline__ void count_apply(int32_t i, int32_t i0, int32_t n_total,
                                            const uint32_t* __restrict__ count, const uint32_t* __restrict__ woff,
                                            uint32_t* __restrict__ off_id, PrimPack* pk)
{
    const bool ok = i < n_total;
    uint32_t t;
    const uint32_t ex = wave_excl_scan_u32(ok ? count[i] : 0u, &t);
    if (ok) {
        const uint32_t o = woff[i0 >> 6] + ex;
        off_id[i] = o;
        pk[i].base = o;
    }
}

__global__ void __launch_bounds__(256) k_count_apply(int32_t n_total, const uint32_t* __restrict__ count,
                                                     const uint32_t* __restrict__ woff, uint32_t* __restrict__ off_id,
                                                     PrimPack* __restrict__ pk)
{
    const int32_t i0 = (int32_t)(blockIdx.x * 256u + (threadIdx.x & ~63u));   // lane 0 of the wave
    if (i0 >= n_total) return;   // wave-uniform
    count_apply(i0 + lane_id(), i0, n_total, count, woff, off_id, pk);
}

// Depth-rank order of the packed per-primitive data: pkr[r] = the PrimPack
// of primitive order[r] (its base field is not read from pkr), and the
// count sum of each 64 ranks into wsum_r for the emission's offsets.  One
// gather here lets the emission read coalesced.  The same threads also
// apply the count offsets by primitive index (count_apply), which only the
// backward and this kernel's successors read.
__global__ void __launch_bounds__(256) k_rank_pack(int32_t n_total, const uint32_t* __restrict__ order, PrimPack* pk,
                                                   PrimPack* __restrict__ pkr, uint32_t* __restrict__ wsum_r,
                                                   const uint32_t* __restrict__ count,
                                                   const uint32_t* __restrict__ woff_c, uint32_t* __restrict__ off_id)
{
    const int32_t r0 = (int32_t)(blockIdx.x * 256u + (threadIdx.x & ~63u));   // lane 0 of the wave
    if (r0 >= n_total) return;   // wave-uniform
    const int32_t r = r0 + lane_id();
    uint32_t c = 0;
    if (r < n_total) {
        const PrimPack q = pk[order[r]];
        pkr[r] = q;
        c = q.count;
    }
    const uint32_t ws = wave_sum_u32(c);
    if (lane_id() == 0) wsum_r[r0 >> 6] = ws;
    count_apply(r, r0, n_total, count, woff_c, off_id, pk);
}

// Writes the instances of the primitive of rank r at its offset (woff[r /
// 64], the scanned count sum of the ranks before its wave, plus the counts of
// the lanes before it): key = global tile, value = primitive, tiles of the
// pixel box row-major.  Ranks are primitive indices (order == NULL; pkx =
// per-primitive pack) or depth ranks (pkx = per-rank pack, prim = order[r]).  (An instance's
// gradient slot is its primitive's slot base plus the rank of its tile among
// the primitive's kept tiles; the backward derives it from the pack.)
//
// A wave owns 64 consecutive ranks, whose instances form one contiguous run;
// it walks that run 64 entries at a time and each lane finds its entry's
// primitive by a binary search over the 64 start offsets in LDS, so every
// store is coalesced however uneven the per-primitive counts are.
__global__ void __launch_bounds__(256) k_emit(const ImgDesc* __restrict__ descs, int B, int32_t n_total,
                                               KParams kp, const PrimPack* __restrict__ pkx,
                                               const uint32_t* __restrict__ order,
                                               const uint32_t* __restrict__ woff,
                                               const uint32_t* __restrict__ n_eff, uint32_t* __restrict__ keys,
                                               uint32_t* __restrict__ vals)
{
    __shared__ uint32_t s_start[4][kWave], s_prim[4][kWave], s_base[4][kWave], s_tx[4][kWave], s_w[4][kWave],
        s_mlo[4][kWave], s_mhi[4][kWave], s_full[4][kWave];
    const int w = (int)(threadIdx.x >> 6), l = lane_id();
    const int32_t r0 = (int32_t)(blockIdx.x * 256u + (uint32_t)w * kWave);   // rank of lane 0
    if (r0 >= n_total || *n_eff == 0u) return;   // wave-uniform
    const int32_t r = r0 + l;
    uint32_t c = 0, prim = 0, base = 0, tilesx = 1, wd = 1, mlo = 0, mhi = 0, full = 1;
    if (r < n_total) {
        const PrimPack q = pkx[r];
        prim = order ? order[r] : (uint32_t)r;
        c = q.count;
        if (c) {
            const ImgDesc& d = descs[image_of_prim(descs, B, (int32_t)prim)];
            const int32_t tx0 = lo16(q.box0) >> kp.log2_tw, ty0 = hi16(q.box0) >> kp.log2_th;
            const int32_t tx1 = lo16(q.box1) >> kp.log2_tw;
            wd = (uint32_t)(tx1 - tx0 + 1);
            tilesx = (uint32_t)d.tiles_x;
            base = (uint32_t)(d.tile_begin + ty0 * d.tiles_x + tx0);
            mlo = q.mlo;
            mhi = q.mhi;
            full = q.full;
        }
    }
    const uint32_t first = woff[r0 >> 6];   // offset of lane 0
    uint32_t total;
    const uint32_t ex = wave_excl_scan_u32(c, &total);
    // ranks past the end never match (start beyond every entry)
    s_start[w][l] = r < n_total ? ex : 0xffffffffu;
    s_prim[w][l] = prim;
    s_base[w][l] = base;
    s_tx[w][l] = tilesx;
    s_w[w][l] = wd;
    s_mlo[w][l] = mlo;
    s_mhi[w][l] = mhi;
    s_full[w][l] = full;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint32_t k0 = 0; k0 < total; k0 += kWave) {
        const uint32_t k = k0 + (uint32_t)l;
        if (k >= total) break;
        // largest j with start[j] <= k (start[0] = 0; a rank with no instances
        // shares its start with the next one, which the search prefers)
        int j = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1)
            if (s_start[w][j + step] <= k) j += step;
        const uint32_t local = k - s_start[w][j];
        const uint32_t wj = s_w[w][j];
        // position in the tile rectangle: the local-th kept tile
        const uint32_t at = s_full[w][j] ? local
                                         : nth_set_bit(((uint64_t)s_mhi[w][j] << 32) | s_mlo[w][j], local);
        // approximate quotient (off by at most one while it is below 2^22),
        // corrected to the exact one below
        uint32_t dy = (uint32_t)((float)at * __builtin_amdgcn_rcpf((float)wj));
        if (dy * wj > at) --dy;
        else if ((dy + 1u) * wj <= at) ++dy;
        const uint32_t dx = at - dy * wj;
        const uint32_t o = first + k;
        keys[o] = s_base[w][j] + dy * s_tx[w][j] + dx;
        vals[o] = s_prim[w][j];
    }
}

// ranges[t] = [first, last + 1) of tile t in the sorted keys (pre-zeroed).
// Eight consecutive positions per thread (two 16-byte loads; the keys array
// is 256-byte aligned), with the neighbours of the first and last from memory.
constexpr uint32_t kRangePer = 8;
__global__ void __launch_bounds__(256) k_ranges(const uint32_t* __restrict__ keys,
                                                 const uint32_t* __restrict__ n_eff, uint2* __restrict__ ranges)
{
    const uint32_t s0 = (blockIdx.x * 256u + threadIdx.x) * kRangePer;
    const uint32_t K = *n_eff;
    if (s0 >= K) return;
    uint32_t k[kRangePer];
    if (s0 + kRangePer - 1u < K) {
        const uint4* q = reinterpret_cast<const uint4*>(keys + s0);
#pragma unroll
        for (uint32_t j = 0; j < kRangePer / 4u; ++j) {
            const uint4 x = q[j];
            k[4 * j] = x.x;
            k[4 * j + 1] = x.y;
            k[4 * j + 2] = x.z;
            k[4 * j + 3] = x.w;
        }
    } else {
#pragma unroll
        for (uint32_t j = 0; j < kRangePer; ++j) k[j] = s0 + j < K ? keys[s0 + j] : 0u;
    }
    const bool first_starts = s0 == 0u || keys[s0 - 1u] != k[0];
    const bool last_ends = s0 + kRangePer >= K || keys[s0 + kRangePer] != k[kRangePer - 1u];
#pragma unroll
    for (uint32_t j = 0; j < kRangePer; ++j) {
        const uint32_t s = s0 + j;
        if (s >= K) break;
        const bool starts = j == 0 ? first_starts : k[j - 1] != k[j];
        const bool ends = s == K - 1u || (j == kRangePer - 1u ? last_ends : k[j + 1] != k[j]);
        if (starts) ranges[k[j]].x = s;
        if (ends) ranges[k[j]].y = s + 1u;
    }
}

// Longest-first tile order for the persistent queue: a counting sort of the
// tiles by a log-scale length key, 255 - min(255, floor(16 log2(len + 1))),
// by one workgroup with LDS counters.  Within a key the order is whatever the
// LDS atomics give: any order of the tiles renders the same images and
// gradients, the order only brings the long tiles to the front.
__device__ __forceinline__ uint32_t lpt_key(uint2 r)
{
    const float q = 16.0f * __log2f((float)(r.y - r.x) + 1.0f);
    return 255u - min((uint32_t)q, 255u);
}

// Tiles per thread per round (their range loads issued together, so a
// round costs one memory latency for kLptRound tiles), and tiles per
// workgroup of the two-pass form.
constexpr uint32_t kLptPer = 8, kLptRound = 1024u * kLptPer, kLptSlice = 2u * kLptRound;

template <typename Fn>
__device__ __forceinline__ void lpt_rounds(const uint2* __restrict__ ranges, uint32_t t_begin, uint32_t t_end, Fn fn)
{
    for (uint32_t t0 = t_begin; t0 < t_end; t0 += kLptRound) {
        uint32_t key[kLptPer];
#pragma unroll
        for (uint32_t k = 0; k < kLptPer; ++k) {
            const uint32_t t = t0 + k * 1024u + threadIdx.x;
            key[k] = t < t_end ? lpt_key(ranges[t]) : 0u;
        }
#pragma unroll
        for (uint32_t k = 0; k < kLptPer; ++k) fn(t0 + k * 1024u + threadIdx.x, key[k]);
    }
}

// The key of empty tiles (255; half the tiles of a typical frame) is counted
// and placed once per wave rather than once per lane: per-lane LDS atomics on
// one address serialise.  (Called by whole waves: t_end bounds the tiles.)
__device__ __forceinline__ void lpt_count1(uint32_t t, uint32_t key, uint32_t t_end, uint32_t* s_cnt)
{
    const bool in = t < t_end;
    const uint64_t low = __ballot(in && key == 255u);
    if (in && key != 255u) atomicAdd(&s_cnt[key], 1u);
    if (low && lane_id() == 0) atomicAdd(&s_cnt[255], (uint32_t)__popcll(low));
}

__device__ __forceinline__ void lpt_place1(uint32_t t, uint32_t key, uint32_t t_end, uint32_t* s_cnt,
                                           uint32_t* __restrict__ order)
{
    const int l = lane_id();
    const uint64_t lt = (l == 0) ? 0ull : (~0ull >> (64 - l));
    const bool in = t < t_end;
    const uint64_t low = __ballot(in && key == 255u);
    uint32_t at = 0u;
    if (low && l == 0) at = atomicAdd(&s_cnt[255], (uint32_t)__popcll(low));
    at = (uint32_t)__shfl((int)at, 0, kWave);
    if (in) order[key == 255u ? at + (uint32_t)__popcll(low & lt) : atomicAdd(&s_cnt[key], 1u)] = t;
}

__device__ __forceinline__ void lpt_count(const uint2* __restrict__ ranges, uint32_t t_begin, uint32_t t_end,
                                          uint32_t* s_cnt)
{
    lpt_rounds(ranges, t_begin, t_end, [&](uint32_t t, uint32_t key) { lpt_count1(t, key, t_end, s_cnt); });
}

__device__ __forceinline__ void lpt_place(const uint2* __restrict__ ranges, uint32_t t_begin, uint32_t t_end,
                                          uint32_t* s_cnt, uint32_t* __restrict__ order)
{
    lpt_rounds(ranges, t_begin, t_end, [&](uint32_t t, uint32_t key) { lpt_place1(t, key, t_end, s_cnt, order); });
}

// Exclusive scan of the 256 counts in place, by the first wave (four per lane).
__device__ __forceinline__ void lpt_scan(uint32_t* s_cnt)
{
    if (threadIdx.x >= kWave) return;
    const uint32_t l = threadIdx.x;
    uint32_t c[4], sum = 0u, tot;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        c[k] = s_cnt[4u * l + k];
        sum += c[k];
    }
    uint32_t ex = wave_excl_scan_u32(sum, &tot);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        s_cnt[4u * l + k] = ex;
        ex += c[k];
    }
}

// Up to kLptSlice tiles: one workgroup counts, scans and places.
__global__ void __launch_bounds__(1024) k_tile_lpt_order(const uint2* __restrict__ ranges, uint32_t n_tiles,
                                                         uint32_t* __restrict__ order)
{
    __shared__ uint32_t s_cnt[256];
    if (threadIdx.x < 256) s_cnt[threadIdx.x] = 0u;
    // the keys of all (at most kLptSlice) tiles, read once for both phases
    constexpr uint32_t R = kLptSlice / kLptRound;
    uint32_t key[R][kLptPer];
#pragma unroll
    for (uint32_t r = 0; r < R; ++r)
#pragma unroll
        for (uint32_t k = 0; k < kLptPer; ++k) {
            const uint32_t t = r * kLptRound + k * 1024u + threadIdx.x;
            key[r][k] = t < n_tiles ? lpt_key(ranges[t]) : 0u;
        }
    __syncthreads();
#pragma unroll
    for (uint32_t r = 0; r < R; ++r)
#pragma unroll
        for (uint32_t k = 0; k < kLptPer; ++k)
            lpt_count1(r * kLptRound + k * 1024u + threadIdx.x, key[r][k], n_tiles, s_cnt);
    __syncthreads();
    lpt_scan(s_cnt);
    __syncthreads();
#pragma unroll
    for (uint32_t r = 0; r < R; ++r)
#pragma unroll
        for (uint32_t k = 0; k < kLptPer; ++k)
            lpt_place1(r * kLptRound + k * 1024u + threadIdx.x, key[r][k], n_tiles, s_cnt, order);
}

// More tiles: workgroup g counts the keys of slice g into counts[g][256] ...
__global__ void __launch_bounds__(1024) k_tile_lpt_count(const uint2* __restrict__ ranges, uint32_t n_tiles,
                                                         uint32_t* __restrict__ counts)
{
    __shared__ uint32_t s_cnt[256];
    if (threadIdx.x < 256) s_cnt[threadIdx.x] = 0u;
    __syncthreads();
    const uint32_t b = blockIdx.x * kLptSlice;
    lpt_count(ranges, b, min(n_tiles, b + kLptSlice), s_cnt);
    __syncthreads();
    if (threadIdx.x < 256) counts[blockIdx.x * 256u + threadIdx.x] = s_cnt[threadIdx.x];
}

// ... then places slice g: a key's tiles start after every smaller key's and
// after those of slices before g.
__global__ void __launch_bounds__(1024) k_tile_lpt_place(const uint2* __restrict__ ranges, uint32_t n_tiles,
                                                         const uint32_t* __restrict__ counts, uint32_t n_slices,
                                                         uint32_t* __restrict__ order)
{
    __shared__ uint32_t s_cnt[256], s_pre[256];
    if (threadIdx.x < 256) {
        uint32_t tot = 0u, pre = 0u;
        for (uint32_t g = 0; g < n_slices; ++g) {
            const uint32_t c = counts[g * 256u + threadIdx.x];
            tot += c;
            pre += g < blockIdx.x ? c : 0u;
        }
        s_cnt[threadIdx.x] = tot;
        s_pre[threadIdx.x] = pre;
    }
    __syncthreads();
    lpt_scan(s_cnt);
    __syncthreads();
    if (threadIdx.x < 256) s_cnt[threadIdx.x] += s_pre[threadIdx.x];
    __syncthreads();
    const uint32_t b = blockIdx.x * kLptSlice;
    lpt_place(ranges, b, min(n_tiles, b + kLptSlice), s_cnt, order);
}

// Fill kernel (used instead of memset so the sequence can live in a graph).
__global__ void __launch_bounds__(256) k_fill_u32(uint32_t* __restrict__ p, uint32_t n, uint32_t v)
{
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < n) p[i] = v;
}

// Two fills in one launch: p[0..n) then q[0..m).
__global__ void __launch_bounds__(256) k_fill2_u32(uint32_t* __restrict__ p, uint32_t n, uint32_t* __restrict__ q,
                                                    uint32_t m, uint32_t v)
{
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < n) p[i] = v;
    else if (i - n < m) q[i - n] = v;
}

// ------------------------------------------------------------- host side

static inline uint32_t blocks_of(uint32_t n) { return (n + 255u) / 256u; }

hipError_t launch_fill2_u32(uint32_t* p, uint32_t n, uint32_t* q, uint32_t m, uint32_t v, hipStream_t s);

hipError_t launch_bin_count(const ImgDesc* descs, int B, int32_t n_total, const KParams& kp, Rec* recs,
                            const void* aux, uint32_t* count, PrimPack* pk, uint32_t* dkey, uint32_t* dval,
                            uint32_t* wsum, const Clear2& clr, hipStream_t s)
{
    if (n_total > 0)
        hipLaunchKernelGGL(k_bin_count, dim3(blocks_of((uint32_t)n_total)), dim3(256), 0, s, descs, B, n_total, kp,
                           recs, (const Aux*)aux, count, pk, dkey, dval, wsum, clr);
    else
        return launch_fill2_u32(clr.p0, clr.n0, clr.p1, clr.n1, 0u, s);
    return hipGetLastError();
}

hipError_t launch_count_apply(int32_t n_total, const uint32_t* count, const uint32_t* woff, uint32_t* off_id,
                              PrimPack* pk, hipStream_t s)
{
    if (n_total > 0)
        hipLaunchKernelGGL(k_count_apply, dim3(blocks_of((uint32_t)n_total)), dim3(256), 0, s, n_total, count, woff,
                           off_id, pk);
    return hipGetLastError();
}

hipError_t launch_rank_pack(int32_t n_total, const uint32_t* order, PrimPack* pk, PrimPack* pkr, uint32_t* wsum_r,
                            const uint32_t* count, const uint32_t* woff_c, uint32_t* off_id, hipStream_t s)
{
    if (n_total > 0)
        hipLaunchKernelGGL(k_rank_pack, dim3(blocks_of((uint32_t)n_total)), dim3(256), 0, s, n_total, order, pk,
                           pkr, wsum_r, count, woff_c, off_id);
    return hipGetLastError();
}

hipError_t launch_emit(const ImgDesc* descs, int B, int32_t n_total, const KParams& kp, const PrimPack* pkx,
                       const uint32_t* order, const uint32_t* woff, const uint32_t* n_eff, uint32_t* keys,
                       uint32_t* vals, hipStream_t s)
{
    if (n_total > 0)
        hipLaunchKernelGGL(k_emit, dim3(blocks_of((uint32_t)n_total)), dim3(256), 0, s, descs, B, n_total, kp, pkx,
                           order, woff, n_eff, keys, vals);
    return hipGetLastError();
}

uint32_t lpt_slices(uint32_t n_tiles) { return (n_tiles + kLptSlice - 1u) / kLptSlice; }

hipError_t launch_tile_lpt_order(const uint2* ranges, uint32_t n_tiles, uint32_t* counts, uint32_t* order,
                                 hipStream_t s)
{
    if (n_tiles == 0) return hipGetLastError();
    const uint32_t g = lpt_slices(n_tiles);
    if (g <= 1) {
        hipLaunchKernelGGL(k_tile_lpt_order, dim3(1), dim3(1024), 0, s, ranges, n_tiles, order);
    } else {
        hipLaunchKernelGGL(k_tile_lpt_count, dim3(g), dim3(1024), 0, s, ranges, n_tiles, counts);
        hipLaunchKernelGGL(k_tile_lpt_place, dim3(g), dim3(1024), 0, s, ranges, n_tiles, counts, g, order);
    }
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t n, uint32_t v, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_u32, dim3(blocks_of(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill2_u32(uint32_t* p, uint32_t n, uint32_t* q, uint32_t m, uint32_t v, hipStream_t s)
{
    if (!q) m = 0;
    if (!p) n = 0;
    if ((uint64_t)n + m >= (1ull << 32)) {
        const hipError_t e = launch_fill_u32(p, n, v, s);
        return e != hipSuccess ? e : launch_fill_u32(q, m, v, s);
    }
    if (n + m > 0) hipLaunchKernelGGL(k_fill2_u32, dim3(blocks_of(n + m)), dim3(256), 0, s, p, n, q, m, v);
    return hipGetLastError();
}

hipError_t launch_ranges(const uint32_t* keys, const uint32_t* n_eff, uint32_t max_k, uint2* ranges, hipStream_t s)
{
    if (max_k > 0)
        hipLaunchKernelGGL(k_ranges, dim3(blocks_of((max_k + kRangePer - 1u) / kRangePer)), dim3(256), 0, s, keys,
                           n_eff, ranges);
    return hipGetLastError();
}

}  // namespace wipes
