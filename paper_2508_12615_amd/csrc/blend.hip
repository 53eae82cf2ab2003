// Per-tile blending of wavelet primitives, forward and backward, for gfx950.
//
// Paper: W' of Eq. 7 (Sec. 4.1) blended by Eq. 4 (additive, 2D fitting) or by
// Eq. 3 (front-to-back alpha compositing, view synthesis).
//
// Work decomposition (both modes):
//  * every 8 x 8 block of a tile gets its own wave (the tile is one
//    workgroup), lane l holding pixel (l & 7, l >> 3) of the block, so the
//    serial walk of a long list is split four ways (16 x 16 tiles) without
//    lengthening the sort, and a small frame still fills the machine;
//  * the wave walks the tile's list in chunks of 64 entries: each lane
//    gathers one entry's record (vector loads; the next chunk's entries and
//    records are in flight while the current chunk blends), tests its pixel
//    box and padded support ellipse against the bounding box of the block
//    pixels still in play, and the hits are packed (ballot + prefix count)
//    into a per-wave LDS stage holding
//    their block-relative, pre-scaled values.  The wave then blends the staged
//    primitives in list order; all lanes read the same LDS address, which the
//    LDS broadcasts.  A primitive that misses the block costs one lane of one
//    box test instead of a serial round trip through memory;
//  * alpha mode shrinks the box as pixels terminate and leaves when none is
//    left (lists are long and skewed in clustered scenes, and pixels stop
//    early); additive mode keeps the box of the block's pixels;
//  * the forward records, per block and list position, whether the
//    primitive contributed to a pixel of the block; the backward walks the
//    same chunks top down (alpha: from the tile's last contributing position)
//    with all block waves in step, replays only the recorded contributors,
//    each wave reducing a primitive's twelve per-pair basis sums over its
//    block into LDS, and the workgroup sums the blocks in a fixed order into
//    the instance's slot.
//
// Gradient slots are numbered in primitive order (an instance's slot is its
// primitive's slot base plus the rank of its tile among the primitive's kept
// tiles), so the projection backward sums a primitive's slots from one
// contiguous run in a fixed order: gradients are deterministic, atomic-free
// and independent of the batch a primitive is rendered in.
//
// Per-pair rule (shared by forward and backward so their FP32 decisions agree
// bit for bit): e2 = -q/2 log2(e) from the pre-scaled conic, E = exp2(e2),
// phase in revolutions ph = (f'/2pi).d + phi0/2pi, K = (1 + cos 2pi ph)/2,
// W' = K E.
#include "common.hpp"

// Multiply-adds within one expression fuse into FMAs here (the rest of the
// library builds with contraction off).  Every include/stop decision goes
// through eval_at, whose arithmetic is spelled out with fmaf, so the forward
// and the backward still take identical decisions; only the rounding of the
// colour and gradient sums changes.
#pragma clang fp contract(on)

namespace wipes {

constexpr int kWpb = 4;   // waves (tiles) per workgroup of the work-counting kernel

// Per-primitive, wave-uniform values (work counting).
struct PrimU {
    float mrx, mry;       // mean relative to the tile origin
    float ca2, cb2, cc2;  // conic scaled by -log2(e)/2 (cb2 includes the factor 2)
    float fxr, fyr;       // frequency in revolutions per pixel
    float ph0;            // carrier phase in revolutions
    float op, r, g, b;
    float ca, cb, cc, fx, fy;   // raw values for the backward
};

constexpr float kConicScale = -0.5f * kLog2e;
constexpr float kTwoLn2 = 1.3862943611198906f;

__device__ __forceinline__ PrimU load_prim(const Rec* __restrict__ recs, uint32_t prim, int ox, int oy,
                                           uint32_t* box0, uint32_t* box1)
{
    const Rec R = recs[prim];
    PrimU u;
    u.mrx = (R.mx - (float)ox) + R.mxl;
    u.mry = (R.my - (float)oy) + R.myl;
    u.ca2 = R.ca * kConicScale;
    u.cb2 = R.cb * (2.0f * kConicScale);
    u.cc2 = R.cc * kConicScale;
    u.fxr = R.fx * kInv2Pi;
    u.fyr = R.fy * kInv2Pi;
    u.ph0 = R.ph;
    u.op = R.op;
    u.r = R.r; u.g = R.g; u.b = R.b;
    u.ca = R.ca; u.cb = R.cb; u.cc = R.cc; u.fx = R.fx; u.fy = R.fy;
    *box0 = R.box0;
    *box1 = R.box1;
    return u;
}

// One (pixel, primitive) evaluation: offsets from the mean, e2 = the
// Gaussian's base-2 exponent minus one, E = exp2(e2) (half the Gaussian
// factor), the phase in turns and W = E (1 + cos phi), which is W' (the
// Gaussian times the raised cosine (1 + cos phi) / 2).  Taking the half
// into the exponent, where the last product of the quadratic form becomes a
// fused multiply-add, saves the instruction that would scale the cosine.
struct PairEval {
    float dx, dy, e2, E, ph, W;
};

__device__ __forceinline__ PairEval eval_at(float mrx, float mry, float ca2, float cb2, float cc2, float fxr, float fyr,
                                            float ph0, float lx, float ly)
{
    PairEval p;
    p.dx = lx - mrx;
    p.dy = ly - mry;
    const float t = fmaf(ca2, p.dx, cb2 * p.dy);
    p.e2 = fmaf(t, p.dx, fmaf(cc2 * p.dy, p.dy, -1.0f));
    p.ph = fmaf(fxr, p.dx, fmaf(fyr, p.dy, ph0));
    p.E = __builtin_amdgcn_exp2f(p.e2);
    p.W = fmaf(p.E, __builtin_amdgcn_cosf(__builtin_amdgcn_fractf(p.ph)), p.E);
    return p;
}

__device__ __forceinline__ PairEval eval_pair(const PrimU& u, float lx, float ly)
{
    return eval_at(u.mrx, u.mry, u.ca2, u.cb2, u.cc2, u.fxr, u.fyr, u.ph0, lx, ly);
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

// Map a wave to its tile (work counting, one wave per tile).  Workgroups are
// remapped so that each of the 8 XCDs (which receive workgroups round-robin)
// walks a contiguous band of tiles.
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

// Next tile from the persistent queue (called by one thread): counter
// `lane` first, then the others in turn once it runs dry, so every tile is
// handed out exactly once and a workgroup never waits on an empty lane while
// another has work.  Returns n_tiles when all are taken.
__device__ __forceinline__ uint32_t pull_tile(uint32_t* __restrict__ queue, uint32_t n_tiles,
                                              const uint32_t* __restrict__ order, uint32_t& lane)
{
    for (int tries = 0; tries < kQueueLanes; ++tries) {
        const uint32_t x = (lane + (uint32_t)tries) % kQueueLanes;
        const uint32_t nx = n_tiles > x ? (n_tiles - x + kQueueLanes - 1) / kQueueLanes : 0u;
        if (nx == 0) continue;
        const uint32_t j = atomicAdd(queue + x * kQueueStride, 1u);
        if (j < nx) {
            lane = x;
            const uint32_t i = x + kQueueLanes * j;
            return order ? order[i] : i;
        }
    }
    return n_tiles;
}

// Issue priority of a wave by its tile's list length: the kernels' time is
// set by the serial walk of the heaviest tiles, so their waves go first on a
// shared SIMD and lighter waves fill the gaps.
__device__ __forceinline__ void prioritise(uint32_t len)
{
    if (len >= 4096u) __builtin_amdgcn_s_setprio(3);
    else if (len >= 1024u) __builtin_amdgcn_s_setprio(2);
    else if (len >= 256u) __builtin_amdgcn_s_setprio(1);
    else __builtin_amdgcn_s_setprio(0);
}

// ------------------------------------------------------------ block waves

// One staged primitive (48 bytes), with the conic and the frequency
// pre-scaled as load_prim does; forward and backward stage the same values,
// so both passes take identical FP32 decisions.  A staged primitive's list position is not
// stored: the j-th staged entry is the j-th set bit of the chunk's hit mask,
// which the (wave-uniform) loops walk with scalar bit scans.
struct __align__(16) Staged {
    float mrx, mry;     // mean relative to the block origin
    float c0, c1, c2;   // conic
    float f0, f1;       // frequency
    float ph;           // carrier phase (revolutions)
    float op, r, g, b;
};
static_assert(sizeof(Staged) == 48, "staged record must be 48 bytes");

struct PixBox {
    int x0, y0, x1, y1;
};

// Bounding box (image pixels) of the set lanes of the ballot m of an 8 x 8
// block at (bx, by) whose lane l holds pixel (l & 7, l >> 3): columns are the
// OR of the eight bytes, rows the non-zero bytes -- scalar bit operations
// only.  An empty set gives an inverted box that no primitive meets.
__device__ __forceinline__ PixBox block_box(uint64_t m, int bx, int by)
{
    PixBox b;
    if (m == 0ull) {
        b.x0 = b.y0 = 1 << 20;
        b.x1 = b.y1 = -(1 << 20);
        return b;
    }
    uint64_t t = m | (m >> 32);
    t |= t >> 16;
    t |= t >> 8;
    const uint32_t cols = (uint32_t)t & 0xffu;
    uint32_t rows = 0;
#pragma unroll
    for (int r = 0; r < 8; ++r) rows |= ((m >> (8 * r)) & 0xffull) ? (1u << r) : 0u;
    b.x0 = bx + __builtin_ctz(cols);
    b.x1 = bx + 31 - __builtin_clz(cols);
    b.y0 = by + __builtin_ctz(rows);
    b.y1 = by + 31 - __builtin_clz(rows);
    return b;
}

__device__ __forceinline__ bool box_meets(uint32_t b0, uint32_t b1, const PixBox& q)
{
    return lo16(b0) <= q.x1 && lo16(b1) >= q.x0 && hi16(b0) <= q.y1 && hi16(b1) >= q.y0;
}

// Whether the support ellipse {q(x) <= Qs} of record R can reach a pixel
// centre of the box q (image pixels): the minimum of the convex quadratic
// q(x) = ca dx^2 + 2 cb dx dy + cc dy^2 over the centre rectangle is 0 if the
// mean lies inside, else it lies on an edge, where it is a clamped 1-D
// minimum.  Qs carries a margin over the blend's own threshold, so a pixel
// the blend would accept is never dropped.
__device__ __forceinline__ bool ellipse_meets(const Rec& R, const PixBox& q, float Qs)
{
    const float mx = R.mx + R.mxl, my = R.my + R.myl;
    const float x0 = (float)q.x0 + 0.5f, x1 = (float)q.x1 + 0.5f;
    const float y0 = (float)q.y0 + 0.5f, y1 = (float)q.y1 + 0.5f;
    // (branch-free: every lane evaluates the whole test)
    const bool inside = (mx >= x0) & (mx <= x1) & (my >= y0) & (my <= y1);
    const float sy = -R.cb * __builtin_amdgcn_rcpf(R.cc), sx = -R.cb * __builtin_amdgcn_rcpf(R.ca);
    auto qv = [&](float dx, float dy) { return fmaf(R.ca * dx, dx, fmaf(2.0f * R.cb * dx, dy, R.cc * dy * dy)); };
    const float dxa = x0 - mx, dxb = x1 - mx, dya = y0 - my, dyb = y1 - my;
    float m = qv(dxa, fminf(fmaxf(sy * dxa, dya), dyb));
    m = fminf(m, qv(dxb, fminf(fmaxf(sy * dxb, dya), dyb)));
    m = fminf(m, qv(fminf(fmaxf(sx * dya, dxa), dxb), dya));
    m = fminf(m, qv(fminf(fmaxf(sx * dyb, dxa), dxb), dyb));
    return inside | (m <= Qs);
}

// box0 of a lane past the end of a chunk: x0 = y0 = 65535 lies beyond every
// image (pixel coordinates stay below 2^15), so it meets no pixel box.
constexpr uint32_t kNoBox = 0xffffffffu;

__device__ __forceinline__ Staged stage_fwd(const Rec& R, int bx, int by)
{
    Staged w;
    w.mrx = (R.mx - (float)bx) + R.mxl;
    w.mry = (R.my - (float)by) + R.myl;
    w.c0 = R.ca * kConicScale;
    w.c1 = R.cb * (2.0f * kConicScale);
    w.c2 = R.cc * kConicScale;
    w.f0 = R.fx * kInv2Pi;
    w.f1 = R.fy * kInv2Pi;
    w.ph = R.ph;
    w.op = R.op;
    w.r = R.r;
    w.g = R.g;
    w.b = R.b;
    return w;
}

// Additive forward: colour premultiplied by the opacity (Eq. 4's weight).
__device__ __forceinline__ Staged stage_add(const Rec& R, int bx, int by)
{
    Staged w = stage_fwd(R, bx, by);
    w.r = R.r * R.op;
    w.g = R.g * R.op;
    w.b = R.b * R.op;
    return w;
}

// Forward of one 8 x 8 block `blk` of tile t (one wave).  Additive mode
// tests primitives against the box of the block's pixels inside the image;
// alpha mode against the box of its pixels still transmitting, which shrinks
// as pixels terminate.
template <int MODE, int TW, int TH>
__device__ __forceinline__ void fwd_block(const ImgDesc* __restrict__ descs, int B, const KParams& kp,
                                          const Rec* __restrict__ recs, const uint32_t* __restrict__ vals,
                                          const uint2* __restrict__ ranges, uint32_t t, int blk,
                                          float* __restrict__ image, float* __restrict__ T_final,
                                          int32_t* __restrict__ last, unsigned long long* __restrict__ cmask,
                                          uint32_t cmask_words, Staged* __restrict__ stage)
{
    const TileGeo G = tile_geo(descs, B, ranges, t, TW, TH);
    prioritise(G.end - G.start);
    const ImgDesc& d = descs[G.b];
    const int l = lane_id();
    const int bx = G.ox + (blk % (TW / 8)) * 8, by = G.oy + (blk / (TW / 8)) * 8;
    const int px = bx + (l & 7), py = by + (l >> 3);
    const bool valid = px < d.W && py < d.H;
    if (__ballot(valid) == 0ull) return;   // block past the image edge
    const float lx = (float)(l & 7) + 0.5f, ly = (float)(l >> 3) + 0.5f;
    const uint64_t below = (1ull << l) - 1ull;
    float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, T = 1.0f;
    int32_t lst = -1;
    // the block's pixels still transmitting, as a wave mask (scalar registers)
    const uint64_t vm = __builtin_amdgcn_ballot_w64(valid);
    uint64_t am = vm;
    PixBox live = block_box(am, bx, by);
    const float thr2 = fmaf(kp.q_add, kConicScale, -1.0f);   // support test on e2 (exponent minus one)
    const float lg2_amin = __builtin_amdgcn_logf(kp.alpha_min);
    unsigned long long* cm_row = cmask ? cmask + (size_t)blk * cmask_words : nullptr;
    if (G.start < G.end) {
        const uint32_t e1 = G.end - 1u;
        // Chunks are the 64-position words of the global list ([base, base +
        // 64) with base a multiple of 64, clipped to the tile's range), so a
        // chunk's contribution bits form one word of the mask.  Lane l holds
        // position base + l.  Records of the current chunk and list entries of
        // the next one are loaded ahead.
        uint32_t base = G.start & ~63u;
        Rec cur = recs[vals[min(max(base + (uint32_t)l, G.start), e1)]];
        if (base + (uint32_t)l < G.start || base + (uint32_t)l > e1) cur.box0 = kNoBox;
        uint32_t pn = vals[min(base + (uint32_t)(kWave + l), e1)];
        for (;;) {
            // support threshold with margin: additive q <= q_add; alpha
            // o W' >= alpha_min needs q <= 2 ln(o / alpha_min) = 2 ln 2 (log2 o - log2 alpha_min)
            // (W' <= G'); the hardware log2 is within a few ulp, far inside the margin
            const float Qs = (MODE == WIPES_2D_ADDITIVE ? kp.q_add
                                                        : kTwoLn2 * (__builtin_amdgcn_logf(cur.op) - lg2_amin)) *
                                 1.001f +
                             1e-3f;
            const bool hit = box_meets(cur.box0, cur.box1, live) & ellipse_meets(cur, live, Qs);
            const uint64_t m = __ballot(hit);
            if (hit)
                stage[__popcll(m & below)] = MODE == WIPES_2D_ADDITIVE ? stage_add(cur, bx, by) : stage_fwd(cur, bx, by);
            const uint32_t cn = base + kWave;
            const bool more = cn < G.end;
            Rec nx{};
            if (more) {   // the next chunk is in flight while this one blends
                nx = recs[pn];
                if (cn + (uint32_t)l > e1) nx.box0 = kNoBox;
                pn = vals[min(cn + (uint32_t)(kWave + l), e1)];
            }
            wave_lds_sync();
            bool left = true;
            uint64_t contrib = 0;   // bit (pos & 63): the primitive at pos contributed to a pixel of the block
            uint64_t rest = m;      // staged positions not yet blended (bit = position - base)
            // the staged entries in order: the k-th set bit of the hit mask is
            // stage[k]; the loop runs while bits are left (scalar work per
            // step matters here: the SIMD's scalar issue is shared with the
            // other waves of the block's CU)
            const Staged* sp = stage;
            const uint64_t am0 = am;
            while (rest) {
                const Staged S = *sp++;
                const uint32_t bp = (uint32_t)__builtin_ctzll(rest);   // this entry's position - base
                const uint64_t bit = 1ull << bp;
                rest ^= bit;
                const float cr = S.r, cg = S.g, cb = S.b;
                const PairEval p = eval_at(S.mrx, S.mry, S.c0, S.c1, S.c2, S.f0, S.f1, S.ph, lx, ly);
                if constexpr (MODE == WIPES_2D_ADDITIVE) {
                    const bool in = p.e2 >= thr2;
                    const float w = in ? p.W : 0.0f;
                    C0 = fmaf(S.r, w, C0);
                    C1 = fmaf(S.g, w, C1);
                    C2 = fmaf(S.b, w, C2);
                    if (__builtin_amdgcn_ballot_w64(in) & vm) contrib |= bit;
                    continue;
                }
                const float a = S.op * p.W;
                // the pixels the pair adds to and the pixels it ends, as wave
                // masks: lane conditions combined with AND stay in scalar
                // registers instead of round trips through vector booleans
                const uint64_t addm = am & __builtin_amdgcn_ballot_w64(a >= kp.alpha_min);
                const bool adds = __builtin_amdgcn_inverse_ballot_w64(addm);
                // branch-free: a pair that does not add gets alpha 0, for which
                // the colour, T and `last` updates are exact identities
                const float al = adds ? __builtin_amdgcn_fmed3f(a, 0.0f, kp.alpha_max) : 0.0f;
                const float wt = T * al;
                C0 = fmaf(wt, cr, C0);
                C1 = fmaf(wt, cg, C1);
                C2 = fmaf(wt, cb, C2);
                T = T - wt;   // T (1 - al)
                lst = adds ? (int32_t)(base + bp) : lst;
                contrib |= addm ? bit : 0ull;
                const uint64_t diedm = addm & __builtin_amdgcn_ballot_w64(T < kp.T_min);
                if (diedm) {
                    am &= ~diedm;
                    if (am == 0ull) {   // every pixel has ended: no entry is left to blend
                        left = false;
                        rest = 0ull;
                    }
                }
            }
            // the box of the pixels still transmitting, for the next chunk's
            // prefilter: once per chunk, not at every pixel's end
            if (left && am != am0) live = block_box(am, bx, by);
            // a word can be shared with the neighbouring tile's list: OR, not store
            if (cm_row && contrib && l == 0) atomicOr(cm_row + (base >> 6), (unsigned long long)contrib);
            if (!left || !more) break;
            wave_lds_sync();   // the stage is rewritten next
            cur = nx;
            base = cn;
        }
    }
    if (valid) {
        const uint32_t pix = (uint32_t)d.pix_begin + (uint32_t)(py * d.W + px);
        float* o = d.out_image ? d.out_image + 3 * (pix - (uint32_t)d.pix_begin) : image + 3 * pix;
        if constexpr (MODE == WIPES_2D_ADDITIVE) {
            o[0] = C0;
            o[1] = C1;
            o[2] = C2;
        } else {
            o[0] = fmaf(T, kp.bg[0], C0);
            o[1] = fmaf(T, kp.bg[1], C1);
            o[2] = fmaf(T, kp.bg[2], C2);
            T_final[pix] = T;
            last[pix] = lst;
        }
    }
}

// Grid form: one workgroup per tile, one wave per block.  Tiles map to
// workgroups one to one, so the XCDs (which take workgroups round-robin)
// share the heavy tiles of a cluster instead of one XCD taking a whole band.
// With `order` (a permutation of the tiles, longest list first) workgroup i
// takes tile order[i]: the hardware dispatcher, which starts workgroups in
// index order as earlier ones retire, then hands out the heavy tiles first
// with no queue atomics and no workgroup barrier between tiles.
template <int MODE, int TW, int TH>
__global__ void __launch_bounds__(TW * TH) k_blend_fwd(const ImgDesc* __restrict__ descs, int B, KParams kp,
                                                             const Rec* __restrict__ recs,
                                                             const uint32_t* __restrict__ vals,
                                                             const uint2* __restrict__ ranges,
                                                             const uint32_t* __restrict__ ovf, uint32_t n_tiles,
                                                             float* __restrict__ image, float* __restrict__ T_final,
                                                             int32_t* __restrict__ last,
                                                             unsigned long long* __restrict__ cmask,
                                                             uint32_t cmask_words, const uint32_t* __restrict__ order)
{
    __shared__ Staged stage[(TW / 8) * (TH / 8)][kWave];
    if (*ovf) return;
    if (blockIdx.x >= n_tiles) return;
    const uint32_t t = order ? order[blockIdx.x] : blockIdx.x;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    fwd_block<MODE, TW, TH>(descs, B, kp, recs, vals, ranges, t, w, image, T_final, last, cmask, cmask_words,
                            stage[w]);
}

// Persistent form: each workgroup pulls whole tiles from the queue (tiles in
// `order`, longest list first, when given).
template <int MODE, int TW, int TH>
__global__ void __launch_bounds__(TW * TH) k_blend_fwd_q(const ImgDesc* __restrict__ descs, int B, KParams kp,
                                                         const Rec* __restrict__ recs,
                                                         const uint32_t* __restrict__ vals,
                                                         const uint2* __restrict__ ranges,
                                                         const uint32_t* __restrict__ ovf, uint32_t n_tiles,
                                                         const uint32_t* __restrict__ order,
                                                         uint32_t* __restrict__ queue, float* __restrict__ image,
                                                         float* __restrict__ T_final, int32_t* __restrict__ last,
                                                         unsigned long long* __restrict__ cmask,
                                                         uint32_t cmask_words)
{
    constexpr int NB = (TW / 8) * (TH / 8);
    __shared__ Staged stage[NB][kWave];
    __shared__ uint32_t qtile;
    if (*ovf) return;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    uint32_t lane = blockIdx.x % kQueueLanes;
    for (;;) {
        if (threadIdx.x == 0) qtile = pull_tile(queue, n_tiles, order, lane);
        __syncthreads();
        const uint32_t t = qtile;
        __syncthreads();   // every wave has read `qtile` before it is rewritten
        if (t >= n_tiles) break;
        fwd_block<MODE, TW, TH>(descs, B, kp, recs, vals, ranges, t, w, image, T_final, last, cmask, cmask_words,
                                stage[w]);
    }
}

// Sum 12 per-lane values over the wave with a halving butterfly on VALU
// cross-lane paths only (no LDS round trips): each step pairs lanes, keeps
// part of the values and adds the partner's copy of that part.  gfx950's
// permlane32/permlane16 swaps exchange the two halves / row pairs of two
// registers in one instruction (12 -> 6 -> 3 values per lane), and DPP
// row_mirror, row_half_mirror and quad_perm pair lanes inside a 16-lane row.
// Pairing lanes by a mirror flips several low bits at once, which is still a
// valid butterfly as long as the lanes that keep a value are chosen by the
// bit the pairing flips last.  The three values left in a row end in lanes
// 0-3 (first), 4-7 (second) and 8-15 (third) of that row, so lane l returns
// the wave total of value reduce12_index(l).
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

__device__ __forceinline__ float wave_reduce12_valu(const float v[12])
{
    const int l = lane_id();
    float u[6], w[3];
#pragma unroll
    for (int j = 0; j < 6; ++j) {   // lanes 0-31 keep v[j], lanes 32-63 keep v[j + 6]
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(v[j]), __float_as_int(v[j + 6]), false, false);
        u[j] = __int_as_float(r[0]) + __int_as_float(r[1]);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {   // even rows keep u[j], odd rows keep u[j + 3]
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(u[j]), __float_as_int(u[j + 3]), false, false);
        w[j] = __int_as_float(r[0]) + __int_as_float(r[1]);
    }
    // row_mirror pairs i with 15 - i: lanes 0-7 go on with w[0] and w[1], lanes 8-15 with w[2]
    const float a0 = w[0] + dpp_mov<0x140>(w[0]);
    const float a1 = w[1] + dpp_mov<0x140>(w[1]);
    const float a2 = w[2] + dpp_mov<0x140>(w[2]);
    const float x = (l & 8) ? a2 : a0;
    // row_half_mirror pairs i with 7 - i inside each half row: lanes 4-7 keep the second value
    const float xs = x + dpp_mov<0x141>(x);
    const float ys = a1 + dpp_mov<0x141>(a1);
    float t = ((l & 12) == 4) ? ys : xs;
    t += dpp_mov<0x4e>(t);   // quad_perm [2, 3, 0, 1]
    t += dpp_mov<0xb1>(t);   // quad_perm [1, 0, 3, 2]
    return t;
}

// Which of the 12 values wave_reduce12_valu leaves in lane l; lanes whose
// (l & 15) is 0, 4 or 8 are the first of their group.
__device__ __forceinline__ int reduce12_index(int l)
{
    const int i = l & 15;
    return 6 * (l >> 5) + 3 * ((l >> 4) & 1) + (i < 4 ? 0 : i < 8 ? 1 : 2);
}

// ------------------------------------------------------------ backward

// Gradient slot layout per instance: 12 floats, sums over the pixels of the
// tile of (dq dx, dq dy, dq dx^2, dq dx dy, dq dy^2, dphi dx, dphi dy,
// dL/do, dL/dr, dL/dg, dL/db, dphi), with dq = dL/dq, dphi = dL/dphi and
// (dx, dy) the pixel's offset from the mean.  The gradients with respect to
// mu', the conic and f' are linear in these sums with the primitive's own
// conic and f' as coefficients (dL/dmu'x = -2 (ca S_qx + cb S_qy) - f'x S_phi,
// dL/dcb = 2 S_qxy, ...), so the projection backward applies them once per
// primitive instead of every pair paying for them.  The same holds for the
// opacity factors: with d = dL/d(o W') of the pair, G the Gaussian factor
// and W' = G (1 + cos phi) / 2, dL/dq = -o/2 W' d and dL/dphi =
// -o/2 G sin(phi) d = -o (G/2) sin(phi) d.  The slots hold the dq terms (the
// first five values) without -o/2 and the dphi terms (values 5, 6 and the
// last), built from the evaluation's G/2, without -o; the projection
// backward multiplies them by -o/2 and -o.
constexpr int kSlot = 12;

// Per-pair gradient terms shared by both modes: d = dL/d(o W') of the pair,
// v[7] = W' d already set (the opacity term, which is also dq / (-o/2)).
__device__ __forceinline__ void pair_grads(float v[12], const PairEval& p, float d)
{
    const float sn = __builtin_amdgcn_sinf(__builtin_amdgcn_fractf(p.ph));
    const float dq = v[7];                 // dL/dq / (-o/2)
    const float dph = (p.E * sn) * d;      // dL/dphi (radians) / (-o): p.E is half the Gaussian factor
    const float qx = dq * p.dx, qy = dq * p.dy;
    v[0] = qx;
    v[1] = qy;
    v[2] = qx * p.dx;
    v[3] = qx * p.dy;
    v[4] = qy * p.dy;
    v[5] = dph * p.dx;
    v[6] = dph * p.dy;
    v[11] = dph;
}

// Gradient slot of an instance -- primitive with pack q on tile (tx, ty) of
// its image: the primitive's slot base plus the rank of the tile among the
// primitive's kept tiles, row-major over its tile rectangle, which is the
// order the emission numbers them in.
template <int TW, int TH>
__device__ __forceinline__ uint32_t slot_of(const PrimPack& q, int tx, int ty)
{
    const int tx0 = lo16(q.box0) / TW, ty0 = hi16(q.box0) / TH, tx1 = lo16(q.box1) / TW;
    const uint32_t k = (uint32_t)((ty - ty0) * (tx1 - tx0 + 1) + (tx - tx0));
    if (q.full) return q.base + k;
    const uint64_t mask = ((uint64_t)q.mhi << 32) | q.mlo;
    return q.base + (uint32_t)__popcll(mask & ((1ull << k) - 1ull));   // k < 64 for a culled rectangle
}

// Backward of tile t by the whole workgroup (wave w = block w).  The waves
// walk the tile's list in the same chunks of 64 positions, top down from the
// tile's last contributing position (alpha; the list end for additive); each
// wave stages the chunk's primitives that meet its contributing pixels,
// replays them back to front (alpha: recovering T and the colour behind from
// the forward's T_final), reduces each primitive's gradients over the block,
// and leaves them in LDS; then the workgroup adds the blocks in a fixed order
// and writes the chunk's slots.
template <int MODE, int TW, int TH>
__device__ __forceinline__ void bwd_tile(const ImgDesc* __restrict__ descs, int B, const KParams& kp,
                                               const Rec* __restrict__ recs, const uint32_t* __restrict__ vals,
                                               const PrimPack* __restrict__ pk, const uint2* __restrict__ ranges,
                                               uint32_t t, const float* __restrict__ T_final,
                                               const int32_t* __restrict__ last, const float* __restrict__ dLdC,
                                               float* __restrict__ slots, uint32_t* __restrict__ smark,
                                               const unsigned long long* __restrict__ cmask, uint32_t cmask_words,
                                               Staged (*stage)[kWave], float* __restrict__ part,
                                               uint32_t* __restrict__ top, uint64_t* __restrict__ hitm)
{
    constexpr int NBX = TW / 8, NB = (TW / 8) * (TH / 8), NT = NB * kWave;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int l = lane_id(), tid = (int)threadIdx.x;
    const TileGeo G = tile_geo(descs, B, ranges, t, TW, TH);
    prioritise(G.end - G.start);
    const ImgDesc& d = descs[G.b];
    const int bx = G.ox + (w % NBX) * 8, by = G.oy + (w / NBX) * 8;
    const int px = bx + (l & 7), py = by + (l >> 3);
    const bool valid = px < d.W && py < d.H;
    const uint32_t pix = valid ? (uint32_t)d.pix_begin + (uint32_t)(py * d.W + px) : 0u;
    // a `last` outside this tile's list (from a mismatched forward) can only
    // give wrong gradients, never an access outside the list
    const int32_t lst = MODE == WIPES_2D_ADDITIVE ? (valid ? (int32_t)G.end - 1 : -1)
                                                  : min(valid ? last[pix] : -1, (int32_t)G.end - 1);
    const bool on = lst >= (int32_t)G.start;
    float T = 0.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
    if (on) {
        if constexpr (MODE == WIPES_3D_ALPHA) T = T_final[pix];
        g0 = dLdC[3 * pix];
        g1 = dLdC[3 * pix + 1];
        g2 = dLdC[3 * pix + 2];
    }
    float Sg = kp.bg[0] * g0 + kp.bg[1] * g1 + kp.bg[2] * g2;   // dL/dC . colour behind (alpha)
    const float thr2 = fmaf(kp.q_add, kConicScale, -1.0f);   // support test on e2, as in the forward
    const float lx = (float)(l & 7) + 0.5f, ly = (float)(l >> 3) + 0.5f;
    const int32_t btop = __builtin_amdgcn_readfirstlane(wave_max_i32(on ? lst : -1));
    if (l == 0) top[w] = (uint32_t)(btop + 1);
    __syncthreads();
    uint32_t hi = G.start;
#pragma unroll
    for (int k = 0; k < NB; ++k) hi = max(hi, top[k]);
    // positions no pixel reached write nothing: their slots stay unmarked in
    // `smark` and the projection backward reads them as zero
    if (hi <= G.start) return;   // uniform over the workgroup
    const uint64_t below = (1ull << l) - 1ull;
    // The block partials and hit masks alternate between two buffers from
    // chunk to chunk, so one workgroup barrier per chunk suffices: the barrier
    // after the next chunk's replay also orders every thread's combine of
    // this chunk before its buffer is written again.
    uint32_t pbuf = 0;
    Staged* st = stage[w];
    // the lanes that hold the wave totals of the twelve slot values, and which value
    const bool red_lane = (l & 3) == 0 && (l & 15) <= 8;
    const int red_idx = reduce12_index(l);
    const unsigned long long* cm_row = cmask + (size_t)w * cmask_words;
    // Chunks are the 64-position words of the global list clipped to [start,
    // hi), walked top down; lane l holds position (c0 & ~63) + l.  A chunk's
    // hits are the positions whose primitive the forward found contributing
    // to this block (its contribution word), up to the block's last position.
    auto lo_of = [&](uint32_t c1) { return max(G.start, (c1 - 1u) & ~63u); };
    auto hits_of = [&](uint32_t c0, uint32_t c1) -> uint64_t {
        if (btop < (int32_t)c0) return 0ull;
        const uint32_t b = c0 & ~63u;
        const uint32_t lo = c0 - b, hb = min(c1 - 1u, (uint32_t)btop) - b;
        return cm_row[b >> 6] & ((~0ull >> (63u - hb)) & (~0ull << lo));
    };
    // List entries are read for every lane, at positions clamped into the
    // tile's list, so that they are in flight together with the chunk's
    // contribution word instead of waiting for it; only the hit lanes' record
    // loads depend on the word.  Records are loaded two chunks ahead (a
    // chunk with few hits in this block gives its loads little time), list
    // entries and hits three.  A chunk that does not exist has c0 = c1 = start.
    const uint32_t e1 = G.end - 1u;
    uint32_t c1 = hi, c0 = lo_of(hi);
    const uint32_t p0 = vals[min((c0 & ~63u) + (uint32_t)l, e1)];
    uint64_t m = hits_of(c0, c1);
    Rec cur{};
    if ((m >> l) & 1ull) cur = recs[p0];
    // the next chunk: hits and records
    uint32_t n1 = c0, n0 = c0 > G.start ? lo_of(c0) : c0;
    uint64_t mn = c0 > G.start ? hits_of(n0, n1) : 0ull;
    Rec nx1{};
    {
        const uint32_t p1 = vals[min((n0 & ~63u) + (uint32_t)l, e1)];
        if ((mn >> l) & 1ull) nx1 = recs[p1];
    }
    // the chunk after it: hits and list entries
    uint32_t nn1 = n0, nn0 = n0 > G.start ? lo_of(n0) : n0;
    uint64_t mnn = n0 > G.start ? hits_of(nn0, nn1) : 0ull;
    uint32_t pn2 = vals[min((nn0 & ~63u) + (uint32_t)l, e1)];
    // The combine step gives four threads to each list position of the chunk
    // (the first three take four slot values each, as one 16-byte piece), in
    // CR rounds of NT / 4 positions.  The
    // positions' primitives are loaded a chunk ahead (in the previous chunk's
    // prologue) and, in one round, their packs after the previous chunk's
    // replay, so the combine finds both in registers.
    constexpr int CR = NT >= 4 * kWave ? 1 : (4 * kWave) / NT;
    constexpr uint32_t CP = (uint32_t)NT / 4u;
    const uint32_t co0 = (uint32_t)tid >> 2, cc4 = ((uint32_t)tid & 3u) * 4u;
    const int tcx = G.ox / TW, tcy = G.oy / TH;   // this tile in its image
    auto combine_entries = [&](uint32_t lo, uint32_t hi1, bool (&cm)[CR], uint32_t (&cp)[CR]) {
        const uint32_t bb = lo & ~63u;
#pragma unroll
        for (int r = 0; r < CR; ++r) {
            const uint32_t co = co0 + (uint32_t)r * CP;
            cm[r] = co < (uint32_t)kWave && bb + co >= lo && bb + co < hi1;
            cp[r] = cm[r] ? vals[bb + co] : 0u;
        }
    };
    bool cmine[CR];
    uint32_t cprim[CR];
    combine_entries(c0, c1, cmine, cprim);
    PrimPack cq{};
    if (CR == 1 && cmine[0]) cq = pk[cprim[0]];
    for (;;) {
        const uint32_t b = c0 & ~63u;
        float* pcur = part + (size_t)pbuf * (NB * kWave * kSlot);
        uint64_t* hcur = hitm + pbuf * NB;
        float* mine = pcur + (size_t)w * kWave * kSlot;
        bool cmine_n[CR] = {};
        uint32_t cprim_n[CR] = {};
        if (c0 > G.start) combine_entries(n0, n1, cmine_n, cprim_n);
        if ((m >> l) & 1ull) {
            st[__popcll(m & below)] = stage_fwd(cur, bx, by);
        } else {
            float4* z = reinterpret_cast<float4*>(mine + l * kSlot);
            z[0] = make_float4(0.f, 0.f, 0.f, 0.f);
            z[1] = make_float4(0.f, 0.f, 0.f, 0.f);
            z[2] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        const bool more = c0 > G.start;   // uniform over the workgroup
        // the records of the chunk after next (and the entries of the one
        // after that) go in flight; the next chunk's are already
        Rec nx2{};
        uint32_t m31 = nn0, m30 = nn0, p3 = 0;
        uint64_t h3 = 0ull;
        if (n0 > G.start) {
            if ((mnn >> l) & 1ull) nx2 = recs[pn2];
            if (nn0 > G.start) {
                m30 = lo_of(nn0);
                h3 = hits_of(m30, m31);
                p3 = vals[min((m30 & ~63u) + (uint32_t)l, e1)];
            }
        }
        if (l == 0) hcur[w] = m;
        wave_lds_sync();
        const int nh = __popcll(m);
        // bp: the staged entry's position - b (its bit in m)
        auto replay = [&](const Staged& S, uint32_t bp) {
            __builtin_assume(bp < 64u);
            // branch-free: a pair that takes no part gets zero weight, for which
            // every update is an exact identity and every gradient term is zero
            float v[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) v[k] = 0.0f;
            const PairEval p = eval_at(S.mrx, S.mry, S.c0, S.c1, S.c2, S.f0, S.f1, S.ph, lx, ly);
            const float a = S.op * p.W;
            const bool reach = on && (int32_t)(b + bp) <= lst;
            bool takes;
            float da;
            if constexpr (MODE == WIPES_2D_ADDITIVE) {
                takes = reach && p.e2 >= thr2;
                const float cg = S.r * g0 + S.g * g1 + S.b * g2;
                const float ow = takes ? a : 0.0f;
                v[8] = ow * g0;
                v[9] = ow * g1;
                v[10] = ow * g2;
                da = takes ? cg : 0.0f;
                v[7] = p.W * da;
            } else {
                takes = reach && a >= kp.alpha_min;
                const float al = takes ? fminf(a, kp.alpha_max) : 0.0f;
                // T before this pair; the hardware reciprocal (1 ulp) keeps the
                // recovery within a few ulp of the forward's T.  A pair that takes
                // no part has al = 0 and keeps T exactly: the reciprocal of 1 is
                // exactly 1 (checked on the device), so no select is needed.
                const float Tb = T * __builtin_amdgcn_rcpf(1.0f - al);
                const float cg = S.r * g0 + S.g * g1 + S.b * g2;
                const float dal = Tb * (cg - Sg);
                const float wt = Tb * al;
                v[8] = wt * g0;
                v[9] = wt * g1;
                v[10] = wt * g2;
                Sg = fmaf(al, cg - Sg, Sg);
                T = Tb;
                da = (takes && a <= kp.alpha_max) ? dal : 0.0f;
                v[7] = p.W * da;
            }
            pair_grads(v, p, da);
            // (a primitive no pixel takes reduces to exact zeros: every term has a zero factor)
            float tot = wave_reduce12_valu(v);
            // the whole reduction runs with every lane on: left to itself the
            // compiler moves its last DPP add under the store's lane mask,
            // where the add can no longer read its neighbour in the same
            // instruction (two extra moves per replay)
            asm volatile("" : "+v"(tot));
            if (red_lane) mine[bp * kSlot + red_idx] = tot;
        };
        // back to front, two records a round in alternating registers: each
        // is read from the stage one replay ahead, without register copies;
        // positions come off the top of the hit mask
        uint64_t rest = m;
        auto top_pos = [&]() {
            const uint32_t bp = 63u - (uint32_t)__builtin_clzll(rest);
            rest &= ~(1ull << bp);
            return bp;
        };
        Staged Sa = st[nh > 0 ? nh - 1 : 0];
        for (int j = nh - 1; j >= 0; j -= 2) {
            const Staged Sb = st[j > 0 ? j - 1 : 0];
            replay(Sa, top_pos());
            if (j == 0) break;
            Sa = st[j > 1 ? j - 2 : 0];
            replay(Sb, top_pos());
        }
        PrimPack cq_n{};
        if (CR == 1 && cmine_n[0]) cq_n = pk[cprim_n[0]];
        __syncthreads();
        // positions some block staged get their slot written and marked
        uint64_t anyhit = 0ull;
#pragma unroll
        for (int k = 0; k < NB; ++k) anyhit |= hcur[k];
#pragma unroll
        for (int r = 0; r < CR; ++r) {
            const uint32_t co = co0 + (uint32_t)r * CP;
            if (cc4 < (uint32_t)kSlot && cmine[r] && ((anyhit >> co) & 1ull)) {
                const uint32_t ce = slot_of<TW, TH>(CR == 1 ? cq : pk[cprim[r]], tcx, tcy);
                // 16-byte pieces: a position's 12 values are 48 bytes in LDS and in the slots
                const uint32_t rr = co * kSlot + cc4;
                float4 sum = *reinterpret_cast<const float4*>(pcur + rr);
#pragma unroll
                for (int k = 1; k < NB; ++k) {   // blocks added in order
                    const float4 x = *reinterpret_cast<const float4*>(pcur + (size_t)k * kWave * kSlot + rr);
                    sum.x += x.x;
                    sum.y += x.y;
                    sum.z += x.z;
                    sum.w += x.w;
                }
                *reinterpret_cast<float4*>(slots + (size_t)ce * kSlot + cc4) = sum;
                if (cc4 == 0) atomicOr(smark + (ce >> 5), 1u << (ce & 31u));
            }
        }
        pbuf ^= 1u;
        if (!more) break;
#pragma unroll
        for (int r = 0; r < CR; ++r) {
            cmine[r] = cmine_n[r];
            cprim[r] = cprim_n[r];
        }
        cq = cq_n;
        cur = nx1;
        nx1 = nx2;
        m = mn;
        mn = mnn;
        mnn = h3;
        pn2 = p3;
        c1 = n1;
        c0 = n0;
        n1 = nn1;
        n0 = nn0;
        nn1 = m31;
        nn0 = m30;
    }
}

template <int MODE, int TW, int TH>
__global__ void __launch_bounds__(TW * TH) k_blend_bwd(const ImgDesc* __restrict__ descs, int B, KParams kp,
                                                             const Rec* __restrict__ recs,
                                                             const uint32_t* __restrict__ vals,
                                                             const PrimPack* __restrict__ pk,
                                                             const uint2* __restrict__ ranges,
                                                             const uint32_t* __restrict__ ovf, uint32_t n_tiles,
                                                             const float* __restrict__ T_final,
                                                             const int32_t* __restrict__ last,
                                                             const float* __restrict__ dLdC,
                                                             float* __restrict__ slots,
                                                             uint32_t* __restrict__ valid,
                                                             const unsigned long long* __restrict__ cmask,
                                                             uint32_t cmask_words, const uint32_t* __restrict__ order)
{
    constexpr int NB = (TW / 8) * (TH / 8);
    __shared__ Staged stage[NB][kWave];
    __shared__ __attribute__((aligned(16))) float part[2 * NB * kWave * kSlot];
    __shared__ uint32_t top[NB];
    __shared__ uint64_t hitm[2 * NB];
    if (*ovf) return;
    if (blockIdx.x >= n_tiles) return;
    const uint32_t t = order ? order[blockIdx.x] : blockIdx.x;
    bwd_tile<MODE, TW, TH>(descs, B, kp, recs, vals, pk, ranges, t, T_final, last, dLdC, slots, valid, cmask,
                           cmask_words, stage, part, top, hitm);
}

// Persistent form: each workgroup pulls whole tiles from the queue.
template <int MODE, int TW, int TH>
__global__ void __launch_bounds__(TW * TH) k_blend_bwd_q(const ImgDesc* __restrict__ descs, int B, KParams kp,
                                                               const Rec* __restrict__ recs,
                                                               const uint32_t* __restrict__ vals,
                                                               const PrimPack* __restrict__ pk,
                                                               const uint2* __restrict__ ranges,
                                                               const uint32_t* __restrict__ ovf, uint32_t n_tiles,
                                                               const uint32_t* __restrict__ order,
                                                               uint32_t* __restrict__ queue,
                                                               const float* __restrict__ T_final,
                                                               const int32_t* __restrict__ last,
                                                               const float* __restrict__ dLdC,
                                                               float* __restrict__ slots,
                                                               uint32_t* __restrict__ valid,
                                                               const unsigned long long* __restrict__ cmask,
                                                               uint32_t cmask_words)
{
    constexpr int NB = (TW / 8) * (TH / 8);
    __shared__ Staged stage[NB][kWave];
    __shared__ __attribute__((aligned(16))) float part[2 * NB * kWave * kSlot];
    __shared__ uint32_t top[NB];
    __shared__ uint64_t hitm[2 * NB];
    __shared__ uint32_t qtile;
    if (*ovf) return;
    uint32_t lane = blockIdx.x % kQueueLanes;
    for (;;) {
        if (threadIdx.x == 0) qtile = pull_tile(queue, n_tiles, order, lane);
        __syncthreads();
        const uint32_t t = qtile;
        __syncthreads();   // every wave has read `qtile` before it is rewritten
        if (t >= n_tiles) break;
        bwd_tile<MODE, TW, TH>(descs, B, kp, recs, vals, pk, ranges, t, T_final, last, dLdC, slots, valid, cmask,
                               cmask_words, stage, part, top, hitm);
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
        const float thr = fmaf(kq, MODE == WIPES_2D_ADDITIVE ? kp.q_add : 2.0f * logf(u.op / kp.alpha_min), -1.0f);
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
                         unsigned long long* cmask, uint32_t cmask_words, hipStream_t s)
{
    constexpr uint32_t NB = (TW / 8) * (TH / 8);
    if (queue) {
        const uint32_t nb = max(1u, persistent_blocks * kWpb / NB);   // same number of waves
        hipLaunchKernelGGL((k_blend_fwd_q<MODE, TW, TH>), dim3(nb), dim3(TW * TH), 0, s, descs, B, kp, recs, vals,
                           ranges, ovf, n_tiles, order, queue, image, T_final, last, cmask, cmask_words);
        return;
    }
    if (n_tiles == 0) return;
    hipLaunchKernelGGL((k_blend_fwd<MODE, TW, TH>), dim3(n_tiles), dim3(TW * TH), 0, s, descs, B, kp, recs, vals,
                       ranges, ovf, n_tiles, image, T_final, last, cmask, cmask_words, order);
}

template <int MODE, int TW, int TH>
static void launch_bwd_t(const ImgDesc* descs, int B, const KParams& kp, const Rec* recs, const uint32_t* vals,
                         const PrimPack* pk, const uint2* ranges, const uint32_t* ovf, uint32_t n_tiles,
                         const uint32_t* order, uint32_t* queue, uint32_t persistent_blocks, const float* T_final,
                         const int32_t* last, const float* dLdC, float* slots, uint32_t* valid,
                         const unsigned long long* cmask, uint32_t cmask_words, hipStream_t s)
{
    constexpr uint32_t NB = (TW / 8) * (TH / 8);
    if (queue) {
        const uint32_t nb = max(1u, persistent_blocks * kWpb / NB);
        hipLaunchKernelGGL((k_blend_bwd_q<MODE, TW, TH>), dim3(nb), dim3(TW * TH), 0, s, descs, B, kp, recs, vals,
                           pk, ranges, ovf, n_tiles, order, queue, T_final, last, dLdC, slots, valid, cmask,
                           cmask_words);
        return;
    }
    if (n_tiles == 0) return;
    hipLaunchKernelGGL((k_blend_bwd<MODE, TW, TH>), dim3(n_tiles), dim3(TW * TH), 0, s, descs, B, kp, recs, vals,
                       pk, ranges, ovf, n_tiles, T_final, last, dLdC, slots, valid, cmask, cmask_words, order);
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
                            unsigned long long* cmask, uint32_t cmask_words, hipStream_t s)
{
    if (kp.mode == WIPES_2D_ADDITIVE)
        WIPES_TILE_DISPATCH(launch_fwd_t, WIPES_2D_ADDITIVE, descs, B, kp, recs, vals, ranges, ovf, n_tiles, order,
                            queue, persistent_blocks, image, T_final, last, cmask, cmask_words, s);
    else
        WIPES_TILE_DISPATCH(launch_fwd_t, WIPES_3D_ALPHA, descs, B, kp, recs, vals, ranges, ovf, n_tiles, order,
                            queue, persistent_blocks, image, T_final, last, cmask, cmask_words, s);
    return hipGetLastError();
}

hipError_t launch_blend_bwd(const ImgDesc* descs, int B, const KParams& kp, const Rec* recs, const uint32_t* vals,
                            const PrimPack* pk, const uint2* ranges, const uint32_t* ovf, uint32_t n_tiles,
                            const uint32_t* order, uint32_t* queue, uint32_t persistent_blocks, const float* T_final,
                            const int32_t* last, const float* dLdC, float* slots, uint32_t* valid,
                            const unsigned long long* cmask, uint32_t cmask_words, hipStream_t s)
{
    if (kp.mode == WIPES_2D_ADDITIVE)
        WIPES_TILE_DISPATCH(launch_bwd_t, WIPES_2D_ADDITIVE, descs, B, kp, recs, vals, pk, ranges, ovf, n_tiles,
                            order, queue, persistent_blocks, T_final, last, dLdC, slots, valid, cmask, cmask_words, s);
    else
        WIPES_TILE_DISPATCH(launch_bwd_t, WIPES_3D_ALPHA, descs, B, kp, recs, vals, pk, ranges, ovf, n_tiles, order,
                            queue, persistent_blocks, T_final, last, dLdC, slots, valid, cmask, cmask_words, s);
    return hipGetLastError();
}

}  // namespace wipes
