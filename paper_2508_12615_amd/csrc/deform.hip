// Deformation network of Eq. 8 (Sec. 4.3): per primitive, offsets of its
// position, frequency and covariance, (dx, df, dq, ds) = F(gamma(x), gamma(t)),
// with the D-3DGS configuration the paper keeps (Sec. 5.3): positional
// encodings of 10 (position) and 6 (time) frequencies, 8 ReLU layers of 256
// units with the encoding joining the fifth layer's output, 13 outputs.  It is
// the one dense contraction of the method, so it runs on the matrix cores.
//
// Precision: FP32-class products from bf16 MFMAs.  Every operand x is split
// into hi = bf16(x) and lo = bf16(x - hi) (together 16 significant bits) and a
// product is hi*hi + hi*lo + lo*hi, accumulated in FP32 (the dropped lo*lo
// and the split residuals are below 2^-16 relative).  WIPES_DEFORM_BF16 keeps
// hi*hi only (three times fewer matrix instructions, ~2^-8 relative).
//
// Row kernels (forward, and the backward through the layers): one workgroup
// of 4 waves per 64 primitives, two workgroups per CU (each holds its rows'
// activations in 66 KB of LDS: 64 rows x 256 hidden units as bf16 hi/lo
// pairs), so one workgroup's epilogue and barriers overlap the other's
// matrix products.  Each wave computes 64 output units for all 64 rows -- 4
// tiles of v_mfma_f32_32x32x16_bf16 -- so every weight fragment it streams
// from L2 feeds two row tiles and every activation fragment it reads from
// LDS feeds two unit tiles.  The encoding (76 values per row) is computed
// once per workgroup into a double-buffered LDS stage, 16 columns per K step
// of the first and the sixth layer (exact range reduction, hardware sine and
// cosine in revolutions).  Bias, ReLU and the hi/lo split happen in the
// epilogue, written back into the same LDS rows after a barrier.
//
// Stored arrays (the backward's inputs) are kept per block of 128 rows; the
// two 64-row workgroups of a block each write their half.  For the backward
// the forward stores every layer input per block, column
// major over groups of 32 rows (each lane holds four consecutive rows of one
// unit after the matrix product: one 8-byte store per plane), the layout in
// which the weight-gradient products read their K runs (the rows) as
// contiguous 32-row steps.  The weight copies are stored in matrix-core
// fragment order, so a wave's operand fragment is one contiguous kilobyte.
#include <hip/hip_runtime.h>

#include "api_internal.hpp"

namespace wipes {

namespace dmlp {
constexpr int kLX = 10, kLT = 6;
constexpr int kIn = 3 * (1 + 2 * kLX) + (1 + 2 * kLT);   // 76
constexpr int kInPad = 80;
constexpr int kW = 256;
constexpr int kDepth = 8;
constexpr int kSkip = 5;
constexpr int kOut = 13;
constexpr int kOutPad = 32;
constexpr int kRB = 128;                          // primitives per stored block (two row-kernel workgroups)
constexpr int kAS = kW + 8;                       // LDS row stride of the activations (bf16 elements)
constexpr int kSaveCols = kInPad + kDepth * kW;   // stored layer inputs per row: e, then h_1..h_8
constexpr int kZS = 32 + 8;                       // LDS row stride of the weight-gradient stage
constexpr int kES = 16 + 8;                       // LDS row stride of the forward's encoding stage
}  // namespace dmlp

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Layer l of the split weight copy: K length (padded inputs) and output units (padded).
struct DLayer {
    int klen, n;
};

__host__ __device__ constexpr DLayer dlayer(int l)
{
    using namespace dmlp;
    return l == 0 ? DLayer{kInPad, kW}
                  : l == kSkip ? DLayer{kW + kInPad, kW} : l == kDepth ? DLayer{kW, kOutPad} : DLayer{kW, kW};
}

// Offsets (elements) of layer l's weights [n][klen] in the split weight copy;
// the caller's FP32 parameters are [out][in] row-major per layer (W0 [256,
// 76], b0, ..., W5 [256, 332], b5, ..., Wo [13, 256], bo).
__host__ __device__ inline size_t dw_off(int l)
{
    size_t o = 0;
    for (int i = 0; i < l; ++i) o += (size_t)dlayer(i).n * dlayer(i).klen;
    return o;
}
__host__ __device__ inline size_t dw_total() { return dw_off(dmlp::kDepth + 1); }

// Caller-layout geometry of layer j: fan-in, outputs and offset of W_j in the flat array.
__host__ __device__ inline int dfan(int j) { return j == 0 ? dmlp::kIn : j == dmlp::kSkip ? dmlp::kW + dmlp::kIn : dmlp::kW; }
__host__ __device__ inline int dnout(int j) { return j == dmlp::kDepth ? dmlp::kOut : dmlp::kW; }
__host__ __device__ inline size_t dsrc_off(int j)
{
    size_t o = 0;
    for (int i = 0; i < j; ++i) o += (size_t)dnout(i) * dfan(i) + dnout(i);
    return o;
}

__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo)
{
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

// Four bf16 values as one 8-byte word (element 0 in the low half of .x), and back.
__device__ __forceinline__ uint2 pack4(const __bf16 v[4])
{
    uint32_t b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) b[i] = __builtin_bit_cast(uint16_t, v[i]);
    return make_uint2(b[0] | (b[1] << 16), b[2] | (b[3] << 16));
}
__device__ __forceinline__ float unpack4(uint2 v, int i)
{
    const uint32_t w = i < 2 ? v.x : v.y;
    return __uint_as_float((i & 1) ? (w & 0xffff0000u) : (w << 16));
}

__device__ __forceinline__ f32x16 mfma(const bf16x8& a, const bf16x8& b, const f32x16& c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// The weight copies are in matrix-core fragment order: for each tile of 32
// units and K step of 16 the 64 lanes' 8-element runs are contiguous (one
// operand fragment is 1 KB), lane l holding unit 32 tile + l % 32 and K
// 16 step + 8 (l / 32) .. + 7; nks = K steps of the matrix.
__host__ __device__ inline size_t frag_index(int unit, int k, int nks)
{
    const int lane = (unit & 31) + 32 * ((k >> 3) & 1);
    return (((size_t)(unit >> 5) * nks + (k >> 4)) * 64 + lane) * 8 + (k & 7);
}
// Offset (elements) of the fragment of (unit tile, K step) in such a copy.
__host__ __device__ inline size_t frag_at(int tile, int ks, int nks) { return ((size_t)tile * nks + ks) * 512; }

// Per-block stored arrays of ncols columns x 128 rows are kept in groups of 32
// rows, (row / 32, column, row % 32), so that one 32-row step of the weight
// gradients reads contiguous runs and a lane's four consecutive rows of one
// column are one 8-byte word.
__host__ __device__ inline size_t cm(int c, int r, int ncols) { return ((size_t)(r >> 5) * ncols + c) * 32 + (r & 31); }

// Pre-split copy of the weights: hi/lo bf16 arrays [n][klen] per layer (in
// fragment order), K
// padded with zeros (layer 0: 76 -> 80; the skip layer: hidden 256 then
// encoding 76 then 4 zeros) and the output layer's rows padded 13 -> 32; and
// the biases [layer][256] (the output layer's 13 then zeros).
__global__ void __launch_bounds__(256) k_deform_split(const float* __restrict__ params, __bf16* __restrict__ whi,
                                                      __bf16* __restrict__ wlo, float* __restrict__ bias)
{
    using namespace dmlp;
    const size_t i = (size_t)blockIdx.x * 256u + threadIdx.x;
    if (i < dw_total()) {
        int l = 0;
        while (l < kDepth && i >= dw_off(l + 1)) ++l;
        const DLayer L = dlayer(l);
        const size_t q = i - dw_off(l);
        const int r = (int)(q / (size_t)L.klen), c = (int)(q % (size_t)L.klen);
        const float v = (r < dnout(l) && c < dfan(l)) ? params[dsrc_off(l) + (size_t)r * dfan(l) + c] : 0.0f;
        const size_t o = dw_off(l) + frag_index(r, c, L.klen / 16);
        split_bf16(v, whi[o], wlo[o]);
    }
    if (i < (size_t)(kDepth + 1) * kW) {
        const int l = (int)(i / kW), r = (int)(i % kW);
        bias[i] = r < dnout(l) ? params[dsrc_off(l) + (size_t)dnout(l) * dfan(l) + r] : 0.0f;
    }
}

// Encoding entry j (0..75) of position x and time t, FP32 with exact range
// reduction: sin(2^k pi p) = sin(2 pi r), r = fract(2^(k-1) p), and the power
// of two scaling is exact.
__device__ __forceinline__ float encode_entry(int j, const float x[3], float t)
{
    using namespace dmlp;
    float p;
    int blk;
    if (j < 3 * (1 + 2 * kLX)) {
        blk = j / 3;
        p = x[j % 3];
    } else {
        blk = j - 3 * (1 + 2 * kLX);
        p = t;
    }
    if (blk == 0) return p;
    const int k = (blk - 1) >> 1;
    const float r = __builtin_amdgcn_fractf(ldexpf(p, k - 1));
    return (blk & 1) ? __builtin_amdgcn_sinf(r) : __builtin_amdgcn_cosf(r);
}

// Stored layer inputs of block b: plane 0 (hi) then plane 1 (lo), each
// kSaveCols columns x 128 rows in the row-group order of cm(); column c < 80
// is encoding entry c, column 80 + 256 (j - 1) + u is unit u of h_j (the
// input of layer j).
__host__ __device__ inline size_t save_block(size_t b) { return b * dmlp::kSaveCols * 2 * dmlp::kRB; }
__host__ __device__ constexpr size_t save_col_h(int j) { return (size_t)dmlp::kInPad + (size_t)(j - 1) * dmlp::kW; }
// ReLU masks of h_1..h_8 per block, stored after the layer inputs of all blocks: [layer][unit] of four
// 32-bit words, bit r % 32 of word r / 32 set when row r's pre-activation of the unit is positive (32 KB
// per block; the backward reads these instead of the 64 KB hi plane of each h_j).
__host__ __device__ constexpr size_t mask_words_per_block() { return (size_t)dmlp::kDepth * dmlp::kW * 4; }

// Copy-out of a layer's RB x 256 activations (or gradients) from LDS (row major, hi and lo arrays) to a
// stored per-block array of 128-row blocks in the row-group order of cm(), the RB rows starting at row
// rb of the block: chunk c (0 .. 2 RB 256 / 8 - 1) is 8 rows of one unit of one plane -- r8 = c % 4,
// unit (c / 4) % 256, row group (c / 1024) % (RB / 32), plane c / (256 RB / 8) -- read as 8 LDS values
// and written as one 16-byte store, consecutive chunks contiguous in memory.  With mbytes the hi
// plane's chunks also store their ReLU mask byte (bit i: row 8 r8 + i of the group is positive).
template <int RB>
constexpr int copy_chunks() { return 2 * RB * dmlp::kW / 8; }
constexpr int kCopyChunks = copy_chunks<dmlp::kRB>();
template <int RB = dmlp::kRB>
__device__ __forceinline__ void copy_chunk(int c, const __bf16* shi, const __bf16* slo, __bf16* dst,
                                           size_t plane_stride, int ncols, int col0, uint8_t* mbytes, int rb = 0)
{
    using namespace dmlp;
    constexpr int GB = RB / 32, PS = RB == 128 ? 12 : 11;   // row groups; chunks per plane = 1 << PS
    static_assert((1 << PS) == RB * kW / 8, "chunks per plane");
    const int r8 = c & 3, u = (c >> 2) & (kW - 1), g = (c >> 10) & (GB - 1), p = c >> PS;
    const int r0 = 32 * g + 8 * r8;
    const __bf16* src = p ? slo : shi;
    __bf16 v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = src[(r0 + i) * kAS + u];
    const uint2 a = pack4(v), b = pack4(v + 4);
    *reinterpret_cast<uint4*>(dst + (size_t)p * plane_stride + cm(col0 + u, rb + r0, ncols)) =
        make_uint4(a.x, a.y, b.x, b.y);
    if (mbytes && p == 0) {
        uint32_t m = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) m |= (float)v[i] > 0.0f ? 1u << i : 0u;
        mbytes[u * 16 + (rb / 32 + g) * 4 + r8] = (uint8_t)m;
    }
}

// RB rows per workgroup: 128 (one workgroup per CU) or 64 (two workgroups
// per CU, so that one's epilogue and LDS traffic overlap the other's
// products).  The stored forward writes the backward's blocks of 128 rows:
// with RB = 64 workgroup 2 b + h fills rows 64 h .. 64 h + 63 of block b.
template <bool SPLIT, bool KEEP, int RB>
__global__ void __launch_bounds__(256, 128 / RB) k_deform_fwd(int32_t n, const float* __restrict__ mean, float t,
                                                       const __bf16* __restrict__ whi,
                                                       const __bf16* __restrict__ wlo,
                                                       const float* __restrict__ bias, float* __restrict__ delta,
                                                       __bf16* __restrict__ save, uint32_t* __restrict__ mask)
{
    using namespace dmlp;
    static_assert(RB == 128 || RB == 64, "64 or 128 rows per workgroup");
    static_assert(kRB == 128, "stored blocks of 128 rows");
    constexpr int RT = RB / 32;    // row tiles (each wave: all of them, for its 64 units)
    constexpr int RPT = RB / 16;   // encoding rows per thread and stage
    __shared__ __attribute__((aligned(16))) __bf16 ahi[RB * kAS];
    __shared__ __attribute__((aligned(16))) __bf16 alo[RB * kAS];
    // encoding columns 16 s .. 16 s + 15 of every row, two stages; the block's positions
    __shared__ __attribute__((aligned(16))) __bf16 ehi[2][RB * kES];
    __shared__ __attribute__((aligned(16))) __bf16 elo[2][RB * kES];
    __shared__ float xs[RB * 3];
    const int tid = (int)threadIdx.x, w = tid >> 6, l = tid & 63;
    // lane roles in v_mfma_f32_32x32x16_bf16: A row / B column = l % 32, K run 8 (l / 32) .. + 7;
    // result element e of a lane: column l % 32, row 8 (e / 4) + 4 (l / 32) + e % 4
    const int lr = l & 31, lk = (l >> 5) * 8, hs = l >> 5;
    const int32_t row0 = (int32_t)blockIdx.x * RB;
    const uint32_t sblk = blockIdx.x / (kRB / RB);          // the stored block
    const int rb = RB == kRB ? 0 : 64 * (blockIdx.x & 1);   // this workgroup's first row in it
    __bf16* sv = KEEP ? save + save_block(sblk) : nullptr;
    for (int q = tid; q < RB * 3; q += 256)
        xs[q] = row0 + q / 3 < n ? mean[3 * (size_t)row0 + q] : 0.0f;
    __syncthreads();
    // Encoding columns 16 s .. + 15 into stage b, computed once for the workgroup: thread t takes
    // column 16 s + t / 16 (uniform over 16 lanes) for rows RPT (t % 16) .. + RPT - 1; in layer 0 of
    // the stored forward it also stores them for the backward (eight consecutive rows of one
    // column: 16 bytes per plane).
    auto enc_stage = [&](int st, int b, bool store) __attribute__((always_inline)) {
        const int jj = tid >> 4, r0 = RPT * (tid & 15), j = 16 * st + jj;
        __bf16 eh[RPT], el[RPT];
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const float x3[3] = {xs[3 * (r0 + i)], xs[3 * (r0 + i) + 1], xs[3 * (r0 + i) + 2]};
            const float v = j < kIn ? encode_entry(j, x3, t) : 0.0f;
            split_bf16(v, eh[i], el[i]);
            ehi[b][(r0 + i) * kES + jj] = eh[i];
            elo[b][(r0 + i) * kES + jj] = el[i];
        }
        if constexpr (KEEP) {
            if (store) {
                if constexpr (RPT == 8) {
                    const uint4 hv = make_uint4(pack4(eh).x, pack4(eh).y, pack4(eh + 4).x, pack4(eh + 4).y);
                    const uint4 lv = make_uint4(pack4(el).x, pack4(el).y, pack4(el + 4).x, pack4(el + 4).y);
                    *reinterpret_cast<uint4*>(sv + cm(j, rb + r0, kSaveCols)) = hv;
                    *reinterpret_cast<uint4*>(sv + (size_t)kSaveCols * kRB + cm(j, rb + r0, kSaveCols)) = lv;
                } else {   // four consecutive rows of one column: 8 bytes per plane
                    *reinterpret_cast<uint2*>(sv + cm(j, rb + r0, kSaveCols)) = pack4(eh);
                    *reinterpret_cast<uint2*>(sv + (size_t)kSaveCols * kRB + cm(j, rb + r0, kSaveCols)) = pack4(el);
                }
            }
        }
    };
    // hidden layers: this wave's units 64 w .. 64 w + 63 (two tiles) for the RT row tiles
    for (int layer = 0; layer < kDepth; ++layer) {
        const int klen = dlayer(layer).klen;
        const int nks = klen / 16;
        const __bf16* wh = whi + dw_off(layer) + 8 * l;
        const __bf16* wl = wlo + dw_off(layer) + 8 * l;
        f32x16 acc[2][RT];
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int bt = 0; bt < RT; ++bt)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[q][bt][e] = 0.0f;
        // weight fragments of K step k (weight column k) are loaded one step ahead of their products
        auto load_b = [&](int k, bf16x8(&bh)[2], bf16x8(&bl)[2]) __attribute__((always_inline)) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const size_t o = frag_at(2 * w + q, k >> 4, nks);
                bh[q] = *reinterpret_cast<const bf16x8*>(wh + o);
                if (SPLIT) bl[q] = *reinterpret_cast<const bf16x8*>(wl + o);
            }
        };
        auto mma = [&](int bt, const bf16x8& ah, const bf16x8& al, const bf16x8(&bh)[2], const bf16x8(&bl)[2])
            __attribute__((always_inline)) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                acc[q][bt] = mfma(ah, bh[q], acc[q][bt]);
                if (SPLIT) {
                    acc[q][bt] = mfma(ah, bl[q], acc[q][bt]);
                    acc[q][bt] = mfma(al, bh[q], acc[q][bt]);
                }
            }
        };
        // activation fragments of K step k (LDS), and one K step's products
        auto load_a = [&](int k, bf16x8(&ah)[RT], bf16x8(&al)[RT]) __attribute__((always_inline)) {
#pragma unroll
            for (int bt = 0; bt < RT; ++bt) {
                const int ao = (32 * bt + lr) * kAS + k + lk;
                ah[bt] = *reinterpret_cast<const bf16x8*>(ahi + ao);
                if (SPLIT) al[bt] = *reinterpret_cast<const bf16x8*>(alo + ao);
            }
        };
        auto step_h = [&](const bf16x8(&ah)[RT], const bf16x8(&al)[RT], const bf16x8(&bh)[2], const bf16x8(&bl)[2])
            __attribute__((always_inline)) {
#pragma unroll
            for (int bt = 0; bt < RT; ++bt) mma(bt, ah[bt], al[bt], bh, bl);
        };
        // one K step over the encoding (fragments from stage b)
        auto step_e = [&](int b, const bf16x8(&bh)[2], const bf16x8(&bl)[2]) __attribute__((always_inline)) {
#pragma unroll
            for (int bt = 0; bt < RT; ++bt) {
                const int eo2 = (32 * bt + lr) * kES + lk;
                mma(bt, *reinterpret_cast<const bf16x8*>(&ehi[b][eo2]), *reinterpret_cast<const bf16x8*>(&elo[b][eo2]),
                    bh, bl);
            }
        };
        bf16x8 bh0[2], bl0[2], bh1[2], bl1[2];
        if (layer >= 1) {   // K over the hidden units: weight columns 0 .. 255
            // software pipeline: the fragments of step k + 1 are in flight during step k's
            // products (the scheduling barriers keep the compiler from sinking them); the stored
            // copy of this layer's input h_layer (and its ReLU mask bytes) goes out a few chunks per
            // step, its stores overlapping the products
            bf16x8 ah0[RT], al0[RT], ah1[RT], al1[RT];
            uint8_t* mb = KEEP ? reinterpret_cast<uint8_t*>(mask + mask_words_per_block() * sblk) +
                                     (size_t)(layer - 1) * kW * 16
                               : nullptr;
            load_b(0, bh0, bl0);
            load_a(0, ah0, al0);
#pragma unroll 1
            for (int k = 0; k < kW; k += 32) {
                load_b(k + 16, bh1, bl1);
                load_a(k + 16, ah1, al1);
                if constexpr (KEEP) {
                    constexpr int CPS = copy_chunks<RB>() / 256 / (kW / 32);   // chunks per thread and step
#pragma unroll
                    for (int i = 0; i < CPS; ++i)
                        copy_chunk<RB>(tid + 256 * ((k / 32) * CPS + i), ahi, alo, sv, (size_t)kSaveCols * kRB,
                                       kSaveCols, (int)save_col_h(layer), mb, rb);
                }
                __builtin_amdgcn_sched_barrier(0);
                step_h(ah0, al0, bh0, bl0);
                __builtin_amdgcn_sched_barrier(0);
                if (k + 32 < kW) {
                    load_b(k + 32, bh0, bl0);
                    load_a(k + 32, ah0, al0);
                }
                __builtin_amdgcn_sched_barrier(0);
                step_h(ah1, al1, bh1, bl1);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        if (layer == 0 || layer == kSkip) {   // K over the encoding: weight columns eo .. eo + 79
            const int eo = layer == 0 ? 0 : kW;
            const bool store = KEEP && layer == 0;
            load_b(eo, bh0, bl0);
            enc_stage(0, 0, store);
            __syncthreads();
            // step st reads stage st % 2 while stage (st + 1) % 2 -- last read in step st - 1, before
            // the barrier that ended it -- is computed; weights one step ahead as above
#pragma unroll 1
            for (int k = 0; k < kInPad; k += 32) {
                const int st = k / 16;
                if (k + 16 < kInPad) {
                    load_b(eo + k + 16, bh1, bl1);
                    enc_stage(st + 1, 1, store);
                }
                step_e(0, bh0, bl0);
                __syncthreads();
                if (k + 16 >= kInPad) break;
                if (k + 32 < kInPad) {
                    load_b(eo + k + 32, bh0, bl0);
                    enc_stage(st + 2, 0, store);
                }
                step_e(1, bh1, bl1);
                __syncthreads();
            }
        }
        __syncthreads();   // every wave has read this layer's input rows
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int col = 64 * w + 32 * q + lr;
            const float bcol = bias[(size_t)layer * kW + col];
#pragma unroll
            for (int bt = 0; bt < RT; ++bt) {
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int r = 32 * bt + 8 * g + 4 * hs;   // this lane's rows r .. r + 3
                    __bf16 hh[4], hl[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        split_bf16(fmaxf(acc[q][bt][4 * g + i] + bcol, 0.0f), hh[i], hl[i]);
                        ahi[(r + i) * kAS + col] = hh[i];
                        alo[(r + i) * kAS + col] = hl[i];
                    }
                }
            }
        }
        __syncthreads();   // the next layer reads the rows just written
    }
    // output layer: units 0..31 (13 real) of row tile w, K over the 256 hidden units (waves
    // past the block's row tiles only help store h_8)
    {
        const __bf16* wh = whi + dw_off(kDepth) + 8 * l;
        const __bf16* wl = wlo + dw_off(kDepth) + 8 * l;
        f32x16 acc;
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[e] = 0.0f;
        uint8_t* mb = KEEP ? reinterpret_cast<uint8_t*>(mask + mask_words_per_block() * sblk) +
                                 (size_t)(kDepth - 1) * kW * 16
                           : nullptr;
#pragma unroll 4
        for (int k = 0; k < kW; k += 16) {
            if constexpr (KEEP) {   // the stored copy of h_8, a few chunks per step
                constexpr int CPS = copy_chunks<RB>() / 256 / (kW / 16);
#pragma unroll
                for (int i = 0; i < CPS; ++i)
                    copy_chunk<RB>(tid + 256 * ((k / 16) * CPS + i), ahi, alo, sv, (size_t)kSaveCols * kRB,
                                   kSaveCols, (int)save_col_h(kDepth), mb, rb);
            }
            if (w >= RT) continue;   // wave-uniform
            const int ao = (32 * w + lr) * kAS + k + lk;
            const bf16x8 ah = *reinterpret_cast<const bf16x8*>(ahi + ao);
            const bf16x8 bh = *reinterpret_cast<const bf16x8*>(wh + frag_at(0, k >> 4, kW / 16));
            acc = mfma(ah, bh, acc);
            if (SPLIT) {
                const bf16x8 al = *reinterpret_cast<const bf16x8*>(alo + ao);
                const bf16x8 bl = *reinterpret_cast<const bf16x8*>(wl + frag_at(0, k >> 4, kW / 16));
                acc = mfma(ah, bl, acc);
                acc = mfma(al, bh, acc);
            }
        }
        const float bcol = bias[(size_t)kDepth * kW + lr];
        if (w < RT) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int32_t p = row0 + 32 * w + 8 * (e >> 2) + 4 * hs + (e & 3);
                if (lr < kOut && p < n) delta[(size_t)p * kOut + lr] = acc[e] + bcol;
            }
        }
    }
}

// The mask words of a stored forward (after the layer inputs of every block).
static uint32_t* save_masks(__bf16* save, int64_t n)
{
    const int64_t blocks = (n + dmlp::kRB - 1) / dmlp::kRB;
    return reinterpret_cast<uint32_t*>(save + save_block((size_t)blocks));
}

hipError_t launch_deform_fwd(int32_t n, const float* mean, float t, const float* params, void* ws, int split,
                             float* delta, void* save, hipStream_t s)
{
    using namespace dmlp;
    __bf16* whi = (__bf16*)ws;
    __bf16* wlo = whi + dw_total();
    float* bias = (float*)(wlo + dw_total());
    hipLaunchKernelGGL(k_deform_split, dim3((unsigned)((dw_total() + 255) / 256)), dim3(256), 0, s, params, whi,
                       wlo, bias);
    if (n > 0) {
        // the stored forward fills whole blocks of 128 rows (the backward reads every row of a block)
        const dim3 grid64((unsigned)((n + 63) / 64)), grid64k((unsigned)(2 * ((n + kRB - 1) / kRB)));
        __bf16* sv = (__bf16*)save;
        uint32_t* mk = save ? save_masks(sv, n) : nullptr;
        if (split && save)
            hipLaunchKernelGGL((k_deform_fwd<true, true, 64>), grid64k, dim3(256), 0, s, n, mean, t, whi, wlo, bias,
                               delta, sv, mk);
        else if (split)
            hipLaunchKernelGGL((k_deform_fwd<true, false, 64>), grid64, dim3(256), 0, s, n, mean, t, whi, wlo, bias,
                               delta, sv, mk);
        else if (save)
            hipLaunchKernelGGL((k_deform_fwd<false, true, 64>), grid64k, dim3(256), 0, s, n, mean, t, whi, wlo,
                               bias, delta, sv, mk);
        else
            hipLaunchKernelGGL((k_deform_fwd<false, false, 64>), grid64, dim3(256), 0, s, n, mean, t, whi, wlo, bias,
                               delta, sv, mk);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ backward
//
// Rows kernel, per 64 rows (two workgroups per 128-row stored block), the
// forward's tiling with the transposed split weights as the B operand:
// dIn_j = dZ_j W_j for j = 8 .. 0 (dZ_8 = dL/d offsets; dZ_{j-1} = dIn_j
// where the stored h_j > 0), the encoding's gradient collected from layer 0
// and from the skip layer's encoding inputs, then dL/dmean through the
// encoding's derivative.  Each dZ_j is also stored per block column major
// over the rows, with its column sums per workgroup (the bias gradients).
//
// Weight gradients dW_j = sum over rows of dZ_j^T a_j: one workgroup of 8
// waves per (chunk of blocks, layer part) stages 32 rows of dZ_j and a_j at a
// time in LDS and accumulates its layer's whole 256 x 256 (at most) product,
// each wave a block of 4 x 2 (or 1 x 3, 1 x 1) tiles of 32 x 32;
// a last kernel adds the chunks' partial sums in a fixed order (deterministic)
// into the caller's parameter layout.

// Backward product of layer j: K = output width Kb, output columns nT (the
// layer's input width padded to 32).
__host__ __device__ constexpr int dkb(int j) { return dlayer(j).n; }
__host__ __device__ constexpr int dnt(int j) { return j == 0 ? 96 : j == dmlp::kSkip ? 352 : dmlp::kW; }
__host__ __device__ inline size_t dwt_off(int j)
{
    size_t o = 0;
    for (int i = 0; i < j; ++i) o += (size_t)dnt(i) * dkb(i);
    return o;
}
__host__ __device__ inline size_t dwt_total() { return dwt_off(dmlp::kDepth + 1); }

// Transposed split weights WT_j [nT][Kb] (fragment order): WT_j[in][out] =
// W_j[out][in], zero outside the layer's real inputs and outputs.
__global__ void __launch_bounds__(256) k_deform_splitT(const float* __restrict__ params, __bf16* __restrict__ thi,
                                                       __bf16* __restrict__ tlo)
{
    using namespace dmlp;
    const size_t i = (size_t)blockIdx.x * 256u + threadIdx.x;
    if (i >= dwt_total()) return;
    int j = 0;
    while (j < kDepth && i >= dwt_off(j + 1)) ++j;
    const size_t q = i - dwt_off(j);
    const int in = (int)(q / (size_t)dkb(j)), out = (int)(q % (size_t)dkb(j));
    const float v = (in < dfan(j) && out < dnout(j)) ? params[dsrc_off(j) + (size_t)out * dfan(j) + in] : 0.0f;
    const size_t o = dwt_off(j) + frag_index(in, out, dkb(j) / 16);
    split_bf16(v, thi[o], tlo[o]);
}

// Per-block dZ storage: dZ_0..dZ_7 256 units, dZ_8 32 units, each plane 0
// (hi) then plane 1 (lo), units x 128 rows in the row-group order of cm().
__host__ __device__ constexpr size_t dz_cols_total() { return (size_t)dmlp::kDepth * dmlp::kW + dmlp::kOutPad; }
__host__ __device__ inline size_t dz_region(int j) { return (size_t)j * dmlp::kW * 2 * dmlp::kRB; }
__host__ __device__ constexpr int dz_units(int j) { return j == dmlp::kDepth ? dmlp::kOutPad : dmlp::kW; }

// RB = 64: two workgroups per CU; workgroup 2 b + h takes rows 64 h .. 64 h
// + 63 of the 128-row block b (its stored inputs, masks and dZ), and keeps
// bias partials of its own.
template <bool SPLIT, int RB>
__global__ void __launch_bounds__(256, 128 / RB) k_deform_bwd_rows(int32_t n, const float* __restrict__ mean,
                                                            const float* __restrict__ ddelta,
                                                            const __bf16* __restrict__ thi,
                                                            const __bf16* __restrict__ tlo,
                                                            __bf16* __restrict__ dz, float* __restrict__ dbp,
                                                            float* __restrict__ de_scr, float* __restrict__ dmean,
                                                            const uint32_t* __restrict__ mask)
{
    using namespace dmlp;
    static_assert(RB == 128 || RB == 64, "64 or 128 rows per workgroup");
    constexpr int RT = RB / 32;
    __shared__ __attribute__((aligned(16))) __bf16 ghi[RB * kAS];
    __shared__ __attribute__((aligned(16))) __bf16 glo[RB * kAS];
    const int tid = (int)threadIdx.x, w = tid >> 6, l = tid & 63;
    const int lr = l & 31, lk = (l >> 5) * 8, hs = l >> 5;
    const size_t blk = blockIdx.x / (kRB / RB);              // the 128-row block
    const int rb = RB == kRB ? 0 : 64 * (blockIdx.x & 1);    // this workgroup's first row in it
    const int32_t row0 = (int32_t)blockIdx.x * RB;
    __bf16* dzb = dz + blk * dz_cols_total() * 2 * kRB;
    float* dbb = dbp + (size_t)blockIdx.x * (kDepth + 1) * kW;
    // dZ_8 = dL/d offsets (13 of 32 units; rows past n are zero), in LDS and stored
    for (int q = tid; q < RB * kOutPad; q += 256) {
        const int r = q % RB, c = q / RB;
        const int32_t p = row0 + r;
        const float v = (c < kOut && p < n) ? ddelta[(size_t)p * kOut + c] : 0.0f;
        __bf16 h, o;
        split_bf16(v, h, o);
        ghi[r * kAS + c] = h;
        glo[r * kAS + c] = o;
        dzb[dz_region(kDepth) + cm(c, rb + r, kOutPad)] = h;
        dzb[dz_region(kDepth) + (size_t)kOutPad * kRB + cm(c, rb + r, kOutPad)] = o;
    }
    if (tid < kOutPad) {   // bias gradient of the output layer: column sums of dZ_8, row order
        float s = 0.0f;
        for (int r = 0; r < RB; ++r) {
            const int32_t p = row0 + r;
            s += (tid < kOut && p < n) ? ddelta[(size_t)p * kOut + tid] : 0.0f;
        }
        dbb[(size_t)kDepth * kW + tid] = s;
    }
    __syncthreads();
    for (int j = kDepth; j >= 0; --j) {
        const int Kb = dkb(j);
        const __bf16* th = thi + dwt_off(j);
        const __bf16* tl = tlo + dwt_off(j);
        const bool hpass = j >= 1;                            // input units 0..255 are hidden units
        const bool epass = (j == 0 || j == kSkip) && w < 3;   // encoding inputs: 3 tiles of 32
        const int eo = j == 0 ? 0 : kW;                       // their first row in WT_j
        // the ReLU mask words of h_j for this lane's two units (one per row tile of this
        // workgroup), in flight during the products
        uint32_t mk[2][RT];
        if (hpass) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const uint32_t* mw = mask + mask_words_per_block() * blk + ((size_t)(j - 1) * kW + 64 * w + 32 * q + lr) * 4;
                if constexpr (RT == 4) {
                    const uint4 v = *reinterpret_cast<const uint4*>(mw);
                    mk[q][0] = v.x; mk[q][1] = v.y; mk[q][2] = v.z; mk[q][3] = v.w;
                } else {
                    const uint2 v = *reinterpret_cast<const uint2*>(mw + rb / 32);
                    mk[q][0] = v.x; mk[q][1] = v.y;
                }
            }
        }
        if (!SPLIT && j == 0) {   // dZ_0 from LDS to its stored copy (layer 0 has no hidden-unit K loop to spread it over)
            for (int c = tid; c < copy_chunks<RB>(); c += 256)
                copy_chunk<RB>(c, ghi, glo, dzb + dz_region(0), (size_t)kW * kRB, kW, 0, nullptr, rb);
        }
        // encoding inputs first: the skip layer's part goes to scratch, and layer 0's is added to
        // it by the same lanes (same elements); the position gradient reads the sum
        f32x16 acce[RT];
#pragma unroll
        for (int bt = 0; bt < RT; ++bt)
#pragma unroll
            for (int e = 0; e < 16; ++e) acce[bt][e] = 0.0f;
        if (epass) {
            auto load_e = [&](int k, bf16x8& bh, bf16x8& bl) __attribute__((always_inline)) {
                const size_t wo = frag_at(eo / 32 + w, k >> 4, Kb / 16) + 8 * l;
                bh = *reinterpret_cast<const bf16x8*>(th + wo);
                if (SPLIT) bl = *reinterpret_cast<const bf16x8*>(tl + wo);
            };
            auto step_e = [&](int k, const bf16x8& bh, const bf16x8& bl) __attribute__((always_inline)) {
#pragma unroll
                for (int bt = 0; bt < RT; ++bt) {
                    const int ao = (32 * bt + lr) * kAS + k + lk;
                    const bf16x8 ah = *reinterpret_cast<const bf16x8*>(ghi + ao);
                    acce[bt] = mfma(ah, bh, acce[bt]);
                    if (SPLIT) {
                        const bf16x8 al = *reinterpret_cast<const bf16x8*>(glo + ao);
                        acce[bt] = mfma(ah, bl, acce[bt]);
                        acce[bt] = mfma(al, bh, acce[bt]);
                    }
                }
            };
            bf16x8 eh0, el0, eh1, el1;
            load_e(0, eh0, el0);
            for (int k = 0; k < Kb; k += 32) {
                load_e(k + 16, eh1, el1);
                step_e(k, eh0, el0);
                if (k + 32 < Kb) load_e(k + 32, eh0, el0);
                step_e(k + 16, eh1, el1);
            }
            const int u = 32 * w + lr;
#pragma unroll
            for (int bt = 0; bt < RT; ++bt)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int r = 32 * bt + 8 * (e >> 2) + 4 * hs + (e & 3);
                    float* sc = de_scr + (size_t)(row0 + r) * kInPad + u;
                    if (u < kInPad) *sc = j == kSkip ? acce[bt][e] : acce[bt][e] + *sc;
                }
        }
        f32x16 acc[2][RT];
#pragma unroll
        for (int bt = 0; bt < RT; ++bt)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[0][bt][e] = acc[1][bt][e] = 0.0f;
        if (hpass) {
            auto load_h = [&](int k, bf16x8(&bh)[2], bf16x8(&bl)[2]) __attribute__((always_inline)) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const size_t wo = frag_at(2 * w + q, k >> 4, Kb / 16) + 8 * l;
                    bh[q] = *reinterpret_cast<const bf16x8*>(th + wo);
                    if (SPLIT) bl[q] = *reinterpret_cast<const bf16x8*>(tl + wo);
                }
            };
            auto load_a = [&](int k, bf16x8(&ah)[RT], bf16x8(&al)[RT]) __attribute__((always_inline)) {
#pragma unroll
                for (int bt = 0; bt < RT; ++bt) {
                    const int ao = (32 * bt + lr) * kAS + k + lk;
                    ah[bt] = *reinterpret_cast<const bf16x8*>(ghi + ao);
                    if (SPLIT) al[bt] = *reinterpret_cast<const bf16x8*>(glo + ao);
                }
            };
            auto step_h = [&](const bf16x8(&ah)[RT], const bf16x8(&al)[RT], const bf16x8(&bh)[2],
                              const bf16x8(&bl)[2]) __attribute__((always_inline)) {
#pragma unroll
                for (int bt = 0; bt < RT; ++bt) {
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        acc[q][bt] = mfma(ah[bt], bh[q], acc[q][bt]);
                        if (SPLIT) {
                            acc[q][bt] = mfma(ah[bt], bl[q], acc[q][bt]);
                            acc[q][bt] = mfma(al[bt], bh[q], acc[q][bt]);
                        }
                    }
                }
            };
            // software pipeline as in the forward.  In the one-product (bf16) form dZ_j (j < 8: dZ_8
            // was stored directly) goes to its stored copy a few 16-byte chunks per step, the stores
            // overlapping the products; the three-product form has no registers to spare for it
            // (it would spill) and stores dZ_{j-1} in one pass after the epilogue instead
            bf16x8 bh0[2], bl0[2], bh1[2], bl1[2], ah0[RT], al0[RT], ah1[RT], al1[RT];
            load_h(0, bh0, bl0);
            load_a(0, ah0, al0);
#pragma unroll 1
            for (int k = 0; k < Kb; k += 32) {
                load_h(k + 16, bh1, bl1);
                load_a(k + 16, ah1, al1);
                if (!SPLIT && j < kDepth) {   // Kb = kW here: kW / 32 steps
                    constexpr int CPS = copy_chunks<RB>() / 256 / (kW / 32);   // chunks per thread and step
                    static_assert(CPS * 256 * (kW / 32) == copy_chunks<RB>(), "the copy divides over the steps");
#pragma unroll
                    for (int i = 0; i < CPS; ++i)
                        copy_chunk<RB>(tid + 256 * ((k / 32) * CPS + i), ghi, glo, dzb + dz_region(j),
                                       (size_t)kW * kRB, kW, 0, nullptr, rb);
                }
                __builtin_amdgcn_sched_barrier(0);
                step_h(ah0, al0, bh0, bl0);
                __builtin_amdgcn_sched_barrier(0);
                if (k + 32 < Kb) {
                    load_h(k + 32, bh0, bl0);
                    load_a(k + 32, ah0, al0);
                }
                __builtin_amdgcn_sched_barrier(0);
                step_h(ah1, al1, bh1, bl1);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        __syncthreads();   // every wave has read dZ_j
        if (hpass) {
            // dZ_{j-1} = dIn_j where the pre-activation of h_j was positive, into LDS, with its column sums
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int u = 64 * w + 32 * q + lr;
                float cs = 0.0f;
#pragma unroll
                for (int bt = 0; bt < RT; ++bt) {
                    const uint32_t mw = mk[q][bt];
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        const int r = 32 * bt + 8 * g + 4 * hs;
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const float d = (mw >> (8 * g + 4 * hs + i)) & 1u ? acc[q][bt][4 * g + i] : 0.0f;
                            split_bf16(d, ghi[(r + i) * kAS + u], glo[(r + i) * kAS + u]);
                            cs += d;
                        }
                    }
                }
                cs += __shfl_xor(cs, 32, kWave);   // the other half of the rows
                if (hs == 0) dbb[(size_t)(j - 1) * kW + u] = cs;
            }
        }
        __syncthreads();   // the next layer reads dZ_{j-1}
        if (SPLIT && hpass) {   // dZ_{j-1} from LDS to its stored copy (16-byte chunks, contiguous over the workgroup)
            for (int c = tid; c < copy_chunks<RB>(); c += 256)
                copy_chunk<RB>(c, ghi, glo, dzb + dz_region(j - 1), (size_t)kW * kRB, kW, 0, nullptr, rb);
        }
    }
    // dL/dmean: the encoding's derivative, FP32 with the forward's range reduction
    const float* des = de_scr + (size_t)row0 * kInPad;   // written by this workgroup before the last barrier
    for (int q = tid; q < RB * 3; q += 256) {
        const int r = q / 3, c = q % 3;
        const int32_t p = row0 + r;
        if (p >= n) continue;
        const float x = mean[3 * (size_t)p + c];
        float g = des[r * kInPad + c];
        for (int k = 0; k < kLX; ++k) {
            const float rr = __builtin_amdgcn_fractf(ldexpf(x, k - 1));
            const float wgt = ldexpf(3.14159265358979f, k);   // 2^k pi
            g += des[r * kInPad + 3 + 6 * k + c] * wgt * __builtin_amdgcn_cosf(rr);
            g -= des[r * kInPad + 6 + 6 * k + c] * wgt * __builtin_amdgcn_sinf(rr);
        }
        dmean[3 * (size_t)p + c] = g;
    }
}

// Parts of the weight-gradient products: layer, output units and inputs in
// tiles of 32, the stored input columns that feed them (zero beyond), and the
// first column of the part in layer j's padded [n][klen] product.
struct WPart {
    int j, mt, nt;
    int acol, avalid;
    int ccol;
};
constexpr int kWParts = 10;

__host__ __device__ constexpr WPart wpart(int v)
{
    using namespace dmlp;
    return v == 0   ? WPart{0, 8, 3, 0, kInPad, 0}
           : v <= 4 ? WPart{v, 8, 8, (int)save_col_h(v), kW, 0}
           : v == 5 ? WPart{kSkip, 8, 8, (int)save_col_h(kSkip), kW, 0}
           : v == 6 ? WPart{kSkip, 8, 3, 0, kInPad, kW}
           : v <= 8 ? WPart{v - 1, 8, 8, (int)save_col_h(v - 1), kW, 0}
                    : WPart{kDepth, 1, 8, (int)save_col_h(kDepth), kW, 0};
}

// The weight-gradient kernel maps waves to tiles for these three part shapes only.
constexpr bool wpart_shapes_known()
{
    for (int v = 0; v < kWParts; ++v) {
        const WPart P = wpart(v);
        if (!((P.mt == 8 && P.nt == 8) || (P.mt == 8 && P.nt == 3) || (P.mt == 1 && P.nt == 8))) return false;
    }
    return true;
}
static_assert(wpart_shapes_known(), "weight-gradient part shapes");

template <bool SPLIT>
__global__ void __launch_bounds__(512) k_deform_wgrad(int32_t n_blocks, int blocks_per_chunk,
                                                      const __bf16* __restrict__ dz, const __bf16* __restrict__ save,
                                                      float* __restrict__ part)
{
    using namespace dmlp;
    // two stages (the next one fills while the current one feeds the products):
    // dZ_j [unit][32 rows] and a_j [input][32 rows], hi and lo planes each
    __shared__ __attribute__((aligned(16))) __bf16 zs[2][2][kW * kZS];
    __shared__ __attribute__((aligned(16))) __bf16 as[2][2][kW * kZS];
    const WPart P = wpart((int)blockIdx.y);
    const int tid = (int)threadIdx.x, w = tid >> 6, l = tid & 63;
    const int lr = l & 31, lk = (l >> 5) * 8, hs = l >> 5;
    const int M = 32 * P.mt, N = 32 * P.nt, T = P.mt * P.nt;
    const int zu = dz_units(P.j);
    const int32_t b0 = (int32_t)blockIdx.x * blocks_per_chunk, b1 = min(n_blocks, b0 + blocks_per_chunk);
    const int steps = (b1 - b0) * (kRB / 32);
    f32x16 acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[i][e] = 0.0f;
    // this thread's 16-byte pieces of a stage: piece q = tid + 512 i (i < 4) is unit q / 8,
    // plane (q / 4) % 2, rows 8 (q % 4) .. + 7 of the step
    uint4 rz0, rz1, rz2, rz3, ra0, ra1, ra2, ra3;
    auto gpiece = [&](int st, int i, uint4& z, uint4& a) __attribute__((always_inline)) {
        const int32_t b = b0 + st / (kRB / 32);
        const int ks = (st % (kRB / 32)) * 32;
        const int q = tid + 512 * i;
        const int u = q >> 3, p = (q >> 2) & 1, c = q & 3;
        const __bf16* zb = dz + (size_t)b * dz_cols_total() * 2 * kRB + dz_region(P.j);
        const __bf16* sb = save + save_block((size_t)b);
        z = make_uint4(0u, 0u, 0u, 0u);
        a = make_uint4(0u, 0u, 0u, 0u);
        if (q < M * 8) z = *reinterpret_cast<const uint4*>(zb + (size_t)p * zu * kRB + cm(u, ks, zu) + 8 * c);
        if (q < N * 8 && u < P.avalid)
            a = *reinterpret_cast<const uint4*>(sb + (size_t)p * kSaveCols * kRB + cm(P.acol + u, ks, kSaveCols) +
                                                8 * c);
    };
    auto spiece = [&](int buf, int i, const uint4& z, const uint4& a) __attribute__((always_inline)) {
        const int q = tid + 512 * i;
        const int u = q >> 3, p = (q >> 2) & 1, c = q & 3;
        if (q < M * 8) *reinterpret_cast<uint4*>(&zs[buf][p][u * kZS + 8 * c]) = z;
        if (q < N * 8) *reinterpret_cast<uint4*>(&as[buf][p][u * kZS + 8 * c]) = a;
    };
    auto gload = [&](int st) __attribute__((always_inline)) {
        gpiece(st, 0, rz0, ra0);
        gpiece(st, 1, rz1, ra1);
        gpiece(st, 2, rz2, ra2);
        gpiece(st, 3, rz3, ra3);
    };
    auto sstore = [&](int buf) __attribute__((always_inline)) {
        spiece(buf, 0, rz0, ra0);
        spiece(buf, 1, rz1, ra1);
        spiece(buf, 2, rz2, ra2);
        spiece(buf, 3, rz3, ra3);
    };
    if (steps > 0) {
        gload(0);
        sstore(0);
    }
    __syncthreads();
    const DLayer L = dlayer(P.j);
    float* pc = part + (size_t)blockIdx.x * dw_total() + dw_off(P.j);
    // Each wave takes an RM x RN block of 32x32 tiles at (mi0, ni0), so it reads
    // RM + RN fragment pairs from LDS per 16-deep step for RM * RN products.
    auto run = [&](auto rmc, auto rnc, int mi0, int ni0) __attribute__((always_inline)) {
        constexpr int RM = decltype(rmc)::value, RN = decltype(rnc)::value;
        for (int st = 0; st < steps; ++st) {
            const int cur = st & 1;
            if (st + 1 < steps) gload(st + 1);   // in flight during this step's products
#pragma unroll
            for (int kk = 0; kk < 32; kk += 16) {
                bf16x8 ah[RM], al[RM], bh[RN], bl[RN];
#pragma unroll
                for (int a = 0; a < RM; ++a) {
                    const int ao = (32 * (mi0 + a) + lr) * kZS + kk + lk;
                    ah[a] = *reinterpret_cast<const bf16x8*>(&zs[cur][0][ao]);
                    if (SPLIT) al[a] = *reinterpret_cast<const bf16x8*>(&zs[cur][1][ao]);
                }
#pragma unroll
                for (int b = 0; b < RN; ++b) {
                    const int bo = (32 * (ni0 + b) + lr) * kZS + kk + lk;
                    bh[b] = *reinterpret_cast<const bf16x8*>(&as[cur][0][bo]);
                    if (SPLIT) bl[b] = *reinterpret_cast<const bf16x8*>(&as[cur][1][bo]);
                }
#pragma unroll
                for (int a = 0; a < RM; ++a)
#pragma unroll
                    for (int b = 0; b < RN; ++b) {
                        f32x16& c = acc[a * RN + b];
                        c = mfma(ah[a], bh[b], c);
                        if (SPLIT) {
                            c = mfma(ah[a], bl[b], c);
                            c = mfma(al[a], bh[b], c);
                        }
                    }
            }
            // the other stage was last read in the previous step, before the barrier that ended it
            if (st + 1 < steps) sstore(cur ^ 1);
            __syncthreads();
        }
        // result element e of tile (mi, ni): unit 32 mi + 8 (e / 4) + 4 (l / 32) + e % 4, input 32 ni + l % 32
#pragma unroll
        for (int i = 0; i < RM * RN; ++i) {
            const int mi = mi0 + i / RN, ni = ni0 + i % RN;
            const int col = 32 * ni + lr;
            if (col >= P.avalid) continue;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int row = 32 * mi + 8 * (e >> 2) + 4 * hs + (e & 3);
                pc[(size_t)row * L.klen + P.ccol + col] = acc[i][e];
            }
        }
    };
    using I1 = std::integral_constant<int, 1>;
    if (P.nt == 8 && P.mt == 8)   // 8 x 8 tiles: waves in 2 x 4, 4 x 2 tiles each
        run(std::integral_constant<int, 4>{}, std::integral_constant<int, 2>{}, 4 * (w & 1), 2 * (w >> 1));
    else if (P.nt == 3)           // 8 x 3 tiles: one row of tiles per wave
        run(I1{}, std::integral_constant<int, 3>{}, w, 0);
    else                          // 1 x 8 tiles: one tile per wave
        run(I1{}, I1{}, 0, w);
}

// Bias gradients per chunk: thread r of (chunk k, layer j) sums unit r of
// layer j over the chunk's blocks, in block order.
__global__ void __launch_bounds__(256) k_deform_bias_part(int32_t n_blocks, int blocks_per_chunk,
                                                          const float* __restrict__ dbp, float* __restrict__ bpart)
{
    using namespace dmlp;
    const int r = (int)threadIdx.x, chunk = (int)blockIdx.x, j = (int)blockIdx.y;
    const int32_t b0 = chunk * blocks_per_chunk, b1 = min(n_blocks, b0 + blocks_per_chunk);
    float acc = 0.0f;
    for (int32_t b = b0; b < b1; ++b) acc += dbp[((size_t)b * (kDepth + 1) + j) * kW + r];
    bpart[((size_t)chunk * (kDepth + 1) + j) * kW + r] = acc;
}

// Sum the chunks' partial weight and bias gradients in a fixed order into the
// caller's parameter layout.
__global__ void __launch_bounds__(256) k_deform_reduce(int chunks, const float* __restrict__ part,
                                                       const float* __restrict__ bpart, float* __restrict__ dparams)
{
    using namespace dmlp;
    const size_t i = (size_t)blockIdx.x * 256u + threadIdx.x;
    if (i >= dsrc_off(kDepth + 1)) return;
    int j = 0;
    while (j < kDepth && i >= dsrc_off(j + 1)) ++j;
    const size_t q = i - dsrc_off(j);
    const int fan = dfan(j), no = dnout(j);
    float acc = 0.0f;
    if (q < (size_t)no * fan) {   // weight (out r, in c): padded column c (the padding follows the inputs)
        const int r = (int)(q / (size_t)fan), c = (int)(q % (size_t)fan);
        const size_t pi = dw_off(j) + (size_t)r * dlayer(j).klen + c;
        for (int k = 0; k < chunks; ++k) acc += part[(size_t)k * dw_total() + pi];
    } else {                      // bias
        const int r = (int)(q - (size_t)no * fan);
        for (int k = 0; k < chunks; ++k) acc += bpart[((size_t)k * (kDepth + 1) + j) * kW + r];
    }
    dparams[i] = acc;
}

// Chunks of blocks of the weight-gradient products: about 100 per layer part
// (a thousand workgroups in all), at least one block each.
static int wgrad_blocks_per_chunk(int32_t n_blocks) { return std::max<int32_t>(1, (n_blocks + 99) / 100); }

static size_t up256(size_t b) { return (b + 255) / 256 * 256; }

size_t deform_weight_bytes()
{
    return up256(dw_total() * 2 * sizeof(__bf16) + (size_t)(dmlp::kDepth + 1) * dmlp::kW * sizeof(float));
}

size_t deform_save_bytes(int64_t n)
{
    const int64_t blocks = (n + dmlp::kRB - 1) / dmlp::kRB;
    return up256(save_block((size_t)blocks) * sizeof(__bf16) + (size_t)blocks * mask_words_per_block() * 4);
}

// Backward scratch: WT | dZ per block | bias partials per half block | encoding
// gradient of the skip layer | bias partials per chunk | weight partials per chunk.
struct BwdScratch {
    size_t wt, dz, dbp, de, bpart, part, total;
};

static BwdScratch bwd_scratch(int64_t n)
{
    using namespace dmlp;
    const int32_t blocks = (int32_t)((n + kRB - 1) / kRB);
    const int bpc = wgrad_blocks_per_chunk(blocks);
    const int32_t chunks = std::max<int32_t>(1, (blocks + bpc - 1) / bpc);
    BwdScratch s;
    s.wt = 0;
    s.dz = s.wt + up256(dwt_total() * 2 * sizeof(__bf16));
    s.dbp = s.dz + up256((size_t)blocks * dz_cols_total() * 2 * kRB * sizeof(__bf16));
    s.de = s.dbp + up256((size_t)2 * blocks * (kDepth + 1) * kW * sizeof(float));   // per 64-row workgroup
    s.bpart = s.de + up256((size_t)blocks * kRB * kInPad * sizeof(float));
    s.part = s.bpart + up256((size_t)chunks * (kDepth + 1) * kW * sizeof(float));
    s.total = s.part + up256((size_t)chunks * dw_total() * sizeof(float));
    return s;
}

size_t deform_bwd_scratch_bytes(int64_t n) { return bwd_scratch(n).total; }

hipError_t launch_deform_bwd(int32_t n, const float* mean, const float* params, void* ws, int split,
                             const float* ddelta, float* dparams, float* dmean, hipStream_t s)
{
    using namespace dmlp;
    const int32_t blocks = (n + kRB - 1) / kRB;
    const int bpc = wgrad_blocks_per_chunk(blocks);
    const int chunks = (blocks + bpc - 1) / bpc;
    char* base = (char*)ws;
    const __bf16* save = (const __bf16*)(base + deform_weight_bytes());
    char* scr = base + deform_weight_bytes() + deform_save_bytes(n);
    const BwdScratch L = bwd_scratch(n);
    __bf16* thi = (__bf16*)(scr + L.wt);
    __bf16* tlo = thi + dwt_total();
    __bf16* dz = (__bf16*)(scr + L.dz);
    float* dbp = (float*)(scr + L.dbp);
    float* de = (float*)(scr + L.de);
    float* bpart = (float*)(scr + L.bpart);
    float* part = (float*)(scr + L.part);
    hipLaunchKernelGGL(k_deform_splitT, dim3((unsigned)((dwt_total() + 255) / 256)), dim3(256), 0, s, params, thi,
                       tlo);
    if (blocks > 0) {
        // two 64-row workgroups per block: every row of every block gets its dZ (zero past n)
        if (split)
            hipLaunchKernelGGL((k_deform_bwd_rows<true, 64>), dim3((unsigned)(2 * blocks)), dim3(256), 0, s, n, mean,
                               ddelta, thi, tlo, dz, dbp, de, dmean, save_masks((__bf16*)save, n));
        else
            hipLaunchKernelGGL((k_deform_bwd_rows<false, 64>), dim3((unsigned)(2 * blocks)), dim3(256), 0, s, n,
                               mean, ddelta, thi, tlo, dz, dbp, de, dmean, save_masks((__bf16*)save, n));
        const dim3 grid((unsigned)chunks, (unsigned)kWParts);
        if (split)
            hipLaunchKernelGGL(k_deform_wgrad<true>, grid, dim3(512), 0, s, blocks, bpc, dz, save, part);
        else
            hipLaunchKernelGGL(k_deform_wgrad<false>, grid, dim3(512), 0, s, blocks, bpc, dz, save, part);
        // bias partials of the 64-row halves, summed in order over each chunk's blocks
        hipLaunchKernelGGL(k_deform_bias_part, dim3((unsigned)chunks, (unsigned)(kDepth + 1)), dim3(256), 0, s,
                           2 * blocks, 2 * bpc, dbp, bpart);
    }
    const size_t total = dsrc_off(kDepth + 1);
    hipLaunchKernelGGL(k_deform_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       blocks > 0 ? chunks : 0, part, bpart, dparams);
    return hipGetLastError();
}

// The deformed primitive set: mean + dx, freq + df, quat + dq, scale + ds.  One
// thread per output value, over [mean 3n | freq 3n | quat 4n | scale 3n], so the
// parameter arrays are read and written coalesced (the offsets' rows of 13 are
// gathered, consecutive threads on neighbouring rows).
// (no __restrict__: the outputs may alias the inputs)
__global__ void __launch_bounds__(256) k_deform_apply(int32_t n, const float* off, const float* mean, const float* freq,
                                                      const float* quat, const float* scale, float* omean,
                                                      float* ofreq, float* oquat, float* oscale)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n3 = 3 * (int64_t)n;
    if (e >= 13 * (int64_t)n) return;
    const float* src;
    float* dst;
    int64_t k;   // element within the array
    int width, col0;
    if (e < n3) { src = mean; dst = omean; k = e; width = 3; col0 = 0; }
    else if (e < 2 * n3) { src = freq; dst = ofreq; k = e - n3; width = 3; col0 = 3; }
    else if (e < 2 * n3 + 4 * (int64_t)n) { src = quat; dst = oquat; k = e - 2 * n3; width = 4; col0 = 6; }
    else { src = scale; dst = oscale; k = e - 2 * n3 - 4 * (int64_t)n; width = 3; col0 = 10; }
    const int64_t row = k / width;
    dst[k] = src[k] + off[row * dmlp::kOut + col0 + (k - row * width)];
}

}  // namespace wipes

using namespace wipes;

extern "C" {

int64_t wipes_deform_param_count(void)
{
    return (int64_t)dsrc_off(dmlp::kDepth + 1);
}

wipes_status wipes_deform_workspace_size(int64_t n, int32_t with_backward, size_t* bytes)
{
    if (n < 0 || n >= (1ll << 31) || !bytes) return fail(nullptr, WIPES_ERR_INVALID, "n out of range or bytes NULL");
    size_t b = deform_weight_bytes();
    if (with_backward) b += deform_save_bytes(n) + deform_bwd_scratch_bytes(n);
    *bytes = b;
    return WIPES_OK;
}

static wipes_status deform_check(wipes_ctx* ctx, int32_t precision, const float* params, int64_t n,
                                 const float* mean, void* workspace, size_t workspace_bytes, int32_t with_backward)
{
    if (!ctx) return fail(nullptr, WIPES_ERR_INVALID, "ctx must not be NULL");
    if (precision != WIPES_DEFORM_BF16X3 && precision != WIPES_DEFORM_BF16)
        return fail(ctx, WIPES_ERR_INVALID, "bad precision");
    if (n < 0 || n >= (1ll << 31)) return fail(ctx, WIPES_ERR_INVALID, "n out of range");
    if (!params || !workspace || (n > 0 && !mean))
        return fail(ctx, WIPES_ERR_INVALID, "params, workspace and mean must be set");
    size_t need = 0;
    wipes_deform_workspace_size(n, with_backward, &need);
    if (workspace_bytes < need)
        return fail(ctx, WIPES_ERR_NOMEM, "deform workspace too small (%zu < %zu)", workspace_bytes, need);
    return WIPES_OK;
}

wipes_status wipes_deform_fwd(wipes_ctx* ctx, int32_t precision, const float* params, int64_t n, const float* mean,
                              float time, float* offsets, void* workspace, size_t workspace_bytes,
                              int32_t keep_for_backward, void* stream)
{
    wipes_status st = deform_check(ctx, precision, params, n, mean, workspace, workspace_bytes, keep_for_backward);
    if (st != WIPES_OK) return st;
    if (n > 0 && !offsets) return fail(ctx, WIPES_ERR_INVALID, "offsets must be set");
    char* save = keep_for_backward ? (char*)workspace + deform_weight_bytes() : nullptr;
    const hipError_t e = launch_deform_fwd((int32_t)n, mean, time, params, workspace,
                                           precision == WIPES_DEFORM_BF16X3, offsets, save, (hipStream_t)stream);
    return e == hipSuccess ? WIPES_OK : hip_fail(ctx, e, "deform fwd");
}

wipes_status wipes_deform_bwd(wipes_ctx* ctx, int32_t precision, const float* params, int64_t n, const float* mean,
                              float time, const float* d_offsets, void* workspace, size_t workspace_bytes,
                              float* d_params, float* d_mean, void* stream)
{
    (void)time;   // the stored layer inputs carry it
    wipes_status st = deform_check(ctx, precision, params, n, mean, workspace, workspace_bytes, 1);
    if (st != WIPES_OK) return st;
    if (!d_params || (n > 0 && (!d_offsets || !d_mean)))
        return fail(ctx, WIPES_ERR_INVALID, "d_offsets, d_params and d_mean must be set");
    const hipError_t e = launch_deform_bwd((int32_t)n, mean, params, workspace, precision == WIPES_DEFORM_BF16X3,
                                           d_offsets, d_params, d_mean, (hipStream_t)stream);
    return e == hipSuccess ? WIPES_OK : hip_fail(ctx, e, "deform bwd");
}

wipes_status wipes_deform_apply(wipes_ctx* ctx, int64_t n, const float* offsets, const float* mean,
                                const float* freq, const float* quat, const float* scale, float* out_mean,
                                float* out_freq, float* out_quat, float* out_scale, void* stream)
{
    if (!ctx) return fail(nullptr, WIPES_ERR_INVALID, "ctx must not be NULL");
    if (n < 0 || n >= (1ll << 31)) return fail(ctx, WIPES_ERR_INVALID, "n out of range");
    if (n > 0 && (!offsets || !mean || !freq || !quat || !scale || !out_mean || !out_freq || !out_quat || !out_scale))
        return fail(ctx, WIPES_ERR_INVALID, "every array must be set");
    if (n > 0)
        hipLaunchKernelGGL(k_deform_apply, dim3((unsigned)((13 * n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                           (int32_t)n, offsets, mean, freq, quat, scale, out_mean, out_freq, out_quat, out_scale);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? WIPES_OK : hip_fail(ctx, e, "deform apply");
}

}  // extern "C"
