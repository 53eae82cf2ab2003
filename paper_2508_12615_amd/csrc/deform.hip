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
// Forward kernel: one workgroup (4 waves) per 32 primitives.  The 32 rows of
// activations live in LDS as bf16 hi/lo pairs, one row = [256 hidden | 76
// encoding | 4 zero], so the first layer reads the encoding block and the
// skip layer reads hidden + encoding in one contiguous K range.  Each wave
// computes 64 of the 256 output columns (two 32x32 tiles of
// v_mfma_f32_32x32x16_bf16), streaming its weight fragments from the
// pre-split weight copy (L2-resident: every workgroup reads the same 2 MB).
// Bias, ReLU and the hi/lo split happen in the epilogue, written back into
// the same LDS rows after a barrier.  For the backward the kernel can store
// every layer input per tile, column-major over the 32 rows (the layout the
// weight-gradient products read as contiguous K runs).
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
constexpr int kRows = 32;                  // primitives per workgroup
constexpr int kRowLen = kW + kInPad;       // 336: [hidden | encoding | zero]
constexpr int kRowStride = kRowLen + 8;    // LDS row stride (bf16 elements)
constexpr int kSaveCols = kInPad + kDepth * kW;   // layer inputs stored per tile: e and h1..h8
}  // namespace dmlp

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Layer l: K range [k0, k0 + klen) of an activation row, output columns n.
struct DLayer {
    int k0, klen, n;
};

__host__ __device__ constexpr DLayer dlayer(int l)
{
    using namespace dmlp;
    return l == 0 ? DLayer{kW, kInPad, kW}
                  : l == kSkip ? DLayer{0, kRowLen, kW} : l == kDepth ? DLayer{0, kW, kOutPad} : DLayer{0, kW, kW};
}

// Offsets (elements) of layer l's weights [n][klen] and bias in the split
// weight copy; the caller's FP32 parameters are [out][in] row-major per layer
// (W0 [256, 76], b0, ..., W5 [256, 332], b5, ..., Wo [13, 256], bo).
__host__ __device__ inline size_t dw_off(int l)
{
    size_t o = 0;
    for (int i = 0; i < l; ++i) o += (size_t)dlayer(i).n * dlayer(i).klen;
    return o;
}
__host__ __device__ inline size_t dw_total() { return dw_off(dmlp::kDepth + 1); }

__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo)
{
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

// Pre-split copy of the weights: hi/lo bf16 arrays [n][klen] per layer, K
// padded with zeros (layer 0: 76 -> 80 in the encoding block; the skip layer:
// hidden 256 then encoding 76 then 4 zeros) and the output layer's rows
// padded 13 -> 32.  Source index of (layer, row r, padded column c).
__global__ void __launch_bounds__(256) k_deform_split(const float* __restrict__ params, __bf16* __restrict__ whi,
                                                      __bf16* __restrict__ wlo, float* __restrict__ bias)
{
    using namespace dmlp;
    const size_t i = (size_t)blockIdx.x * 256u + threadIdx.x;
    const size_t total = dw_total();
    // source offsets of each layer in the caller's flat array
    if (i < total) {
        int l = 0;
        while (l < kDepth && i >= dw_off(l + 1)) ++l;
        const DLayer L = dlayer(l);
        const size_t j = i - dw_off(l);
        const int r = (int)(j / (size_t)L.klen), c = (int)(j % (size_t)L.klen);
        size_t src = 0;
        int fan_in = 0, nout = 0;
        for (int q = 0; q <= l; ++q) {
            fan_in = q == 0 ? kIn : q == kSkip ? kW + kIn : kW;
            nout = q == kDepth ? kOut : kW;
            if (q < l) src += (size_t)nout * fan_in + nout;
        }
        int sc = -1;   // source column
        if (l == 0) sc = c < kIn ? c : -1;
        else if (l == kSkip) sc = c < kW + kIn ? c : -1;
        else sc = c;
        const float v = (r < nout && sc >= 0) ? params[src + (size_t)r * fan_in + sc] : 0.0f;
        split_bf16(v, whi[i], wlo[i]);
    }
    // biases: [layer][256] (the output layer's 13 then zeros)
    if (i < (size_t)(kDepth + 1) * kW) {
        const int l = (int)(i / kW), r = (int)(i % kW);
        size_t src = 0;
        for (int q = 0; q < l; ++q) {
            const int fi = q == 0 ? kIn : q == kSkip ? kW + kIn : kW;
            const int no = q == kDepth ? kOut : kW;
            src += (size_t)no * fi + no;
        }
        const int fi = l == 0 ? kIn : l == kSkip ? kW + kIn : kW;
        const int no = l == kDepth ? kOut : kW;
        bias[i] = r < no ? params[src + (size_t)no * fi + r] : 0.0f;
    }
}

// Encoding entry j (0..75) of position x and time t, FP32 with exact range
// reduction: sin(2^k pi p) = sin(2 pi r), r = fract(2^(k-1) p), and the power
// of two scaling is exact.
__device__ __forceinline__ float encode_entry(int j, const float x[3], float t)
{
    using namespace dmlp;
    float p;
    int k, kind;   // kind 0: the value itself, 1: sin, 2: cos
    if (j < 3 * (1 + 2 * kLX)) {
        const int blk = j / 3;
        p = x[j % 3];
        kind = blk == 0 ? 0 : ((blk - 1) & 1) + 1;
        k = blk == 0 ? 0 : (blk - 1) >> 1;
    } else {
        const int blk = j - 3 * (1 + 2 * kLX);
        p = t;
        kind = blk == 0 ? 0 : ((blk - 1) & 1) + 1;
        k = blk == 0 ? 0 : (blk - 1) >> 1;
    }
    if (kind == 0) return p;
    const float r = __builtin_amdgcn_fractf(ldexpf(p, k - 1));
    return kind == 1 ? __builtin_amdgcn_sinf(r) : __builtin_amdgcn_cosf(r);
}

template <bool SPLIT>
__global__ void __launch_bounds__(256) k_deform_fwd(int32_t n, const float* __restrict__ mean, float t,
                                                    const __bf16* __restrict__ whi, const __bf16* __restrict__ wlo,
                                                    const float* __restrict__ bias, float* __restrict__ delta,
                                                    __bf16* __restrict__ save)
{
    using namespace dmlp;
    __shared__ __attribute__((aligned(16))) __bf16 ahi[kRows * kRowStride];
    __shared__ __attribute__((aligned(16))) __bf16 alo[kRows * kRowStride];
    const int tid = (int)threadIdx.x, w = tid >> 6, l = tid & 63;
    const int32_t row0 = (int32_t)blockIdx.x * kRows;
    // encoding block (columns 256..335) of every row; zero the padding
    for (int q = tid; q < kRows * kInPad; q += 256) {
        const int r = q / kInPad, j = q % kInPad;
        const int32_t p = row0 + r;
        float v = 0.0f;
        if (j < kIn && p < n) {
            const float x[3] = {mean[3 * (size_t)p], mean[3 * (size_t)p + 1], mean[3 * (size_t)p + 2]};
            v = encode_entry(j, x, t);
        }
        split_bf16(v, ahi[r * kRowStride + kW + j], alo[r * kRowStride + kW + j]);
    }
    __syncthreads();
    const size_t tile = blockIdx.x;
    // lane roles in v_mfma_f32_32x32x16_bf16: A row / B column = l % 32, K sub-block 8 (l / 32)
    const int lr = l & 31, lk = (l >> 5) * 8;
    for (int layer = 0; layer <= kDepth; ++layer) {
        const DLayer L = dlayer(layer);
        const bool out_layer = layer == kDepth;
        if (save && layer >= 1) {   // layer input (hidden block), column-major over the 32 rows
            __bf16* sh = save + ((tile * kSaveCols * 2) + (size_t)(kInPad + (layer - 1) * kW) * 2) * kRows;
            for (int q = tid; q < kW * kRows; q += 256) {
                const int c = q / kRows, r = q % kRows;
                sh[(size_t)c * kRows + r] = ahi[r * kRowStride + c];
                sh[(size_t)kW * kRows + (size_t)c * kRows + r] = alo[r * kRowStride + c];
            }
        } else if (save && layer == 0) {   // the encoding
            __bf16* sh = save + tile * kSaveCols * 2 * kRows;
            for (int q = tid; q < kInPad * kRows; q += 256) {
                const int c = q / kRows, r = q % kRows;
                sh[(size_t)c * kRows + r] = ahi[r * kRowStride + kW + c];
                sh[(size_t)kInPad * kRows + (size_t)c * kRows + r] = alo[r * kRowStride + kW + c];
            }
        }
        const int ntile = out_layer ? (w == 0 ? 1 : 0) : 2;   // 32-column tiles of this wave
        f32x16 acc[2];
        for (int q = 0; q < 2; ++q)
            for (int e = 0; e < 16; ++e) acc[q][e] = 0.0f;
        if (ntile > 0) {
            const __bf16* wh = whi + dw_off(layer);
            const __bf16* wl = wlo + dw_off(layer);
            const int c0 = out_layer ? 0 : 64 * w;
            for (int k = 0; k < L.klen; k += 16) {
                const bf16x8 a_h = *reinterpret_cast<const bf16x8*>(ahi + lr * kRowStride + L.k0 + k + lk);
                const bf16x8 a_l = *reinterpret_cast<const bf16x8*>(alo + lr * kRowStride + L.k0 + k + lk);
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    if (q >= ntile) break;
                    const size_t wo = (size_t)(c0 + 32 * q + lr) * L.klen + k + lk;
                    const bf16x8 b_h = *reinterpret_cast<const bf16x8*>(wh + wo);
                    acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_h, b_h, acc[q], 0, 0, 0);
                    if (SPLIT) {
                        const bf16x8 b_l = *reinterpret_cast<const bf16x8*>(wl + wo);
                        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_h, b_l, acc[q], 0, 0, 0);
                        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_l, b_h, acc[q], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();   // every wave has read this layer's input rows
        // epilogue: D layout of a 32x32 tile -- lane l holds column l % 32,
        // element e holds row 8 (e / 4) + 4 (l / 32) + e % 4
        for (int q = 0; q < ntile; ++q) {
            const int col = (out_layer ? 0 : 64 * w) + 32 * q + lr;
            const float bcol = bias[(size_t)layer * kW + col];
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int r = 8 * (e >> 2) + 4 * (l >> 5) + (e & 3);
                const float z = acc[q][e] + bcol;
                if (out_layer) {
                    const int32_t p = row0 + r;
                    if (col < kOut && p < n) delta[(size_t)p * kOut + col] = z;
                } else {
                    split_bf16(fmaxf(z, 0.0f), ahi[r * kRowStride + col], alo[r * kRowStride + col]);
                }
            }
        }
        __syncthreads();   // the next layer reads the rows just written
    }
}

hipError_t launch_deform_fwd(int32_t n, const float* mean, float t, const float* params, void* ws, int split,
                             float* delta, void* save, hipStream_t s)
{
    using namespace dmlp;
    __bf16* whi = (__bf16*)ws;
    __bf16* wlo = whi + dw_total();
    float* bias = (float*)(wlo + dw_total());
    const size_t total = dw_total();
    hipLaunchKernelGGL(k_deform_split, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, params, whi, wlo,
                       bias);
    if (n > 0) {
        const dim3 grid((unsigned)((n + kRows - 1) / kRows));
        if (split)
            hipLaunchKernelGGL(k_deform_fwd<true>, grid, dim3(256), 0, s, n, mean, t, whi, wlo, bias, delta,
                               (__bf16*)save);
        else
            hipLaunchKernelGGL(k_deform_fwd<false>, grid, dim3(256), 0, s, n, mean, t, whi, wlo, bias, delta,
                               (__bf16*)save);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ backward
//
// dIn_j = dZ_j W_j for layer j (dZ_8 = dL/d offsets; dZ_{j-1} = dIn_j masked by
// the ReLU of the layer input h_j, read from the stored forward activations),
// the encoding's gradient collected from layer 0 and the skip layer, then
// dL/dmean through the encoding's derivative -- one workgroup per 32 rows,
// the same matrix-core tiling as the forward, with the transposed split
// weights as the B operand.  Each dZ_j is also stored per tile, column-major
// over the rows, with its column sums (the bias gradients); a second kernel
// forms the weight gradients dW_j = sum over rows of dZ_j^T a_j as split-K
// matrix products over chunks of tiles, and a third adds the chunks in a
// fixed order (deterministic) into the caller's parameter layout.

// Backward GEMM of layer j: K = out width Kb, output columns nT (the layer's
// input width padded to 32).
__host__ __device__ constexpr int dkb(int j) { return dlayer(j).n; }
__host__ __device__ constexpr int dnt(int j) { return j == 0 ? 96 : j == dmlp::kSkip ? 352 : dmlp::kW; }
__host__ __device__ inline size_t dwt_off(int j)
{
    size_t o = 0;
    for (int i = 0; i < j; ++i) o += (size_t)dnt(i) * dkb(i);
    return o;
}
__host__ __device__ inline size_t dwt_total() { return dwt_off(dmlp::kDepth + 1); }

// Caller-layout geometry of layer j: fan-in, outputs and offset of W_j in the flat array.
__host__ __device__ inline int dfan(int j) { return j == 0 ? dmlp::kIn : j == dmlp::kSkip ? dmlp::kW + dmlp::kIn : dmlp::kW; }
__host__ __device__ inline int dnout(int j) { return j == dmlp::kDepth ? dmlp::kOut : dmlp::kW; }
__host__ __device__ inline size_t dsrc_off(int j)
{
    size_t o = 0;
    for (int i = 0; i < j; ++i) o += (size_t)dnout(i) * dfan(i) + dnout(i);
    return o;
}

// Transposed split weights WT_j [nT][Kb]: WT_j[in][out] = W_j[out][in], zero
// outside the layer's real inputs and outputs.
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
    split_bf16(v, thi[i], tlo[i]);
}

// Stored forward activation a_j (j >= 1: h_j; hi part) at column c, row r of a tile.
__device__ __forceinline__ const __bf16* saved_block(const __bf16* save, size_t tile, int j)
{
    using namespace dmlp;
    // block start of a_j: e (j = 0) at 0, h_j at kInPad + (j - 1) kW columns; each block is hi then lo
    const size_t col0 = j == 0 ? 0 : (size_t)kInPad + (size_t)(j - 1) * kW;
    return save + (tile * kSaveCols * 2 + col0 * 2) * kRows;
}

// Per-tile dZ storage: layers 0..7 256 columns, layer 8 32 columns, each hi then lo, column-major over the rows.
__host__ __device__ constexpr size_t dz_cols_total() { return (size_t)dmlp::kDepth * dmlp::kW + dmlp::kOutPad; }
__host__ __device__ inline size_t dz_block(int j) { return (size_t)j * dmlp::kW * 2 * dmlp::kRows; }

template <bool SPLIT>
__global__ void __launch_bounds__(256) k_deform_bwd_rows(int32_t n, const float* __restrict__ mean, float t,
                                                         const float* __restrict__ ddelta,
                                                         const __bf16* __restrict__ thi,
                                                         const __bf16* __restrict__ tlo,
                                                         const __bf16* __restrict__ save, __bf16* __restrict__ dz,
                                                         float* __restrict__ dbp, float* __restrict__ dmean)
{
    using namespace dmlp;
    constexpr int kGs = kW + 8;   // LDS row stride of the dZ operand
    __shared__ __attribute__((aligned(16))) __bf16 ghi[kRows * kGs];
    __shared__ __attribute__((aligned(16))) __bf16 glo[kRows * kGs];
    __shared__ float de[kRows * kInPad];
    __shared__ float dbs[kW];
    const int tid = (int)threadIdx.x, w = tid >> 6, l = tid & 63;
    const size_t tile = blockIdx.x;
    const int32_t row0 = (int32_t)blockIdx.x * kRows;
    const int lr = l & 31, lk = (l >> 5) * 8;
    __bf16* dzt = dz + tile * dz_cols_total() * 2 * kRows;
    // dZ_8 = dL/d offsets (13 columns of 32), rows past n are zero
    for (int q = tid; q < kRows * kOutPad; q += 256) {
        const int r = q / kOutPad, c = q % kOutPad;
        const int32_t p = row0 + r;
        const float v = (c < kOut && p < n) ? ddelta[(size_t)p * kOut + c] : 0.0f;
        split_bf16(v, ghi[r * kGs + c], glo[r * kGs + c]);
        __bf16* b8 = dzt + dz_block(kDepth);
        b8[(size_t)c * kRows + r] = ghi[r * kGs + c];
        b8[(size_t)kOutPad * kRows + (size_t)c * kRows + r] = glo[r * kGs + c];
    }
    for (int q = tid; q < kRows * kInPad; q += 256) de[q] = 0.0f;
    if (tid < kOutPad) {   // bias gradient of the output layer: column sums of dZ_8
        float sacc = 0.0f;
        for (int r = 0; r < kRows; ++r) {
            const int32_t p = row0 + r;
            sacc += (tid < kOut && p < n) ? ddelta[(size_t)p * kOut + tid] : 0.0f;
        }
        dbp[(tile * (kDepth + 1) + kDepth) * kW + tid] = sacc;
    }
    __syncthreads();
    for (int j = kDepth; j >= 0; --j) {
        const int Kb = dkb(j), NT = dnt(j);
        const int ntiles = NT / 32;
        const __bf16* th = thi + dwt_off(j);
        const __bf16* tl = tlo + dwt_off(j);
        f32x16 acc[3];
        for (int q = 0; q < 3; ++q)
            for (int e = 0; e < 16; ++e) acc[q][e] = 0.0f;
        // this wave's 32-column tiles: w, w + 4, w + 8 (< ntiles)
        for (int k = 0; k < Kb; k += 16) {
            const bf16x8 a_h = *reinterpret_cast<const bf16x8*>(ghi + lr * kGs + k + lk);
            const bf16x8 a_l = *reinterpret_cast<const bf16x8*>(glo + lr * kGs + k + lk);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int ct = w + 4 * q;
                if (ct >= ntiles) break;
                const size_t wo = (size_t)(32 * ct + lr) * Kb + k + lk;
                const bf16x8 b_h = *reinterpret_cast<const bf16x8*>(th + wo);
                acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_h, b_h, acc[q], 0, 0, 0);
                if (SPLIT) {
                    const bf16x8 b_l = *reinterpret_cast<const bf16x8*>(tl + wo);
                    acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_h, b_l, acc[q], 0, 0, 0);
                    acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_l, b_h, acc[q], 0, 0, 0);
                }
            }
        }
        __syncthreads();   // every wave has read dZ_j
        if (tid < kW) dbs[tid] = 0.0f;
        __syncthreads();
        // epilogue: lane l holds column 32 ct + l % 32 and rows 8 (e / 4) + 4 (l / 32) + e % 4
        const __bf16* hs = j >= 1 ? saved_block(save, tile, j) : nullptr;   // a_j = h_j (its first 256 columns)
        for (int q = 0; q < 3; ++q) {
            const int ct = w + 4 * q;
            if (ct >= ntiles) break;
            const int col = 32 * ct + lr;
            float csum = 0.0f;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int r = 8 * (e >> 2) + 4 * (l >> 5) + (e & 3);
                const float v = acc[q][e];
                if (j >= 1 && col < kW) {
                    // dZ_{j-1} = dIn_j where h_j > 0
                    const float h = (float)hs[(size_t)col * kRows + r];
                    const float d = h > 0.0f ? v : 0.0f;
                    split_bf16(d, ghi[r * kGs + col], glo[r * kGs + col]);
                    csum += d;
                } else {
                    // encoding block: layer 0 (columns 0..79) or the skip layer (256..335)
                    const int ec = j == 0 ? col : col - kW;
                    if (ec < kInPad) de[r * kInPad + ec] += v;
                }
            }
            if (j >= 1 && col < kW) {   // column sum over the 32 rows (two lane halves)
                csum += __shfl_xor(csum, 32, kWave);
                if (l < 32) dbs[col] = csum;
            }
        }
        __syncthreads();
        if (j >= 1) {
            // store dZ_{j-1} column-major with its bias gradient
            __bf16* bz = dzt + dz_block(j - 1);
            for (int q = tid; q < kW * kRows; q += 256) {
                const int c = q / kRows, r = q % kRows;
                bz[(size_t)c * kRows + r] = ghi[r * kGs + c];
                bz[(size_t)kW * kRows + (size_t)c * kRows + r] = glo[r * kGs + c];
            }
            if (tid < kW) dbp[(tile * (kDepth + 1) + (j - 1)) * kW + tid] = dbs[tid];
            __syncthreads();
        }
    }
    __syncthreads();   // the encoding gradient is complete
    // dL/dmean: the encoding's derivative, FP32 with the forward's range reduction
    if (tid < kRows * 3) {
        const int r = tid / 3, c = tid % 3;
        const int32_t p = row0 + r;
        if (p < n) {
            const float x = mean[3 * (size_t)p + c];
            float g = de[r * kInPad + c];
            for (int k = 0; k < kLX; ++k) {
                const float rr = __builtin_amdgcn_fractf(ldexpf(x, k - 1));
                const float wgt = ldexpf(3.14159265358979f, k);   // 2^k pi
                g += de[r * kInPad + 3 + 6 * k + c] * wgt * __builtin_amdgcn_cosf(rr);
                g -= de[r * kInPad + 6 + 6 * k + c] * wgt * __builtin_amdgcn_sinf(rr);
            }
            dmean[3 * (size_t)p + c] = g;
        }
    }
}

// Weight gradients of layer j, split over chunks of tiles: each wave owns one
// 32 x 32 tile of C = sum over rows of dZ_j^T a_j (rows out, columns in, the
// padded layout of the split weights) and writes its chunk's partial sum.
template <bool SPLIT>
__global__ void __launch_bounds__(256) k_deform_wgrad(int j, int32_t n_tiles, int tiles_per_chunk,
                                                      const __bf16* __restrict__ dz, const __bf16* __restrict__ save,
                                                      float* __restrict__ part)
{
    using namespace dmlp;
    const DLayer L = dlayer(j);
    const int mt = L.n / 32, nt = (L.klen + 31) / 32;
    const int w = (int)(threadIdx.x >> 6), l = (int)(threadIdx.x & 63);
    const int ctile = (int)blockIdx.x * 4 + w;
    if (ctile >= mt * nt) return;   // whole wave
    const int mi = ctile / nt, ni = ctile % nt;
    const int chunk = (int)blockIdx.y;
    const int32_t t0 = chunk * tiles_per_chunk, t1 = min(n_tiles, t0 + tiles_per_chunk);
    const int lr = l & 31, lk = (l >> 5) * 8;
    const int m = 32 * mi + lr;    // output unit (A row)
    const int c = 32 * ni + lr;    // input column (B column) in the layer's padded input
    // where input column c lives in the stored activations: block, column, valid
    int blk, bc;
    bool cvalid = c < L.klen;
    if (j == 0) { blk = 0; bc = c; cvalid = c < kInPad; }
    else if (j == kSkip) { blk = c < kW ? j : 0; bc = c < kW ? c : c - kW; cvalid = bc < (c < kW ? kW : kInPad); }
    else { blk = j; bc = c; }
    const int bcols = blk == 0 ? kInPad : kW;   // columns of that block (hi plane size)
    const int zcols = j == kDepth ? kOutPad : kW;
    f32x16 acc;
    for (int e = 0; e < 16; ++e) acc[e] = 0.0f;
    for (int32_t tt = t0; tt < t1; ++tt) {
        const __bf16* zb = dz + (size_t)tt * dz_cols_total() * 2 * kRows + dz_block(j);
        const __bf16* sb = saved_block(save, (size_t)tt, blk);
#pragma unroll
        for (int k = 0; k < kRows; k += 16) {
            const bf16x8 a_h = *reinterpret_cast<const bf16x8*>(zb + (size_t)m * kRows + k + lk);
            bf16x8 b_h, b_l;
            if (cvalid) {
                b_h = *reinterpret_cast<const bf16x8*>(sb + (size_t)bc * kRows + k + lk);
                b_l = *reinterpret_cast<const bf16x8*>(sb + (size_t)bcols * kRows + (size_t)bc * kRows + k + lk);
            } else {
                for (int e = 0; e < 8; ++e) b_h[e] = b_l[e] = (__bf16)0.0f;
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_h, b_h, acc, 0, 0, 0);
            if (SPLIT) {
                const bf16x8 a_l = *reinterpret_cast<const bf16x8*>(zb + (size_t)zcols * kRows + (size_t)m * kRows + k + lk);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_h, b_l, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_l, b_h, acc, 0, 0, 0);
            }
        }
    }
    // D: lane l holds C column 32 ni + l % 32, rows 32 mi + 8 (e / 4) + 4 (l / 32) + e % 4
    float* pc = part + (size_t)chunk * dw_total() + dw_off(j);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int row = 32 * mi + 8 * (e >> 2) + 4 * (l >> 5) + (e & 3);
        const int col = 32 * ni + lr;
        if (col < L.klen) pc[(size_t)row * L.klen + col] = acc[e];
    }
}

// Bias gradients per chunk of tiles: thread r of chunk k sums unit r of every
// layer over the chunk's tiles, in tile order.
__global__ void __launch_bounds__(256) k_deform_bias_part(int32_t n_tiles, int tiles_per_chunk,
                                                          const float* __restrict__ dbp, float* __restrict__ bpart)
{
    using namespace dmlp;
    const int r = (int)threadIdx.x, chunk = (int)blockIdx.x;
    const int32_t t0 = chunk * tiles_per_chunk, t1 = min(n_tiles, t0 + tiles_per_chunk);
    for (int j = 0; j <= kDepth; ++j) {
        float acc = 0.0f;
        for (int32_t tt = t0; tt < t1; ++tt) acc += dbp[((size_t)tt * (kDepth + 1) + j) * kW + r];
        bpart[((size_t)chunk * (kDepth + 1) + j) * kW + r] = acc;
    }
}

// Sum the chunks' partial weight and bias gradients in a fixed order into the
// caller's parameter layout.
__global__ void __launch_bounds__(256) k_deform_reduce(int chunks, const float* __restrict__ part,
                                                       const float* __restrict__ bpart, float* __restrict__ dparams)
{
    using namespace dmlp;
    const size_t i = (size_t)blockIdx.x * 256u + threadIdx.x;
    const size_t total = dsrc_off(kDepth + 1);
    if (i >= total) return;
    int j = 0;
    while (j < kDepth && i >= dsrc_off(j + 1)) ++j;
    const size_t q = i - dsrc_off(j);
    const int fan = dfan(j), no = dnout(j);
    float acc = 0.0f;
    if (q < (size_t)no * fan) {   // weight (out r, in c) -> padded column c (same index: padding comes after)
        const int r = (int)(q / (size_t)fan), c = (int)(q % (size_t)fan);
        const size_t pi = dw_off(j) + (size_t)r * dlayer(j).klen + c;
        for (int k = 0; k < chunks; ++k) acc += part[(size_t)k * dw_total() + pi];
    } else {                      // bias
        const int r = (int)(q - (size_t)no * fan);
        for (int k = 0; k < chunks; ++k) acc += bpart[((size_t)k * (kDepth + 1) + j) * kW + r];
    }
    dparams[i] = acc;
}

constexpr int kTilesPerChunk = 128;

hipError_t launch_deform_bwd(int32_t n, const float* mean, float t, const float* params, void* ws, int split,
                             const float* ddelta, float* dparams, float* dmean, hipStream_t s)
{
    using namespace dmlp;
    const int32_t n_tiles = (n + kRows - 1) / kRows;
    const int chunks = (n_tiles + kTilesPerChunk - 1) / kTilesPerChunk;
    char* base = (char*)ws;
    const size_t wbytes = (dw_total() * 2 * sizeof(__bf16) + (size_t)(kDepth + 1) * kW * sizeof(float) + 255) / 256 * 256;
    const __bf16* save = (const __bf16*)(base + wbytes);
    const size_t sbytes = ((size_t)n_tiles * kSaveCols * 2 * kRows * sizeof(__bf16) + 255) / 256 * 256;
    char* scr = base + wbytes + sbytes;
    __bf16* thi = (__bf16*)scr;
    __bf16* tlo = thi + dwt_total();
    char* after_t = scr + (dwt_total() * 2 * sizeof(__bf16) + 255) / 256 * 256;
    __bf16* dz = (__bf16*)after_t;
    float* dbp = (float*)(after_t + ((size_t)n_tiles * dz_cols_total() * 2 * kRows * sizeof(__bf16) + 255) / 256 * 256);
    float* bpart = dbp + ((size_t)n_tiles * (kDepth + 1) * kW + 63) / 64 * 64;
    float* part = bpart + (size_t)std::max(chunks, 1) * (kDepth + 1) * kW;
    hipLaunchKernelGGL(k_deform_splitT, dim3((unsigned)((dwt_total() + 255) / 256)), dim3(256), 0, s, params, thi,
                       tlo);
    if (n_tiles > 0) {
        if (split)
            hipLaunchKernelGGL(k_deform_bwd_rows<true>, dim3((unsigned)n_tiles), dim3(256), 0, s, n, mean, t, ddelta,
                               thi, tlo, save, dz, dbp, dmean);
        else
            hipLaunchKernelGGL(k_deform_bwd_rows<false>, dim3((unsigned)n_tiles), dim3(256), 0, s, n, mean, t,
                               ddelta, thi, tlo, save, dz, dbp, dmean);
        for (int j = 0; j <= kDepth; ++j) {
            const DLayer L = dlayer(j);
            const int ct = (L.n / 32) * ((L.klen + 31) / 32);
            const dim3 grid((unsigned)((ct + 3) / 4), (unsigned)chunks);
            if (split)
                hipLaunchKernelGGL(k_deform_wgrad<true>, grid, dim3(256), 0, s, j, n_tiles, kTilesPerChunk, dz, save,
                                   part);
            else
                hipLaunchKernelGGL(k_deform_wgrad<false>, grid, dim3(256), 0, s, j, n_tiles, kTilesPerChunk, dz, save,
                                   part);
        }
    }
    if (n_tiles > 0)
        hipLaunchKernelGGL(k_deform_bias_part, dim3((unsigned)chunks), dim3(256), 0, s, n_tiles, kTilesPerChunk, dbp,
                           bpart);
    const size_t total = dsrc_off(kDepth + 1);
    hipLaunchKernelGGL(k_deform_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       n_tiles > 0 ? chunks : 0, part, bpart, dparams);
    return hipGetLastError();
}

size_t deform_weight_bytes()
{
    return (dw_total() * 2 * sizeof(__bf16) + (size_t)(dmlp::kDepth + 1) * dmlp::kW * sizeof(float) + 255) / 256 * 256;
}

size_t deform_save_bytes(int64_t n)
{
    const int64_t tiles = (n + dmlp::kRows - 1) / dmlp::kRows;
    return ((size_t)tiles * dmlp::kSaveCols * 2 * dmlp::kRows * sizeof(__bf16) + 255) / 256 * 256;
}

size_t deform_bwd_scratch_bytes(int64_t n)
{
    using namespace dmlp;
    const int64_t tiles = (n + kRows - 1) / kRows;
    const int64_t chunks = (tiles + kTilesPerChunk - 1) / kTilesPerChunk;
    return (dwt_total() * 2 * sizeof(__bf16) + 255) / 256 * 256 +
           ((size_t)tiles * dz_cols_total() * 2 * kRows * sizeof(__bf16) + 255) / 256 * 256 +
           ((size_t)tiles * (kDepth + 1) * kW + 63) / 64 * 64 * sizeof(float) +
           (size_t)std::max<int64_t>(chunks, 1) * ((kDepth + 1) * kW + dw_total()) * sizeof(float);
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
    wipes_status st = deform_check(ctx, precision, params, n, mean, workspace, workspace_bytes, 1);
    if (st != WIPES_OK) return st;
    if (!d_params || (n > 0 && (!d_offsets || !d_mean)))
        return fail(ctx, WIPES_ERR_INVALID, "d_offsets, d_params and d_mean must be set");
    const hipError_t e = launch_deform_bwd((int32_t)n, mean, time, params, workspace,
                                           precision == WIPES_DEFORM_BF16X3, d_offsets, d_params, d_mean,
                                           (hipStream_t)stream);
    return e == hipSuccess ? WIPES_OK : hip_fail(ctx, e, "deform bwd");
}

}  // extern "C"
