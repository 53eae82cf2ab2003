// Device-wide exclusive scan and stable LSD radix sort of (uint32 key, uint32 value).
//
// Both are written for 64-lane waves: a workgroup of 256 threads owns a tile
// of elements (4096; 2048 for radix sorts of up to 2^21 keys, which need the
// extra workgroups to fill the chip), each wave a contiguous quarter of it,
// so loads are fully coalesced and the in-tile order (wave, round, lane) is
// the element order.
// The radix pass ranks a wave's 64 elements per round with ballot-based digit
// matching (one ballot per digit bit), accumulates per-wave digit counters in
// LDS, then stages the tile in LDS in sorted order and writes it out so that
// runs of equal digits go to HBM as contiguous stores.
//
// Element counts may live in device memory (instance counts produced on the
// device are never read back inside a captured graph); grids are sized by an
// upper bound and surplus workgroups exit.
#include <algorithm>

#include "common.hpp"

namespace wipes {

constexpr int kTile = 4096;      // elements per workgroup
constexpr int kItems = 16;       // per thread
constexpr int kBlock = 256;

__device__ __forceinline__ uint32_t load_n(uint32_t n_host, const uint32_t* __restrict__ n_dev)
{
    return n_dev ? *n_dev : n_host;
}

// ------------------------------------------------------------------ scan

// block_sums[b] = sum of vals[gather ? gather[i] : i] over the tile of block b.
template <int ITEMS>
__global__ void __launch_bounds__(kBlock) k_block_reduce(const uint32_t* __restrict__ vals,
                                                         const uint32_t* __restrict__ gather, uint32_t n_host,
                                                         const uint32_t* __restrict__ n_dev,
                                                         uint32_t* __restrict__ block_sums)
{
    __shared__ uint32_t s_w[kBlock / kWave];
    const uint32_t n = load_n(n_host, n_dev);
    const uint32_t base = blockIdx.x * (uint32_t)(ITEMS * kBlock);
    uint32_t acc = 0;
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t i = base + j * kBlock + threadIdx.x;
        if (i < n) acc += vals[gather ? gather[i] : i];
    }
    acc = wave_sum_u32(acc);
    if (lane_id() == 0) s_w[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kBlock / kWave; ++w) t += s_w[w];
        block_sums[blockIdx.x] = t;
    }
}

// Exclusive scan of block_sums[0..nb) in place (one workgroup); *total = sum.
// If cap != 0 and the total exceeds it, *n_eff = 0 and *overflow = 1, else
// *n_eff = total (n_eff/overflow may be NULL).
__global__ void __launch_bounds__(kBlock) k_scan_block_sums(uint32_t* __restrict__ block_sums, uint32_t nb,
                                                            uint32_t* __restrict__ total, uint32_t cap,
                                                            uint32_t* __restrict__ n_eff,
                                                            uint32_t* __restrict__ overflow,
                                                            uint32_t* __restrict__ total_host)
{
    // a thread scans 8 consecutive sums in registers: one block-wide combine
    // per 2048 sums
    constexpr int IPT = 8, NW = kBlock / kWave;
    __shared__ uint32_t s_w[NW];
    const int w = threadIdx.x / kWave;
    uint32_t carry = 0;
    for (uint32_t c = 0; c < nb; c += IPT * kBlock) {
        const uint32_t i0 = c + threadIdx.x * (uint32_t)IPT;
        uint32_t v[IPT], sum = 0;
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            v[j] = i0 + j < nb ? block_sums[i0 + j] : 0u;
            sum += v[j];
        }
        uint32_t wt;
        uint32_t ex = wave_excl_scan_u32(sum, &wt);
        if (lane_id() == 0) s_w[w] = wt;
        __syncthreads();
        uint32_t tot = 0;
#pragma unroll
        for (int x = 0; x < NW; ++x) {
            const uint32_t t = s_w[x];
            if (x < w) ex += t;
            tot += t;
        }
        ex += carry;
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            if (i0 + j < nb) block_sums[i0 + j] = ex;
            ex += v[j];
        }
        carry += tot;
        __syncthreads();   // s_w is rewritten by the next chunk
    }
    if (threadIdx.x == 0) {
        const uint32_t t = carry;
        *total = t;
        if (total_host) {   // pinned host word: the host reads it once this kernel has completed
            *total_host = t;
            __threadfence_system();
        }
        if (n_eff) {
            const bool over = cap != 0u && t > cap;
            *n_eff = over ? 0u : t;
            if (overflow) *overflow = over ? 1u : 0u;
        }
    }
}

// out[i] = exclusive prefix of vals (through gather) + scanned block sum.
template <int ITEMS>
__global__ void __launch_bounds__(kBlock) k_scan_apply(const uint32_t* __restrict__ vals,
                                                       const uint32_t* __restrict__ gather, uint32_t n_host,
                                                       const uint32_t* __restrict__ n_dev,
                                                       const uint32_t* __restrict__ block_sums,
                                                       uint32_t* __restrict__ out, uint32_t* __restrict__ out2,
                                                       uint32_t stride2)
{
    __shared__ uint32_t s_w[kBlock / kWave];
    const uint32_t n = load_n(n_host, n_dev);
    const uint32_t base = blockIdx.x * (uint32_t)(ITEMS * kBlock);
    // each wave owns a contiguous quarter of the tile: 16 rounds of 64
    const int w = threadIdx.x / kWave, l = lane_id();
    const uint32_t wbase = base + (uint32_t)w * (uint32_t)(ITEMS * kBlock / 4);
    uint32_t v[ITEMS];
    uint32_t wsum = 0;
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t i = wbase + j * kWave + l;
        v[j] = i < n ? vals[gather ? gather[i] : i] : 0u;
        wsum += v[j];
    }
    wsum = wave_sum_u32(wsum);
    if (l == 0) s_w[w] = wsum;
    __syncthreads();
    uint32_t run = block_sums[blockIdx.x];
    for (int k = 0; k < w; ++k) run += s_w[k];
    for (int j = 0; j < ITEMS; ++j) {
        uint32_t t;
        const uint32_t ex = wave_excl_scan_u32(v[j], &t);
        const uint32_t i = wbase + j * kWave + l;
        if (i < n) {
            out[i] = run + ex;
            if (out2) out2[(size_t)i * stride2] = run + ex;
        }
        run += t;
    }
}

// ------------------------------------------------------------ radix sort

// hist[d * nblocks + b] = number of elements of tile b with digit d.
// Each thread counts ITEMS consecutive keys and adds a run of equal digits
// with one LDS atomic: after a pass over the low digits the next digit comes
// in long runs, and lanes adding to one counter at once are serialised.
template <int BITS, int ITEMS>
__global__ void __launch_bounds__(kBlock) k_radix_hist(const uint32_t* __restrict__ keys, uint32_t n_host,
                                                       const uint32_t* __restrict__ n_dev, int shift,
                                                       uint32_t nblocks, uint32_t* __restrict__ hist)
{
    static_assert(ITEMS % 4 == 0, "keys are read four at a time");
    constexpr int ND = 1 << BITS;
    __shared__ uint32_t s_h[ND];
    for (int d = threadIdx.x; d < ND; d += kBlock) s_h[d] = 0;
    __syncthreads();
    const uint32_t n = load_n(n_host, n_dev);
    const uint32_t i0 = blockIdx.x * (uint32_t)(ITEMS * kBlock) + threadIdx.x * (uint32_t)ITEMS;
    if (i0 < n) {
        uint32_t k[ITEMS];
        if (i0 + ITEMS <= n) {
            const uint4* q = reinterpret_cast<const uint4*>(keys + i0);
#pragma unroll
            for (int j = 0; j < ITEMS / 4; ++j) {
                const uint4 x = q[j];
                k[4 * j] = x.x;
                k[4 * j + 1] = x.y;
                k[4 * j + 2] = x.z;
                k[4 * j + 3] = x.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) k[j] = i0 + j < n ? keys[i0 + j] : 0u;
        }
        const uint32_t m = min((uint32_t)ITEMS, n - i0);   // valid keys of this thread, >= 1
        uint32_t prev = (k[0] >> shift) & (ND - 1), run = 1;
#pragma unroll
        for (int j = 1; j < ITEMS; ++j) {
            if ((uint32_t)j < m) {
                const uint32_t d = (k[j] >> shift) & (ND - 1);
                if (d == prev) {
                    ++run;
                } else {
                    atomicAdd(&s_h[prev], run);
                    prev = d;
                    run = 1;
                }
            }
        }
        atomicAdd(&s_h[prev], run);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < ND; d += kBlock) hist[(uint32_t)d * nblocks + blockIdx.x] = s_h[d];
}

// Exclusive scan of each digit's row of hist across blocks; row totals to
// dtot.  A thread scans IPT consecutive entries in registers, so a row of up
// to IPT * kBlock blocks takes one block-wide combine (two barriers).
template <int IPT>
__global__ void __launch_bounds__(kBlock) k_radix_rowscan(uint32_t* __restrict__ hist, uint32_t nblocks,
                                                          uint32_t* __restrict__ dtot)
{
    constexpr int NW = kBlock / kWave;
    __shared__ uint32_t s_w[NW];
    uint32_t* row = hist + (uint32_t)blockIdx.x * nblocks;
    const int w = threadIdx.x / kWave;
    uint32_t carry = 0;
    for (uint32_t c = 0; c < nblocks; c += IPT * kBlock) {
        const uint32_t i0 = c + threadIdx.x * (uint32_t)IPT;
        uint32_t v[IPT], sum = 0;
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            v[j] = i0 + j < nblocks ? row[i0 + j] : 0u;
            sum += v[j];
        }
        uint32_t wt;
        uint32_t ex = wave_excl_scan_u32(sum, &wt);
        if (lane_id() == 0) s_w[w] = wt;
        __syncthreads();
        uint32_t tot = 0;
#pragma unroll
        for (int x = 0; x < NW; ++x) {
            const uint32_t t = s_w[x];
            if (x < w) ex += t;
            tot += t;
        }
        ex += carry;
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            if (i0 + j < nblocks) row[i0 + j] = ex;
            ex += v[j];
        }
        carry += tot;
        __syncthreads();   // s_w is rewritten by the next chunk
    }
    if (threadIdx.x == 0) dtot[blockIdx.x] = carry;
}

// W: a second payload (w_in/w_out) is permuted with the values.
template <int BITS, bool W, int ITEMS>
__global__ void __launch_bounds__(kBlock) k_radix_scatter(const uint32_t* __restrict__ keys_in,
                                                          const uint32_t* __restrict__ vals_in,
                                                          const uint32_t* __restrict__ w_in, uint32_t n_host,
                                                          const uint32_t* __restrict__ n_dev, int shift,
                                                          uint32_t nblocks, const uint32_t* __restrict__ hist,
                                                          const uint32_t* __restrict__ dtot,
                                                          uint32_t* __restrict__ keys_out,
                                                          uint32_t* __restrict__ vals_out,
                                                          uint32_t* __restrict__ w_out)
{
    constexpr int ND = 1 << BITS;
    constexpr int NW = kBlock / kWave;
    constexpr int TILE = ITEMS * kBlock;
    __shared__ uint32_t s_keys[TILE];
    __shared__ uint32_t s_vals[TILE];
    __shared__ uint32_t s_w[W ? TILE : 1];
    __shared__ uint32_t s_wcnt[NW][ND];
    __shared__ uint32_t s_dbase[ND];
    __shared__ uint32_t s_gbase[ND];
    __shared__ uint32_t s_part[2][NW];

    const uint32_t n = load_n(n_host, n_dev);
    const uint32_t base = blockIdx.x * TILE;
    if (base >= n) return;
    const int w = threadIdx.x / kWave, l = lane_id();
    for (int d = threadIdx.x; d < NW * ND; d += kBlock) (&s_wcnt[0][0])[d] = 0;
    __syncthreads();

    const uint32_t wbase = base + (uint32_t)w * (TILE / NW);
    const uint64_t lt_mask = (l == 0) ? 0ull : (~0ull >> (64 - l));
    uint32_t k[ITEMS], v[ITEMS], ww[W ? ITEMS : 1], rk[ITEMS];
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t i = wbase + j * kWave + l;
        const bool ok = i < n;
        k[j] = ok ? keys_in[i] : 0u;
        v[j] = ok ? vals_in[i] : 0u;
        if (W) ww[j] = ok ? w_in[i] : 0u;
    }
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t i = wbase + j * kWave + l;
        const bool ok = i < n;
        const uint32_t dig = (k[j] >> shift) & (ND - 1);
        uint64_t peers = __ballot(ok);
        for (int b = 0; b < BITS; ++b) {
            const bool bit = (dig >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t before = (uint32_t)__popcll(peers & lt_mask);
        uint32_t old = 0;
        if (ok) old = s_wcnt[w][dig];
        rk[j] = old + before;
        // the lowest lane of each digit group publishes the new count; every
        // lane of the wave has read the old value above (in-order LDS per wave)
        if (ok && before == 0) s_wcnt[w][dig] = old + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // per digit: exclusive prefix over waves, then over digits within the tile
    for (int d = threadIdx.x; d < ND; d += kBlock) {
        uint32_t run = 0;
        for (int ww = 0; ww < NW; ++ww) {
            const uint32_t c = s_wcnt[ww][d];
            s_wcnt[ww][d] = run;
            run += c;
        }
        s_dbase[d] = run;   // tile total of digit d (scanned below)
    }
    __syncthreads();
    {
        // exclusive scans of the ND tile totals and of the ND global digit
        // totals over the whole workgroup: thread t owns DPT consecutive
        // digits (all loads issued up front), waves combine through LDS
        constexpr int DPT = (ND + kBlock - 1) / kBlock;
        const int d0 = threadIdx.x * DPT;
        uint32_t tt[DPT], gt[DPT], hb[DPT], st = 0, sg = 0;
        for (int i = 0; i < DPT; ++i) {
            const int d = d0 + i;
            tt[i] = d < ND ? s_dbase[d] : 0u;
            gt[i] = d < ND ? dtot[d] : 0u;
            hb[i] = d < ND ? hist[(uint32_t)d * nblocks + blockIdx.x] : 0u;
            st += tt[i];
            sg += gt[i];
        }
        uint32_t wt, wg;
        uint32_t ot = wave_excl_scan_u32(st, &wt);
        uint32_t og = wave_excl_scan_u32(sg, &wg);
        if (l == 0) {
            s_part[0][w] = wt;
            s_part[1][w] = wg;
        }
        __syncthreads();
        for (int x = 0; x < w; ++x) {
            ot += s_part[0][x];
            og += s_part[1][x];
        }
        for (int i = 0; i < DPT; ++i) {
            const int d = d0 + i;
            if (d < ND) {
                s_dbase[d] = ot;
                s_gbase[d] = og + hb[i];
            }
            ot += tt[i];
            og += gt[i];
        }
    }
    __syncthreads();
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t i = wbase + j * kWave + l;
        if (i < n) {
            const uint32_t dig = (k[j] >> shift) & (ND - 1);
            const uint32_t pos = s_dbase[dig] + s_wcnt[w][dig] + rk[j];
            s_keys[pos] = k[j];
            s_vals[pos] = v[j];
            if (W) s_w[pos] = ww[j];
        }
    }
    __syncthreads();
    const uint32_t cnt = min((uint32_t)TILE, n - base);
    for (uint32_t p = threadIdx.x; p < cnt; p += kBlock) {
        const uint32_t key = s_keys[p];
        const uint32_t dig = (key >> shift) & (ND - 1);
        const uint32_t g = s_gbase[dig] + (p - s_dbase[dig]);
        keys_out[g] = key;
        vals_out[g] = s_vals[p];
        if (W) w_out[g] = s_w[p];
    }
}

// ------------------------------------------------------------- host side

// Scans of up to 2^21 values use 2048-value workgroups (8 per thread), which
// a scan of ~1 M values needs to fill the chip; larger ones 4096.
static uint32_t scan_tile(uint32_t max_n) { return max_n <= (1u << 21) ? 8u * kBlock : (uint32_t)kTile; }
uint32_t scan_blocks(uint32_t max_n) { return (max_n + scan_tile(max_n) - 1) / scan_tile(max_n); }

hipError_t scan_excl(const uint32_t* vals, const uint32_t* gather, uint32_t n_host, const uint32_t* n_dev,
                     uint32_t max_n, uint32_t* block_sums, uint32_t* out, uint32_t* total, uint32_t cap,
                     uint32_t* n_eff, uint32_t* overflow, hipStream_t s, uint32_t* total_host, uint32_t* out2,
                     uint32_t stride2)
{
    const uint32_t nb = scan_blocks(max_n);
    const bool small = scan_tile(max_n) != (uint32_t)kTile;
    if (nb > 0) {
        if (small)
            hipLaunchKernelGGL(k_block_reduce<8>, dim3(nb), dim3(kBlock), 0, s, vals, gather, n_host, n_dev,
                               block_sums);
        else
            hipLaunchKernelGGL(k_block_reduce<kItems>, dim3(nb), dim3(kBlock), 0, s, vals, gather, n_host, n_dev,
                               block_sums);
    }
    hipLaunchKernelGGL(k_scan_block_sums, dim3(1), dim3(kBlock), 0, s, block_sums, nb, total, cap, n_eff, overflow,
                       total_host);
    if (nb > 0) {
        if (small)
            hipLaunchKernelGGL(k_scan_apply<8>, dim3(nb), dim3(kBlock), 0, s, vals, gather, n_host, n_dev,
                               block_sums, out, out2, stride2);
        else
            hipLaunchKernelGGL(k_scan_apply<kItems>, dim3(nb), dim3(kBlock), 0, s, vals, gather, n_host, n_dev,
                               block_sums, out, out2, stride2);
    }
    return hipGetLastError();
}

template <int BITS, int ITEMS>
static void radix_pass_t(const uint32_t* ki, const uint32_t* vi, const uint32_t* wi, uint32_t* ko, uint32_t* vo,
                         uint32_t* wo, uint32_t n_host, const uint32_t* n_dev, uint32_t nb, int shift, uint32_t* hist,
                         uint32_t* dtot, hipStream_t s)
{
    hipLaunchKernelGGL((k_radix_hist<BITS, ITEMS>), dim3(nb), dim3(kBlock), 0, s, ki, n_host, n_dev, shift, nb, hist);
    hipLaunchKernelGGL(k_radix_rowscan<8>, dim3(1 << BITS), dim3(kBlock), 0, s, hist, nb, dtot);
    if (wi)
        hipLaunchKernelGGL((k_radix_scatter<BITS, true, ITEMS>), dim3(nb), dim3(kBlock), 0, s, ki, vi, wi, n_host,
                           n_dev, shift, nb, hist, dtot, ko, vo, wo);
    else
        hipLaunchKernelGGL((k_radix_scatter<BITS, false, ITEMS>), dim3(nb), dim3(kBlock), 0, s, ki, vi, nullptr,
                           n_host, n_dev, shift, nb, hist, dtot, ko, vo, nullptr);
}

// Sorts of up to kSmallSort keys use 2048-key workgroups (8 keys per
// thread): twice the workgroups of 4096-key ones, which a sort of ~1 M keys
// needs to occupy the chip; larger sorts keep 4096 for longer runs of equal
// digits in the scatter's stores.
constexpr uint32_t kSmallSort = 1u << 21;
uint32_t radix_tile(uint32_t max_n) { return max_n <= kSmallSort ? 8u * kBlock : (uint32_t)kTile; }

// Workgroups of a radix sort of at most max_n keys (what its histograms hold).
uint32_t radix_blocks(uint32_t max_n) { return (max_n + radix_tile(max_n) - 1u) / radix_tile(max_n); }

// The most workgroups any sort of up to cap keys uses (the block count is not
// monotonic in the key count where the tile size changes).
uint32_t radix_max_blocks(uint32_t cap)
{
    return std::max(radix_blocks(cap), radix_blocks(std::min(cap, kSmallSort)));
}

template <int BITS>
static void radix_pass(const uint32_t* ki, const uint32_t* vi, const uint32_t* wi, uint32_t* ko, uint32_t* vo,
                       uint32_t* wo, uint32_t n_host, const uint32_t* n_dev, uint32_t nb, int shift, uint32_t* hist,
                       uint32_t* dtot, bool small, hipStream_t s)
{
    if (small)
        radix_pass_t<BITS, 8>(ki, vi, wi, ko, vo, wo, n_host, n_dev, nb, shift, hist, dtot, s);
    else
        radix_pass_t<BITS, kItems>(ki, vi, wi, ko, vo, wo, n_host, n_dev, nb, shift, hist, dtot, s);
}

// Passes of at most 8-bit digits.  (Wider digits save passes but shorten the
// runs of equal digits in a 4096-element tile, so the scatter's stores stop
// coalescing: three 11-bit passes over 1M depth keys measured slower than
// four 8-bit ones.)
int radix_passes(int nbits) { return nbits <= 0 ? 0 : (nbits + 7) / 8; }
int radix_digit_bits(int nbits)
{
    const int np = radix_passes(nbits);
    return np == 0 ? 0 : (nbits + np - 1) / np;
}

hipError_t radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, uint32_t n_host,
                      const uint32_t* n_dev, uint32_t max_n, int nbits, uint32_t* hist, uint32_t* dtot,
                      int* result_in_1, hipStream_t s, uint32_t* w0, uint32_t* w1)
{
    const int np = radix_passes(nbits);
    *result_in_1 = 0;
    const bool small = radix_tile(max_n) != (uint32_t)kTile;
    const uint32_t nb = radix_blocks(max_n);
    if (np == 0 || nb == 0) return hipGetLastError();
    const int bits = radix_digit_bits(nbits);
    uint32_t *ki = k0, *vi = v0, *wi = w0, *ko = k1, *vo = v1, *wo = w1;
    for (int p = 0; p < np; ++p) {
        const int shift = p * bits;
        switch (bits) {
        case 1: radix_pass<1>(ki, vi, wi, ko, vo, wo, n_host, n_dev, nb, shift, hist, dtot, small, s); break;
        case 2: radix_pass<2>(ki, vi, wi, ko, vo, wo, n_host, n_dev, nb, shift, hist, dtot, small, s); break;
        case 3: radix_pass<3>(ki, vi, wi, ko, vo, wo, n_host, n_dev, nb, shift, hist, dtot, small, s); break;
        case 4: radix_pass<4>(ki, vi, wi, ko, vo, wo, n_host, n_dev, nb, shift, hist, dtot, small, s); break;
        case 5: radix_pass<5>(ki, vi, wi, ko, vo, wo, n_host, n_dev, nb, shift, hist, dtot, small, s); break;
        case 6: radix_pass<6>(ki, vi, wi, ko, vo, wo, n_host, n_dev, nb, shift, hist, dtot, small, s); break;
        case 7: radix_pass<7>(ki, vi, wi, ko, vo, wo, n_host, n_dev, nb, shift, hist, dtot, small, s); break;
        case 8: radix_pass<8>(ki, vi, wi, ko, vo, wo, n_host, n_dev, nb, shift, hist, dtot, small, s); break;
        default: return hipErrorInvalidValue;
        }
        uint32_t* t;
        t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
        t = wi; wi = wo; wo = t;
    }
    *result_in_1 = (np & 1);
    return hipGetLastError();
}

}  // namespace wipes
