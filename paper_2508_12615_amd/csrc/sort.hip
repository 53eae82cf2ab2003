// Scan of partial sums and stable LSD radix sort of (uint32 key, uint32 value).
//
// The scan is the middle step of an exclusive prefix: the kernels that
// produce the values also write one sum per 64 of them, one workgroup scans
// those sums here, and the kernels that need the per-element offsets add the
// prefix within their wave themselves -- two launches fewer per prefix, which
// on this chip costs more than the work they did.
//
// The radix sort is written for 64-lane waves: a workgroup of 256 threads
// owns a tile of elements (4096; 2048 for sorts of up to 2^21 keys, which
// need the extra workgroups to fill the chip), each wave a contiguous quarter
// of it, so loads are fully coalesced and the in-tile order (wave, round,
// lane) is the element order.  A pass ranks a wave's 64 elements per round
// with ballot-based digit matching (one ballot per digit bit), accumulates
// per-wave digit counters in LDS, then stages the tile in LDS in sorted order
// and writes it out so that runs of equal digits go to HBM as contiguous
// stores.
//
// Element counts may live in device memory (instance counts produced on the
// device are never read back inside a captured graph); grids are sized by an
// upper bound and surplus workgroups exit.
#include <algorithm>
#include <type_traits>

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

// Exclusive scan of block_sums[0..nb) in place (one workgroup of 1024
// threads); *total = sum.  If cap != 0 and the total exceeds it, *n_eff = 0
// and *overflow = 1, else *n_eff = total (n_eff/overflow may be NULL).
// A round covers 4096 sums: each thread reads four consecutive ones with one
// 16-byte load (the wave's loads are one contiguous kilobyte), and the
// workgroup combines the threads' sums once per round.
constexpr int kSumsBlock = 1024;
__global__ void __launch_bounds__(kSumsBlock) k_scan_block_sums(uint32_t* __restrict__ block_sums, uint32_t nb,
                                                                uint32_t* __restrict__ total, uint32_t cap,
                                                                uint32_t* __restrict__ n_eff,
                                                                uint32_t* __restrict__ overflow,
                                                                uint32_t* __restrict__ total_host,
                                                                uint32_t* __restrict__ clr, uint32_t nclr)
{
    for (uint32_t k = threadIdx.x; k < nclr; k += kSumsBlock) clr[k] = 0u;
    constexpr int NW = kSumsBlock / kWave;
    __shared__ uint32_t s_w[NW];
    const int w = threadIdx.x / kWave;
    uint32_t carry = 0;
    for (uint32_t c = 0; c < nb; c += 4u * kSumsBlock) {
        const uint32_t i0 = c + threadIdx.x * 4u;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (i0 + 4u <= nb) {
            v = *reinterpret_cast<const uint4*>(block_sums + i0);
        } else if (i0 < nb) {
            v.x = block_sums[i0];
            if (i0 + 1u < nb) v.y = block_sums[i0 + 1u];
            if (i0 + 2u < nb) v.z = block_sums[i0 + 2u];
        }
        uint32_t wt;
        uint32_t ex = wave_excl_scan_u32(v.x + v.y + v.z + v.w, &wt);
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
        const uint4 o = make_uint4(ex, ex + v.x, ex + v.x + v.y, ex + v.x + v.y + v.z);
        if (i0 + 4u <= nb) {
            *reinterpret_cast<uint4*>(block_sums + i0) = o;
        } else if (i0 < nb) {
            block_sums[i0] = o.x;
            if (i0 + 1u < nb) block_sums[i0 + 1u] = o.y;
            if (i0 + 2u < nb) block_sums[i0 + 2u] = o.z;
        }
        carry += tot;
        __syncthreads();   // s_w is rewritten by the next round
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

// K16: the keys fit in 16 bits and are staged in LDS as such (6 bytes per
// element instead of 8), with 16-bit per-wave digit counters: six workgroups
// per CU instead of four, so a 6.3 M-key sort runs in one round of
// workgroups rather than one and a half.
template <int BITS, bool K16, int ITEMS>
__global__ void __launch_bounds__(kBlock) k_radix_scatter(const uint32_t* __restrict__ keys_in,
                                                          const uint32_t* __restrict__ vals_in, uint32_t n_host,
                                                          const uint32_t* __restrict__ n_dev, int shift,
                                                          uint32_t nblocks, const uint32_t* __restrict__ hist,
                                                          const uint32_t* __restrict__ dtot,
                                                          uint32_t* __restrict__ keys_out,
                                                          uint32_t* __restrict__ vals_out)
{
    constexpr int ND = 1 << BITS;
    constexpr int NW = kBlock / kWave;
    constexpr int TILE = ITEMS * kBlock;
    using KeyT = typename std::conditional<K16, uint16_t, uint32_t>::type;
    using CntT = KeyT;   // per-wave digit counts and their prefixes (at most a tile)
    static_assert(!K16 || TILE <= 65535, "16-bit counters");
    __shared__ KeyT s_keys[TILE];
    __shared__ uint32_t s_vals[TILE];
    __shared__ CntT s_wcnt[NW][ND];
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
    uint32_t k[ITEMS], v[ITEMS], rk[ITEMS];
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t i = wbase + j * kWave + l;
        const bool ok = i < n;
        k[j] = ok ? keys_in[i] : 0u;
        v[j] = ok ? vals_in[i] : 0u;
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
        if (ok && before == 0) s_wcnt[w][dig] = (CntT)(old + (uint32_t)__popcll(peers));
    }
    __syncthreads();
    // per digit: exclusive prefix over waves, then over digits within the tile
    for (int d = threadIdx.x; d < ND; d += kBlock) {
        uint32_t run = 0;
        for (int ww = 0; ww < NW; ++ww) {
            const uint32_t c = s_wcnt[ww][d];
            s_wcnt[ww][d] = (CntT)run;
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
            s_keys[pos] = (KeyT)k[j];
            s_vals[pos] = v[j];
        }
    }
    __syncthreads();
    const uint32_t cnt = min((uint32_t)TILE, n - base);
    for (uint32_t p = threadIdx.x; p < cnt; p += kBlock) {
        const uint32_t key = (uint32_t)s_keys[p];
        const uint32_t dig = (key >> shift) & (ND - 1);
        const uint32_t g = s_gbase[dig] + (p - s_dbase[dig]);
        keys_out[g] = key;
        vals_out[g] = s_vals[p];
    }
}

// ------------------------------------------------------------- host side

hipError_t scan_sums(uint32_t* sums, uint32_t n, uint32_t* total, uint32_t cap, uint32_t* n_eff, uint32_t* overflow,
                     uint32_t* total_host, hipStream_t s, uint32_t* clr, uint32_t nclr)
{
    hipLaunchKernelGGL(k_scan_block_sums, dim3(1), dim3(kSumsBlock), 0, s, sums, n, total, cap, n_eff, overflow,
                       total_host, clr, nclr);
    return hipGetLastError();
}

template <int BITS, bool K16, int ITEMS>
static void radix_pass_t(const uint32_t* ki, const uint32_t* vi, uint32_t* ko, uint32_t* vo, uint32_t n_host,
                         const uint32_t* n_dev, uint32_t nb, int shift, uint32_t* hist, uint32_t* dtot, hipStream_t s)
{
    hipLaunchKernelGGL((k_radix_hist<BITS, ITEMS>), dim3(nb), dim3(kBlock), 0, s, ki, n_host, n_dev, shift, nb, hist);
    hipLaunchKernelGGL(k_radix_rowscan<8>, dim3(1 << BITS), dim3(kBlock), 0, s, hist, nb, dtot);
    hipLaunchKernelGGL((k_radix_scatter<BITS, K16, ITEMS>), dim3(nb), dim3(kBlock), 0, s, ki, vi, n_host, n_dev,
                       shift, nb, hist, dtot, ko, vo);
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
static void radix_pass(const uint32_t* ki, const uint32_t* vi, uint32_t* ko, uint32_t* vo, uint32_t n_host,
                       const uint32_t* n_dev, uint32_t nb, int shift, uint32_t* hist, uint32_t* dtot, bool small,
                       bool k16, hipStream_t s)
{
    if (small)
        radix_pass_t<BITS, false, 8>(ki, vi, ko, vo, n_host, n_dev, nb, shift, hist, dtot, s);
    else if (k16)
        radix_pass_t<BITS, true, kItems>(ki, vi, ko, vo, n_host, n_dev, nb, shift, hist, dtot, s);
    else
        radix_pass_t<BITS, false, kItems>(ki, vi, ko, vo, n_host, n_dev, nb, shift, hist, dtot, s);
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
                      int* result_in_1, hipStream_t s)
{
    const int np = radix_passes(nbits);
    *result_in_1 = 0;
    const bool small = radix_tile(max_n) != (uint32_t)kTile;
    const bool k16 = nbits <= 16;   // (the keys then fit in 16 bits)
    const uint32_t nb = radix_blocks(max_n);
    if (np == 0 || nb == 0) return hipGetLastError();
    const int bits = radix_digit_bits(nbits);
    uint32_t *ki = k0, *vi = v0, *ko = k1, *vo = v1;
    for (int p = 0; p < np; ++p) {
        const int shift = p * bits;
        switch (bits) {
        case 1: radix_pass<1>(ki, vi, ko, vo, n_host, n_dev, nb, shift, hist, dtot, small, k16, s); break;
        case 2: radix_pass<2>(ki, vi, ko, vo, n_host, n_dev, nb, shift, hist, dtot, small, k16, s); break;
        case 3: radix_pass<3>(ki, vi, ko, vo, n_host, n_dev, nb, shift, hist, dtot, small, k16, s); break;
        case 4: radix_pass<4>(ki, vi, ko, vo, n_host, n_dev, nb, shift, hist, dtot, small, k16, s); break;
        case 5: radix_pass<5>(ki, vi, ko, vo, n_host, n_dev, nb, shift, hist, dtot, small, k16, s); break;
        case 6: radix_pass<6>(ki, vi, ko, vo, n_host, n_dev, nb, shift, hist, dtot, small, k16, s); break;
        case 7: radix_pass<7>(ki, vi, ko, vo, n_host, n_dev, nb, shift, hist, dtot, small, k16, s); break;
        case 8: radix_pass<8>(ki, vi, ko, vo, n_host, n_dev, nb, shift, hist, dtot, small, k16, s); break;
        default: return hipErrorInvalidValue;
        }
        std::swap(ki, ko);
        std::swap(vi, vo);
    }
    *result_in_1 = (np & 1);
    return hipGetLastError();
}

}  // namespace wipes
