// Device-side definitions shared by the gfx950 kernels of the wavelet rasterizer.
//
// Layout decisions (MI355X / CDNA4):
//  * one 64-byte screen record per primitive, so a wave fetches a whole
//    record with wave-uniform (scalar) loads while blending;
//  * per-image descriptors in device memory, so a single launch covers a
//    batch of images of different sizes;
//  * all integer index arithmetic in 32 bits (instances, tiles, pixels of one
//    launch stay below 2^31; the host checks).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/wipes.h"

namespace wipes {

constexpr int kWave = 64;

// Persistent tile queue: kQueueLanes counters, kQueueStride words apart (one
// 256-byte line each); counter x hands out the tiles at positions x, x + 8,
// x + 16, ... of the tile order, so the XCDs (which take workgroups
// round-robin) pull from different lines instead of all contending for one.
constexpr int kQueueLanes = 8;
constexpr int kQueueStride = 64;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kInv2Pi = 0.15915494309189535f;

// Screen record (mirrors wipes_screen_record).  The mean is mx + mxl in
// exact arithmetic (mx = FP32 rounding, mxl = FP32 rounding of the rest).
struct __align__(64) Rec {
    float mx, my, ca, cb, cc, fx, fy, op, r, g, b, mxl, myl;
    float ph;   // carrier phase in revolutions (phi0 / 2 pi)
    uint32_t box0, box1;
};
static_assert(sizeof(Rec) == 64, "screen record must be 64 bytes");

// Per-primitive inputs of the binning stage, written by the projection.
struct Aux {
    float rx, ry;   // padded support half-extents (pixels); rx < 0 marks a culled primitive
    float depth;    // FP32 depth key (alpha mode)
    float Qs;       // padded support threshold: the ellipse q <= Qs holds every pixel the blend accepts
};

// Per-primitive binning result, read by the emission in two 16-byte loads:
// instance count, pixel box, slot base (filled in depth order), and the
// kept tiles of the box's tile rectangle (bit k = k-th tile row-major) when
// the rectangle has at most 64 tiles (full = 1: every tile kept).
struct __align__(16) PrimPack {
    uint32_t count, box0, box1, base;
    uint32_t mlo, mhi, full, pad;
};

// Per-image descriptor, uploaded once per call into the screen buffer.
struct __align__(16) ImgDesc {
    const float* mean;
    const float* cov;
    const float* quat;
    const float* scale;
    const float* freq;
    const float* color;
    const float* opac;
    const float* vel;
    const float* phase;   // [n] carrier phase (radians) or null
    const float* sh;      // [n, (deg + 1)^2, 3] spherical-harmonic colour or null
    float* g_mean;
    float* g_cov;
    float* g_quat;
    float* g_scale;
    float* g_freq;
    float* g_color;
    float* g_opac;
    float* g_vel;
    float* g_phase;
    float* g_sh;
    float* out_image;     // optional per-image colour output (forward)
    int32_t prim_begin;   // first global record index of this image
    int32_t n;            // primitives of this image
    int32_t pix_begin;    // first pixel of this image in the per-pixel arrays
    int32_t tile_begin;   // first global tile of this image
    int32_t W, H, tiles_x, tiles_y;
    float fx, fy, cx, cy;
    float view[12];       // rows 0..2 of the world->camera matrix
    float time;
    float limx, limy;     // guard band of x/z and y/z
    float cam_c[3];       // camera centre in world coordinates (spherical-harmonic view direction)
};

// A descriptor table small enough to travel as a kernel argument (the
// kernel that receives it may read it from there and store it for the
// kernels after it).
constexpr int kDescArgMax = 8;
struct DescArgs {
    ImgDesc d[kDescArgMax];
};

// Two word ranges a kernel zeroes on its way (p0/p1 may be null with n 0).
struct Clear2 {
    uint32_t* p0;
    uint32_t n0;
    uint32_t* p1;
    uint32_t n1;
};

// Rasterizer constants as the kernels see them.
struct KParams {
    int32_t mode, cov, tile_w, tile_h, log2_tw, log2_th;
    int32_t freq_xform, sh_degree;
    float alpha_min, alpha_max, T_min, q_add, blur_eps, near_plane;
    float bg[3];
};

// Index of the image owning global element `i` given ascending begin offsets.
// B is small (<= a few hundred); the search is wave-uniform in practice.
template <typename GetBegin>
__device__ __forceinline__ int find_owner(int B, int32_t i, GetBegin begin)
{
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (begin(mid) <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int image_of_prim(const ImgDesc* __restrict__ d, int B, int32_t i)
{
    return find_owner(B, i, [&](int b) { return d[b].prim_begin; });
}

__device__ __forceinline__ int image_of_tile(const ImgDesc* __restrict__ d, int B, int32_t t)
{
    return find_owner(B, t, [&](int b) { return d[b].tile_begin; });
}

__device__ __forceinline__ uint32_t pack16(int32_t a, int32_t b)
{
    return (uint32_t)(a & 0xffff) | ((uint32_t)(b & 0xffff) << 16);
}

__device__ __forceinline__ int32_t lo16(uint32_t v) { return (int32_t)(v & 0xffffu); }
__device__ __forceinline__ int32_t hi16(uint32_t v) { return (int32_t)(v >> 16); }

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Orders this wave's LDS accesses (one wave's LDS instructions execute in
// program order; the fences keep the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave-wide sum, max (results in every lane).
__device__ __forceinline__ int32_t wave_max_i32(int32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o, kWave);
    return v;
}

// Exclusive prefix sum within the wave; returns the wave total in *total.
__device__ __forceinline__ uint32_t wave_excl_scan_u32(uint32_t v, uint32_t* total)
{
    const int l = lane_id();
    uint32_t x = v;
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t y = (uint32_t)__shfl_up((int)x, o, kWave);
        if (l >= o) x += y;
    }
    *total = (uint32_t)__shfl((int)x, kWave - 1, kWave);
    return x - v;
}

}  // namespace wipes
