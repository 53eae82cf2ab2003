// Autotuner: times the render path of a given batch for every supported tile
// shape and launch form (grid; persistent queue in tile order; persistent
// queue longest list first; grid longest list first) and returns the fastest.  The per-pixel rule is
// tile-independent, so every candidate computes the same image (to FP32
// rounding of tile-relative coordinates); only speed differs.  This is an
// offline call: it allocates and frees its own scratch and synchronises.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "api_internal.hpp"

using namespace wipes;

namespace {

struct Cand {
    int tw, th, persistent;
};

const Cand kCands[] = {{8, 8, 0},  {16, 8, 0},  {8, 16, 0},  {16, 16, 0},  {32, 8, 0},  {32, 16, 0},
                       {8, 8, 1},  {16, 8, 1},  {8, 16, 1},  {16, 16, 1},  {32, 8, 1},  {32, 16, 1},
                       {8, 8, 2},  {16, 8, 2},  {8, 16, 2},  {16, 16, 2},  {32, 8, 2},  {32, 16, 2},
                       {8, 8, 3},  {16, 8, 3},  {8, 16, 3},  {16, 16, 3},  {32, 8, 3},  {32, 16, 3}};
constexpr int kNCand = sizeof(kCands) / sizeof(kCands[0]);

struct Scratch {
    std::vector<void*> ptrs;
    ~Scratch()
    {
        for (void* p : ptrs) (void)hipFree(p);
    }
    void* get(size_t n)
    {
        void* p = nullptr;
        if (hipMalloc(&p, n < 256 ? 256 : n) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return p;
    }
};

}  // namespace

extern "C" {

int32_t wipes_autotune_candidates(int32_t* tile_w, int32_t* tile_h, int32_t* persistent, int32_t max)
{
    for (int i = 0; i < kNCand && i < max; ++i) {
        if (tile_w) tile_w[i] = kCands[i].tw;
        if (tile_h) tile_h[i] = kCands[i].th;
        if (persistent) persistent[i] = kCands[i].persistent;
    }
    return kNCand;
}

wipes_status wipes_autotune(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, int32_t with_backward,
                            int32_t reps, wipes_params* best, double* times_ms, void* stream)
{
    if (!ctx || !best) return fail(ctx, WIPES_ERR_INVALID, "ctx and best must be set");
    wipes_status st = validate(ctx, p, b, false);
    if (st != WIPES_OK) return st;
    if (reps < 1) reps = 3;
    hipStream_t s = (hipStream_t)stream;
    Scratch mem;
    const Layout L0 = layout_of(p, b, 0, 0);
    float* image = (float*)mem.get((size_t)L0.pixels * 12);
    float* T = (float*)mem.get((size_t)L0.pixels * 4);
    int32_t* last = (int32_t*)mem.get((size_t)L0.pixels * 4);
    float* dL = (float*)mem.get((size_t)L0.pixels * 12);
    if (!image || !T || !last || !dL) return fail(ctx, WIPES_ERR_NOMEM, "autotune scratch");
    hipError_t e = launch_fill_u32((uint32_t*)dL, (uint32_t)(L0.pixels * 3), 0x38d1b717u /* 1e-4f */, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "autotune fill");
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(ctx, WIPES_ERR_DEVICE, "autotune events");
    double best_ms = 1e300;
    int best_i = -1;
    for (int i = 0; i < kNCand; ++i) {
        wipes_params q = *p;
        q.tile_w = kCands[i].tw;
        q.tile_h = kCands[i].th;
        q.persistent = kCands[i].persistent;
        size_t sb = 0, bb = 0;
        // size bins from a first sort with a generous capacity, then reuse
        int64_t cap = 4 * L0.n + 65536;
        void* screen = nullptr;
        void* bins = nullptr;
        int64_t K = 0;
        for (int attempt = 0; attempt < 3; ++attempt) {
            if ((st = wipes_workspace_size(&q, b, cap, with_backward, &sb, &bb)) != WIPES_OK) break;
            screen = mem.get(sb);
            bins = mem.get(bb);
            if (!screen || !bins) {
                st = fail(ctx, WIPES_ERR_NOMEM, "autotune workspace");
                break;
            }
            wipes_buffer sbuf{screen, sb, 0, 0, 0}, bbuf{bins, bb, cap, with_backward, 0};
            if ((st = wipes_project(ctx, &q, b, &sbuf, s)) != WIPES_OK) break;
            st = wipes_bin_sort(ctx, &q, b, &sbuf, &bbuf, &K, s);
            if (st != WIPES_ERR_CAPACITY) break;
            cap = (int64_t)(K * 1.2) + 4096;
        }
        if (st != WIPES_OK) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return st;
        }
        wipes_buffer sbuf{screen, sb, 0, 0, 0}, bbuf{bins, bb, cap, with_backward, 0};
        double tot = 0.0;
        for (int r = 0; r <= reps; ++r) {   // first round warms up
            (void)hipEventRecord(e0, s);
            st = wipes_project(ctx, &q, b, &sbuf, s);
            if (st == WIPES_OK) st = wipes_bin_sort(ctx, &q, b, &sbuf, &bbuf, &K, s);
            if (st == WIPES_OK) st = wipes_render_fwd(ctx, &q, b, &sbuf, &bbuf, image, T, last, s);
            if (st == WIPES_OK && with_backward)
                st = wipes_render_bwd(ctx, &q, b, &sbuf, &bbuf, T, last, dL, nullptr, s);
            (void)hipEventRecord(e1, s);
            if (st != WIPES_OK) break;
            if (hipEventSynchronize(e1) != hipSuccess) {
                st = fail(ctx, WIPES_ERR_DEVICE, "autotune sync");
                break;
            }
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (r > 0) tot += ms;
        }
        if (st != WIPES_OK) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return st;
        }
        const double mean = tot / reps;
        if (times_ms) times_ms[i] = mean;
        if (mean < best_ms) {
            best_ms = mean;
            best_i = i;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *best = *p;
    best->tile_w = kCands[best_i].tw;
    best->tile_h = kCands[best_i].th;
    best->persistent = kCands[best_i].persistent;
    return WIPES_OK;
}

}  // extern "C"
