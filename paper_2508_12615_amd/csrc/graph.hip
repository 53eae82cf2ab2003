// hipGraph capture of the whole render step for a fixed batch:
//   project -> bin/sort (no host synchronisation: grids sized by the bins
//   capacity, instance count read on the device) -> forward blend ->
//   [L2 loss gradient] -> backward blend -> projection backward.
// Replaying the graph costs one launch instead of ~30, which is what makes
// many small images (uneven 2D fits) worth batching.  The descriptor table is
// uploaded before capture and must stay valid (same batch, same buffers) for
// the graph's lifetime.  Clears inside the graph use fill kernels, never
// memset nodes.
#include <hip/hip_runtime.h>

#include "api_internal.hpp"

namespace wipes {

// dL/dC of L = sum over images of mean over that image's 3 W H values of
// (C - target)^2:  2 (C - target) / (3 W H).  One thread per pixel; the
// image is looked up once per wave (for the wave's first pixel, with
// wave-uniform loads), and a lane past that image's end searches on its own.
__global__ void __launch_bounds__(256) k_l2_grad(const ImgDesc* __restrict__ descs, int B, int32_t npix,
                                                  const float* __restrict__ image, const float* __restrict__ target,
                                                  float* __restrict__ grad)
{
    const int32_t p0 = __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x * 256u + (threadIdx.x & ~63u)));
    if (p0 >= npix) return;   // wave-uniform
    int b = find_owner(B, p0, [&](int k) { return descs[k].pix_begin; });
    const int32_t p = (int32_t)(blockIdx.x * 256u + threadIdx.x);
    if (p >= npix) return;
    if (b + 1 < B && p >= descs[b + 1].pix_begin) b = find_owner(B, p, [&](int k) { return descs[k].pix_begin; });
    const float scale = 2.0f / (3.0f * (float)descs[b].W * (float)descs[b].H);
    for (int c = 0; c < 3; ++c) grad[3 * p + c] = scale * (image[3 * p + c] - target[3 * p + c]);
}

hipError_t launch_l2_grad(const ImgDesc* descs, int B, int32_t npix, const float* image, const float* target,
                          float* grad, hipStream_t s)
{
    if (npix > 0)
        hipLaunchKernelGGL(k_l2_grad, dim3(((uint32_t)npix + 255u) / 256u), dim3(256), 0, s, descs, B, npix, image,
                           target, grad);
    return hipGetLastError();
}

}  // namespace wipes

using namespace wipes;

struct wipes_graph {
    wipes_ctx* ctx = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

wipes_status wipes_l2_grad(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, const wipes_buffer* screen,
                           const float* image, const float* target, float* dL_dimage, void* stream)
{
    if (!ctx) return fail(nullptr, WIPES_ERR_INVALID, "ctx must not be NULL");
    wipes_status st = validate(ctx, p, b, false);
    if (st != WIPES_OK) return st;
    if (!image || !target || !dL_dimage) return fail(ctx, WIPES_ERR_INVALID, "image, target and dL_dimage must be set");
    const Layout L = layout_of(p, b, 0, 0);
    if (!screen || !screen->base || screen->bytes < L.screen_bytes)
        return fail(ctx, WIPES_ERR_NOMEM, "screen buffer missing or too small");
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_descs(ctx, p, b, L, screen->base, s)) != WIPES_OK) return st;
    hipError_t e = launch_l2_grad((const ImgDesc*)((char*)screen->base + L.s_descs), L.B, (int32_t)L.pixels, image,
                                  target, dL_dimage, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "l2 grad");
    return WIPES_OK;
}

wipes_status wipes_graph_capture(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, wipes_buffer* screen,
                                 wipes_buffer* bins, float* image, float* T_final, int32_t* last, const float* target,
                                 float* dL_dimage, int32_t backward, wipes_graph** out)
{
    if (!ctx || !out) return fail(ctx, WIPES_ERR_INVALID, "ctx and out must not be NULL");
    *out = nullptr;
    wipes_status st = validate(ctx, p, b, backward != 0);
    if (st != WIPES_OK) return st;
    if (!screen || !bins || !image) return fail(ctx, WIPES_ERR_INVALID, "screen, bins and image must be set");
    if (p->mode == WIPES_3D_ALPHA && (!T_final || !last))
        return fail(ctx, WIPES_ERR_INVALID, "alpha mode needs T_final and last");
    if (backward && (!dL_dimage || !bins->with_backward))
        return fail(ctx, WIPES_ERR_INVALID, "backward needs dL_dimage and a bins buffer sized with_backward");
    const Layout L = layout_of(p, b, bins->capacity, bins->with_backward != 0);
    if (screen->bytes < L.screen_bytes || bins->bytes < L.bins_bytes)
        return fail(ctx, WIPES_ERR_NOMEM, "workspace too small for this batch and capacity");
    hipStream_t s = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(ctx, e, "graph stream");
    // descriptors first, outside the graph
    if ((st = upload_descs(ctx, p, b, L, screen->base, s)) != WIPES_OK) {
        (void)hipStreamDestroy(s);
        return st;
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(s);
        return hip_fail(ctx, e, "graph upload sync");
    }
    wipes_graph* g = new wipes_graph();
    g->ctx = ctx;
    ctx->capturing = true;
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        ctx->capturing = false;
        delete g;
        (void)hipStreamDestroy(s);
        return hip_fail(ctx, e, "begin capture");
    }
    char* base = (char*)screen->base;
    const ImgDesc* descs = (const ImgDesc*)(base + L.s_descs);
    e = launch_project(descs, L.B, (int32_t)L.n, kparams(p), (Rec*)(base + L.s_recs), (Aux*)(base + L.s_aux), s);
    if (e == hipSuccess) {
        st = bin_sort_core(ctx, p, b, L, screen->base, bins->base, nullptr, s);
        if (st == WIPES_OK) st = render_fwd_core(ctx, p, b, L, screen->base, bins->base, image, T_final, last, s);
        if (st == WIPES_OK && target && dL_dimage) {
            e = launch_l2_grad(descs, L.B, (int32_t)L.pixels, image, target, dL_dimage, s);
            if (e != hipSuccess) st = hip_fail(ctx, e, "l2 grad");
        }
        if (st == WIPES_OK && backward)
            st = render_bwd_core(ctx, p, b, L, screen->base, bins->base, T_final, last, dL_dimage, nullptr, s);
    } else {
        st = hip_fail(ctx, e, "project");
    }
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    ctx->capturing = false;
    (void)hipStreamDestroy(s);
    if (st != WIPES_OK || e2 != hipSuccess) {
        if (graph) hipGraphDestroy(graph);
        delete g;
        return st != WIPES_OK ? st : hip_fail(ctx, e2, "end capture");
    }
    g->graph = graph;
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        delete g;
        return hip_fail(ctx, e, "graph instantiate");
    }
    *out = g;
    return WIPES_OK;
}

wipes_status wipes_graph_launch(wipes_graph* g, void* stream)
{
    if (!g || !g->exec) return fail(nullptr, WIPES_ERR_INVALID, "graph must not be NULL");
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(g->ctx, e, "graph launch");
    return WIPES_OK;
}

void wipes_graph_destroy(wipes_graph* g)
{
    if (!g) return;
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"
