// Adam over the parameter groups of a fit in one launch, with the step count
// and the overflow guard on the device, so that a fitting step (render
// replay + optimiser) needs no host synchronisation.  The update follows the
// optimiser of the 2D fitting experiments (Sec. 5.1), written as the usual
// bias-corrected form: m as a lerp towards g, v as beta2 v + (1 - beta2) g^2,
// the step size lr / (1 - beta1^t) and the denominator
// sqrt(v) / sqrt(1 - beta2^t) + eps with both corrections formed in FP64 and
// rounded once to FP32.
#include <hip/hip_runtime.h>

#include <cmath>

#include "api_internal.hpp"

namespace wipes {

struct AdamArgs {
    float* p[WIPES_ADAM_MAX_GROUPS];
    const float* g[WIPES_ADAM_MAX_GROUPS];
    float* m[WIPES_ADAM_MAX_GROUPS];
    float* v[WIPES_ADAM_MAX_GROUPS];
    double lr[WIPES_ADAM_MAX_GROUPS];
    uint32_t off[WIPES_ADAM_MAX_GROUPS + 1];   // first element of each group in the joint index
    int ng;
    double beta1, beta2;
    float w1, b2, w2, eps;                      // 1 - beta1, beta2, 1 - beta2, eps in FP32
};

__global__ void __launch_bounds__(256) k_adam(AdamArgs a, const uint32_t* __restrict__ step,
                                               const uint32_t* __restrict__ skip)
{
    if (skip && *skip) return;
    const double t = (double)(*step + 1u);
    const double bc1 = 1.0 - pow(a.beta1, t), bc2s = sqrt(1.0 - pow(a.beta2, t));
    const uint32_t total = a.off[a.ng];
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < total; i += gridDim.x * 256u) {
        int k = 0;
        while (k + 1 < a.ng && i >= a.off[k + 1]) ++k;
        const uint32_t j = i - a.off[k];
        const float step_size = (float)(a.lr[k] / bc1), corr = (float)bc2s;
        const float g = a.g[k][j];
        float m = a.m[k][j], v = a.v[k][j];
        m = m + a.w1 * (g - m);
        v = v * a.b2;
        v = v + a.w2 * g * g;
        const float denom = sqrtf(v) / corr + a.eps;
        a.p[k][j] = a.p[k][j] + (-step_size) * (m / denom);
        a.m[k][j] = m;
        a.v[k][j] = v;
    }
}

// Advances the step count after the update (a separate launch: every
// workgroup of the update reads the old count).
__global__ void k_adam_count(uint32_t* __restrict__ step, const uint32_t* __restrict__ skip)
{
    if (threadIdx.x == 0 && !(skip && *skip)) *step = *step + 1u;
}

}  // namespace wipes

using namespace wipes;

extern "C" wipes_status wipes_adam(wipes_ctx* ctx, int32_t n_groups, const wipes_adam_group* groups, double beta1,
                                   double beta2, double eps, uint32_t* step, const wipes_params* p,
                                   const wipes_batch* batch, const wipes_buffer* screen, void* stream)
{
    if (!ctx) return fail(nullptr, WIPES_ERR_INVALID, "ctx must not be NULL");
    if (n_groups < 1 || n_groups > WIPES_ADAM_MAX_GROUPS || !groups || !step)
        return fail(ctx, WIPES_ERR_INVALID, "need 1..%d groups and a step counter", WIPES_ADAM_MAX_GROUPS);
    AdamArgs a{};
    a.ng = n_groups;
    int64_t total = 0;
    for (int k = 0; k < n_groups; ++k) {
        const wipes_adam_group& gr = groups[k];
        if (gr.n < 0 || (gr.n > 0 && (!gr.param || !gr.grad || !gr.m || !gr.v)))
            return fail(ctx, WIPES_ERR_INVALID, "group %d: negative size or NULL array", k);
        a.p[k] = gr.param;
        a.g[k] = gr.grad;
        a.m[k] = gr.m;
        a.v[k] = gr.v;
        a.lr[k] = gr.lr;
        a.off[k] = (uint32_t)total;
        total += gr.n;
        if (total >= (1ll << 31)) return fail(ctx, WIPES_ERR_INVALID, "more than 2^31 elements");
    }
    a.off[n_groups] = (uint32_t)total;
    a.beta1 = beta1;
    a.beta2 = beta2;
    a.w1 = (float)(1.0 - beta1);
    a.b2 = (float)beta2;
    a.w2 = (float)(1.0 - beta2);
    a.eps = (float)eps;
    const uint32_t* skip = nullptr;
    if (screen) {
        const wipes_status st = validate(ctx, p, batch, false);
        if (st != WIPES_OK) return st;
        const Layout L = layout_of(p, batch, 0, 0);
        if (!screen->base || screen->bytes < L.screen_bytes)
            return fail(ctx, WIPES_ERR_NOMEM, "screen buffer missing or too small");
        skip = (const uint32_t*)((const char*)screen->base + L.s_ctrl) + kCtrlOverflow;
    }
    hipStream_t s = (hipStream_t)stream;
    const uint32_t blocks = (uint32_t)std::min<int64_t>((total + 255) / 256, 4096);
    if (blocks > 0) hipLaunchKernelGGL(k_adam, dim3(blocks), dim3(256), 0, s, a, step, skip);
    hipLaunchKernelGGL(k_adam_count, dim3(1), dim3(64), 0, s, step, skip);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? WIPES_OK : hip_fail(ctx, e, "adam");
}
