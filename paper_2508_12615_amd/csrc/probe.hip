// Issue-rate probes for the roofline of the blend kernels: how many lane
// operations per second the chip sustains for an FP32 fused multiply-add and
// for each transcendental the per-pixel rule uses (exp2, cos, sin, rcp).  The
// blend's algorithmic cost per support pair counts these, so their measured
// rates replace the nominal quarter rate of the transcendental unit.
//
// Each lane runs kChains independent dependency chains (enough to hide the
// unit's latency at full occupancy) for `iters` rounds; the grid fills every
// SIMD of the chip many times over.  The chains converge to fixed points, so
// the values stay finite and no operand is special.
#include <hip/hip_runtime.h>

#include <cstring>

#include "api_internal.hpp"

namespace wipes {

constexpr int kChains = 8;

template <int OP>
__device__ __forceinline__ float probe_op(float x)
{
    if constexpr (OP == 0) return fmaf(x, 0.999f, 0.001f);
    if constexpr (OP == 1) return __builtin_amdgcn_exp2f(-x);
    if constexpr (OP == 2) return __builtin_amdgcn_cosf(x);
    if constexpr (OP == 3) return __builtin_amdgcn_sinf(x);
    return __builtin_amdgcn_rcpf(x);
}

template <int OP>
__global__ void __launch_bounds__(256) k_probe(int iters, float* __restrict__ sink)
{
    float v[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) v[c] = 0.3f + 0.05f * (float)c + 1e-6f * (float)threadIdx.x;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) v[c] = probe_op<OP>(v[c]);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += v[c];
    // a result that is never exactly this value keeps the work alive
    if (sink != nullptr && s == -12345.0f) sink[blockIdx.x] = s;
}

}  // namespace wipes

using namespace wipes;

extern "C" wipes_status wipes_probe_issue_rate(wipes_ctx* ctx, int32_t op, double* lane_ops_per_s, void* stream)
{
    if (!ctx || !lane_ops_per_s || op < 0 || op > 4)
        return fail(ctx, WIPES_ERR_INVALID, "probe: ctx, op in 0..4 and the output must be given");
    hipStream_t s = (hipStream_t)stream;
    const int iters = 4096;
    const uint32_t blocks = (uint32_t)ctx->n_cu * 64u;   // 16 waves per SIMD, many times over
    float* sink = nullptr;   // (never written: see k_probe)
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    auto launch = [&]() {
        switch (op) {
        case 0: hipLaunchKernelGGL(k_probe<0>, dim3(blocks), dim3(256), 0, s, iters, sink); break;
        case 1: hipLaunchKernelGGL(k_probe<1>, dim3(blocks), dim3(256), 0, s, iters, sink); break;
        case 2: hipLaunchKernelGGL(k_probe<2>, dim3(blocks), dim3(256), 0, s, iters, sink); break;
        case 3: hipLaunchKernelGGL(k_probe<3>, dim3(blocks), dim3(256), 0, s, iters, sink); break;
        default: hipLaunchKernelGGL(k_probe<4>, dim3(blocks), dim3(256), 0, s, iters, sink); break;
        }
        return hipGetLastError();
    };
    if (e == hipSuccess) e = launch();   // warm-up
    if (e == hipSuccess) e = hipEventRecord(a, s);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) return hip_fail(ctx, e, "probe");
    const double ops = (double)blocks * 256.0 * (double)iters * (double)kChains;
    *lane_ops_per_s = ops / ((double)ms * 1e-3);
    return WIPES_OK;
}
