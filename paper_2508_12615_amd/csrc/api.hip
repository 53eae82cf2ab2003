// C ABI of the wavelet rasterizer: argument validation, workspace layout,
// descriptor upload and stage sequencing.  No allocation on the render path:
// every device buffer is the caller's.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "api_internal.hpp"

using namespace wipes;

// --------------------------------------------------------------- helpers

namespace wipes {

static thread_local std::string g_err_no_ctx;

wipes_status fail(wipes_ctx* ctx, wipes_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf; else g_err_no_ctx = buf;
    return st;
}

wipes_status hip_fail(wipes_ctx* ctx, hipError_t e, const char* where)
{
    return fail(ctx, WIPES_ERR_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

static int ilog2(int v)
{
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

bool tile_ok(int tw, int th)
{
    return (tw == 8 && th == 8) || (tw == 16 && th == 8) || (tw == 16 && th == 16) || (tw == 32 && th == 8) ||
           (tw == 8 && th == 16) || (tw == 32 && th == 16);
}

KParams kparams(const wipes_params* p)
{
    KParams k;
    k.mode = p->mode;
    k.cov = p->cov;
    k.tile_w = p->tile_w;
    k.tile_h = p->tile_h;
    k.log2_tw = ilog2(p->tile_w);
    k.log2_th = ilog2(p->tile_h);
    k.freq_xform = p->freq_xform;
    k.sh_degree = p->sh_degree;
    k.alpha_min = p->alpha_min;
    k.alpha_max = p->alpha_max;
    k.T_min = p->T_min;
    k.q_add = p->q_add;
    k.blur_eps = p->blur_eps;
    k.near_plane = p->near_plane;
    k.bg[0] = p->bg[0];
    k.bg[1] = p->bg[1];
    k.bg[2] = p->bg[2];
    return k;
}

wipes_status validate(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, bool need_grads)
{
    if (!p || !b) return fail(ctx, WIPES_ERR_INVALID, "params and batch must not be NULL");
    if (p->mode != WIPES_2D_ADDITIVE && p->mode != WIPES_3D_ALPHA) return fail(ctx, WIPES_ERR_INVALID, "bad mode");
    if (p->mode == WIPES_2D_ADDITIVE && p->cov != WIPES_COV_CHOLESKY && p->cov != WIPES_COV_RS)
        return fail(ctx, WIPES_ERR_INVALID, "2D mode needs cov CHOLESKY or RS");
    if (p->mode == WIPES_3D_ALPHA && p->cov != WIPES_COV_QUAT_SCALE)
        return fail(ctx, WIPES_ERR_INVALID, "3D mode needs cov QUAT_SCALE");
    if (p->freq_xform != WIPES_FREQ_VECTOR && p->freq_xform != WIPES_FREQ_COVECTOR)
        return fail(ctx, WIPES_ERR_INVALID, "bad freq_xform");
    if (p->sh_degree < -1 || p->sh_degree > 3) return fail(ctx, WIPES_ERR_INVALID, "sh_degree must be -1..3");
    if (p->sh_degree >= 0 && p->mode != WIPES_3D_ALPHA)
        return fail(ctx, WIPES_ERR_INVALID, "spherical-harmonic colour needs 3D mode");
    if (p->persistent < 0 || p->persistent > 3)
        return fail(ctx, WIPES_ERR_INVALID, "persistent must be 0..3 (blend launch form)");
    if (p->lds_batch != 0 && p->lds_batch != 64)
        return fail(ctx, WIPES_ERR_INVALID, "lds_batch must be 0 or 64 (the blend stages one 64-position word)");
    if (!tile_ok(p->tile_w, p->tile_h)) return fail(ctx, WIPES_ERR_INVALID, "unsupported tile %dx%d", p->tile_w, p->tile_h);
    if (!(p->alpha_min > 0.0f) || !(p->alpha_max > p->alpha_min) || !(p->alpha_max < 1.0f) || !(p->T_min > 0.0f) ||
        !(p->q_add > 0.0f) || !(p->blur_eps >= 0.0f) || !(p->near_plane > 0.0f) || !(p->fov_guard > 0.0f))
        return fail(ctx, WIPES_ERR_INVALID, "rasterizer constants out of range");
    if (b->n_images < 1 || b->n_images > kMaxImages || !b->images)
        return fail(ctx, WIPES_ERR_INVALID, "batch must hold 1..%d images", kMaxImages);
    int64_t prims = 0, pix = 0, tiles = 0;
    for (int i = 0; i < b->n_images; ++i) {
        const wipes_image& im = b->images[i];
        const wipes_prims& q = im.prims;
        if (im.cam.width < 1 || im.cam.height < 1 || im.cam.width > 32768 || im.cam.height > 32768)
            return fail(ctx, WIPES_ERR_INVALID, "image %d: size %dx%d out of range", i, im.cam.width, im.cam.height);
        if (q.n < 0) return fail(ctx, WIPES_ERR_INVALID, "image %d: negative primitive count", i);
        if (q.n > 0) {
            if (!q.mean || !q.freq || !q.opacity)
                return fail(ctx, WIPES_ERR_INVALID, "image %d: mean/freq/opacity must be set", i);
            if (p->sh_degree < 0 && !q.color) return fail(ctx, WIPES_ERR_INVALID, "image %d: color missing", i);
            if (p->sh_degree >= 0 && !q.sh)
                return fail(ctx, WIPES_ERR_INVALID, "image %d: sh_degree %d needs sh coefficients", i, p->sh_degree);
            if (p->mode == WIPES_2D_ADDITIVE && !q.cov) return fail(ctx, WIPES_ERR_INVALID, "image %d: cov missing", i);
            if (p->mode == WIPES_3D_ALPHA) {
                if (!q.quat || !q.scale) return fail(ctx, WIPES_ERR_INVALID, "image %d: quat/scale missing", i);
                if (!(im.cam.fx > 0.0f) || !(im.cam.fy > 0.0f))
                    return fail(ctx, WIPES_ERR_INVALID, "image %d: focal lengths must be positive", i);
            }
        }
        if (need_grads) {
            const wipes_prims_grad& g = im.grads;
            if (g.velocity && !q.velocity)
                return fail(ctx, WIPES_ERR_INVALID, "image %d: velocity gradient without velocity", i);
            if (g.sh && p->sh_degree < 0)
                return fail(ctx, WIPES_ERR_INVALID, "image %d: sh gradient without spherical-harmonic colour", i);
        }
        prims += q.n;
        pix += (int64_t)im.cam.width * im.cam.height;
        tiles += (int64_t)((im.cam.width + p->tile_w - 1) / p->tile_w) * ((im.cam.height + p->tile_h - 1) / p->tile_h);
    }
    if (prims >= (1ll << 31) || pix * 3 >= (1ll << 31) || tiles >= (1ll << 31))
        return fail(ctx, WIPES_ERR_INVALID, "batch too large (primitives, pixels*3 and tiles must stay below 2^31)");
    return WIPES_OK;
}

Layout layout_of(const wipes_params* p, const wipes_batch* b, int64_t cap, int with_bwd)
{
    Layout L{};
    L.B = b->n_images;
    L.alpha = p->mode == WIPES_3D_ALPHA;
    for (int i = 0; i < b->n_images; ++i) {
        const wipes_camera& c = b->images[i].cam;
        L.n += b->images[i].prims.n;
        L.pixels += (int64_t)c.width * c.height;
        L.tiles += (int64_t)((c.width + p->tile_w - 1) / p->tile_w) * ((c.height + p->tile_h - 1) / p->tile_h);
    }
    L.cap = cap;
    const int64_t n = L.n;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    L.s_recs = take((size_t)n * 64);
    L.s_aux = take((size_t)n * 16);
    L.s_count = take((size_t)n * 4);
    L.s_off_id = take((size_t)n * 4);
    L.s_pk = take((size_t)n * sizeof(PrimPack));
    if (L.alpha) {
        L.s_pkr = take((size_t)n * sizeof(PrimPack));
        L.s_dkey_a = take((size_t)n * 4);
        L.s_dval_a = take((size_t)n * 4);
        L.s_dkey_b = take((size_t)n * 4);
        L.s_dval_b = take((size_t)n * 4);
        L.s_dhist = take(((size_t)1 << radix_digit_bits(32)) * ((size_t)radix_max_blocks((uint32_t)n) + 1) * 4);
        L.s_ddtot = take(((size_t)1 << radix_digit_bits(32)) * 4);
    }
    L.s_bsum = take((size_t)((n + 63) / 64 + 1) * 4);
    L.s_bsum2 = take((size_t)((n + 63) / 64 + 1) * 4);
    L.s_ctrl = take(kCtrlWords * 4);
    L.s_descs = take((size_t)L.B * sizeof(ImgDesc));
    L.screen_bytes = o;

    const int64_t nb_t = (L.tiles + 4095) / 4096 + 1;
    // tile sort bits and where its result lands
    int bits = 0;
    while (bits < 32 && (1ll << bits) < L.tiles) ++bits;
    L.tile_bits = std::max(bits, 1);
    L.tile_result_b = radix_passes(L.tile_bits) & 1;
    L.depth_result_b = radix_passes(32) & 1;
    // digit histograms of the tile sort
    const size_t nd_bins = (size_t)1 << radix_digit_bits(L.tile_bits);
    o = 0;
    L.b_keys_a = take((size_t)cap * 4);
    L.b_vals_a = take((size_t)cap * 4);
    L.b_keys_b = take((size_t)cap * 4);
    L.b_vals_b = take((size_t)cap * 4);
    L.b_hist = take(nd_bins * std::max((int64_t)radix_max_blocks((uint32_t)cap) + 1, nb_t) * 4);
    L.b_dtot = take(nd_bins * 4);
    L.b_ranges = take((size_t)L.tiles * 8);
    L.b_order = take((size_t)L.tiles * 4);   // longest-first tile order
    L.b_lpt = take((size_t)(lpt_slices((uint32_t)L.tiles) + 1) * 256 * 4);   // its per-slice key counts
    L.b_tbsum = take((size_t)(nb_t + 1) * 4);
    if (with_bwd) {
        L.b_slots = take((size_t)cap * 48);
        // contribution mask: (tile_w/8)(tile_h/8) block rows of cap/64 + 2 words
        L.cmask_words = (uint32_t)(cap / 64 + 2);
        L.b_cmask = take((size_t)(p->tile_w / 8) * (p->tile_h / 8) * L.cmask_words * 8);
        L.b_svalid = take((size_t)(cap / 32 + 2) * 4);
    }
    L.bins_bytes = o;
    L.with_bwd = with_bwd;
    return L;
}

void fill_descs(const wipes_params* p, const wipes_batch* b, std::vector<ImgDesc>& out)
{
    out.resize(b->n_images);
    int32_t prim = 0, pix = 0, tile = 0;
    for (int i = 0; i < b->n_images; ++i) {
        const wipes_image& im = b->images[i];
        ImgDesc& d = out[i];
        memset(&d, 0, sizeof(d));
        d.mean = im.prims.mean;
        d.cov = im.prims.cov;
        d.quat = im.prims.quat;
        d.scale = im.prims.scale;
        d.freq = im.prims.freq;
        d.color = im.prims.color;
        d.opac = im.prims.opacity;
        d.vel = im.prims.velocity;
        d.phase = im.prims.phase;
        d.sh = p->sh_degree >= 0 ? im.prims.sh : nullptr;
        d.g_mean = im.grads.mean;
        d.g_cov = im.grads.cov;
        d.g_quat = im.grads.quat;
        d.g_scale = im.grads.scale;
        d.g_freq = im.grads.freq;
        d.g_color = im.grads.color;
        d.g_opac = im.grads.opacity;
        d.g_vel = im.grads.velocity;
        d.g_phase = im.grads.phase;
        d.g_sh = p->sh_degree >= 0 ? im.grads.sh : nullptr;
        d.out_image = im.out_image;
        d.prim_begin = prim;
        d.n = (int32_t)im.prims.n;
        d.pix_begin = pix;
        d.tile_begin = tile;
        d.W = im.cam.width;
        d.H = im.cam.height;
        d.tiles_x = (d.W + p->tile_w - 1) / p->tile_w;
        d.tiles_y = (d.H + p->tile_h - 1) / p->tile_h;
        d.fx = im.cam.fx;
        d.fy = im.cam.fy;
        d.cx = im.cam.cx;
        d.cy = im.cam.cy;
        for (int k = 0; k < 12; ++k) d.view[k] = im.cam.viewmat[k];
        d.time = im.cam.time;
        d.limx = p->mode == WIPES_3D_ALPHA ? p->fov_guard * 0.5f * (float)d.W / im.cam.fx : 0.0f;
        d.limy = p->mode == WIPES_3D_ALPHA ? p->fov_guard * 0.5f * (float)d.H / im.cam.fy : 0.0f;
        // camera centre -R^T w of the world->camera map [R | w]
        const float* V = im.cam.viewmat;
        for (int k = 0; k < 3; ++k)
            d.cam_c[k] = (float)-((double)V[k] * V[3] + (double)V[4 + k] * V[7] + (double)V[8 + k] * V[11]);
        prim += d.n;
        pix += d.W * d.H;
        tile += d.tiles_x * d.tiles_y;
    }
}

// Tables of up to kDescArgMax images travel as a kernel argument and one
// wave writes them into the screen buffer: no copy from host memory, whose
// blit and the wait after it cost more than the blend of a small image.

__global__ void __launch_bounds__(64) k_put_descs(DescArgs a, int n, ImgDesc* __restrict__ out)
{
    const uint32_t* src = reinterpret_cast<const uint32_t*>(a.d);
    uint32_t* dst = reinterpret_cast<uint32_t*>(out);
    const uint32_t words = (uint32_t)n * (uint32_t)(sizeof(ImgDesc) / 4);
    for (uint32_t k = threadIdx.x; k < words; k += 64u) dst[k] = src[k];
}

// Copy the descriptor table into the screen buffer (stream-ordered): small
// tables as a kernel argument, larger ones through a ring of pinned staging
// slots (a slot is reused only after its previous copy has completed).
// Skipped while a graph is being captured (the table is uploaded before
// capture and stays valid for the graph's lifetime).
static wipes_status put_descs(wipes_ctx* ctx, const std::vector<ImgDesc>& h, char* dst, hipStream_t s);

wipes_status upload_descs(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, const Layout& L, void* screen,
                          hipStream_t s, bool reuse, bool defer)
{
    ctx->desc_pend = false;
    if (ctx->capturing) return WIPES_OK;
    std::vector<ImgDesc>& h = ctx->desc_tmp;   // swapped with desc_last below: both keep their storage
    fill_descs(p, b, h);
    const size_t bytes = h.size() * sizeof(ImgDesc);
    char* dst = (char*)screen + L.s_descs;
    // the table this context wrote last is still in place for the later
    // stages of the same frame (they read the screen buffer that the
    // projection filled, so it cannot have been overwritten meanwhile)
    if (reuse && ctx->desc_dst == dst && ctx->desc_last.size() == h.size() &&
        memcmp(ctx->desc_last.data(), h.data(), bytes) == 0)
        return WIPES_OK;
    // does the new table differ from the stored one in gradient pointers only?
    bool grads_only = ctx->desc_dst == dst && ctx->desc_last.size() == h.size();
    for (size_t k = 0; grads_only && k < h.size(); ++k) {
        ImgDesc x = ctx->desc_last[k], y = h[k];
        x.g_mean = x.g_cov = x.g_quat = x.g_scale = x.g_freq = x.g_color = x.g_opac = x.g_vel = nullptr;
        y.g_mean = y.g_cov = y.g_quat = y.g_scale = y.g_freq = y.g_color = y.g_opac = y.g_vel = nullptr;
        x.g_phase = x.g_sh = y.g_phase = y.g_sh = nullptr;
        grads_only = memcmp(&x, &y, sizeof(ImgDesc)) == 0;
    }
    ctx->desc_dst = nullptr;
    if (defer && h.size() <= (size_t)kDescArgMax) {
        // the caller's first launch (launch_fill2_put, or the projection
        // backward after a fresh bin_sort) writes the table
        ctx->desc_pend_grads_only = grads_only;
        memset(&ctx->desc_pend_args, 0, sizeof(DescArgs));
        memcpy(ctx->desc_pend_args.d, h.data(), bytes);
        ctx->desc_pend_n = (int)h.size();
        ctx->desc_pend_dst = dst;
        ctx->desc_pend = true;
        ctx->desc_last.swap(h);
        return WIPES_OK;
    }
    wipes_status st = put_descs(ctx, h, dst, s);
    if (st == WIPES_OK) {
        ctx->desc_dst = dst;
        ctx->desc_last.swap(h);
    }
    return st;
}

// Two fills (p[0..n), q[0..m)) and, when a table is pending, its copy
// (words 32-bit words) into the screen buffer, in one launch.
__global__ void __launch_bounds__(256) k_fill2_put(uint32_t* __restrict__ p, uint32_t n, uint32_t* __restrict__ q,
                                                   uint32_t m, uint32_t v, DescArgs a, uint32_t words,
                                                   uint32_t* __restrict__ out)
{
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < n) p[i] = v;
    else if (i - n < m) q[i - n] = v;
    if (i < words) out[i] = reinterpret_cast<const uint32_t*>(a.d)[i];
}

hipError_t launch_fill2_put(wipes_ctx* ctx, uint32_t* p, uint32_t n, uint32_t* q, uint32_t m, uint32_t v,
                            hipStream_t s)
{
    if (!ctx->desc_pend) return launch_fill2_u32(p, n, q, m, v, s);
    if (!q) m = 0;
    if (!p) n = 0;
    const uint32_t words = (uint32_t)ctx->desc_pend_n * (uint32_t)(sizeof(ImgDesc) / 4);
    hipError_t e = hipSuccess;
    if ((uint64_t)n + m >= (1ull << 32)) {   // (not in one launch)
        e = launch_fill2_u32(p, n, q, m, v, s);
        n = m = 0;
    }
    if (e == hipSuccess) {
        const uint32_t cnt = std::max(n + m, words);
        hipLaunchKernelGGL(k_fill2_put, dim3((cnt + 255u) / 256u), dim3(256), 0, s, p, n, q, m, v,
                           ctx->desc_pend_args, words, reinterpret_cast<uint32_t*>(ctx->desc_pend_dst));
        e = hipGetLastError();
    }
    ctx->desc_pend = false;
    if (e == hipSuccess) ctx->desc_dst = ctx->desc_pend_dst;
    return e;
}

static wipes_status put_descs(wipes_ctx* ctx, const std::vector<ImgDesc>& h, char* dst, hipStream_t s)
{
    const size_t bytes = h.size() * sizeof(ImgDesc);
    if (h.size() <= (size_t)kDescArgMax) {
        DescArgs a;
        memset(&a, 0, sizeof(a));
        memcpy(a.d, h.data(), bytes);
        hipLaunchKernelGGL(k_put_descs, dim3(1), dim3(64), 0, s, a, (int)h.size(), reinterpret_cast<ImgDesc*>(dst));
        const hipError_t e = hipGetLastError();
        return e == hipSuccess ? WIPES_OK : hip_fail(ctx, e, "descriptor upload");
    }
    StagingSlot& slot = ctx->ring[ctx->ring_next];
    ctx->ring_next = (ctx->ring_next + 1) % kRing;
    hipError_t e;
    if (slot.used) {
        e = hipEventSynchronize(slot.ev);
        if (e != hipSuccess) return hip_fail(ctx, e, "staging event");
    }
    memcpy(slot.host, h.data(), bytes);
    e = hipMemcpyAsync(dst, slot.host, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "descriptor upload");
    e = hipEventRecord(slot.ev, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "staging event record");
    slot.used = true;
    return WIPES_OK;
}

static hipEvent_t prof_event(wipes_ctx* c)
{
    if (!c->prof.pool.empty()) {
        hipEvent_t e = c->prof.pool.back();
        c->prof.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

StageScope::StageScope(wipes_ctx* ctx, int stage, hipStream_t stream) : c(ctx), st(stage), s(stream)
{
    if (c && c->prof.on && !c->capturing) {
        a = prof_event(c);
        if (a) (void)hipEventRecord(a, s);
    }
}

StageScope::~StageScope()
{
    if (!a) return;
    hipEvent_t b = prof_event(c);
    if (!b) return;
    (void)hipEventRecord(b, s);
    c->prof.rec[st].push_back({a, b});
}

}  // namespace wipes

// --------------------------------------------------------------- static workspace

// Device workspace of wipes_render_fwd_noalloc, for callers that cannot
// allocate: every device the library runs on holds its own copy until the
// process ends.  In host code `scratch` names a host-side stand-in, not the
// device array: host code only ever uses the device address that
// hipGetSymbolAddress gives for the current device at context creation
// (wipes_ctx::scratch).
static __device__ __align__(256) unsigned char scratch[WIPES_NOALLOC_WORKSPACE_BYTES];

// --------------------------------------------------------------- C ABI

extern "C" {

void wipes_params_default(int32_t mode, wipes_params* p)
{
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->mode = mode;
    p->cov = mode == WIPES_3D_ALPHA ? WIPES_COV_QUAT_SCALE : WIPES_COV_RS;
    p->freq_xform = WIPES_FREQ_VECTOR;
    p->tile_w = 16;
    p->tile_h = 16;
    p->persistent = 3;
    p->alpha_min = 1.0f / 255.0f;
    p->alpha_max = 0.99f;
    p->T_min = 1e-4f;
    p->q_add = 9.0f;
    p->blur_eps = mode == WIPES_3D_ALPHA ? 0.3f : 0.0f;
    p->near_plane = 0.01f;
    p->fov_guard = 1.3f;
    p->sh_degree = -1;
    p->lds_batch = 0;
}

wipes_status wipes_ctx_create(int32_t device, wipes_ctx** out)
{
    if (!out) return fail(nullptr, WIPES_ERR_INVALID, "out must not be NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(nullptr, WIPES_ERR_INVALID, "device %d out of range", device);
    e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
    wipes_ctx* c = new wipes_ctx();
    c->device = device;
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(nullptr, e, "hipGetDeviceProperties");
    }
    c->n_cu = prop.multiProcessorCount;
    e = hipHostMalloc((void**)&c->k_host, 256, hipHostMallocMapped);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&c->k_host_dev, c->k_host, 0);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->k_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        wipes_ctx_destroy(c);
        return hip_fail(nullptr, e, "instance-count readback allocation");
    }
    // this device's copy of the static workspace (the device is current)
    e = hipGetSymbolAddress((void**)&c->scratch, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
        c->scratch = nullptr;
        wipes_ctx_destroy(c);
        return hip_fail(nullptr, e, "static workspace address");
    }
    for (int i = 0; i < kRing; ++i) {
        e = hipHostMalloc(&c->ring[i].host, kStagingBytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ring[i].ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            wipes_ctx_destroy(c);
            return hip_fail(nullptr, e, "staging allocation");
        }
    }
    *out = c;
    return WIPES_OK;
}

void wipes_ctx_destroy(wipes_ctx* ctx)
{
    if (!ctx) return;
    for (int st = 0; st < kStN; ++st)
        for (auto& pr : ctx->prof.rec[st]) {
            (void)hipEventSynchronize(pr.second);
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (hipEvent_t e : ctx->prof.pool) (void)hipEventDestroy(e);
    for (int i = 0; i < kRing; ++i) {
        if (ctx->ring[i].ev) {
            (void)hipEventSynchronize(ctx->ring[i].ev);
            (void)hipEventDestroy(ctx->ring[i].ev);
        }
        if (ctx->ring[i].host) hipHostFree(ctx->ring[i].host);
    }
    if (ctx->k_ev) {
        (void)hipEventSynchronize(ctx->k_ev);
        (void)hipEventDestroy(ctx->k_ev);
    }
    if (ctx->k_host) hipHostFree(ctx->k_host);
    delete ctx;
}

const char* wipes_last_error(const wipes_ctx* ctx)
{
    return ctx ? ctx->err.c_str() : g_err_no_ctx.c_str();
}

wipes_status wipes_workspace_size(const wipes_params* p, const wipes_batch* b, int64_t capacity_instances,
                                  int32_t with_backward, size_t* screen_bytes, size_t* bins_bytes)
{
    wipes_status st = validate(nullptr, p, b, false);
    if (st != WIPES_OK) return st;
    if (capacity_instances < 0 || capacity_instances >= (1ll << 31))
        return fail(nullptr, WIPES_ERR_INVALID, "capacity out of range");
    const Layout L = layout_of(p, b, capacity_instances, with_backward);
    if (screen_bytes) *screen_bytes = L.screen_bytes;
    if (bins_bytes) *bins_bytes = L.bins_bytes;
    return WIPES_OK;
}

static wipes_status check_buf(wipes_ctx* ctx, const wipes_buffer* buf, size_t need, const char* what)
{
    if (!buf || !buf->base) return fail(ctx, WIPES_ERR_INVALID, "%s buffer missing", what);
    if (buf->bytes < need) return fail(ctx, WIPES_ERR_NOMEM, "%s buffer too small (%zu < %zu)", what, buf->bytes, need);
    return WIPES_OK;
}

// Common prologue: ctx, params, batch, buffers; returns the layout for the bins capacity.
static wipes_status prologue(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, const wipes_buffer* screen,
                             const wipes_buffer* bins, bool need_grads, bool need_bwd_bins, Layout* L)
{
    if (!ctx) return fail(nullptr, WIPES_ERR_INVALID, "ctx must not be NULL");
    wipes_status st = validate(ctx, p, b, need_grads);
    if (st != WIPES_OK) return st;
    int64_t cap = 0;
    int wb = 0;
    if (bins) {
        if (bins->capacity < 0 || bins->capacity >= (1ll << 31))
            return fail(ctx, WIPES_ERR_INVALID, "bins capacity out of range");
        cap = bins->capacity;
        wb = bins->with_backward != 0;
        if (need_bwd_bins && !wb) return fail(ctx, WIPES_ERR_INVALID, "bins buffer was not sized with_backward");
    }
    *L = layout_of(p, b, cap, wb);
    if ((st = check_buf(ctx, screen, L->screen_bytes, "screen")) != WIPES_OK) return st;
    if (bins && (st = check_buf(ctx, bins, L->bins_bytes, "bins")) != WIPES_OK) return st;
    return WIPES_OK;
}

wipes_status wipes_project(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, wipes_buffer* screen,
                           void* stream)
{
    Layout L;
    wipes_status st = prologue(ctx, p, b, screen, nullptr, false, false, &L);
    if (st != WIPES_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    // the projection always writes the table (a new frame may follow a
    // different one in this screen buffer); a small one travels with the
    // projection's own launch
    const bool defer = L.n > 0;
    if ((st = upload_descs(ctx, p, b, L, screen->base, s, false, defer)) != WIPES_OK) return st;
    char* base = (char*)screen->base;
    StageScope sc(ctx, kStProject, s);
    const bool pend = ctx->desc_pend;
    ctx->desc_pend = false;
    hipError_t e = launch_project((const ImgDesc*)(base + L.s_descs), L.B, (int32_t)L.n, kparams(p),
                                  (Rec*)(base + L.s_recs), (Aux*)(base + L.s_aux), s,
                                  pend ? &ctx->desc_pend_args : nullptr, pend ? ctx->desc_pend_n : 0);
    if (e != hipSuccess) return hip_fail(ctx, e, "project");
    if (pend) ctx->desc_dst = ctx->desc_pend_dst;
    return WIPES_OK;
}

wipes_status wipes_bin_sort(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, wipes_buffer* screen,
                            wipes_buffer* bins, int64_t* n_instances_out, void* stream)
{
    Layout L;
    if (!bins) return fail(ctx, WIPES_ERR_INVALID, "bins buffer missing");
    wipes_status st = prologue(ctx, p, b, screen, bins, false, false, &L);
    if (st != WIPES_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_descs(ctx, p, b, L, screen->base, s, true)) != WIPES_OK) return st;
    return bin_sort_core(ctx, p, b, L, screen->base, bins->base, n_instances_out, s);
}

wipes_status wipes_render_fwd(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, const wipes_buffer* screen,
                              const wipes_buffer* bins, float* image, float* T_final, int32_t* last, void* stream)
{
    Layout L;
    if (!bins) return fail(ctx, WIPES_ERR_INVALID, "bins buffer missing");
    wipes_status st = prologue(ctx, p, b, screen, bins, false, false, &L);
    if (st != WIPES_OK) return st;
    if (!image) return fail(ctx, WIPES_ERR_INVALID, "image must not be NULL");
    if (p->mode == WIPES_3D_ALPHA && (!T_final || !last))
        return fail(ctx, WIPES_ERR_INVALID, "alpha mode needs T_final and last");
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_descs(ctx, p, b, L, screen->base, s, true, true)) != WIPES_OK) return st;
    return render_fwd_core(ctx, p, b, L, screen->base, bins->base, image, T_final, last, s);
}

wipes_status wipes_render_bwd(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, const wipes_buffer* screen,
                              const wipes_buffer* bins, const float* T_final, const int32_t* last,
                              const float* dL_dimage, float* dscreen, void* stream)
{
    Layout L;
    if (!bins) return fail(ctx, WIPES_ERR_INVALID, "bins buffer missing");
    wipes_status st = prologue(ctx, p, b, screen, bins, true, true, &L);
    if (st != WIPES_OK) return st;
    if (!dL_dimage) return fail(ctx, WIPES_ERR_INVALID, "dL_dimage must not be NULL");
    if (p->mode == WIPES_3D_ALPHA && (!T_final || !last))
        return fail(ctx, WIPES_ERR_INVALID, "alpha mode needs T_final and last");
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_descs(ctx, p, b, L, screen->base, s, true, true)) != WIPES_OK) return st;
    return render_bwd_core(ctx, p, b, L, screen->base, bins->base, T_final, last, dL_dimage, dscreen, s);
}

wipes_status wipes_render_fwd_noalloc(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, float* image,
                                      float* T_final, int32_t* last, int64_t* n_instances_out, void* stream)
{
    if (!ctx) return fail(nullptr, WIPES_ERR_INVALID, "ctx must not be NULL");
    wipes_status st = validate(ctx, p, b, false);
    if (st != WIPES_OK) return st;
    if (!image) return fail(ctx, WIPES_ERR_INVALID, "image must not be NULL");
    if (p->mode == WIPES_3D_ALPHA && (!T_final || !last))
        return fail(ctx, WIPES_ERR_INVALID, "alpha mode needs T_final and last");
    if (!ctx->scratch) return fail(ctx, WIPES_ERR_DEVICE, "static workspace unavailable on this device");
    // the screen workspace first, the bins after it with the largest
    // instance capacity that fits (host arithmetic only)
    const size_t total = (size_t)WIPES_NOALLOC_WORKSPACE_BYTES;
    const size_t sbytes = align_up(layout_of(p, b, 0, 0).screen_bytes, 256);
    const size_t bmin = layout_of(p, b, 1, 0).bins_bytes;
    if (sbytes > total || total - sbytes < bmin)
        return fail(ctx, WIPES_ERR_CAPACITY,
                    "batch needs %zu bytes of projection workspace plus %zu of bins; the static workspace holds %zu",
                    sbytes, bmin, total);
    const size_t rest = total - sbytes;
    int64_t lo = 1, hi = std::min<int64_t>((int64_t)(rest / 16) + 1, (1ll << 31) - 1);   // bins > 16 B/instance
    while (lo < hi) {   // largest capacity whose bins fit in `rest`
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (layout_of(p, b, mid, 0).bins_bytes <= rest) lo = mid; else hi = mid - 1;
    }
    wipes_buffer screen{ctx->scratch, sbytes, 0, 0, 0};
    wipes_buffer bins{ctx->scratch + sbytes, rest, lo, 0, 0};
    // no profiling events here: creating one may allocate
    const bool prof = ctx->prof.on;
    ctx->prof.on = false;
    st = wipes_project(ctx, p, b, &screen, stream);
    if (st == WIPES_OK) st = wipes_bin_sort(ctx, p, b, &screen, &bins, n_instances_out, stream);
    if (st == WIPES_ERR_CAPACITY)
        (void)fail(ctx, st, "frame needs %lld instances; the static workspace holds %lld for this batch",
                   n_instances_out ? (long long)*n_instances_out : -1ll, (long long)lo);
    if (st == WIPES_OK) st = wipes_render_fwd(ctx, p, b, &screen, &bins, image, T_final, last, stream);
    ctx->prof.on = prof;
    return st;
}

wipes_status wipes_check_overflow(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b,
                                  const wipes_buffer* screen, int64_t* required_instances, void* stream)
{
    Layout L;
    wipes_status st = prologue(ctx, p, b, screen, nullptr, false, false, &L);
    if (st != WIPES_OK) return st;
    if (!required_instances) return fail(ctx, WIPES_ERR_INVALID, "required_instances must not be NULL");
    uint32_t ctrl[kCtrlHead];
    hipError_t e = hipMemcpyAsync(ctrl, (char*)screen->base + L.s_ctrl, sizeof(ctrl), hipMemcpyDeviceToHost,
                                  (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "check_overflow");
    *required_instances = ctrl[kCtrlK];
    return ctrl[kCtrlOverflow] ? WIPES_ERR_CAPACITY : WIPES_OK;
}

wipes_status wipes_bins_view(const wipes_params* p, const wipes_batch* b, const wipes_buffer* screen,
                             const wipes_buffer* bins, const uint32_t** keys, const uint32_t** vals,
                             const uint32_t** ranges, int64_t* n_tiles)
{
    Layout L;
    wipes_ctx tmp;
    wipes_status st = prologue(&tmp, p, b, screen, bins, false, false, &L);
    if (!bins) return fail(nullptr, WIPES_ERR_INVALID, "bins buffer missing");
    if (st != WIPES_OK) return fail(nullptr, st, "%s", tmp.err.c_str());
    const char* base = (const char*)bins->base;
    if (keys) *keys = (const uint32_t*)(base + (L.tile_result_b ? L.b_keys_b : L.b_keys_a));
    if (vals) *vals = (const uint32_t*)(base + (L.tile_result_b ? L.b_vals_b : L.b_vals_a));
    if (ranges) *ranges = (const uint32_t*)(base + L.b_ranges);
    if (n_tiles) *n_tiles = L.tiles;
    return WIPES_OK;
}

static const char* kStageNames[kStN] = {"project", "bin_count", "scan", "depth_sort", "rank_scan", "emit",
                                        "tile_sort", "ranges", "blend_fwd", "blend_bwd", "project_bwd"};

const char* wipes_stage_name(int32_t stage)
{
    return (stage >= 0 && stage < kStN) ? kStageNames[stage] : "";
}

wipes_status wipes_profile_enable(wipes_ctx* ctx, int32_t enable)
{
    if (!ctx) return fail(nullptr, WIPES_ERR_INVALID, "ctx must not be NULL");
    ctx->prof.on = enable != 0;
    return WIPES_OK;
}

wipes_status wipes_profile_read(wipes_ctx* ctx, double* ms, int64_t* launches, int32_t n)
{
    if (!ctx || !ms || !launches || n < kStN) return fail(ctx, WIPES_ERR_INVALID, "need arrays of WIPES_N_STAGES");
    for (int st = 0; st < kStN; ++st) {
        double tot = 0.0;
        for (auto& pr : ctx->prof.rec[st]) {
            hipError_t e = hipEventSynchronize(pr.second);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, pr.first, pr.second);
            if (e != hipSuccess) return hip_fail(ctx, e, "profile read");
            tot += t;
            ctx->prof.pool.push_back(pr.first);
            ctx->prof.pool.push_back(pr.second);
        }
        ms[st] = tot;
        launches[st] = (int64_t)ctx->prof.rec[st].size();
        ctx->prof.rec[st].clear();
    }
    return WIPES_OK;
}

wipes_status wipes_render_stats(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b,
                                const wipes_buffer* screen, const wipes_buffer* bins, const float* T_final,
                                const int32_t* last, uint64_t* out, void* stream)
{
    Layout L;
    if (!bins || !out) return fail(ctx, WIPES_ERR_INVALID, "bins and out must be set");
    wipes_status st = prologue(ctx, p, b, screen, bins, false, false, &L);
    if (st != WIPES_OK) return st;
    if (p->mode == WIPES_3D_ALPHA && (!T_final || !last))
        return fail(ctx, WIPES_ERR_INVALID, "alpha mode needs T_final and last");
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload_descs(ctx, p, b, L, screen->base, s, true)) != WIPES_OK) return st;
    return render_stats_core(ctx, p, b, L, screen->base, bins->base, T_final, last, out, s);
}

}  // extern "C"
