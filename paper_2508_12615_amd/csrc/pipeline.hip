// Stage sequencing of the render path: bin/sort, forward blend, backward.
//
// bin_sort (one stream, no allocation):
//   count  -> scan (index order, capacity check)   -> [alpha: depth sort of all
//   primitives by FP32 key, then scan in depth order] -> emit -> tile sort ->
//   ranges [-> longest-first tile order for the persistent queue].
// The tile sort's key is the global tile index only; depth order comes from
// emitting instances in depth order into a stable sort (see binning.hip), so
// the 45-bit (tile, depth) sort of the 3DGS pipeline becomes a 32-bit sort over
// primitives plus a ceil(log2 tiles)-bit sort over instances.
#include <hip/hip_runtime.h>

#include "api_internal.hpp"

namespace wipes {

struct Views {
    Rec* recs;
    Aux* aux;
    uint32_t *count, *off_id, *dkey_a, *dval_a, *dkey_b, *dval_b, *dhist, *ddtot, *bsum, *bsum2, *ctrl;
    ImgDesc* descs;
    PrimPack *pk, *pkr;
    uint32_t *keys_a, *vals_a, *keys_b, *vals_b, *hist, *dtot, *order, *tbsum;
    uint2* ranges;
    float* slots;
    unsigned long long* cmask;
    uint32_t* svalid;
};

static Views views(const Layout& L, const void* screen, const void* bins)
{
    char* s = (char*)screen;
    char* b = (char*)bins;
    Views v{};
    v.recs = (Rec*)(s + L.s_recs);
    v.aux = (Aux*)(s + L.s_aux);
    v.count = (uint32_t*)(s + L.s_count);
    v.off_id = (uint32_t*)(s + L.s_off_id);
    v.pk = (PrimPack*)(s + L.s_pk);
    if (L.alpha) {
        v.dkey_a = (uint32_t*)(s + L.s_dkey_a);
        v.dval_a = (uint32_t*)(s + L.s_dval_a);
        v.dkey_b = (uint32_t*)(s + L.s_dkey_b);
        v.dval_b = (uint32_t*)(s + L.s_dval_b);
        v.pkr = (PrimPack*)(s + L.s_pkr);
        v.dhist = (uint32_t*)(s + L.s_dhist);
        v.ddtot = (uint32_t*)(s + L.s_ddtot);
    }
    v.bsum = (uint32_t*)(s + L.s_bsum);
    v.bsum2 = (uint32_t*)(s + L.s_bsum2);
    v.ctrl = (uint32_t*)(s + L.s_ctrl);
    v.descs = (ImgDesc*)(s + L.s_descs);
    if (b) {
        v.keys_a = (uint32_t*)(b + L.b_keys_a);
        v.vals_a = (uint32_t*)(b + L.b_vals_a);
        v.keys_b = (uint32_t*)(b + L.b_keys_b);
        v.vals_b = (uint32_t*)(b + L.b_vals_b);
        v.hist = (uint32_t*)(b + L.b_hist);
        v.dtot = (uint32_t*)(b + L.b_dtot);
        v.ranges = (uint2*)(b + L.b_ranges);
        v.order = (uint32_t*)(b + L.b_order);
        v.tbsum = (uint32_t*)(b + L.b_tbsum);
        if (L.with_bwd) {
            v.slots = (float*)(b + L.b_slots);
            v.cmask = (unsigned long long*)(b + L.b_cmask);
            v.svalid = (uint32_t*)(b + L.b_svalid);
        }
    }
    return v;
}

// The longest-first tile order (persistent 2 and 3), written by bin_sort_core.
static const uint32_t* tile_order(const Layout& L, const Views& v)
{
    (void)L;
    return v.order;
}

#define HIP_TRY(call, what)                                    \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, what);  \
    } while (0)

wipes_status bin_sort_core(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, const Layout& L,
                           void* screen, void* bins, int64_t* n_instances_out, hipStream_t s)
{
    (void)b;
    const Views v = views(L, screen, bins);
    const KParams kp = kparams(p);
    const uint32_t n = (uint32_t)L.n;
    const uint32_t nw = (n + 63u) / 64u;   // count sums, one per 64 primitives (or depth ranks)
    {
        StageScope sc(ctx, kStCount, s);
        // (the count kernel also zeroes the tile ranges for the end of this
        // call, and with backward bins the contribution mask and slot marks
        // of the renders that follow)
        uint32_t* cm = v.cmask ? (uint32_t*)v.cmask : nullptr;
        const uint32_t ncm = v.cmask ? (uint32_t)((L.b_svalid + (size_t)(L.cap / 32 + 2) * 4 - L.b_cmask) / 4) : 0u;
        const Clear2 clr{cm, ncm, (uint32_t*)v.ranges, (uint32_t)(2 * L.tiles)};
        HIP_TRY(launch_bin_count(v.descs, L.B, (int32_t)n, kp, v.recs, v.aux, v.count, v.pk, v.dkey_a, v.dval_a,
                                 v.bsum, clr, s),
                "count");
    }
    // K, capacity check -> n_eff, overflow flag
    {
        StageScope sc(ctx, kStScan, s);
        // the scan also stores K into the pinned host word when the caller
        // wants it; the host waits for it only before the emission, so the
        // round trip overlaps the depth sort
        // (and zeroes both persistent-queue counter sets)
        HIP_TRY(scan_sums(v.bsum, nw, v.ctrl + kCtrlK, (uint32_t)L.cap, v.ctrl + kCtrlNEff, v.ctrl + kCtrlOverflow,
                          n_instances_out ? ctx->k_host_dev : nullptr, s, v.ctrl + kCtrlQueueFwd,
                          (uint32_t)(kCtrlWords - kCtrlQueueFwd)),
                "scan");
    }
    if (!ctx->capturing) {   // the first forward and backward render after this need not clear again
        ctx->fresh_screen = screen;
        ctx->fresh_bins = bins;
        ctx->fresh_fwd = ctx->fresh_bwd = true;
    }
    if (n_instances_out) HIP_TRY(hipEventRecord(ctx->k_ev, s), "read K event");
    const uint32_t* order = nullptr;
    const uint32_t* woff = v.bsum;
    if (L.alpha) {
        int in_b = 0;
        {
            StageScope sc(ctx, kStDepthSort, s);
            HIP_TRY(radix_sort(v.dkey_a, v.dval_a, v.dkey_b, v.dval_b, n, nullptr, n, 32, v.dhist, v.ddtot, &in_b, s),
                    "depth sort");
        }
        order = in_b ? v.dval_b : v.dval_a;
        {
            StageScope sc(ctx, kStRankScan, s);
            // the packs in depth order with the count sums of each 64 ranks;
            // the same launch numbers each primitive's gradient slots (its
            // instance offset: the backward finds an instance's slot from its
            // primitive's pack)
            HIP_TRY(launch_rank_pack((int32_t)n, order, v.pk, v.pkr, v.bsum2, v.count, v.bsum, v.off_id, s),
                    "rank pack");
            HIP_TRY(scan_sums(v.bsum2, nw, v.ctrl + 3, 0u, nullptr, nullptr, nullptr, s), "rank scan");
        }
        woff = v.bsum2;
    } else {
        StageScope sc(ctx, kStRankScan, s);
        HIP_TRY(launch_count_apply((int32_t)n, v.count, v.bsum, v.off_id, v.pk, s), "count offsets");
    }
    uint32_t max_k = (uint32_t)L.cap;
    if (n_instances_out) {
        HIP_TRY(hipEventSynchronize(ctx->k_ev), "sync K");
        const uint32_t K = *ctx->k_host;
        *n_instances_out = K;
        if ((int64_t)K > L.cap) return fail(ctx, WIPES_ERR_CAPACITY, "%u instances exceed capacity %lld", K, (long long)L.cap);
        max_k = K;
    }
    {
        StageScope sc(ctx, kStEmit, s);
        HIP_TRY(launch_emit(v.descs, L.B, (int32_t)n, kp, L.alpha ? v.pkr : v.pk, order, woff, v.ctrl + kCtrlNEff,
                            v.keys_a, v.vals_a, s),
                "emit");
    }
    int in_b = 0;
    {
        StageScope sc(ctx, kStTileSort, s);
        HIP_TRY(radix_sort(v.keys_a, v.vals_a, v.keys_b, v.vals_b, 0, v.ctrl + kCtrlNEff, max_k, L.tile_bits, v.hist,
                           v.dtot, &in_b, s),
                "tile sort");
    }
    const uint32_t* skeys = in_b ? v.keys_b : v.keys_a;
    StageScope sc(ctx, kStRanges, s);
    HIP_TRY(launch_ranges(skeys, v.ctrl + kCtrlNEff, max_k, v.ranges, s), "ranges");
    if (p->persistent >= 2)   // longest tile list first (persistent queue or ordered grid)
        HIP_TRY(launch_tile_lpt_order(v.ranges, (uint32_t)L.tiles, (uint32_t*)((char*)bins + L.b_lpt), v.order, s),
                "lpt order");
    return WIPES_OK;
}

wipes_status render_fwd_core(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, const Layout& L,
                             const void* screen, const void* bins, float* image, float* T_final, int32_t* last,
                             hipStream_t s)
{
    (void)b;
    const Views v = views(L, screen, bins);
    const KParams kp = kparams(p);
    const uint32_t* svals = L.tile_result_b ? v.vals_b : v.vals_a;
    uint32_t* queue = nullptr;
    uint32_t pblocks = 0;
    const uint32_t* order = p->persistent >= 2 ? tile_order(L, v) : nullptr;
    if (p->persistent == 1 || p->persistent == 2) {
        queue = v.ctrl + kCtrlQueueFwd;
        pblocks = (uint32_t)ctx->n_cu * 8u;
    }
    // queue counters, and the mask in which the forward records which
    // primitives contribute to each block (for the backward), cleared in one
    // launch -- unless bin_sort has just cleared them
    const bool fresh = !ctx->capturing && ctx->fresh_fwd && ctx->fresh_screen == screen && ctx->fresh_bins == bins;
    ctx->fresh_fwd = false;
    const size_t mwords = v.cmask && !fresh ? (size_t)(p->tile_w / 8) * (p->tile_h / 8) * L.cmask_words * 2 : 0;
    if (!fresh || ctx->desc_pend)
        HIP_TRY(launch_fill2_put(ctx, fresh ? nullptr : queue, queue && !fresh ? kQueueLanes * kQueueStride : 0u,
                                 (uint32_t*)v.cmask, (uint32_t)mwords, 0u, s),
                "queue reset / mask clear");
    StageScope sc(ctx, kStBlendFwd, s);
    HIP_TRY(launch_blend_fwd(v.descs, L.B, kp, v.recs, svals, v.ranges, v.ctrl + kCtrlOverflow, (uint32_t)L.tiles,
                             order, queue, pblocks, image, T_final, last, v.cmask, L.cmask_words, s),
            "blend fwd");
    return WIPES_OK;
}

wipes_status render_bwd_core(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, const Layout& L,
                             const void* screen, const void* bins, const float* T_final, const int32_t* last,
                             const float* dLdC, float* dscreen, hipStream_t s)
{
    (void)b;
    const Views v = views(L, screen, bins);
    const KParams kp = kparams(p);
    const uint32_t* svals = L.tile_result_b ? v.vals_b : v.vals_a;
    uint32_t* queue = nullptr;
    uint32_t pblocks = 0;
    const uint32_t* order = p->persistent >= 2 ? tile_order(L, v) : nullptr;
    if (p->persistent == 1 || p->persistent == 2) {
        queue = v.ctrl + kCtrlQueueBwd;
        pblocks = (uint32_t)ctx->n_cu * 8u;
    }
    // queue counters and slot marks cleared -- unless bin_sort has just
    // cleared them; then a pending descriptor table that differs from the
    // stored one only in gradient pointers (the blend reads none) travels
    // with the projection backward, the only kernel that uses them
    const bool fresh = !ctx->capturing && ctx->fresh_bwd && ctx->fresh_screen == screen &&
                       ctx->fresh_bins == bins && (!ctx->desc_pend || ctx->desc_pend_grads_only);
    ctx->fresh_bwd = false;
    const bool pend_pbwd = fresh && ctx->desc_pend;
    if (!fresh)
        HIP_TRY(launch_fill2_put(ctx, queue, queue ? kQueueLanes * kQueueStride : 0u, v.svalid,
                                 (uint32_t)(L.cap / 32 + 2), 0u, s),
                "queue reset / slot marks clear");
    if (pend_pbwd) ctx->desc_pend = false;
    {
        StageScope sc(ctx, kStBlendBwd, s);
        HIP_TRY(launch_blend_bwd(v.descs, L.B, kp, v.recs, svals, v.pk, v.ranges, v.ctrl + kCtrlOverflow,
                                 (uint32_t)L.tiles, order, queue, pblocks, T_final, last, dLdC, v.slots, v.svalid,
                                 v.cmask, L.cmask_words, s),
                "blend bwd");
    }
    StageScope sc(ctx, kStProjectBwd, s);
    HIP_TRY(launch_project_bwd(v.descs, L.B, (int32_t)L.n, kp, v.recs, v.count, v.off_id, v.slots, v.svalid,
                               v.ctrl + kCtrlOverflow, dscreen, s, pend_pbwd ? &ctx->desc_pend_args : nullptr,
                               pend_pbwd ? ctx->desc_pend_n : 0),
            "project bwd");
    if (pend_pbwd && L.n > 0) ctx->desc_dst = ctx->desc_pend_dst;
    return WIPES_OK;
}

wipes_status render_stats_core(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, const Layout& L,
                               const void* screen, const void* bins, const float* T_final, const int32_t* last,
                               uint64_t* out, hipStream_t s)
{
    (void)b;
    const Views v = views(L, screen, bins);
    const KParams kp = kparams(p);
    const uint32_t* svals = L.tile_result_b ? v.vals_b : v.vals_a;
    // the queue counters double as scratch for the four totals (8 bytes each)
    unsigned long long* acc = (unsigned long long*)(v.ctrl + 8);
    HIP_TRY(launch_fill_u32(v.ctrl + 8, 8, 0u, s), "stats reset");
    HIP_TRY(launch_pair_stats(v.descs, L.B, kp, v.recs, svals, v.ranges, v.ctrl + kCtrlOverflow, (uint32_t)L.tiles,
                              T_final, last, acc, s),
            "stats");
    unsigned long long h[4];
    HIP_TRY(hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, s), "stats read");
    HIP_TRY(hipStreamSynchronize(s), "stats sync");
    for (int k = 0; k < 4; ++k) out[k] = h[k];
    return WIPES_OK;
}

}  // namespace wipes
