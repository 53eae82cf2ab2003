// Host-side internals of the C ABI: workspace layout, context, stage
// sequencing and the launchers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <string>
#include <vector>

#include "common.hpp"

constexpr int kMaxImages = 1024;
constexpr int kRing = 8;
constexpr size_t kStagingBytes = (size_t)kMaxImages * sizeof(wipes::ImgDesc);

// device control words at Layout::s_ctrl
// (words 0..kCtrlHead-1 are read back by wipes_check_overflow; 8..15 hold
// the work-count totals; the two persistent queues follow, one 256-byte line
// per counter)
enum {
    kCtrlK = 0,
    kCtrlNEff = 1,
    kCtrlOverflow = 2,
    kCtrlHead = 16,
    kCtrlQueueFwd = 64,
    kCtrlQueueBwd = kCtrlQueueFwd + wipes::kQueueLanes * wipes::kQueueStride,
    kCtrlWords = kCtrlQueueBwd + wipes::kQueueLanes * wipes::kQueueStride
};

struct StagingSlot {
    void* host = nullptr;
    hipEvent_t ev = nullptr;
    bool used = false;
};

// Render-path stages bracketed by profiling events (order = WIPES_STAGE_*).
enum Stage {
    kStProject = 0, kStCount, kStScan, kStDepthSort, kStRankScan, kStEmit, kStTileSort, kStRanges,
    kStBlendFwd, kStBlendBwd, kStProjectBwd, kStN
};

struct Profiler {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> rec[kStN];
    std::vector<hipEvent_t> pool;
};

struct wipes_ctx {
    int device = 0;
    int n_cu = 256;
    std::string err;
    StagingSlot ring[kRing];
    int ring_next = 0;
    bool capturing = false;      // descriptor uploads are skipped while capturing a graph
    uint32_t* k_host = nullptr;  // pinned word: instance count read back by bin_sort
    uint32_t* k_host_dev = nullptr;   // the same word as the device addresses it
    hipEvent_t k_ev = nullptr;   // recorded after the kernel that writes it
    const void* desc_dst = nullptr;          // where the last descriptor table went
    std::vector<wipes::ImgDesc> desc_last;   // and what it held
    bool desc_pend = false;                  // a table waits for launch_fill2_put
    bool desc_pend_grads_only = false;       // it differs from the stored one in gradient pointers only
    // bin_sort zeroed the queue counters, contribution mask and slot marks of
    // this (screen, bins) pair: the next forward / backward render need not
    const void* fresh_screen = nullptr;
    const void* fresh_bins = nullptr;
    bool fresh_fwd = false, fresh_bwd = false;
    int desc_pend_n = 0;
    char* desc_pend_dst = nullptr;
    wipes::DescArgs desc_pend_args;
    std::vector<wipes::ImgDesc> desc_tmp;    // reused for each new table (no per-call reallocation)
    Profiler prof;
    unsigned char* scratch = nullptr;        // this device's copy of the static workspace (device address)
};

namespace wipes {

// Byte offsets of every array in the screen and bins buffers.
struct Layout {
    int B = 0;
    bool alpha = false;
    int with_bwd = 0;
    int64_t n = 0, pixels = 0, tiles = 0, cap = 0;
    // screen buffer
    size_t s_recs, s_aux, s_count, s_off_id, s_dkey_a, s_dval_a, s_dkey_b, s_dval_b, s_dhist, s_ddtot;
    size_t s_pk, s_pkr;   // packed {count, box0, box1, slot base, ...} per primitive / per depth rank
    size_t s_bsum, s_bsum2;   // count sums per 64 primitives / per 64 depth ranks, scanned in place
    size_t s_ctrl, s_descs, screen_bytes;
    // bins buffer
    size_t b_keys_a, b_vals_a, b_keys_b, b_vals_b, b_hist, b_dtot, b_ranges, b_order, b_lpt, b_tbsum, b_slots;
    size_t b_cmask;           // per 8x8 block of a tile, one bit per list position (backward only)
    size_t b_svalid;          // one bit per gradient slot: written by this backward (backward only)
    uint32_t cmask_words;     // 64-bit words per block row of the mask
    size_t bins_bytes;
    int tile_bits = 1;
    int tile_result_b = 0;    // tile sort result in the *_b arrays
    int depth_result_b = 0;   // depth sort result in the *_b arrays
};

wipes_status fail(wipes_ctx* ctx, wipes_status st, const char* fmt, ...);
wipes_status hip_fail(wipes_ctx* ctx, hipError_t e, const char* where);
wipes_status validate(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, bool need_grads);
bool tile_ok(int tw, int th);
KParams kparams(const wipes_params* p);
Layout layout_of(const wipes_params* p, const wipes_batch* b, int64_t cap, int with_bwd);
void fill_descs(const wipes_params* p, const wipes_batch* b, std::vector<ImgDesc>& out);
// reuse: skip the upload when this context's last upload put the same table
// at the same place (for the stages after the projection of one frame).
// defer: a small table is left pending for the caller's first launch, which
// must be launch_fill2_put.
wipes_status upload_descs(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, const Layout& L, void* screen,
                          hipStream_t s, bool reuse = false, bool defer = false);
// launch_fill2_u32 that also writes a pending descriptor table
hipError_t launch_fill2_put(wipes_ctx* ctx, uint32_t* p, uint32_t n, uint32_t* q, uint32_t m, uint32_t v,
                            hipStream_t s);

// Brackets one stage with events when profiling is on (never while capturing).
struct StageScope {
    wipes_ctx* c;
    int st;
    hipStream_t s;
    hipEvent_t a = nullptr;
    StageScope(wipes_ctx* ctx, int stage, hipStream_t stream);
    ~StageScope();
};

// stage sequencing (pipeline.hip)
wipes_status bin_sort_core(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, const Layout& L,
                           void* screen, void* bins, int64_t* n_instances_out, hipStream_t s);
wipes_status render_fwd_core(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, const Layout& L,
                             const void* screen, const void* bins, float* image, float* T_final, int32_t* last,
                             hipStream_t s);
wipes_status render_bwd_core(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, const Layout& L,
                             const void* screen, const void* bins, const float* T_final, const int32_t* last,
                             const float* dLdC, float* dscreen, hipStream_t s);

wipes_status render_stats_core(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* b, const Layout& L,
                               const void* screen, const void* bins, const float* T_final, const int32_t* last,
                               uint64_t* out, hipStream_t s);

// kernel launchers
// da/nda: a descriptor table passed as the argument (nda images), which the
// kernel reads from there and stores at descs (nda = 0: read descs)
hipError_t launch_project(const ImgDesc* descs, int B, int32_t n_total, const KParams& kp, Rec* recs, Aux* aux,
                          hipStream_t s, const DescArgs* da = nullptr, int nda = 0);
// Counting: per primitive its kept tile count (count, pk), depth keys; per 64
// primitives the count sum (wsum); clr: two word ranges that the kernel
// zeroes on its way (the tile ranges of this bin_sort).
hipError_t launch_bin_count(const ImgDesc* descs, int B, int32_t n_total, const KParams& kp, Rec* recs,
                            const void* aux, uint32_t* count, PrimPack* pk, uint32_t* dkey, uint32_t* dval,
                            uint32_t* wsum, const Clear2& clr, hipStream_t s);
// off_id[i] = pk[i].base = exclusive prefix of count (woff: scanned wave sums)
hipError_t launch_count_apply(int32_t n_total, const uint32_t* count, const uint32_t* woff, uint32_t* off_id,
                              PrimPack* pk, hipStream_t s);
// pkr[r] = pk[order[r]], wsum_r: count sums of 64 ranks; and count_apply
hipError_t launch_rank_pack(int32_t n_total, const uint32_t* order, PrimPack* pk, PrimPack* pkr, uint32_t* wsum_r,
                            const uint32_t* count, const uint32_t* woff_c, uint32_t* off_id, hipStream_t s);
hipError_t launch_emit(const ImgDesc* descs, int B, int32_t n_total, const KParams& kp, const PrimPack* pkx,
                       const uint32_t* order, const uint32_t* woff, const uint32_t* n_eff, uint32_t* keys,
                       uint32_t* vals, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t n, uint32_t v, hipStream_t s);
uint32_t lpt_slices(uint32_t n_tiles);   // workgroups of the two-pass longest-first order (256 counts each)
hipError_t launch_tile_lpt_order(const uint2* ranges, uint32_t n_tiles, uint32_t* counts, uint32_t* order,
                                 hipStream_t s);
hipError_t launch_fill2_u32(uint32_t* p, uint32_t n, uint32_t* q, uint32_t m, uint32_t v, hipStream_t s);
hipError_t launch_ranges(const uint32_t* keys, const uint32_t* n_eff, uint32_t max_k, uint2* ranges, hipStream_t s);
// Exclusive scan of sums[0..n) in place by one workgroup; *total = sum, and
// with n_eff set: *n_eff = total, or 0 with *overflow = 1 when cap != 0 and
// total > cap; total_host (pinned) also gets the total when set.
// clr[0..nclr) is zeroed on the way.
hipError_t scan_sums(uint32_t* sums, uint32_t n, uint32_t* total, uint32_t cap, uint32_t* n_eff, uint32_t* overflow,
                     uint32_t* total_host, hipStream_t s, uint32_t* clr = nullptr, uint32_t nclr = 0);
   // out2[i * stride2] = out[i] too
int radix_passes(int nbits);
int radix_digit_bits(int nbits);   // digit width of each pass of radix_sort
uint32_t radix_max_blocks(uint32_t cap);   // histogram columns a sort of up to cap keys needs
// Stable LSD sort of (key, value) over the low nbits of the keys; ping-pongs
// between the *0 and *1 arrays, *result_in_1 tells where the result is.  With
// nbits <= 16 the keys must be below 2^16 (they are staged in 16 bits).
hipError_t radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, uint32_t n_host,
                      const uint32_t* n_dev, uint32_t max_n, int nbits, uint32_t* hist, uint32_t* dtot,
                      int* result_in_1, hipStream_t s);
hipError_t launch_blend_fwd(const ImgDesc* descs, int B, const KParams& kp, const Rec* recs, const uint32_t* vals,
                            const uint2* ranges, const uint32_t* ovf, uint32_t n_tiles, const uint32_t* order,
                            uint32_t* queue, uint32_t persistent_blocks, float* image, float* T_final, int32_t* last,
                            unsigned long long* cmask, uint32_t cmask_words, hipStream_t s);
hipError_t launch_blend_bwd(const ImgDesc* descs, int B, const KParams& kp, const Rec* recs, const uint32_t* vals,
                            const PrimPack* pk, const uint2* ranges, const uint32_t* ovf, uint32_t n_tiles,
                            const uint32_t* order, uint32_t* queue, uint32_t persistent_blocks, const float* T_final,
                            const int32_t* last, const float* dLdC, float* slots, uint32_t* valid,
                            const unsigned long long* cmask, uint32_t cmask_words, hipStream_t s);
hipError_t launch_l2_grad(const ImgDesc* descs, int B, int32_t npix, const float* image, const float* target,
                          float* grad, hipStream_t s);
hipError_t launch_pair_stats(const ImgDesc* descs, int B, const KParams& kp, const Rec* recs, const uint32_t* vals,
                             const uint2* ranges, const uint32_t* ovf, uint32_t n_tiles, const float* T_final,
                             const int32_t* last, unsigned long long* out, hipStream_t s);
// da/nda: as launch_project (the table with this call's gradient pointers)
hipError_t launch_project_bwd(const ImgDesc* descs, int B, int32_t n_total, const KParams& kp, const Rec* recs,
                              const uint32_t* count, const uint32_t* off_id, const float* slots,
                              const uint32_t* valid, const uint32_t* overflow, float* dscreen, hipStream_t s,
                              const DescArgs* da = nullptr, int nda = 0);

}  // namespace wipes
