// Serving: resident scenes, render requests admitted by HBM footprint, and
// continuous batching over two HIP streams.
//
// Two threads own the device work:
//  * the worker admits the longest FIFO prefix of pending requests that fits
//    the free request slots, the batch limit and one contiguous arena block
//    (head-of-line: a request that does not fit blocks those behind it, so
//    nothing starves), then runs projection and binning of the batch on the
//    prep stream (one host synchronisation for the instance count) and the
//    tile-queue forward blend of all its requests -- mixed resolutions, one
//    launch -- on the blend stream, ordered by an event;
//  * the completion thread waits on the oldest in-flight batch's event and
//    retires it the moment the GPU is done (its requests complete, arena
//    memory and request slots return, the worker is woken).
// While batch k blends, batch k+1 is already being projected and sorted, so
// requests that arrive during a launch are admitted as soon as slots and
// memory allow.  Every request's image depends only on its scene, camera and
// the per-pixel rule, so it is the same alone and in any mix.
//
// The admission policy and the arena allocator are plain host code shared
// with wipes_serve_simulate, a discrete-event model with a fake executor that
// the CPU tests drive.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "api_internal.hpp"

using namespace wipes;

namespace {

constexpr size_t kAlign = 256;
size_t al(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over one device block (offsets only).
struct Arena {
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> length

    void reset(size_t n)
    {
        size = n;
        free_.clear();
        if (n) free_[0] = n;
    }
    bool fits(size_t n) const
    {
        n = al(n);
        for (auto& kv : free_)
            if (kv.second >= n) return true;
        return false;
    }
    bool alloc(size_t n, size_t* off)
    {
        n = al(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rem = it->second - n, o2 = it->first + n;
            free_.erase(it);
            if (rem) free_[o2] = rem;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = al(n);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const
    {
        size_t f = 0;
        for (auto& kv : free_) f += kv.second;
        return size - f;
    }
};

// Admission: the longest FIFO prefix (at most max_take of the n waiting
// requests) whose footprint prefix_bytes(k) fits one arena block.
template <typename PrefixBytes>
size_t admit_prefix(size_t n, size_t max_take, const Arena& arena, PrefixBytes prefix_bytes)
{
    size_t take = 0;
    while (take < n && take < max_take && arena.fits(prefix_bytes(take + 1))) ++take;
    return take;
}

struct SScene {
    wipes_prims prims{};
    void* mem = nullptr;
    double k_ratio = 12.0;    // instances per primitive, learned from rendered batches
    int refs = 0;             // pending + in-flight requests
};

struct SReq {
    int32_t scene = 0;
    wipes_camera cam{};
    float* out = nullptr;
    hipEvent_t ready = nullptr;   // recorded on the caller's stream at submit: `out` is free to write after it
    double t_submit = 0.0, t_done = -1.0;
    bool deferred = false;
    bool admitted = false;
};

struct SBatch {
    std::vector<uint64_t> ids;
    size_t off = 0, bytes = 0;
    hipEvent_t prep = nullptr, done = nullptr;
};

}  // namespace

struct wipes_server {
    wipes_ctx* ctx = nullptr;
    int device = 0;
    wipes_serve_config cfg{};
    wipes_params params{};
    void* arena_mem = nullptr;
    Arena arena;
    size_t arena_peak = 0;
    hipStream_t s_prep = nullptr, s_blend = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::map<int32_t, SScene> scenes;
    int32_t next_scene = 0;
    std::unordered_map<uint64_t, SReq> reqs;
    std::deque<uint64_t> pending;
    uint64_t next_id = 1;
    std::deque<SBatch> inflight;
    int launching = 0;        // batches taken off `pending` and not yet in flight
    int slots_used = 0;
    std::thread worker, completer;
    bool stop = false, worker_done = false;
    std::string err;
    std::vector<double> lat_ms;
    double t_first = -1.0, t_last = -1.0;
    int64_t n_admitted = 0, n_deferred = 0, n_batches = 0, n_batched = 0;
    std::vector<hipEvent_t> ev_pool;
};

namespace {

// Takes an event from the pool (caller holds the lock: the completion thread
// returns events to the pool concurrently).
hipEvent_t get_event(wipes_server* S)
{
    if (!S->ev_pool.empty()) {
        hipEvent_t e = S->ev_pool.back();
        S->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
    return e;
}

// Workspace of a batch: screen + bins (forward only) + T_final + last.
size_t batch_bytes(const wipes_params* p, const std::vector<wipes_image>& ims, int64_t cap, Layout* out)
{
    wipes_batch b{(int32_t)ims.size(), ims.data()};
    const Layout L = layout_of(p, &b, cap, 0);
    if (out) *out = L;
    return al(L.screen_bytes) + al(L.bins_bytes) + 2 * al((size_t)L.pixels * 4);
}

// Instance capacity estimate for a batch: requests' primitive counts times the
// learned instances-per-primitive ratio of their scenes (+15 %).
int64_t capacity_for(const std::vector<wipes_image>& ims, const std::vector<double>& ratio)
{
    double k = 0.0;
    for (size_t i = 0; i < ims.size(); ++i) k += (double)ims[i].prims.n * ratio[i];
    return (int64_t)std::min(k * 1.15 + 4096.0, 2.0e9);
}

// Completes the oldest in-flight batch (its done event has been reached).
// Called with the lock held.
void retire_front(wipes_server* S)
{
    SBatch& b = S->inflight.front();
    const double t = now_s();
    for (uint64_t id : b.ids) {
        SReq& r = S->reqs[id];
        r.t_done = t;
        if (r.ready) S->ev_pool.push_back(r.ready);
        r.ready = nullptr;
        S->lat_ms.push_back((t - r.t_submit) * 1e3);
        S->scenes[r.scene].refs--;
        S->slots_used--;
    }
    S->t_last = t;
    S->arena.release(b.off, b.bytes);
    S->ev_pool.push_back(b.prep);
    S->ev_pool.push_back(b.done);
    S->inflight.pop_front();
}

void completer_main(wipes_server* S)
{
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv.wait(lk, [&] { return !S->inflight.empty() || (S->stop && S->worker_done); });
        if (S->inflight.empty()) break;   // stopping, nothing left in flight
        hipEvent_t done = S->inflight.front().done;
        lk.unlock();
        const hipError_t e = hipEventSynchronize(done);
        lk.lock();
        if (e != hipSuccess && S->err.empty()) S->err = hipGetErrorString(e);
        retire_front(S);
        S->cv.notify_all();
    }
}

// Project, bin, sort (prep stream) and blend (blend stream) one batch.
// Called without the lock; takes it only for the arena (shared with the
// completion thread).  *K_out receives the batch's instance count.
wipes_status launch_batch(wipes_server* S, std::vector<wipes_image>& ims, const std::vector<hipEvent_t>& ready,
                          int64_t cap, SBatch& B, int64_t* K_out)
{
    wipes_batch b{(int32_t)ims.size(), ims.data()};
    for (int attempt = 0; attempt < 4; ++attempt) {
        Layout L;
        const size_t bytes = batch_bytes(&S->params, ims, cap, &L);
        size_t off = 0;
        {
            // wait for in-flight batches to free memory (the completion thread
            // releases it and notifies)
            std::unique_lock<std::mutex> lk(S->mu);
            bool ok = false;
            S->cv.wait(lk, [&] { return (ok = S->arena.alloc(bytes, &off)) || S->inflight.empty(); });
            if (!ok) return fail(S->ctx, WIPES_ERR_NOMEM, "batch exceeds the serving arena");
            S->arena_peak = std::max(S->arena_peak, S->arena.used());
        }
        char* base = (char*)S->arena_mem + off;
        wipes_buffer sb{base, L.screen_bytes, 0, 0, 0};
        wipes_buffer bb{base + al(L.screen_bytes), L.bins_bytes, cap, 0, 0};
        float* T = (float*)(base + al(L.screen_bytes) + al(L.bins_bytes));
        int32_t* last = (int32_t*)((char*)T + al((size_t)L.pixels * 4));
        wipes_status st = wipes_project(S->ctx, &S->params, &b, &sb, S->s_prep);
        int64_t K = 0;
        if (st == WIPES_OK) st = wipes_bin_sort(S->ctx, &S->params, &b, &sb, &bb, &K, S->s_prep);
        if (st == WIPES_ERR_CAPACITY || st != WIPES_OK) {
            std::lock_guard<std::mutex> lk(S->mu);
            S->arena.release(off, bytes);
            S->cv.notify_all();
        }
        if (st == WIPES_ERR_CAPACITY) {
            cap = (int64_t)(K * 1.1) + 4096;
            continue;
        }
        if (st != WIPES_OK) return st;
        *K_out = K;
        (void)hipEventRecord(B.prep, S->s_prep);
        (void)hipStreamWaitEvent(S->s_blend, B.prep, 0);
        // the blend writes the callers' buffers: after whatever their streams queued before each submit
        for (hipEvent_t e : ready)
            if (e) (void)hipStreamWaitEvent(S->s_blend, e, 0);
        // every image writes to its request's buffer; the batch image array is unused
        st = wipes_render_fwd(S->ctx, &S->params, &b, &sb, &bb, T, T, last, S->s_blend);
        (void)hipEventRecord(B.done, S->s_blend);
        if (st != WIPES_OK) {
            (void)hipStreamSynchronize(S->s_blend);
            std::lock_guard<std::mutex> lk(S->mu);
            S->arena.release(off, bytes);
            S->cv.notify_all();
            return st;
        }
        B.off = off;
        B.bytes = bytes;
        return WIPES_OK;
    }
    return fail(S->ctx, WIPES_ERR_CAPACITY, "instance estimate kept growing");
}

void worker_main(wipes_server* S)
{
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv.wait(lk, [&] {
            return (S->stop && S->pending.empty()) || (!S->pending.empty() && S->slots_used < S->cfg.max_slots);
        });
        if (S->pending.empty()) break;   // stopping with nothing pending
        // admission
        const size_t free_slots = (size_t)std::max(0, S->cfg.max_slots - S->slots_used);
        const size_t max_take = std::min(free_slots, (size_t)S->cfg.max_batch);
        std::vector<wipes_image> cand;
        std::vector<double> ratio;
        std::vector<int32_t> cand_scene;
        std::vector<hipEvent_t> cand_ready;
        for (size_t i = 0; i < S->pending.size() && i < max_take; ++i) {
            const SReq& r = S->reqs[S->pending[i]];
            const SScene& sc = S->scenes[r.scene];
            wipes_image im{};
            im.cam = r.cam;
            im.prims = sc.prims;
            im.out_image = r.out;
            cand.push_back(im);
            ratio.push_back(sc.k_ratio);
            cand_scene.push_back(r.scene);
            cand_ready.push_back(r.ready);
        }
        const size_t take = admit_prefix(cand.size(), max_take, S->arena, [&](size_t k) {
            std::vector<wipes_image> pre(cand.begin(), cand.begin() + k);
            std::vector<double> rr(ratio.begin(), ratio.begin() + k);
            return batch_bytes(&S->params, pre, capacity_for(pre, rr), nullptr);
        });
        for (size_t i = take; i < S->pending.size(); ++i) {
            // requests that had to wait for slots or memory
            SReq& r = S->reqs[S->pending[i]];
            if (!r.deferred) {
                r.deferred = true;
                S->n_deferred++;
            }
        }
        if (take == 0) {
            if (S->inflight.empty()) {
                // the head request does not fit even an empty arena: it fails
                SReq& r = S->reqs[S->pending.front()];
                r.t_done = now_s();
                if (r.ready) S->ev_pool.push_back(r.ready);
                r.ready = nullptr;
                S->scenes[r.scene].refs--;
                S->pending.pop_front();
                S->err = "request exceeds the serving arena";
                S->cv.notify_all();
                continue;
            }
            // wait for the completion thread to free memory
            const size_t n_inflight = S->inflight.size();
            S->cv.wait(lk, [&] { return S->inflight.size() < n_inflight; });
            continue;
        }
        SBatch B;
        for (size_t i = 0; i < take; ++i) {
            B.ids.push_back(S->pending.front());
            S->reqs[S->pending.front()].admitted = true;
            S->pending.pop_front();
        }
        cand.resize(take);
        ratio.resize(take);
        cand_scene.resize(take);
        cand_ready.resize(take);
        const int64_t cap = capacity_for(cand, ratio);
        S->slots_used += (int)take;
        S->n_admitted += (int64_t)take;
        S->launching++;
        // the batch's events come from the pool while the lock is held
        B.prep = get_event(S);
        B.done = get_event(S);
        lk.unlock();
        int64_t K = 0;
        wipes_status st = launch_batch(S, cand, cand_ready, cap, B, &K);
        lk.lock();
        // a batch whose instances outgrew its estimate may not fit even an
        // empty arena: the second half goes back to the head of the queue (in
        // order) and the first half is launched again, down to one request
        while (st == WIPES_ERR_NOMEM && B.ids.size() > 1) {
            const size_t keep = B.ids.size() / 2;
            for (size_t i = B.ids.size(); i-- > keep;) {
                S->reqs[B.ids[i]].admitted = false;
                S->pending.push_front(B.ids[i]);
            }
            S->slots_used -= (int)(B.ids.size() - keep);
            S->n_admitted -= (int64_t)(B.ids.size() - keep);
            B.ids.resize(keep);
            cand.resize(keep);
            ratio.resize(keep);
            cand_scene.resize(keep);
            cand_ready.resize(keep);
            const int64_t cap2 = capacity_for(cand, ratio);
            lk.unlock();
            st = launch_batch(S, cand, cand_ready, cap2, B, &K);
            lk.lock();
        }
        S->launching--;
        if (st != WIPES_OK) {
            // the batch failed: its requests complete without an image; the error is kept
            S->ev_pool.push_back(B.prep);
            S->ev_pool.push_back(B.done);
            S->err = S->ctx->err;
            for (uint64_t id : B.ids) {
                SReq& r = S->reqs[id];
                r.t_done = now_s();
                if (r.ready) S->ev_pool.push_back(r.ready);
                r.ready = nullptr;
                S->scenes[r.scene].refs--;
                S->slots_used--;
            }
            S->cv.notify_all();
            continue;
        }
        // learn instances per primitive for the next footprint estimates
        int64_t nprim = 0;
        for (auto& im : cand) nprim += im.prims.n;
        if (nprim > 0) {
            const double r = (double)K / (double)nprim;
            for (int32_t sid : cand_scene) {
                auto it = S->scenes.find(sid);
                if (it != S->scenes.end()) it->second.k_ratio = std::max(r, 0.9 * it->second.k_ratio);
            }
        }
        S->n_batches++;
        S->n_batched += (int64_t)B.ids.size();
        S->inflight.push_back(std::move(B));
        S->cv.notify_all();
    }
    S->worker_done = true;
    S->cv.notify_all();
}

}  // namespace

extern "C" {

wipes_status wipes_serve_create(const wipes_serve_config* cfg, const wipes_params* p, int32_t device,
                                wipes_server** out)
{
    if (!cfg || !p || !out) return fail(nullptr, WIPES_ERR_INVALID, "config, params and out must be set");
    *out = nullptr;
    if (p->mode != WIPES_3D_ALPHA || cfg->max_slots < 1 || cfg->max_batch < 1 || cfg->max_pending < 1 ||
        cfg->hbm_budget_bytes < (1 << 20) || cfg->persistent < 0 || cfg->persistent > 3)
        return fail(nullptr, WIPES_ERR_INVALID,
                    "serving needs alpha mode, positive limits, >= 1 MiB budget and a launch form 0..3");
    wipes_server* S = new wipes_server();
    S->cfg = *cfg;
    S->params = *p;
    S->params.persistent = cfg->persistent;
    S->device = device;
    wipes_status st = wipes_ctx_create(device, &S->ctx);
    if (st != WIPES_OK) {
        delete S;
        return st;
    }
    hipError_t e = hipMalloc(&S->arena_mem, (size_t)cfg->hbm_budget_bytes);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->s_prep, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->s_blend, hipStreamNonBlocking);
    if (e != hipSuccess) {
        wipes_status r = hip_fail(nullptr, e, "serve create");
        if (S->arena_mem) hipFree(S->arena_mem);
        if (S->s_prep) hipStreamDestroy(S->s_prep);
        wipes_ctx_destroy(S->ctx);
        delete S;
        return r;
    }
    S->arena.reset((size_t)cfg->hbm_budget_bytes);
    S->worker = std::thread(worker_main, S);
    S->completer = std::thread(completer_main, S);
    *out = S;
    return WIPES_OK;
}

wipes_status wipes_serve_load_scene(wipes_server* S, const wipes_prims* prims, int32_t* scene_id)
{
    if (!S || !prims || !scene_id || prims->n <= 0 || !prims->mean || !prims->quat || !prims->scale ||
        !prims->freq || !prims->opacity)
        return fail(nullptr, WIPES_ERR_INVALID, "server, prims (3D, n > 0) and scene_id must be set");
    const int deg = S->params.sh_degree;
    const int K3 = deg >= 0 ? 3 * (deg + 1) * (deg + 1) : 0;
    if (deg < 0 ? !prims->color : !prims->sh)
        return fail(nullptr, WIPES_ERR_INVALID, "scene needs %s", deg < 0 ? "color" : "sh coefficients");
    const int64_t n = prims->n;
    const int per = 3 + 4 + 3 + 3 + (deg < 0 ? 3 : 0) + 1 + (prims->velocity ? 3 : 0) + (prims->phase ? 1 : 0) + K3;
    void* mem = nullptr;
    hipError_t e = hipMalloc(&mem, (size_t)n * per * 4);
    if (e != hipSuccess) return hip_fail(nullptr, e, "scene allocation");
    float* f = (float*)mem;
    SScene sc;
    auto put = [&](const float* src, int k, const float** dst) {
        if (!src) { *dst = nullptr; return hipSuccess; }
        hipError_t r = hipMemcpy(f, src, (size_t)n * k * 4, hipMemcpyDeviceToDevice);
        *dst = f;
        f += (size_t)n * k;
        return r;
    };
    sc.prims.n = n;
    e = put(prims->mean, 3, &sc.prims.mean);
    if (e == hipSuccess) e = put(prims->quat, 4, &sc.prims.quat);
    if (e == hipSuccess) e = put(prims->scale, 3, &sc.prims.scale);
    if (e == hipSuccess) e = put(prims->freq, 3, &sc.prims.freq);
    if (e == hipSuccess) e = put(deg < 0 ? prims->color : nullptr, 3, &sc.prims.color);
    if (e == hipSuccess) e = put(prims->opacity, 1, &sc.prims.opacity);
    if (e == hipSuccess) e = put(prims->velocity, 3, &sc.prims.velocity);
    if (e == hipSuccess) e = put(prims->phase, 1, &sc.prims.phase);
    if (e == hipSuccess) e = put(deg >= 0 ? prims->sh : nullptr, K3, &sc.prims.sh);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        return hip_fail(nullptr, e, "scene copy");
    }
    sc.mem = mem;
    std::lock_guard<std::mutex> lk(S->mu);
    *scene_id = S->next_scene++;
    S->scenes[*scene_id] = sc;
    return WIPES_OK;
}

wipes_status wipes_serve_unload_scene(wipes_server* S, int32_t scene_id)
{
    if (!S) return fail(nullptr, WIPES_ERR_INVALID, "server must be set");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->scenes.find(scene_id);
    if (it == S->scenes.end()) return fail(nullptr, WIPES_ERR_NOTFOUND, "unknown scene %d", scene_id);
    if (it->second.refs > 0) return fail(nullptr, WIPES_ERR_BUSY, "scene %d has requests in flight", scene_id);
    (void)hipFree(it->second.mem);
    S->scenes.erase(it);
    return WIPES_OK;
}

wipes_status wipes_serve_submit(wipes_server* S, int32_t scene_id, const wipes_camera* cam, float* out_image,
                                size_t out_floats, void* stream, uint64_t* req_id)
{
    if (!S || !cam || !out_image || !req_id) return fail(nullptr, WIPES_ERR_INVALID, "arguments must be set");
    if (cam->width < 1 || cam->height < 1 || cam->width > 32768 || cam->height > 32768 || !(cam->fx > 0.0f) ||
        !(cam->fy > 0.0f))
        return fail(nullptr, WIPES_ERR_INVALID, "bad camera");
    const size_t need = (size_t)cam->width * (size_t)cam->height * 3;
    if (out_floats < need)
        return fail(nullptr, WIPES_ERR_NOMEM, "output buffer holds %zu floats, the %dx%d image needs %zu", out_floats,
                    cam->width, cam->height, need);
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->scenes.find(scene_id);
    if (it == S->scenes.end()) return fail(nullptr, WIPES_ERR_NOTFOUND, "unknown scene %d", scene_id);
    if ((int)S->pending.size() >= S->cfg.max_pending) return fail(nullptr, WIPES_ERR_BUSY, "queue full");
    // the server writes `out` only after the work the caller's stream holds now
    hipEvent_t ready = get_event(S);
    if (!ready) return fail(nullptr, WIPES_ERR_DEVICE, "event creation failed");
    const hipError_t e = hipEventRecord(ready, (hipStream_t)stream);
    if (e != hipSuccess) {
        S->ev_pool.push_back(ready);
        return fail(nullptr, WIPES_ERR_DEVICE, "recording the caller's stream: %s", hipGetErrorString(e));
    }
    const uint64_t id = S->next_id++;
    SReq r;
    r.scene = scene_id;
    r.cam = *cam;
    r.out = out_image;
    r.ready = ready;
    r.t_submit = now_s();
    if (S->t_first < 0.0) S->t_first = r.t_submit;
    S->reqs[id] = r;
    it->second.refs++;
    S->pending.push_back(id);
    *req_id = id;
    S->cv.notify_all();
    return WIPES_OK;
}

wipes_status wipes_serve_poll(wipes_server* S, uint64_t req_id, int32_t* done, double* latency_ms)
{
    if (!S || !done) return fail(nullptr, WIPES_ERR_INVALID, "server and done must be set");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(req_id);
    if (it == S->reqs.end()) return fail(nullptr, WIPES_ERR_NOTFOUND, "unknown request");
    *done = it->second.t_done >= 0.0;
    if (latency_ms) *latency_ms = *done ? (it->second.t_done - it->second.t_submit) * 1e3 : -1.0;
    if (*done) S->reqs.erase(it);
    return WIPES_OK;
}

wipes_status wipes_serve_drain(wipes_server* S)
{
    if (!S) return fail(nullptr, WIPES_ERR_INVALID, "server must be set");
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv.wait(lk, [&] { return S->pending.empty() && S->launching == 0 && S->inflight.empty(); });
    if (!S->err.empty()) return fail(nullptr, WIPES_ERR_DEVICE, "%s", S->err.c_str());
    return WIPES_OK;
}

wipes_status wipes_serve_stats(wipes_server* S, wipes_serve_report* st)
{
    if (!S || !st) return fail(nullptr, WIPES_ERR_INVALID, "server and stats must be set");
    std::lock_guard<std::mutex> lk(S->mu);
    std::vector<double> v = S->lat_ms;
    std::sort(v.begin(), v.end());
    auto pct = [&](double q) {
        if (v.empty()) return 0.0;
        const size_t i = (size_t)std::min((double)v.size() - 1, std::ceil(q * v.size()) - 1);
        return v[i];
    };
    st->p50_ms = pct(0.50);
    st->p99_ms = pct(0.99);
    double m = 0.0;
    for (double x : v) m += x;
    st->mean_ms = v.empty() ? 0.0 : m / v.size();
    st->completed = (int64_t)v.size();
    st->frames_per_s = (v.size() > 1 && S->t_last > S->t_first) ? v.size() / (S->t_last - S->t_first) : 0.0;
    st->admitted = S->n_admitted;
    st->deferred = S->n_deferred;
    st->batches = S->n_batches;
    st->mean_batch = S->n_batches ? (double)S->n_batched / S->n_batches : 0.0;
    st->arena_peak_bytes = (int64_t)S->arena_peak;
    return WIPES_OK;
}

wipes_status wipes_serve_reset_stats(wipes_server* S)
{
    if (!S) return fail(nullptr, WIPES_ERR_INVALID, "server must be set");
    std::lock_guard<std::mutex> lk(S->mu);
    S->lat_ms.clear();
    S->t_first = S->t_last = -1.0;
    S->n_admitted = S->n_deferred = S->n_batches = S->n_batched = 0;
    S->arena_peak = S->arena.used();
    return WIPES_OK;
}

void wipes_serve_destroy(wipes_server* S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    if (S->completer.joinable()) S->completer.join();
    (void)hipSetDevice(S->device);
    for (auto& kv : S->scenes) hipFree(kv.second.mem);
    for (hipEvent_t e : S->ev_pool) hipEventDestroy(e);
    if (S->arena_mem) hipFree(S->arena_mem);
    if (S->s_prep) hipStreamDestroy(S->s_prep);
    if (S->s_blend) hipStreamDestroy(S->s_blend);
    wipes_ctx_destroy(S->ctx);
    delete S;
}

// Discrete-event model of the worker with a fake executor: request i arrives
// at t_arrive[i], needs footprint[i] bytes while admitted, its batch's prep
// takes the sum of prep_s over the batch on the prep stream and its blend the
// sum of blend_s on the blend stream (which runs batches one after another,
// overlapping the next batch's prep).  Writes admission and completion times.
// Same admission rule and arena as the real server.
wipes_status wipes_serve_simulate(const wipes_serve_config* cfg, int64_t n, const double* t_arrive,
                                  const int64_t* footprint, const double* prep_s, const double* blend_s,
                                  double* t_admit, double* t_done, int64_t* batch_of, int64_t* arena_peak)
{
    if (!cfg || n < 0 || (n > 0 && (!t_arrive || !footprint || !prep_s || !blend_s || !t_admit || !t_done)))
        return fail(nullptr, WIPES_ERR_INVALID, "bad simulation arguments");
    for (int64_t i = 1; i < n; ++i)
        if (t_arrive[i] < t_arrive[i - 1]) return fail(nullptr, WIPES_ERR_INVALID, "arrivals must be sorted");
    for (int64_t i = 0; i < n; ++i)
        if (footprint[i] < 0 || (size_t)al((size_t)footprint[i]) > (size_t)cfg->hbm_budget_bytes)
            return fail(nullptr, WIPES_ERR_INVALID, "request %lld never fits the budget", (long long)i);
    Arena arena;
    arena.reset((size_t)cfg->hbm_budget_bytes);
    struct Fl { double t_done; size_t off, bytes; std::vector<int64_t> ids; };
    std::vector<Fl> flight;
    std::deque<int64_t> pend;
    int64_t next = 0, done_cnt = 0, batch_no = 0;
    int slots = 0;
    double t = 0.0, prep_free = 0.0, blend_free = 0.0;
    size_t peak = 0;
    while (done_cnt < n) {
        // arrivals up to now
        while (next < n && t_arrive[next] <= t) pend.push_back(next++);
        // retire
        for (size_t k = 0; k < flight.size();) {
            if (flight[k].t_done <= t) {
                for (int64_t id : flight[k].ids) {
                    t_done[id] = flight[k].t_done;
                    --slots;
                    ++done_cnt;
                }
                arena.release(flight[k].off, flight[k].bytes);
                flight.erase(flight.begin() + k);
            } else {
                ++k;
            }
        }
        // admit (the worker is busy until its previous prep has finished)
        if (t >= prep_free && !pend.empty()) {
            const size_t max_take = std::min((size_t)std::max(0, cfg->max_slots - slots), (size_t)cfg->max_batch);
            const size_t take = admit_prefix(pend.size(), max_take, arena, [&](size_t k) {
                size_t b = 0;
                for (size_t i = 0; i < k; ++i) b += al((size_t)footprint[pend[i]]);
                return b;
            });
            if (take > 0) {
                Fl f;
                size_t bytes = 0;
                double prep = 0.0, blend = 0.0;
                for (size_t i = 0; i < take; ++i) {
                    const int64_t id = pend.front();
                    pend.pop_front();
                    f.ids.push_back(id);
                    t_admit[id] = t;
                    if (batch_of) batch_of[id] = batch_no;
                    bytes += al((size_t)footprint[id]);
                    prep += prep_s[id];
                    blend += blend_s[id];
                }
                arena.alloc(bytes, &f.off);
                f.bytes = bytes;
                peak = std::max(peak, arena.used());
                slots += (int)take;
                prep_free = t + prep;
                blend_free = std::max(blend_free, prep_free) + blend;
                f.t_done = blend_free;
                flight.push_back(f);
                ++batch_no;
                continue;   // try to admit more at the same instant only after prep
            }
        }
        // advance to the next event
        double tn = 1e300;
        if (next < n) tn = std::min(tn, t_arrive[next]);
        for (auto& f : flight) tn = std::min(tn, f.t_done);
        if (prep_free > t) tn = std::min(tn, prep_free);
        if (tn == 1e300) break;
        t = std::max(t, tn);
    }
    if (arena_peak) *arena_peak = (int64_t)peak;
    return done_cnt == n ? WIPES_OK : fail(nullptr, WIPES_ERR_BUSY, "simulation did not complete");
}

}  // extern "C"
