// Request loop of the renderer: resident scenes, a host queue of view
// requests, and worker threads that turn the queued requests of one scene into
// one batched forward pass on their own stream (continuous batching).  The
// device buffers of the passes are frames owned by the server and shared by
// its workers: a batch takes an idle frame of its scene (grown when the batch
// exceeds it), so the steady state allocates nothing, and every frame, idle
// or in use, counts against the HBM budget.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "runtime.hpp"

namespace cs {

namespace {

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    int32_t scene = 0;
    cs_camera cam{};
    float *out = nullptr;
    double t_submit = 0.0, t_start = 0.0, t_done = 0.0;
    int status = 0;
    bool done = false;
};

// Device memory of a batched forward pass (to admit a batch whose frame must
// be created or grown): per (view, convex) instance the record and 60 bytes of
// keys, ids, counts, offsets, binning records and hull, a quarter more for the
// capacity rounding of frames; an allowance of 16 (tile, instance) pairs x 16
// bytes (two ping-pong pairs of 4-byte arrays); 8 bytes of per-pixel state;
// and a fixed 2 MiB (view table, counters, work-counter slots).
size_t estimate_bytes(const cs_scene &s, int64_t views, int64_t pixels)
{
    const int64_t inst = (int64_t)s.n * views;
    return (size_t)((double)(inst * (rec_stride(s.k) + 60)) * 1.25) + (size_t)(inst * 16 * 16 + pixels * 8 + (2 << 20));
}

} // namespace

constexpr int MAX_IDLE_PER_SCENE = 8;

struct Server {
    cs_ctx *owner = nullptr;
    cs_serve_config cfg{};
    size_t budget = 0; // 0 = unlimited
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Request> reqs;
    std::map<int32_t, cs_scene> scenes;
    int32_t next_scene = 1;
    uint64_t next_id = 1;
    bool stop = false, paused = false;
    // frames: idle ones by scene (and last use), the bytes of all of them
    struct Idle {
        Frame *F;
        int32_t scene;
        uint64_t tick;
    };
    std::vector<Idle> idle;
    size_t held = 0, peak = 0;
    uint64_t tick = 0;
    int64_t submitted = 0, completed = 0, failed = 0, batches = 0, batch_reqs = 0, running = 0, frames_created = 0;
    double sum_queue_ms = 0.0, sum_run_ms = 0.0;
    std::vector<std::thread> workers;

    // Under the lock: the requests of the oldest request's scene, in arrival
    // order, up to max_batch, with an idle frame of that scene (or none), when
    // the device memory the batch may add fits the budget after idle frames of
    // other scenes are dropped (into `drop`, to be freed outside the lock).
    // A batch always runs when nothing else does.
    bool take(std::vector<uint64_t> &ids, Frame *&frame, std::vector<Frame *> &drop)
    {
        ids.clear();
        frame = nullptr;
        if (queue.empty() || paused) return false;
        const Request &first = reqs[queue.front()];
        auto sit = scenes.find(first.scene);
        if (sit == scenes.end()) { // scene gone: fail it
            Request &r = reqs[queue.front()];
            r.status = CS_EINVAL;
            r.done = true;
            r.t_done = now_ms();
            ++failed;
            queue.pop_front();
            cv_done.notify_all();
            return false;
        }
        const cs_scene &sc = sit->second;
        const int tile = cfg.params.tile > 0 ? cfg.params.tile : 16;
        int64_t pix = 0, tiles = 0;
        std::vector<uint64_t> pick;
        for (uint64_t id : queue) {
            if ((int)pick.size() >= cfg.max_batch) break;
            const Request &r = reqs[id];
            if (r.scene != first.scene) continue;
            pick.push_back(id);
            pix += (int64_t)r.cam.width * r.cam.height;
            tiles += (int64_t)((r.cam.width + tile - 1) / tile) * ((r.cam.height + tile - 1) / tile);
        }
        // the smallest idle frame of this scene that fits the batch and is at
        // most 4x its size (a much larger one would run its capacity-sized sort
        // grids for nothing); none: a new frame of the batch's size
        const size_t inst = (size_t)sc.n * pick.size();
        int best = -1;
        for (size_t i = 0; i < idle.size(); ++i) {
            const Frame *f = idle[i].F;
            if (idle[i].scene != first.scene || f->cap_inst < inst || f->cap_inst > 4 * inst + 4096 ||
                f->cap_tiles < (size_t)tiles || f->cap_pix < (size_t)pix)
                continue;
            if (best < 0 || f->cap_inst < idle[best].F->cap_inst) best = (int)i;
        }
        const size_t have = best >= 0 ? idle[best].F->bytes_held : 0;
        const size_t need = estimate_bytes(sc, (int64_t)pick.size(), pix);
        const size_t grow = need > have ? need - have : 0;
        if (budget) {
            // drop idle frames of other scenes, least recently used first, while short
            while (held + grow > budget) {
                int lru = -1;
                for (size_t i = 0; i < idle.size(); ++i)
                    if ((int)i != best && (lru < 0 || idle[i].tick < idle[lru].tick)) lru = (int)i;
                if (lru < 0) {
                    if (running > 0) return false; // wait for running batches
                    break;                         // alone: run anyway
                }
                held -= idle[lru].F->bytes_held;
                drop.push_back(idle[lru].F);
                idle.erase(idle.begin() + lru);
                if (best > lru) --best;
            }
        }
        if (best >= 0) {
            frame = idle[best].F;
            idle.erase(idle.begin() + best);
        }
        for (uint64_t id : pick) {
            for (auto it = queue.begin(); it != queue.end(); ++it)
                if (*it == id) {
                    queue.erase(it);
                    break;
                }
        }
        ids = pick;
        return true;
    }

    void worker(int device)
    {
        (void)hipSetDevice(device);
        cs_ctx *ctx = nullptr;
        hipStream_t st = nullptr;
        hipEvent_t done_ev = nullptr;
        int init = cs_create(device, 0, &ctx);
        if (init == CS_OK && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) init = CS_EHIP;
        if (init == CS_OK && hipEventCreateWithFlags(&done_ev, hipEventDisableTiming) != hipSuccess) init = CS_EHIP;
        cs_params prm = cfg.params;
        prm.flags &= ~(CS_FLAG_GRAPH | CS_FLAG_AUTOTUNE | CS_FLAG_TIMING);
        std::vector<uint64_t> ids;
        std::vector<cs_camera> cams;
        std::vector<float *> outs;
        std::vector<Frame *> drop;
        for (;;) {
            Frame *F = nullptr;
            cs_scene sc{};
            int32_t scene_id = 0;
            drop.clear();
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return stop || (!paused && !queue.empty()); });
                if (stop) break;
                if (!take(ids, F, drop)) {
                    lk.unlock();
                    release_idle(drop);
                    lk.lock();
                    // waiting for memory held by running batches: woken when one ends
                    cv_work.wait_for(lk, std::chrono::milliseconds(5));
                    continue;
                }
                scene_id = reqs[ids[0]].scene;
                sc = scenes[scene_id];
                cams.clear();
                outs.clear();
                const double t = now_ms();
                for (uint64_t id : ids) {
                    Request &r = reqs[id];
                    r.t_start = t;
                    cams.push_back(r.cam);
                    outs.push_back(r.out);
                }
                running += (int64_t)ids.size();
            }
            release_idle(drop);
            const size_t before = F ? F->bytes_held : 0;
            bool created = false;
            int rc = init;
            if (rc == CS_OK)
                rc = forward_batch_on(ctx, &F, &sc, (int32_t)ids.size(), cams.data(), &prm, outs.data(), st, &created);
            // completion by polling an event: a blocking wait wakes up late
            if (rc == CS_OK && hipEventRecord(done_ev, st) != hipSuccess) rc = CS_EHIP;
            if (rc == CS_OK) {
                hipError_t e;
                while ((e = hipEventQuery(done_ev)) == hipErrorNotReady) std::this_thread::yield();
                if (e != hipSuccess) rc = CS_EHIP;
            } else if (st) {
                (void)hipStreamSynchronize(st);
            }
            const double t = now_ms();
            {
                std::lock_guard<std::mutex> lk(mu);
                held -= before;
                if (F) {
                    if (rc == CS_OK) {
                        held += F->bytes_held;
                        idle.push_back({F, scene_id, ++tick});
                        // at most MAX_IDLE_PER_SCENE idle frames of a scene (sizes of
                        // the batches it meets): the least recently used goes
                        int count = 0, lru = -1;
                        for (size_t i = 0; i < idle.size(); ++i)
                            if (idle[i].scene == scene_id) {
                                ++count;
                                if (lru < 0 || idle[i].tick < idle[lru].tick) lru = (int)i;
                            }
                        if (count > MAX_IDLE_PER_SCENE) {
                            held -= idle[lru].F->bytes_held;
                            drop.push_back(idle[lru].F);
                            idle.erase(idle.begin() + lru);
                        }
                    } else {
                        F->st = nullptr;
                        delete F;
                    }
                }
                peak = std::max(peak, held);
                frames_created += created ? 1 : 0;
                for (uint64_t id : ids) {
                    Request &r = reqs[id];
                    r.status = rc;
                    r.t_done = t;
                    r.done = true;
                    sum_queue_ms += r.t_start - r.t_submit;
                    sum_run_ms += t - r.t_start;
                }
                running -= (int64_t)ids.size();
                ++batches;
                batch_reqs += (int64_t)ids.size();
                (rc == CS_OK ? completed : failed) += (int64_t)ids.size();
            }
            cv_done.notify_all();
            cv_work.notify_all();
            release_idle(drop);
        }
        if (done_ev) (void)hipEventDestroy(done_ev);
        if (ctx) cs_destroy(ctx);
        if (st) (void)hipStreamDestroy(st);
    }

    // Idle frames leave: their buffers go back on the null stream (their last
    // stream may belong to another worker).
    static void release_idle(std::vector<Frame *> &frames)
    {
        for (Frame *d : frames) {
            d->st = nullptr;
            delete d;
        }
        frames.clear();
    }

    // After the workers have joined: free the idle frames.
    void free_frames()
    {
        (void)hipDeviceSynchronize();
        std::vector<Frame *> all;
        for (Idle &i : idle) all.push_back(i.F);
        idle.clear();
        release_idle(all);
        held = 0;
    }
};

} // namespace cs

using namespace cs;

extern "C" {

int cs_serve_start(cs_ctx *ctx, const cs_serve_config *cfg)
{
    if (!ctx || !cfg) return fail(CS_EINVAL, "ctx or config is NULL");
    if (ctx->server) return fail(CS_EINVAL, "server already running on this context");
    if (cfg->workers < 1 || cfg->workers > 16) return fail(CS_EINVAL, "workers = %d outside [1, 16]", cfg->workers);
    if (cfg->max_batch < 1 || cfg->max_batch > MAX_VIEWS)
        return fail(CS_EINVAL, "max_batch = %d outside [1, %d]", cfg->max_batch, MAX_VIEWS);
    if (cfg->max_queue < 1) return fail(CS_EINVAL, "max_queue must be >= 1");
    Server *S = new Server;
    S->owner = ctx;
    S->cfg = *cfg;
    S->budget = cfg->hbm_budget_bytes ? cfg->hbm_budget_bytes : ctx->budget;
    S->paused = cfg->start_paused != 0;
    ctx->server = S;
    for (int w = 0; w < cfg->workers; ++w) S->workers.emplace_back([S, dev = ctx->device] { S->worker(dev); });
    return CS_OK;
}

int cs_serve_resume(cs_ctx *ctx)
{
    if (!ctx || !ctx->server) return fail(CS_EINVAL, "no server on this context");
    Server *S = ctx->server;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->paused = false;
    }
    S->cv_work.notify_all();
    return CS_OK;
}

int cs_serve_stop(cs_ctx *ctx)
{
    if (!ctx || !ctx->server) return CS_OK;
    Server *S = ctx->server;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto &t : S->workers) t.join();
    S->free_frames();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        for (uint64_t id : S->queue) {
            Request &r = S->reqs[id];
            r.status = CS_EBUSY;
            r.done = true;
            ++S->failed;
        }
        S->queue.clear();
    }
    S->cv_done.notify_all();
    ctx->server = nullptr;
    delete S;
    return CS_OK;
}

int cs_scene_register(cs_ctx *ctx, const cs_scene *scene, int32_t *scene_id)
{
    if (!ctx || !ctx->server || !scene_id) return fail(CS_EINVAL, "no server or NULL argument");
    if (!scene) return fail(CS_EINVAL, "scene is NULL");
    if (scene->k < 3 || scene->k > CS_MAX_K || scene->sh_degree < 0 || scene->sh_degree > 3 || scene->n < 0)
        return fail(CS_EINVAL, "bad scene shape");
    Server *S = ctx->server;
    std::lock_guard<std::mutex> lk(S->mu);
    *scene_id = S->next_scene++;
    S->scenes[*scene_id] = *scene;
    return CS_OK;
}

int cs_scene_unregister(cs_ctx *ctx, int32_t scene_id)
{
    if (!ctx || !ctx->server) return fail(CS_EINVAL, "no server on this context");
    Server *S = ctx->server;
    std::lock_guard<std::mutex> lk(S->mu);
    if (!S->scenes.erase(scene_id)) return fail(CS_EINVAL, "unknown scene %d", scene_id);
    return CS_OK;
}

int cs_serve_submit(cs_ctx *ctx, int32_t scene_id, const cs_camera *cam, float *out_rgb, uint64_t *request_id)
{
    if (!ctx || !ctx->server || !cam || !out_rgb || !request_id) return fail(CS_EINVAL, "NULL argument");
    if (cam->width <= 0 || cam->height <= 0 || cam->width > 16384 || cam->height > 16384 || !(cam->fx > 0.0f) ||
        !(cam->fy > 0.0f) || !(cam->znear > 0.0f))
        return fail(CS_EINVAL, "bad camera");
    Server *S = ctx->server;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->scenes.find(scene_id);
        if (it == S->scenes.end()) return fail(CS_EINVAL, "unknown scene %d", scene_id);
        if ((int)S->queue.size() >= S->cfg.max_queue) return fail(CS_EBUSY, "serving queue full");
        const size_t b = estimate_bytes(it->second, 1, (int64_t)cam->width * cam->height);
        if (S->budget && b > S->budget)
            return fail(CS_ENOMEM, "request needs ~%zu bytes, budget %zu", b, S->budget);
        const uint64_t id = S->next_id++;
        Request &r = S->reqs[id];
        r.scene = scene_id;
        r.cam = *cam;
        r.out = out_rgb;
        r.t_submit = now_ms();
        S->queue.push_back(id);
        ++S->submitted;
        *request_id = id;
    }
    S->cv_work.notify_one();
    return CS_OK;
}

int cs_serve_wait(cs_ctx *ctx, uint64_t request_id, double *latency_ms)
{
    if (!ctx || !ctx->server) return fail(CS_EINVAL, "no server on this context");
    Server *S = ctx->server;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(request_id);
    if (it == S->reqs.end()) return fail(CS_EINVAL, "unknown request %llu", (unsigned long long)request_id);
    S->cv_done.wait(lk, [&] { return S->reqs[request_id].done; });
    Request r = S->reqs[request_id];
    S->reqs.erase(request_id);
    if (latency_ms) *latency_ms = r.t_done - r.t_submit;
    if (r.status != CS_OK) return fail(r.status, "request %llu failed (%d)", (unsigned long long)request_id, r.status);
    return CS_OK;
}

int cs_serve_get_stats(cs_ctx *ctx, cs_serve_stats *out)
{
    if (!ctx || !ctx->server || !out) return fail(CS_EINVAL, "no server or NULL argument");
    Server *S = ctx->server;
    std::lock_guard<std::mutex> lk(S->mu);
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->failed = S->failed;
    out->batches = S->batches;
    out->mean_batch = S->batches ? (double)S->batch_reqs / S->batches : 0.0;
    out->peak_bytes = S->peak;
    out->queued = (int64_t)S->queue.size();
    out->running = S->running;
    out->frames_created = S->frames_created;
    out->frame_bytes = S->held;
    const int64_t fin = S->completed + S->failed;
    out->mean_queue_ms = fin ? S->sum_queue_ms / (double)fin : 0.0;
    out->mean_run_ms = fin ? S->sum_run_ms / (double)fin : 0.0;
    return CS_OK;
}

} // extern "C"
