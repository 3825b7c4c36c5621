// Serving form: continuous batching of scene frames from many streams.
//
// mhc_submit copies a frame into a FIFO. A scheduler thread keeps up to
// `max_inflight_ticks` ticks on the GPU, each on its own stream with its own
// device workspace (an equal share of the HBM budget) and pinned staging.
// Whenever a tick slot is free it admits queued frames in arrival order while
// they fit the slot's memory and the tick's frame / check caps, plans the
// tick on the host (while earlier ticks still run), uploads one scene image,
// launches trajectory generation, collision recognition and risk for all its
// frames, and queues the copy of their results back to pinned memory. When a
// tick's event completes, every frame's results are copied to the caller's
// buffers and its waiters are released. A frame's results do not depend on
// which tick carried it or what else was in it.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime.h"

using namespace mhc;

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Bound on the resident collision waves of any GPU this library runs on
// (sizes the slot table in the admission estimate).
constexpr int kMaxCollisionWaves = 1 << 16;

enum FrameState { QUEUED, ADMITTED, DONE };

struct Frame {
    uint64_t ticket = 0;
    int32_t stream_id = 0;
    // owned copy of the scene
    std::vector<mhc_object> objs;
    std::vector<std::vector<double>> arrays;
    mhc_scene scene{};
    mhc_result dst{};
    int64_t n_traj = 0, n_hits = 0, checks = 0;
    size_t bytes = 0;  // device bytes upper bound
    FrameState state = QUEUED;
    mhc_status status = MHC_OK;
    mhc_timing timing{};
};

struct TickSlot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    char *dbuf = nullptr;
    size_t dbytes = 0;
    char *pin_in = nullptr;
    size_t pin_in_bytes = 0;
    char *pin_out = nullptr;
    size_t pin_out_bytes = 0;
    bool busy = false;
    int64_t launched_ns = 0;
    int64_t tick = 0;
    Layout L;
    std::vector<std::shared_ptr<Frame>> frames;
    std::vector<mhc_result> dsts;  // per frame: its host buffers
    ResultPlan results;            // the tick's outputs staged in pin_out
};

}  // namespace

struct mhc_server {
    mhc_ctx *ctx = nullptr;
    mhc_server_cfg cfg{};
    size_t slot_bytes = 0;
    size_t slot_usable = 0;  // slot bytes minus the per-tick collision slot table
    std::vector<TickSlot> slots;
    std::thread thread;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Frame>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Frame>> frames;
    uint64_t next_ticket = 1;
    bool stopping = false;
    std::string fatal;
    // statistics
    int64_t submitted = 0, completed = 0, rejected = 0, deferred = 0, ticks = 0, checks = 0;
    std::vector<double> latency_ms;
    int64_t start_ns = 0;
};

namespace {

// Upper bound of the device bytes a frame adds to a tick (every buffer of the
// workspace layout, with one collision segment per work unit).
void frame_sizes(const mhc_scene *s, int max_waves, bool hits, Frame &f)
{
    int64_t n_traj = 0, pose = 0, n_units = 0, n_hits = 0, vals = 0, n_pairs = 0;
    const int n = s->n_objects;
    for (int a = 0; a < n; ++a) {
        const int64_t T = (int64_t)s->objects[a].n_u * s->objects[a].n_w;
        n_traj += T;
        pose += align256((size_t)s->horizon * T * (s->objects[a].kind == MHC_VEHICLE ? 16 : 8));
        vals += s->objects[a].n_u + s->objects[a].n_w + (s->objects[a].score ? T : 0);
    }
    for (int a = 0; a < n; ++a)
        for (int b = a + 1; b < n; ++b) {
            if (s->pairs == MHC_PAIRS_EGO && a != 0) continue;
            const int64_t Ta = (int64_t)s->objects[a].n_u * s->objects[a].n_w;
            const int64_t Tb = (int64_t)s->objects[b].n_u * s->objects[b].n_w;
            n_hits += Ta * Tb;
            // one collision segment per work unit, for the variant and the
            // time split (up to 4 parts, 16 items a unit) that cut this pair
            // into the most units
            const bool poly = scene_has_outline(s);
            const int cls = pair_class(s->objects[a].kind, s->objects[b].kind, s->overlap,
                                       poly && s->objects[a].n_vertices > 0, poly && s->objects[b].n_vertices > 0);
            int64_t most = 0;
            for (int v = 0; v < N_VARIANTS; ++v) {
                const int64_t items = (Ta + kTiles[v][cls].ri - 1) / kTiles[v][cls].ri *
                                      ((Tb + kTiles[v][cls].rj - 1) / kTiles[v][cls].rj);
                const int64_t per = WAVE >> MAX_TSHIFT;
                most = std::max(most, (items + per - 1) / per);
            }
            n_units += most;
            ++n_pairs;
        }
    const int64_t n_q = n_traj * n;
    size_t bytes = 0;
    bytes += align256(n * sizeof(DObj)) + align256(vals * 8) + align256(n_pairs * sizeof(DPair));
    bytes += align256((scene_has_outline(s) ? n : 0) * sizeof(DPoly));
    bytes += align256((n_units + 1) * sizeof(WorkItem));
    bytes += pose + align256(n_traj * 8) * 3 + align256(n_q * 8) * 2;  // p*2^62, p, traj crit; q sums, q
    bytes += align256((n_traj / WG + n) * 8) + align256(n * 4);         // risk partials and counters
    bytes += align256(hits ? n_hits * 2 : 0) + align256(n * 8);
    if (s->timeline) {
        // per-slot sums (W >= n lanes per trajectory), attribution scratch
        // and output, the criticality over time (scratch and output), crit_t
        // and attrib
        int64_t W = 1;
        while (W < n) W <<= 1;
        bytes += align256((size_t)n_traj * W * s->horizon * 8) + align256(n_q * 8) * 2;
        bytes += align256((size_t)n_traj * s->horizon * 8) * 2 + align256((size_t)n * s->horizon * 8) +
                 align256((size_t)n * n * 8);
    }
    bytes += 16 * 256;                              // alignment slack of the tables
    bytes += align256(((size_t)max_waves + 1) * 4);  // the collision plan's slot table
    f.n_traj = n_traj;
    f.n_hits = n_hits;
    f.checks = n_hits * s->horizon;
    f.bytes = bytes;
}

std::shared_ptr<Frame> copy_frame(const mhc_scene *s)
{
    auto f = std::make_shared<Frame>();
    f->objs.assign(s->objects, s->objects + s->n_objects);
    for (auto &o : f->objs) {
        f->arrays.emplace_back(o.u, o.u + o.n_u);
        o.u = f->arrays.back().data();
        f->arrays.emplace_back(o.w, o.w + o.n_w);
        o.w = f->arrays.back().data();
        if (o.score) {
            f->arrays.emplace_back(o.score, o.score + (size_t)o.n_u * o.n_w);
            o.score = f->arrays.back().data();
        }
        if (o.n_vertices > 0) {
            f->arrays.emplace_back(o.vertices, o.vertices + 2 * (size_t)o.n_vertices);
            o.vertices = f->arrays.back().data();
        }
    }
    f->scene = *s;
    f->scene.objects = f->objs.data();
    return f;
}

hipError_t grow_pinned(char **p, size_t *have, size_t want)
{
    if (*have >= want) return hipSuccess;
    if (*p) hipHostFree(*p);
    *p = nullptr;
    *have = 0;
    const size_t sz = std::max(want + want / 4, (size_t)1 << 20);
    hipError_t e = hipHostMalloc(reinterpret_cast<void **>(p), sz, hipHostMallocDefault);
    if (e == hipSuccess) *have = sz;
    return e;
}

// Launch one tick (scheduler thread, lock not held).
hipError_t launch_tick(mhc_server *srv, TickSlot &t)
{
    std::vector<mhc_scene> scenes;
    scenes.reserve(t.frames.size());
    for (auto &f : t.frames) scenes.push_back(f->scene);
    mhc_ctx *ctx = srv->ctx;
    const int v = ctx->variant_for(scenes.data(), (int)scenes.size());
    bool keep_hits = false;
    for (auto &f : t.frames) keep_hits |= f->dst.first_hit != nullptr;
    build_layout(scenes.data(), (int)scenes.size(), v, ctx->max_waves(v, scenes.data(), (int)scenes.size()), t.L,
                 keep_hits);
    if (t.L.total_bytes > t.dbytes) return hipErrorOutOfMemory;  // admission bounds exclude this
    hipError_t e = grow_pinned(&t.pin_in, &t.pin_in_bytes, t.L.image_bytes);
    if (e != hipSuccess) return e;
    t.dsts.clear();
    for (auto &f : t.frames) t.dsts.push_back(f->dst);
    // every output of the tick in one transfer per output region, staged in
    // pinned memory so that nothing blocks this thread
    t.results = plan_results(t.L, (int)t.frames.size(), t.dsts.data(), true);
    e = grow_pinned(&t.pin_out, &t.pin_out_bytes, t.results.staged);
    if (e != hipSuccess) return e;
    pack_image(t.L, t.pin_in);
    e = hipMemcpyAsync(t.dbuf, t.pin_in, t.L.image_bytes, hipMemcpyHostToDevice, t.stream);
    if (e != hipSuccess) return e;
    Launch X = make_launch(t.L, t.dbuf, nullptr, keep_hits, ctx->n_cu);
    e = launch_all(X, t.stream);
    if (e != hipSuccess) return e;
    e = enqueue_results(t.results, t.L, (int)t.frames.size(), t.dbuf, t.pin_out, t.dsts.data(), t.stream);
    if (e != hipSuccess) return e;
    return hipEventRecord(t.done, t.stream);
}

void finish_tick(mhc_server *srv, TickSlot &t, mhc_status st)
{
    if (st == MHC_OK) scatter_results(t.results, t.L, (int)t.frames.size(), t.pin_out, t.dsts.data());
    const int64_t done = now_ns();  // every result is in its host buffer
    for (auto &fp : t.frames) {
        fp->timing.launch_ns = t.launched_ns;
        fp->timing.done_ns = done;
        fp->timing.tick = t.tick;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    for (auto &fp : t.frames) {
        fp->status = st;
        fp->state = DONE;
        ++srv->completed;
        if (st == MHC_OK) srv->checks += fp->checks;
        srv->latency_ms.push_back((fp->timing.done_ns - fp->timing.submit_ns) * 1e-6);
    }
    t.frames.clear();
    t.busy = false;
    srv->cv_done.notify_all();
}

void scheduler(mhc_server *srv)
{
    hipSetDevice(srv->ctx->device);
    const int64_t watchdog_ns = 30LL * 1000 * 1000 * 1000;
    while (true) {
        // 1. retire finished ticks
        bool any_busy = false;
        for (auto &t : srv->slots) {
            if (!t.busy) continue;
            const hipError_t q = hipEventQuery(t.done);
            if (q == hipSuccess) {
                finish_tick(srv, t, MHC_OK);
            } else if (q != hipErrorNotReady || now_ns() - t.launched_ns > watchdog_ns) {
                {
                    std::lock_guard<std::mutex> lk(srv->mu);
                    srv->fatal = q != hipErrorNotReady ? std::string("tick failed: ") + hipGetErrorString(q)
                                                       : std::string("tick exceeded the watchdog");
                }
                finish_tick(srv, t, MHC_E_DEVICE);
            } else {
                any_busy = true;
            }
        }
        // 2. admit frames into a free slot
        TickSlot *free_slot = nullptr;
        for (auto &t : srv->slots)
            if (!t.busy) {
                free_slot = &t;
                break;
            }
        std::vector<std::shared_ptr<Frame>> take;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            if (srv->queue.empty() && !any_busy) {
                if (srv->stopping) return;
                srv->cv_work.wait_for(lk, std::chrono::milliseconds(5));
                continue;
            }
            if (free_slot && !srv->queue.empty() && srv->fatal.empty()) {
                size_t bytes = 0;
                int64_t checks = 0, objects = 0;
                const int64_t now = now_ns();
                while (!srv->queue.empty() && (int)take.size() < srv->cfg.max_frames_per_tick) {
                    auto &f = srv->queue.front();
                    if (!take.empty() && (bytes + f->bytes > srv->slot_usable ||
                                          checks + f->checks > srv->cfg.max_checks_per_tick ||
                                          objects + f->scene.n_objects > kMaxObjectsPerLaunch))
                        break;
                    bytes += f->bytes;
                    checks += f->checks;
                    objects += f->scene.n_objects;
                    f->state = ADMITTED;
                    f->timing.admit_ns = now;
                    take.push_back(f);
                    srv->queue.pop_front();
                }
                if (!srv->queue.empty()) ++srv->deferred;
            } else if (!srv->fatal.empty() && !srv->queue.empty()) {
                // the device failed: fail everything that is still queued
                for (auto &f : srv->queue) {
                    f->status = MHC_E_DEVICE;
                    f->state = DONE;
                }
                srv->queue.clear();
                srv->cv_done.notify_all();
            }
        }
        if (!take.empty()) {
            TickSlot &t = *free_slot;
            t.frames = std::move(take);
            t.busy = true;
            t.launched_ns = now_ns();
            {
                std::lock_guard<std::mutex> lk(srv->mu);
                t.tick = srv->ticks++;
            }
            const hipError_t e = launch_tick(srv, t);
            if (e != hipSuccess) {
                {
                    std::lock_guard<std::mutex> lk(srv->mu);
                    srv->fatal = std::string("tick launch failed: ") + hipGetErrorString(e);
                }
                finish_tick(srv, t, MHC_E_DEVICE);
            }
            continue;
        }
        if (any_busy) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

}  // namespace

extern "C" mhc_status mhc_server_start(mhc_ctx *ctx, const mhc_server_cfg *cfg, mhc_server **out)
{
    if (!ctx || !out) return MHC_E_INVAL;
    *out = nullptr;
    mhc_server_cfg c = cfg ? *cfg : mhc_server_cfg{};
    if (c.max_inflight_ticks == 0) c.max_inflight_ticks = 2;
    if (c.queue_capacity == 0) c.queue_capacity = 4096;
    if (c.max_frames_per_tick == 0) c.max_frames_per_tick = 256;
    if (c.max_checks_per_tick == 0) c.max_checks_per_tick = 4000000000LL;
    if (c.hbm_budget_bytes == 0) c.hbm_budget_bytes = ctx->budget ? ctx->budget : ((size_t)1 << 30);
    if (c.max_inflight_ticks < 1 || c.max_inflight_ticks > 4 || c.queue_capacity < 1 || c.max_frames_per_tick < 1 ||
        c.max_checks_per_tick < 1) {
        ctx->err = "server config out of range (max_inflight_ticks 1..4, positive caps)";
        return MHC_E_INVAL;
    }
    if (ctx->budget && c.hbm_budget_bytes > ctx->budget) {
        ctx->err = "server budget exceeds the context budget";
        return MHC_E_INVAL;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return MHC_E_DEVICE;
    auto *srv = new mhc_server();
    srv->ctx = ctx;
    srv->cfg = c;
    srv->slot_bytes = (c.hbm_budget_bytes / c.max_inflight_ticks) & ~size_t(255);
    const size_t table = align256(((size_t)kMaxCollisionWaves + 1) * 4);
    if (srv->slot_bytes <= 2 * table) {
        ctx->err = "server budget too small";
        delete srv;
        return MHC_E_INVAL;
    }
    srv->slot_usable = srv->slot_bytes - table;
    srv->slots.resize(c.max_inflight_ticks);
    for (auto &t : srv->slots) {
        if (hipStreamCreateWithFlags(&t.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&t.done, hipEventDisableTiming) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&t.dbuf), srv->slot_bytes) != hipSuccess) {
            ctx->err = "server: cannot create streams or reserve the HBM budget";
            for (auto &u : srv->slots) {
                if (u.dbuf) hipFree(u.dbuf);
                if (u.done) hipEventDestroy(u.done);
                if (u.stream) hipStreamDestroy(u.stream);
            }
            delete srv;
            return MHC_E_NOMEM;
        }
        t.dbytes = srv->slot_bytes;
    }
    srv->start_ns = now_ns();
    srv->thread = std::thread(scheduler, srv);
    *out = srv;
    return MHC_OK;
}

extern "C" mhc_status mhc_submit(mhc_server *srv, int32_t stream_id, const mhc_scene *scene, mhc_result *dst,
                                 uint64_t *ticket)
{
    if (!srv || !ticket) return MHC_E_INVAL;
    std::string err;
    if (!validate_scene(scene, err)) {
        std::lock_guard<std::mutex> lk(srv->mu);
        ++srv->rejected;
        return MHC_E_INVAL;
    }
    if (!dst || !dst->object_crit || !validate_outputs(scene, dst, err)) return MHC_E_INVAL;
    auto f = copy_frame(scene);
    f->dst = *dst;
    frame_sizes(&f->scene, 0, dst->first_hit != nullptr, *f);
    f->stream_id = stream_id;
    f->timing.submit_ns = now_ns();
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) return MHC_E_INVAL;
    if (f->bytes > srv->slot_usable) {
        ++srv->rejected;
        return MHC_E_NOMEM;
    }
    if ((int)srv->queue.size() >= srv->cfg.queue_capacity) {
        ++srv->rejected;
        return MHC_E_BUSY;
    }
    f->ticket = srv->next_ticket++;
    srv->frames[f->ticket] = f;
    srv->queue.push_back(f);
    ++srv->submitted;
    *ticket = f->ticket;
    srv->cv_work.notify_one();
    return MHC_OK;
}

extern "C" mhc_status mhc_wait(mhc_server *srv, uint64_t ticket, int64_t timeout_us, mhc_timing *timing)
{
    if (!srv) return MHC_E_INVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->frames.find(ticket);
    if (it == srv->frames.end()) return MHC_E_INVAL;
    std::shared_ptr<Frame> f = it->second;
    auto ready = [&] { return f->state == DONE; };
    if (timeout_us < 0) {
        srv->cv_done.wait(lk, ready);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
        return MHC_E_TIMEOUT;
    }
    if (timing) *timing = f->timing;
    srv->frames.erase(ticket);
    return f->status;
}

extern "C" mhc_status mhc_server_stats(mhc_server *srv, mhc_stats *out)
{
    if (!srv || !out) return MHC_E_INVAL;
    std::vector<double> lat;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        out->submitted = srv->submitted;
        out->completed = srv->completed;
        out->rejected = srv->rejected;
        out->deferred = srv->deferred;
        out->ticks = srv->ticks;
        out->checks = srv->checks;
        lat = srv->latency_ms;
        const double secs = (now_ns() - srv->start_ns) * 1e-9;
        out->checks_per_s = secs > 0 ? srv->checks / secs : 0.0;
    }
    out->p50_ms = out->p99_ms = out->max_ms = out->mean_ms = 0.0;
    if (!lat.empty()) {
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double q) {
            size_t k = (size_t)std::ceil(q * lat.size());
            return lat[std::min(lat.size() - 1, k ? k - 1 : 0)];
        };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        out->max_ms = lat.back();
        double s = 0;
        for (double x : lat) s += x;
        out->mean_ms = s / lat.size();
    }
    return MHC_OK;
}

extern "C" mhc_status mhc_server_stop(mhc_server *srv)
{
    if (!srv) return MHC_E_INVAL;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
        srv->cv_work.notify_all();
    }
    if (srv->thread.joinable()) srv->thread.join();
    hipSetDevice(srv->ctx->device);
    for (auto &t : srv->slots) {
        if (t.stream) hipStreamSynchronize(t.stream);
        if (t.dbuf) hipFree(t.dbuf);
        if (t.pin_in) hipHostFree(t.pin_in);
        if (t.pin_out) hipHostFree(t.pin_out);
        if (t.done) hipEventDestroy(t.done);
        if (t.stream) hipStreamDestroy(t.stream);
    }
    const mhc_status st = srv->fatal.empty() ? MHC_OK : MHC_E_DEVICE;
    if (st != MHC_OK) srv->ctx->err = srv->fatal;
    delete srv;
    return st;
}
