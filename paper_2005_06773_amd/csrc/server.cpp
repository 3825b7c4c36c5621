// Serving form: continuous batching of scene frames from many streams.
//
// mhc_submit copies a frame into a FIFO. A scheduler thread keeps up to
// `max_inflight_ticks` ticks running at once, one per slot. Whenever a slot
// is free it admits queued frames in arrival order while they fit the slot's
// share of the memory budget and the tick's frame / check caps, and hands the
// tick to an executor. The GPU executor gives every slot its own stream,
// device workspace and pinned staging: it plans the tick on the host (while
// earlier ticks still run), uploads one scene image, launches trajectory
// generation, collision recognition and risk for all its frames (the module
// chain of Fig. 1) and queues the copy of their results back to pinned
// memory; when the tick's event has completed it copies every frame's results
// to the caller's buffers. A frame's results do not depend on which tick
// carried it or what else was in it. Executors written by the caller
// (mhc_server_start_executor) run the same scheduler without a GPU.
//
// A frame of more checks than max_checks_per_tick rides in a tick of its own,
// and with two or more slots such frames may occupy all but one of them, so
// that one slot always stays open to the other frames; those may then go
// ahead of a large frame that waits for a slot. Frames of either kind keep
// their arrival order among themselves. On the GPU such a tick's collision
// plan runs as several launches of at most about min(max_checks_per_tick,
// 1e9) checks each, planned for 4/5 of the resident waves and enqueued one
// ahead of the GPU as the earlier ones end, so that the other slots' kernels
// find room on every CU beside it and between its launches, also where the
// slots' streams share a hardware queue.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include <sys/prctl.h>

#include "runtime.h"

using namespace mhc;

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Deadline of a bounded condition-variable wait. Waits are timed on the
// system clock: with it the standard library waits in
// pthread_cond_timedwait, which thread sanitizers follow (the steady clock's
// pthread_cond_clockwait is not followed by all of them, which then
// misreport the mutex as still held). Only the bounded waits' length depends
// on this clock; latencies are measured on the steady clock.
std::chrono::system_clock::time_point wait_deadline(std::chrono::microseconds d)
{
    return std::chrono::system_clock::now() + d;
}

// Bound on the resident collision waves of any GPU this library runs on
// (sizes the slot table in the admission estimate).
constexpr int kMaxCollisionWaves = 1 << 16;
// Ticks split collision units in time into at most 4 parts: the admission
// bound counts a collision segment per unit of 16 items.
constexpr int kTickMaxTshift = 2;
constexpr int64_t kDefaultWatchdogUs = 30LL * 1000 * 1000;

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
    size_t bytes = 0;    // device bytes upper bound
    bool large = false;  // more checks than one tick may carry
    FrameState state = QUEUED;
    mhc_status status = MHC_OK;
    mhc_timing timing{};
};

using Frames = std::vector<std::shared_ptr<Frame>>;

// Runs the ticks the scheduler forms, at most one per slot at a time. Only
// the scheduler thread calls launch and poll.
class Executor {
public:
    virtual ~Executor() = default;
    // Starts tick `tick` in slot `slot` with these frames.
    virtual mhc_status launch(int slot, int64_t tick, const Frames &frames, std::string &err) = 0;
    // 1: the slot's tick has finished and every frame's results are in its
    //    host buffers; 0: still running; < 0: failed (err says why).
    virtual int poll(int slot, std::string &err) = 0;
    // After the scheduler has stopped: waits for whatever is still running
    // and frees the executor's resources.
    virtual void shutdown() {}
};

// Checks per collision launch of a large tick, at most (about 0.4 ms of the
// GPU): a tick of another slot that shares the large tick's hardware queue
// waits for at most two such launches.
constexpr int64_t kPartChecks = 1000000000;

// One slot of the GPU executor.
struct TickSlot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;          // the tick's results are in pinned memory
    hipEvent_t kernels_done = nullptr;  // a large tick's kernels have ended
    bool copies_pending = false;        // a large tick's result copies are not yet enqueued
    // A large tick's collision parts are enqueued one ahead of the GPU (part
    // k once part k - 2 has ended, part_ev[k % 2]), so that a tick of another
    // slot whose stream shares this one's hardware queue waits for at most
    // two parts, not for the whole frame.
    hipEvent_t part_ev[2] = {nullptr, nullptr};
    Launch X{};                         // the large tick's launch
    int next_part = 0, parts = 0;
    char *dbuf = nullptr;
    size_t dbytes = 0;
    char *pin_in = nullptr;
    size_t pin_in_bytes = 0;
    char *pin_out = nullptr;
    size_t pin_out_bytes = 0;
    // staging buffers outgrown by a later tick, freed when the server stops:
    // hipHostFree waits for every stream of the device, so freeing them here
    // would hold the scheduler thread until the other slots' ticks end
    std::vector<char *> retired;
    Layout L;
    int n_frames = 0;
    std::vector<mhc_result> dsts;  // per frame: its host buffers
    ResultPlan results;            // the tick's outputs staged in pin_out
};

// Pinned staging per slot and direction from the start: a tick of small
// frames (tens of scenes of the batched size mix) fits without growing it.
constexpr size_t kInitialStaging = (size_t)4 << 20;

// Grows a pinned staging buffer to hold `want` bytes, at least doubling it,
// so that a slot's buffers are replaced a logarithmic number of times and
// the retired ones total less than the live one.
hipError_t grow_pinned(char **p, size_t *have, size_t want, std::vector<char *> &retired)
{
    if (*have >= want) return hipSuccess;
    const size_t sz = std::max({want, 2 * *have, (size_t)1 << 20});
    char *fresh = nullptr;
    hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&fresh), sz, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    if (*p) retired.push_back(*p);
    *p = fresh;
    *have = sz;
    return hipSuccess;
}

// The library's own executor: ticks on the GPU of a context. The context's
// tile-variant choices and resident wave counts are copied when the server
// starts, so the context may be used (and retuned) by its own thread while
// the server runs.
class GpuExecutor : public Executor {
public:
    int device = 0, n_cu = 0;
    int64_t max_checks_per_tick = 0;
    Tuning tune;
    int waves[N_VARIANTS][3][2] = {};
    int waves_staged[N_VARIANTS] = {};   // of the LDS-staged instances (plain family, no per-slot sums)
    std::vector<TickSlot> slots;

    int max_waves(int v, const mhc_scene *scenes, int n) const
    {
        int fam = 0, tl = 0;
        for (int k = 0; k < n; ++k) {
            fam = std::max(fam, scene_family(&scenes[k]));
            tl |= scenes[k].timeline != 0;
        }
        return waves[v][fam][tl];
    }

    // Enqueues the next collision part of a large tick; after the last, the
    // risk stage and the event its result copies wait for.
    static hipError_t enqueue_part(TickSlot &t)
    {
        Launch X = t.X;
        X.collide_only = t.next_part + 1;
        hipError_t e = launch_collide(X, t.stream);
        if (e == hipSuccess) e = hipEventRecord(t.part_ev[t.next_part % 2], t.stream);
        ++t.next_part;
        if (e == hipSuccess && t.next_part == t.parts) {
            e = launch_risk(X, t.stream);
            if (e == hipSuccess) e = hipEventRecord(t.kernels_done, t.stream);
        }
        return e;
    }

    mhc_status launch(int slot, int64_t, const Frames &frames, std::string &err) override
    {
        TickSlot &t = slots[slot];
        std::vector<mhc_scene> scenes;
        scenes.reserve(frames.size());
        for (auto &f : frames) scenes.push_back(f->scene);
        const int n = (int)scenes.size();
        const int v = tune.variant_for(scenes.data(), n);
        bool keep_hits = false;
        int64_t checks = 0;
        for (auto &f : frames) {
            keep_hits |= f->dst.first_hit != nullptr;
            checks += f->checks;
        }
        // a tick above the check cap (one large frame) plans its collision
        // work for 4/5 of the resident waves, so that every CU keeps room
        // for the other slots' kernels while it runs
        const bool large = checks > max_checks_per_tick;
        int waves_v = max_waves(v, scenes.data(), n);
        bool plain = true;
        for (int k = 0; k < n; ++k) plain &= scene_family(&scenes[k]) == FAM_PLAIN && !scenes[k].timeline;
        int waves_s = plain ? waves_staged[v] : 0;
        if (large) {
            waves_v = std::max(1, waves_v / 5 * 4);
            waves_s = waves_s / 5 * 4;
        }
        build_layout(scenes.data(), n, v, waves_v, t.L, keep_hits, waves_s, kTickMaxTshift);
        if (t.L.total_bytes > t.dbytes) {  // the admission bound excludes this
            err = "tick workspace above the slot's share of the budget";
            return MHC_E_NOMEM;
        }
        hipError_t e = grow_pinned(&t.pin_in, &t.pin_in_bytes, t.L.image_bytes, t.retired);
        t.n_frames = n;
        t.dsts.clear();
        for (auto &f : frames) t.dsts.push_back(f->dst);
        // every output of the tick in one transfer per output region, staged
        // in pinned memory so that nothing blocks the scheduler thread
        t.results = plan_results(t.L, n, t.dsts.data(), true);
        if (e == hipSuccess) e = grow_pinned(&t.pin_out, &t.pin_out_bytes, t.results.staged, t.retired);
        if (e == hipSuccess) {
            pack_image(t.L, t.pin_in);
            e = hipMemcpyAsync(t.dbuf, t.pin_in, t.L.image_bytes, hipMemcpyHostToDevice, t.stream);
        }
        Launch X = make_launch(t.L, t.dbuf, nullptr, keep_hits, n_cu);
        // A tick above the check cap (one large frame) runs its collision
        // plan as launches of at most about that many checks each, enqueued
        // one ahead of the GPU as the earlier ones end (poll), so that the
        // other slots' ticks get the GPU in between even where their streams
        // share this one's hardware queue. Its result copies are enqueued
        // only once its kernels have ended: a copy enqueued now would wait
        // for them at the head of a copy engine's queue, where the image and
        // result copies of the other slots' ticks would wait behind it.
        t.copies_pending = large;
        if (large) {
            const int64_t per_part = std::min<int64_t>(max_checks_per_tick, kPartChecks);
            X.collide_parts = (int)std::max<int64_t>(2, std::min<int64_t>(64, (t.L.n_checks + per_part - 1) / per_part));
            t.X = X;
            t.parts = X.collide_parts;
            t.next_part = 0;
            if (e == hipSuccess) e = launch_trajgen(X, t.stream);
            while (e == hipSuccess && t.next_part < 2) e = enqueue_part(t);
        } else {
            if (e == hipSuccess) e = launch_all(X, t.stream);
            if (e == hipSuccess) e = enqueue_results(t.results, t.L, n, t.dbuf, t.pin_out, t.dsts.data(), t.stream);
            if (e == hipSuccess) e = hipEventRecord(t.done, t.stream);
        }
        if (e != hipSuccess) {
            err = std::string("tick launch failed: ") + hipGetErrorString(e);
            return MHC_E_DEVICE;
        }
        return MHC_OK;
    }

    int poll(int slot, std::string &err) override
    {
        TickSlot &t = slots[slot];
        while (t.copies_pending && t.next_part < t.parts) {
            const hipError_t k = hipEventQuery(t.part_ev[t.next_part % 2]);  // part next_part - 2
            if (k == hipErrorNotReady) return 0;
            const hipError_t e = k == hipSuccess ? enqueue_part(t) : k;
            if (e != hipSuccess) {
                err = std::string("tick failed: ") + hipGetErrorString(e);
                return -1;
            }
        }
        if (t.copies_pending) {
            const hipError_t k = hipEventQuery(t.kernels_done);
            if (k == hipErrorNotReady) return 0;
            hipError_t e = k;
            if (e == hipSuccess)
                e = enqueue_results(t.results, t.L, t.n_frames, t.dbuf, t.pin_out, t.dsts.data(), t.stream);
            if (e == hipSuccess) e = hipEventRecord(t.done, t.stream);
            if (e != hipSuccess) {
                err = std::string("tick failed: ") + hipGetErrorString(e);
                return -1;
            }
            t.copies_pending = false;
        }
        const hipError_t q = hipEventQuery(t.done);
        if (q == hipErrorNotReady) return 0;
        if (q != hipSuccess) {
            err = std::string("tick failed: ") + hipGetErrorString(q);
            return -1;
        }
        scatter_results(t.results, t.L, t.n_frames, t.pin_out, t.dsts.data());
        return 1;
    }

    void shutdown() override
    {
        (void)hipSetDevice(device);
        for (auto &t : slots) {
            if (t.stream) (void)hipStreamSynchronize(t.stream);
            if (t.dbuf) (void)hipFree(t.dbuf);
            if (t.pin_in) (void)hipHostFree(t.pin_in);
            if (t.pin_out) (void)hipHostFree(t.pin_out);
            for (char *r : t.retired) (void)hipHostFree(r);
            if (t.done) (void)hipEventDestroy(t.done);
            if (t.kernels_done) (void)hipEventDestroy(t.kernels_done);
            for (hipEvent_t &pe : t.part_ev)
                if (pe) (void)hipEventDestroy(pe);
            if (t.stream) (void)hipStreamDestroy(t.stream);
        }
        slots.clear();
    }
};

// An executor given by the caller as C callbacks (mhc_executor).
class CallbackExecutor : public Executor {
public:
    mhc_executor ex{};

    mhc_status launch(int slot, int64_t tick, const Frames &frames, std::string &err) override
    {
        std::vector<mhc_scene> scenes;
        std::vector<mhc_result> dsts;
        for (auto &f : frames) {
            scenes.push_back(f->scene);
            dsts.push_back(f->dst);
        }
        const int32_t st = ex.launch(ex.user, slot, tick, (int32_t)frames.size(), scenes.data(), dsts.data());
        if (st != MHC_OK) {
            err = "executor launch failed with status " + std::to_string(st);
            return st < 0 ? (mhc_status)st : MHC_E_DEVICE;
        }
        return MHC_OK;
    }

    int poll(int slot, std::string &err) override
    {
        const int32_t st = ex.poll(ex.user, slot);
        if (st < 0) err = "executor tick failed with status " + std::to_string(st);
        return st < 0 ? -1 : (st > 0 ? 1 : 0);
    }
};

struct Slot {
    bool busy = false;
    bool large = false;       // carries a frame above max_checks_per_tick
    int64_t launched_ns = 0;
    int64_t tick = 0;
    Frames frames;
};

}  // namespace

struct mhc_server {
    mhc_ctx *ctx = nullptr;   // null for servers on a caller's executor
    std::unique_ptr<Executor> exec;
    mhc_server_cfg cfg{};
    size_t slot_bytes = 0;
    size_t slot_usable = 0;   // slot bytes minus the per-tick collision slot table
    std::vector<Slot> slots;
    std::thread thread;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Frame>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Frame>> frames;
    uint64_t next_ticket = 1;
    bool stopping = false;
    std::string fatal;
    // statistics
    int64_t submitted = 0, completed = 0, rejected = 0, deferred = 0, ticks = 0, checks = 0, late = 0;
    std::vector<double> latency_ms;
    int64_t start_ns = 0;
};

namespace {

// Upper bound of the device bytes a frame adds to a tick (every buffer of the
// workspace layout, with one collision segment per work unit).
void frame_sizes(const mhc_scene *s, int max_waves, bool hits, Frame &f)
{
    int64_t n_traj = 0, pose = 0, n_units = 0, n_hits = 0, vals = 0, n_pairs = 0, k1_blocks = 0;
    const int n = s->n_objects;
    for (int a = 0; a < n; ++a) {
        const int64_t T = (int64_t)s->objects[a].n_u * s->objects[a].n_w;
        n_traj += T;
        // poses; a vehicle's frame block beside them
        const bool vehicle = s->objects[a].kind == MHC_VEHICLE;
        pose += align256((size_t)s->horizon * T * (vehicle ? 16 : 8)) * (vehicle ? 2 : 1);
        vals += s->objects[a].n_u + s->objects[a].n_w + (s->objects[a].score ? T : 0);
        k1_blocks += (T + K1_TPB - 1) / K1_TPB + 1;
    }
    for (int a = 0; a < n; ++a)
        for (int b = a + 1; b < n; ++b) {
            if (s->pairs == MHC_PAIRS_EGO && a != 0) continue;
            const int64_t Ta = (int64_t)s->objects[a].n_u * s->objects[a].n_w;
            const int64_t Tb = (int64_t)s->objects[b].n_u * s->objects[b].n_w;
            n_hits += Ta * Tb;
            // one collision segment per work unit, for the variant and the
            // time split (a tick's: up to 4 parts, 16 items a unit) that cut
            // this pair into the most units (2-D blocks of items are taken
            // where they add at most 1/32 to the units of the row-major cut)
            const bool poly = scene_has_outline(s);
            const int cls = pair_class(s->objects[a].kind, s->objects[b].kind, s->overlap,
                                       poly && s->objects[a].n_vertices > 0, poly && s->objects[b].n_vertices > 0);
            int64_t most = 0;
            for (int v = 0; v < N_VARIANTS; ++v) {
                const int64_t items = (Ta + kTiles[v][cls].ri - 1) / kTiles[v][cls].ri *
                                      ((Tb + kTiles[v][cls].rj - 1) / kTiles[v][cls].rj);
                const int64_t per = WAVE >> kTickMaxTshift;
                most = std::max(most, ((items + per - 1) / per * 33 + 31) / 32);
            }
            n_units += most;
            ++n_pairs;
        }
    const int64_t n_q = n_traj * n;
    size_t bytes = 0;
    bytes += align256(n * sizeof(DObj)) + align256(vals * 8) + align256(n_pairs * sizeof(DPair));
    bytes += align256((scene_has_outline(s) ? n : 0) * sizeof(DPoly));
    bytes += align256((n_units + 1) * sizeof(WorkItem));
    bytes += align256(k1_blocks * 2 * sizeof(int32_t));  // trajectory kernel rows (at most one per block)
    bytes += pose + align256(n_traj * 8) * 3 + align256(n_q * 8) * 2;  // p*2^62, p, traj crit; q sums, q
    bytes += align256(n * 8);                                            // risk kernel's per-object words
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

// Marks a slot's frames done with status st (scheduler thread, lock not held).
void finish_tick(mhc_server *srv, Slot &t, mhc_status st)
{
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
        const double ms = (fp->timing.done_ns - fp->timing.submit_ns) * 1e-6;
        srv->latency_ms.push_back(ms);
        if (srv->cfg.deadline_us > 0 && ms * 1e3 > (double)srv->cfg.deadline_us) ++srv->late;
    }
    t.frames.clear();
    t.busy = false;
    t.large = false;
    srv->cv_done.notify_all();
}

// Frames for a free slot, taken from the queue (lock held). A large frame
// rides alone, and only when large_allowed; other frames are taken in order
// while the tick's caps hold, and may pass a large frame that has to wait.
Frames admit(mhc_server *srv, bool large_allowed, bool *took_large)
{
    Frames take;
    size_t bytes = 0;
    int64_t checks = 0, objects = 0;
    const int64_t now = now_ns();
    *took_large = false;
    for (auto it = srv->queue.begin(); it != srv->queue.end() && (int)take.size() < srv->cfg.max_frames_per_tick;) {
        const std::shared_ptr<Frame> f = *it;
        if (f->large) {
            if (take.empty() && large_allowed) {
                f->state = ADMITTED;
                f->timing.admit_ns = now;
                take.push_back(f);
                srv->queue.erase(it);
                *took_large = true;
                break;
            }
            // it waits for a slot of its own; later large frames wait behind it
            large_allowed = false;
            ++it;
            continue;
        }
        if (!take.empty() && (bytes + f->bytes > srv->slot_usable || checks + f->checks > srv->cfg.max_checks_per_tick ||
                              objects + f->scene.n_objects > kMaxObjectsPerLaunch))
            break;
        bytes += f->bytes;
        checks += f->checks;
        objects += f->scene.n_objects;
        f->state = ADMITTED;
        f->timing.admit_ns = now;
        take.push_back(f);
        it = srv->queue.erase(it);
    }
    return take;
}

// Interval at which the scheduler polls running ticks.
constexpr int kPollUs = 10;

void scheduler(mhc_server *srv)
{
    // The thread polls running ticks every kPollUs; with Linux's default
    // 50 us timer slack each of those sleeps would last about 70 us, which
    // frames that finish in a fraction of a millisecond would wait out.
    (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
    if (srv->ctx) (void)hipSetDevice(srv->ctx->device);
    const int64_t watchdog_ns = srv->cfg.watchdog_us * 1000;
    const int n_slots = (int)srv->slots.size();
    // slots that frames above the check cap may hold at once: all but one
    const int large_slots = n_slots > 1 ? n_slots - 1 : 1;
    std::string err;
    while (true) {
        // 1. retire finished ticks; a tick that fails or outlives the
        // watchdog fails the server
        bool any_busy = false;
        for (int k = 0; k < n_slots; ++k) {
            Slot &t = srv->slots[k];
            if (!t.busy) continue;
            err.clear();
            const int q = srv->exec->poll(k, err);
            if (q > 0) {
                finish_tick(srv, t, MHC_OK);
            } else if (q < 0 || now_ns() - t.launched_ns > watchdog_ns) {
                {
                    std::lock_guard<std::mutex> lk(srv->mu);
                    if (srv->fatal.empty())
                        srv->fatal = q < 0 ? err : "tick " + std::to_string(t.tick) + " exceeded the watchdog";
                }
                finish_tick(srv, t, MHC_E_DEVICE);
            } else {
                any_busy = true;
            }
        }
        // 2. admit frames into a free slot
        int free_slot = -1, large_busy = 0;
        for (int k = 0; k < n_slots; ++k) {
            if (!srv->slots[k].busy && free_slot < 0) free_slot = k;
            large_busy += srv->slots[k].busy && srv->slots[k].large;
        }
        Frames take;
        bool took_large = false;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            if (srv->queue.empty() && !any_busy) {
                if (srv->stopping) return;
                srv->cv_work.wait_until(lk, wait_deadline(std::chrono::milliseconds(5)));
                continue;
            }
            if (!srv->fatal.empty()) {
                // the executor failed: fail everything that is still queued
                for (auto &f : srv->queue) {
                    f->status = MHC_E_DEVICE;
                    f->state = DONE;
                }
                srv->queue.clear();
                srv->cv_done.notify_all();
            } else if (free_slot >= 0 && !srv->queue.empty()) {
                take = admit(srv, large_busy < large_slots, &took_large);
                if (!srv->queue.empty()) ++srv->deferred;
            }
        }
        if (!take.empty()) {
            Slot &t = srv->slots[free_slot];
            t.frames = std::move(take);
            t.busy = true;
            t.large = took_large;
            t.launched_ns = now_ns();
            {
                std::lock_guard<std::mutex> lk(srv->mu);
                t.tick = srv->ticks++;
            }
            err.clear();
            const mhc_status st = srv->exec->launch(free_slot, t.tick, t.frames, err);
            if (st != MHC_OK) {
                {
                    std::lock_guard<std::mutex> lk(srv->mu);
                    if (srv->fatal.empty()) srv->fatal = err;
                }
                finish_tick(srv, t, MHC_E_DEVICE);
            }
            continue;
        }
        if (any_busy) std::this_thread::sleep_for(std::chrono::microseconds(kPollUs));
    }
}

// Fills the defaults of a server configuration and checks it; "" when valid.
std::string complete_cfg(mhc_server_cfg &c, size_t ctx_budget)
{
    if (c.max_inflight_ticks == 0) c.max_inflight_ticks = 2;
    if (c.queue_capacity == 0) c.queue_capacity = 4096;
    if (c.max_frames_per_tick == 0) c.max_frames_per_tick = 256;
    if (c.max_checks_per_tick == 0) c.max_checks_per_tick = 4000000000LL;
    if (c.hbm_budget_bytes == 0) c.hbm_budget_bytes = ctx_budget ? ctx_budget : ((size_t)1 << 30);
    if (c.watchdog_us == 0) c.watchdog_us = kDefaultWatchdogUs;
    if (c.max_inflight_ticks < 1 || c.max_inflight_ticks > 4 || c.queue_capacity < 1 || c.max_frames_per_tick < 1 ||
        c.max_checks_per_tick < 1 || c.watchdog_us < 1 || c.watchdog_us > INT64_MAX / 1000 || c.deadline_us < 0)
        return "server config out of range (max_inflight_ticks 1..4, positive caps and watchdog, deadline >= 0)";
    if (ctx_budget && c.hbm_budget_bytes > ctx_budget) return "server budget exceeds the context budget";
    return "";
}

mhc_server *new_server(const mhc_server_cfg &c, std::string &err)
{
    auto *srv = new mhc_server();
    srv->cfg = c;
    srv->slot_bytes = (c.hbm_budget_bytes / c.max_inflight_ticks) & ~size_t(255);
    const size_t table = align256(((size_t)kMaxCollisionWaves + 1) * 4);
    if (srv->slot_bytes <= 2 * table) {
        err = "server budget too small";
        delete srv;
        return nullptr;
    }
    srv->slot_usable = srv->slot_bytes - table;
    srv->slots.resize(c.max_inflight_ticks);
    return srv;
}

void run_server(mhc_server *srv)
{
    srv->start_ns = now_ns();
    srv->thread = std::thread(scheduler, srv);
}

}  // namespace

extern "C" mhc_status mhc_server_start(mhc_ctx *ctx, const mhc_server_cfg *cfg, mhc_server **out)
{
    if (!ctx || !out) return MHC_E_INVAL;
    *out = nullptr;
    mhc_server_cfg c = cfg ? *cfg : mhc_server_cfg{};
    const std::string bad = complete_cfg(c, ctx->budget);
    if (!bad.empty()) {
        ctx->err = bad;
        return MHC_E_INVAL;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return MHC_E_DEVICE;
    mhc_server *srv = new_server(c, ctx->err);
    if (!srv) return MHC_E_INVAL;
    srv->ctx = ctx;
    auto ex = std::make_unique<GpuExecutor>();
    ex->device = ctx->device;
    ex->n_cu = ctx->n_cu;
    ex->max_checks_per_tick = c.max_checks_per_tick;
    ex->tune = ctx->tune;
    for (int v = 0; v < N_VARIANTS; ++v)
        for (int fam = 0; fam < 3; ++fam)
            for (int tl = 0; tl < 2; ++tl) ex->waves[v][fam][tl] = ctx->max_waves_of(v, fam, tl != 0);
    for (int v = 0; v < N_VARIANTS; ++v) ex->waves_staged[v] = ctx->max_waves_of(v, FAM_PLAIN, false, true);
    ex->slots.resize(c.max_inflight_ticks);
    for (auto &t : ex->slots) {
        if (hipStreamCreateWithFlags(&t.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&t.done, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&t.kernels_done, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&t.part_ev[0], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&t.part_ev[1], hipEventDisableTiming) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&t.dbuf), srv->slot_bytes) != hipSuccess ||
            grow_pinned(&t.pin_in, &t.pin_in_bytes, kInitialStaging, t.retired) != hipSuccess ||
            grow_pinned(&t.pin_out, &t.pin_out_bytes, kInitialStaging, t.retired) != hipSuccess) {
            ctx->err = "server: cannot create streams or reserve the HBM budget";
            ex->shutdown();
            delete srv;
            return MHC_E_NOMEM;
        }
        t.dbytes = srv->slot_bytes;
    }
    srv->exec = std::move(ex);
    run_server(srv);
    *out = srv;
    return MHC_OK;
}

extern "C" mhc_status mhc_server_start_executor(const mhc_server_cfg *cfg, const mhc_executor *ex, mhc_server **out)
{
    if (!out || !ex || !ex->launch || !ex->poll) return MHC_E_INVAL;
    *out = nullptr;
    mhc_server_cfg c = cfg ? *cfg : mhc_server_cfg{};
    if (!complete_cfg(c, 0).empty()) return MHC_E_INVAL;
    std::string err;
    mhc_server *srv = new_server(c, err);
    if (!srv) return MHC_E_INVAL;
    auto cx = std::make_unique<CallbackExecutor>();
    cx->ex = *ex;
    srv->exec = std::move(cx);
    run_server(srv);
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
    f->large = f->checks > srv->cfg.max_checks_per_tick;
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
    } else if (!srv->cv_done.wait_until(lk, wait_deadline(std::chrono::microseconds(timeout_us)), ready)) {
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
        out->late = srv->late;
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
    srv->exec->shutdown();
    const mhc_status st = srv->fatal.empty() ? MHC_OK : MHC_E_DEVICE;
    if (st != MHC_OK && srv->ctx) srv->ctx->err = srv->fatal;
    delete srv;
    return st;
}
