// Autotuning of the collision kernel's micro-tile shape: every compiled
// variant is timed on a scene (or a batch of scenes in one launch) and the
// fastest is kept per size class.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>

#include "runtime.h"

using namespace mhc;

static int ilog2_floor(double x)
{
    int b = 0;
    while (x >= 2.0 && b < 62) {
        x /= 2.0;
        ++b;
    }
    return b;
}

std::array<int, 4> size_class(const mhc_scene *scenes, int n)
{
    double traj = 0.0, objs = 0.0, hsum = 0.0;
    int family = 0;
    for (int k = 0; k < n; ++k) {
        if (scene_has_outline(&scenes[k]))
            family = 2;
        else if (scenes[k].overlap == MHC_OVERLAP_PIP && family < 1)
            family = 1;
        for (int a = 0; a < scenes[k].n_objects; ++a)
            traj += (double)scenes[k].objects[a].n_u * scenes[k].objects[a].n_w;
        objs += scenes[k].n_objects;
        hsum += scenes[k].horizon;
    }
    return {ilog2_floor(traj / std::max(1.0, objs)), ilog2_floor(hsum / std::max(1, n)), family, ilog2_floor(n)};
}

int Tuning::variant_for(const mhc_scene *scenes, int n) const
{
    if (forced_variant >= 0) return forced_variant;
    auto it = tuned.find(size_class(scenes, n));
    return it == tuned.end() ? kDefaultVariant : it->second;
}

#define HIPC(call)                                                               \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess) {                                                  \
            ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);        \
            return MHC_E_DEVICE;                                                 \
        }                                                                        \
    } while (0)

extern "C" mhc_status mhc_set_variant(mhc_ctx *ctx, int32_t variant)
{
    if (!ctx) return MHC_E_INVAL;
    if (variant < -1 || variant >= N_VARIANTS) {
        ctx->err = "variant must be -1 or in [0, MHC_N_VARIANTS)";
        return MHC_E_INVAL;
    }
    ctx->tune.forced_variant = variant;
    return MHC_OK;
}

// Times the collision launch of every variant on the n scenes (one launch
// for all of them, as mhc_evaluate_batch makes it) and records the fastest
// for their size class. The variants are timed in interleaved passes (each
// pass launches every variant in turn, kBackToBack collision launches
// each), each variant on an
// image of its own, so that a change of clock or temperature during the
// tuning weighs on every variant alike. Pass 0 warms up; after `reps`
// timed passes the passes go on while the fastest variant's median over the
// last `reps` passes is still falling (by more than 1 % from the `reps`
// passes before), for at most 0.5 s of tuning and 20 reps passes: a GPU
// that idled before the tuning runs its first milliseconds of launches at a
// lower clock, and a variant's time is its median over the last reps
// passes. Where the variants' images do not fit in device memory together,
// the passes take one variant at a time in the context workspace.
// Collision launches per variant and pass, back to back between two events:
// an event pair around a single launch adds the launch's start-up to it, and
// more so, and unevenly between variants, under a kernel-tracing profiler.
constexpr int kBackToBack = 2;

static mhc_status tune_scenes(mhc_ctx *ctx, int n, const mhc_scene *scenes, int32_t reps, int32_t *best_variant,
                              double *us)
{
    HIPC(hipSetDevice(ctx->device));
    ctx->resident_image.clear();  // the timing launches overwrite the context workspace
    ctx->layout_shape.clear();
    std::vector<Layout> Ls(N_VARIANTS);
    std::vector<size_t> off(N_VARIANTS);
    size_t total = 0;
    for (int v = 0; v < N_VARIANTS; ++v) {
        build_layout(scenes, n, v, ctx->max_waves(v, scenes, n), Ls[v], false, ctx->max_waves_staged(v, scenes, n));
        off[v] = total;
        total += (Ls[v].total_bytes + 255) & ~(size_t)255;
    }
    char *own = nullptr;
    const bool together = (!ctx->budget || total <= ctx->budget) &&
                          hipMalloc(reinterpret_cast<void **>(&own), total) == hipSuccess;
    if (!together) (void)hipGetLastError();  // a failed allocation leaves the one-at-a-time path
    std::vector<std::vector<float>> ms(N_VARIANTS);
    std::vector<hipEvent_t> ev(2 * N_VARIANTS, nullptr);
    hipError_t e = hipSuccess;
    for (auto &x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    auto window_median = [&](int v, size_t end) {  // of passes [end - reps, end) of variant v
        std::vector<float> w(ms[v].begin() + (end - reps), ms[v].begin() + end);
        std::sort(w.begin(), w.end());
        const size_t k = w.size();
        return k % 2 ? (double)w[k / 2] : 0.5 * ((double)w[k / 2 - 1] + (double)w[k / 2]);
    };
    auto run_passes = [&](int v0, int v1, char *const *bases) {
        std::vector<Launch> X;
        for (int v = v0; v < v1; ++v) X.push_back(make_launch(Ls[v], bases[v], nullptr, false, ctx->n_cu));
        const auto t0 = std::chrono::steady_clock::now();
        for (int r = 0; e == hipSuccess; ++r) {
            for (int v = v0; v < v1 && e == hipSuccess; ++v) {
                const Launch &L = X[v - v0];
                e = launch_trajgen(L, ctx->stream);
                if (e == hipSuccess) e = hipEventRecord(ev[2 * v], ctx->stream);
                for (int b = 0; b < kBackToBack && e == hipSuccess; ++b) e = launch_collide(L, ctx->stream);
                if (e == hipSuccess) e = hipEventRecord(ev[2 * v + 1], ctx->stream);
            }
            if (e == hipSuccess) e = hipEventSynchronize(ev[2 * (v1 - 1) + 1]);
            for (int v = v0; v < v1 && e == hipSuccess; ++v) {
                float t = 0.f;
                e = hipEventElapsedTime(&t, ev[2 * v], ev[2 * v + 1]);
                if (r > 0) ms[v].push_back(t / kBackToBack);  // pass 0 warms up
            }
            if (e != hipSuccess || r < reps) continue;  // r timed passes so far
            const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (r >= 20 * reps || secs >= 0.5) break;
            if (r < 2 * reps) continue;  // two windows to compare
            int fast = v0;
            for (int v = v0; v < v1; ++v)
                if (window_median(v, ms[v].size()) < window_median(fast, ms[fast].size())) fast = v;
            const size_t end = ms[fast].size();
            if (window_median(fast, end) > 0.99 * window_median(fast, end - reps)) break;
        }
    };
    mhc_status st = MHC_OK;
    char *bases[N_VARIANTS] = {};
    if (e == hipSuccess && together) {
        for (int v = 0; v < N_VARIANTS && e == hipSuccess; ++v) {
            std::vector<char> img(Ls[v].image_bytes);
            pack_image(Ls[v], img.data());
            bases[v] = own + off[v];
            e = hipMemcpy(bases[v], img.data(), Ls[v].image_bytes, hipMemcpyHostToDevice);
        }
        run_passes(0, N_VARIANTS, bases);
    } else {
        for (int v = 0; v < N_VARIANTS && e == hipSuccess && st == MHC_OK; ++v) {
            st = ensure_device(ctx, Ls[v].total_bytes);
            if (st != MHC_OK) break;
            std::vector<char> img(Ls[v].image_bytes);
            pack_image(Ls[v], img.data());
            bases[v] = static_cast<char *>(ctx->dbuf);
            e = hipMemcpy(bases[v], img.data(), Ls[v].image_bytes, hipMemcpyHostToDevice);
            if (e == hipSuccess) run_passes(v, v + 1, bases);
        }
    }
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    if (own) (void)hipFree(own);
    if (st != MHC_OK) return st;
    if (e != hipSuccess) {
        ctx->err = std::string("autotune launch: ") + hipGetErrorString(e);
        return MHC_E_DEVICE;
    }
    int best = -1;
    double best_us = 0.0;
    for (int v = 0; v < N_VARIANTS; ++v) {
        const double t = 1e3 * window_median(v, ms[v].size());
        if (us) us[v] = t;
        if (best < 0 || t < best_us) {
            best = v;
            best_us = t;
        }
    }
    ctx->tune.tuned[size_class(scenes, n)] = best;
    if (best_variant) *best_variant = best;
    return MHC_OK;
}

extern "C" mhc_status mhc_autotune(mhc_ctx *ctx, const mhc_scene *scene, int32_t reps, int32_t *best_variant,
                                   double *us)
{
    if (!ctx) return MHC_E_INVAL;
    if (reps < 1 || reps > 100000) {
        ctx->err = "reps must be in [1, 100000]";
        return MHC_E_INVAL;
    }
    if (!validate_scene(scene, ctx->err)) return MHC_E_INVAL;
    return tune_scenes(ctx, 1, scene, reps, best_variant, us);
}

extern "C" mhc_status mhc_autotune_batch(mhc_ctx *ctx, int32_t n, const mhc_scene *scenes, int32_t reps,
                                         int32_t *best_variant, double *us)
{
    if (!ctx) return MHC_E_INVAL;
    if (n < 1 || !scenes) {
        ctx->err = "autotune batch needs n >= 1 scenes";
        return MHC_E_INVAL;
    }
    if (reps < 1 || reps > 100000) {
        ctx->err = "reps must be in [1, 100000]";
        return MHC_E_INVAL;
    }
    int64_t total_objects = 0;
    for (int k = 0; k < n; ++k) {
        if (!validate_scene(&scenes[k], ctx->err, k)) return MHC_E_INVAL;
        total_objects += scenes[k].n_objects;
    }
    if (total_objects > kMaxObjectsPerLaunch) {
        ctx->err = "batch holds more than 65535 objects";
        return MHC_E_INVAL;
    }
    return tune_scenes(ctx, n, scenes, reps, best_variant, us);
}

extern "C" mhc_status mhc_tune_save(mhc_ctx *ctx, const char *path)
{
    if (!ctx || !path) return MHC_E_INVAL;
    std::ofstream f(path);
    if (!f) {
        ctx->err = std::string("cannot write ") + path;
        return MHC_E_INVAL;
    }
    f << "{\"gfx950\": {";
    bool firstk = true;
    for (auto &kv : ctx->tune.tuned) {
        f << (firstk ? "" : ", ") << "\"" << kv.first[0] << "," << kv.first[1] << "," << kv.first[2] << ","
          << kv.first[3] << "\": " << kv.second;
        firstk = false;
    }
    f << "}}\n";
    return f ? MHC_OK : MHC_E_INVAL;
}

// Reads the entries of the "gfx950" object: "T,H[,family[,scenes]]": variant.
// Every entry is checked before any is applied, so a malformed file leaves
// the context's choices as they were.
extern "C" mhc_status mhc_tune_load(mhc_ctx *ctx, const char *path)
{
    if (!ctx || !path) return MHC_E_INVAL;
    std::ifstream f(path);
    if (!f) {
        ctx->err = std::string("cannot read ") + path;
        return MHC_E_INVAL;
    }
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    const size_t arch = s.find("\"gfx950\"");
    if (arch == std::string::npos) {
        ctx->err = "tune file has no gfx950 entry";
        return MHC_E_INVAL;
    }
    std::map<std::array<int, 4>, int> got;
    const size_t open = s.find('{', arch);
    const size_t end = open == std::string::npos ? std::string::npos : s.find('}', open);
    if (open == std::string::npos || end == std::string::npos) {
        ctx->err = "malformed tune file";
        return MHC_E_INVAL;
    }
    size_t pos = open;
    while (true) {
        const size_t q = s.find('"', pos + 1);
        if (q == std::string::npos || q > end) break;
        // keys are "T bucket,H bucket,family,scene-count bucket" (family 0
        // rectangles and circles, 1 point-in-polygon rectangles, 2 outlines);
        // a key without the scene-count field is for single scenes, one
        // without the family field also for family 0
        int tb = 0, hb = 0, family = 0, nb = 0, v = -1, used = 0;
        const char *c = s.c_str() + q;
        if (std::sscanf(c, "\"%d,%d,%d,%d\": %d%n", &tb, &hb, &family, &nb, &v, &used) != 5) {
            nb = 0;
            if (std::sscanf(c, "\"%d,%d,%d\": %d%n", &tb, &hb, &family, &v, &used) != 4) {
                family = 0;
                if (std::sscanf(c, "\"%d,%d\": %d%n", &tb, &hb, &v, &used) != 3) v = -1;
            }
        }
        if (v < 0 || v >= N_VARIANTS || family < 0 || family > 2 || tb < 0 || hb < 0 || nb < 0 || tb > 62 ||
            hb > 62 || nb > 62) {
            ctx->err = "malformed tune file entry";
            return MHC_E_INVAL;
        }
        got[{tb, hb, family, nb}] = v;
        pos = q + (size_t)used - 1;
        if (pos >= end) break;
    }
    for (auto &kv : got) ctx->tune.tuned[kv.first] = kv.second;
    return MHC_OK;
}
