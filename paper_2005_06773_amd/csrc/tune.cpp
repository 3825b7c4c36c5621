// Autotuning of the collision kernel's micro-tile shape: every compiled
// variant is timed on a scene (or a batch of scenes in one launch) and the
// fastest is kept per size class.
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
// for their size class.
static mhc_status tune_scenes(mhc_ctx *ctx, int n, const mhc_scene *scenes, int32_t reps, int32_t *best_variant,
                              double *us)
{
    HIPC(hipSetDevice(ctx->device));
    ctx->resident_image.clear();  // the timing launches overwrite the context workspace
    ctx->layout_shape.clear();
    hipEvent_t e0, e1;
    HIPC(hipEventCreate(&e0));
    HIPC(hipEventCreate(&e1));
    int best = -1;
    double best_us = 0.0;
    mhc_status st = MHC_OK;
    for (int v = 0; v < N_VARIANTS && st == MHC_OK; ++v) {
        Layout L;
        build_layout(scenes, n, v, ctx->max_waves(v, scenes, n), L, false, ctx->max_waves_staged(v, scenes, n));
        st = ensure_device(ctx, L.total_bytes);
        if (st != MHC_OK) break;
        char *base = static_cast<char *>(ctx->dbuf);
        std::vector<char> img(L.image_bytes);
        pack_image(L, img.data());
        hipError_t e = hipMemcpy(base, img.data(), L.image_bytes, hipMemcpyHostToDevice);
        Launch X = make_launch(L, base, nullptr, false, ctx->n_cu);
        double total_ms = 0.0;
        for (int r = 0; r <= reps && e == hipSuccess; ++r) {
            e = launch_trajgen(X, ctx->stream);
            if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
            if (e == hipSuccess) e = launch_collide(X, ctx->stream);
            if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (r > 0) total_ms += ms;  // launch 0 warms up
        }
        if (e != hipSuccess) {
            ctx->err = std::string("autotune launch: ") + hipGetErrorString(e);
            st = MHC_E_DEVICE;
            break;
        }
        const double t = total_ms * 1e3 / reps;
        if (us) us[v] = t;
        if (best < 0 || t < best_us) {
            best = v;
            best_us = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != MHC_OK) return st;
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
