// Host-side runtime structures (not part of the public ABI).
#pragma once

#include <array>
#include <functional>
#include <deque>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "mhc.h"
#include "mhc_internal.h"

namespace mhc {

constexpr int kMaxObjects = 4096;
constexpr int kMaxTimelineObjects = 64;   // one lane per collision object in the time-resolved risk kernel
constexpr int64_t kMaxObjectsPerLaunch = 65535;  // trajectory kernel grid y
constexpr int64_t kMaxTraj = 1 << 15;     // trajectories per object (T_a*T_b < 2^31)
constexpr int64_t kMaxPosesPerObject = int64_t(1) << 27;  // pose block < 2 GiB (32-bit buffer offsets)
constexpr int kDefaultVariant = 0;

// Result extents of one scene inside a (possibly multi-scene) layout.
struct SceneExt {
    int n_obj = 0, H = 0;
    int64_t obj0 = 0, traj0 = 0, n_traj = 0, hit0 = 0, n_hits = 0, q0 = 0;
    int64_t n_pairs = 0, checks = 0;
    bool timeline = false;
    int64_t tl_obj0 = 0, tl_traj0 = 0, tl_att0 = 0;  // first crit_t, traj_crit_t, attrib entries
};

// Host tables of one launch plus the byte layout of its device workspace:
// [scene image: tables uploaded in one copy][poses][p * 2^62][integer q sums][per-object counters]
// [p][first hits][q][traj crit][object crit]
// and, when a scene asks for the risk over time:
// [per-slot q sums][attribution scratch][criticality-over-time scratch]
// [crit_t][traj_crit_t][attrib][traj_attrib]
struct Layout {
    std::vector<DObj> objs;
    std::vector<double> vals;
    std::vector<DPair> pairs;
    std::vector<WorkItem> work;     // grouped by collision wave
    std::vector<int32_t> bins;       // [n_bins+1] range of each collision wave in `work`
    std::vector<DPoly> polys;        // polygons of the polygon pairs
    std::vector<SceneExt> sc;
    std::vector<int32_t> k1_rows;    // trajectory kernel rows (object, first block) when objects differ in size
    int64_t n_traj = 0, n_hits = 0, n_q = 0, n_obj = 0, n_checks = 0;
    int k1_x = 0;                 // trajectory kernel grid x (blocks of a row)
    int k1_nrows = 0;             // trajectory kernel grid y (rows)
    int k3_x = 0;                 // risk kernel grid x (chunks of the largest object)
    bool timeline = false;        // some scene asks for the risk over time
    int64_t n_hist = 0, n_tl_traj = 0, n_tl_obj = 0, n_tl_att = 0;
    int64_t k3t_x = 0;            // time-resolved risk kernel grid x (one wave of lanes of the largest object per workgroup)
    int k4t_y = 0;                // time-resolved reduction grid y (rows: slots + objects)
    size_t pose_bytes = 0;
    size_t o_objs = 0, o_vals = 0, o_pairs = 0, o_work = 0, o_bins = 0, o_k1rows = 0, o_polys = 0, image_bytes = 0;
    size_t value_bytes = 0;       // the image's leading part that fill_values rewrites (before the plan)
    size_t o_poses = 0, o_pfix = 0, o_qacc = 0, o_done = 0, o_p = 0, o_hits = 0, o_q = 0, o_tc = 0, o_oc = 0;
    size_t o_hist = 0, o_attw = 0, o_ctw = 0, o_ct = 0, o_tct = 0, o_at = 0, o_tat = 0, total_bytes = 0;
    int variant = 0;
    bool contiguous = false;      // collision plan of contiguous stretches
    int family = 0;               // ClassFamily covering every pair
    bool with_hits = true;        // the workspace holds the first-hit matrix
    bool one_track = false;       // some object follows the one-track model
    bool stage = false;           // the collision launch uses the LDS-staged instance
    double staged_share = 0.0;    // share of the collision cost in 8 x 8 blocks without a time split
};

// Instantiated HIP graphs keyed by what their launch sequence depends on.
struct GraphCache {
    static constexpr size_t kMaxGraphs = 16;
    static constexpr size_t kMaxSeen = 64;
    std::map<std::vector<int64_t>, hipGraphExec_t> graphs;
    std::vector<std::vector<int64_t>> order;  // insertion order, for eviction
    // keys launched without a graph, with the use count at their last launch
    std::deque<std::pair<std::vector<int64_t>, int64_t>> seen;
    int64_t uses = 0;                          // calls of repeated()
    hipStream_t capture = nullptr;
    ~GraphCache();
    void clear();
    hipError_t get(const std::vector<int64_t> &key, const std::function<hipError_t(hipStream_t)> &enqueue,
                   hipGraphExec_t *out);
    // Whether to launch `key` from a graph: it has one, or it comes back
    // within kMaxGraphs launches of its previous (direct) launch, so that a
    // graph captured now is likely still cached at its next use. Shapes used
    // once, or cycling through more shapes than the cache holds, never pay
    // for a capture.
    bool repeated(const std::vector<int64_t> &key);
};

bool validate_scene(const mhc_scene *s, std::string &err, int scene_index = -1);
// The time-resolved outputs of `r` (crit_t, traj_crit_t, attrib, traj_attrib)
// are only allowed for a scene with the timeline flag.
bool validate_outputs(const mhc_scene *s, const mhc_result *r, std::string &err, int scene_index = -1);
// Test class (CLS_*) of an object pair of kinds ka, kb under an overlap mode,
// given whether each has an outline.
int pair_class(int ka, int kb, int overlap, bool outline_a, bool outline_b);
// Relative VALU cost of one test of a class (k_a, k_b: polygon vertex counts).
double class_cost(int cls, int k_a, int k_b);
bool outline_ok(int k, const double *v);
bool scene_has_outline(const mhc_scene *s);
// The class family a scene needs (ClassFamily).
int scene_family(const mhc_scene *s);
// max_waves: resident waves of the collision kernel (0 = one per work unit).
// When the plan's 8 x 8 item blocks without a time split carry at least half
// its cost (plain class family, no risk over time), the launch uses the
// collision instance that stages them in LDS, and the plan is made for that
// instance's resident waves, max_waves_staged (0: the same as max_waves).
// max_tshift caps the time split of the plan's units (S <= 2^max_tshift).
void build_layout(const mhc_scene *scenes, int n_scenes, int variant, int max_waves, Layout &L, bool with_hits,
                  int max_waves_staged = 0, int max_tshift = MAX_TSHIFT);

// The host side of the results of the n scenes of a layout: per output, the
// workspace range [lo, hi) of every requested part and, where staged, its
// offset in a pinned buffer of `staged` bytes (else copied per scene straight
// to the callers' buffers). stage_all stages every output.
struct ResultPlan {
    static constexpr int kOutputs = 9;
    size_t lo[kOutputs], hi[kOutputs], at[kOutputs];
    bool stage[kOutputs];
    size_t staged = 0;
    // staged outputs that lie close together in the workspace come down as
    // one transfer: [copy_lo, copy_hi) of the workspace to pinned + copy_at
    int n_copies = 0;
    size_t copy_lo[kOutputs], copy_hi[kOutputs], copy_at[kOutputs];
};
ResultPlan plan_results(const Layout &L, int n, const mhc_result *res, bool stage_all);
// Enqueues the transfers on s: staged outputs into `pinned`, the others to res.
hipError_t enqueue_results(const ResultPlan &R, const Layout &L, int n, const char *dbase, char *pinned,
                           const mhc_result *res, hipStream_t s);
// After the transfers: copies each scene's staged parts from `pinned` to res.
void scatter_results(const ResultPlan &R, const Layout &L, int n, const char *pinned, const mhc_result *res);
// Per-scene origin subtracted from the positions before they go to the GPU
// (a multiple of 256 m near the middle of the initial positions).
void scene_origin(const mhc_scene &s, double *ox, double *oy);
void fill_values(const mhc_scene *scenes, int n_scenes, Layout &L);
// values_only: only the leading value_bytes (the collision plan is left out).
void pack_image(const Layout &L, char *dst, bool values_only = false);
std::vector<int32_t> shape_of(const mhc_scene *s);
Launch make_launch(const Layout &L, char *base, const mhc_result *dev_out, bool keep_hits, int n_cu);
hipError_t launch_all(const Launch &X, hipStream_t s);

// The collision kernel's tile-variant choices: a forced variant, else the
// autotuned one of the launch's size class, else the default. A context owns
// one; a server copies it when it starts.
struct Tuning {
    int forced_variant = -1;                      // mhc_set_variant
    std::map<std::array<int, 4>, int> tuned;      // size class -> variant (mhc_autotune, mhc_autotune_batch)
    int variant_for(const mhc_scene *scenes, int n) const;
};

}  // namespace mhc

struct mhc_ctx {
    int device = 0;
    int n_cu = 0;
    size_t budget = 0;
    hipStream_t stream = nullptr;
    std::string err;
    void *dbuf = nullptr;         // workspace of the synchronous entry points
    size_t dbuf_bytes = 0;
    char *staging = nullptr;      // pinned host copy of the last scene image
    size_t staging_bytes = 0;
    hipEvent_t staging_ev = nullptr;
    char *res_pin = nullptr;      // pinned host staging of the results of the synchronous calls
    size_t res_pin_bytes = 0;
    char *scratch = nullptr;      // this GPU's address of the allocation-free workspace
    mhc::Layout noalloc_layout;   // host tables of mhc_evaluate_noalloc (storage reused)
    std::vector<char> noalloc_image;   // its scene image (pageable host memory)
    hipEvent_t noalloc_ev = nullptr;   // the last upload from noalloc_image has left it
    mhc::Layout layout;           // reused by mhc_evaluate
    std::vector<int32_t> layout_shape;  // shape (+ variant, waves) `layout` was built for
    // launch key (+ workspace address) of the single-scene image whose
    // collision plan is in the workspace now; empty when other work wrote it
    std::vector<int64_t> resident_image;
    mhc::GraphCache batch_graphs;                 // mhc_evaluate_batch, keyed by batch shape
    mhc::Tuning tune;
    int variant_for(const mhc_scene *scenes, int n) const { return tune.variant_for(scenes, n); }
    int waves_cache[mhc::N_VARIANTS][3][2][2] = {};  // [variant][class family][time-resolved][staged]
    // resident waves on this GPU of the collision kernel that `scenes` need
    // (of its LDS-staged instance: max_waves_staged, 0 where there is none)
    int max_waves(int variant, const mhc_scene *scenes, int n);
    int max_waves_staged(int variant, const mhc_scene *scenes, int n);
    // the same for a variant, class family, time-resolved flag and staging
    int max_waves_of(int variant, int family, bool timeline, bool stage = false);
};

// Autotuning class of a launch: log2 of the mean trajectory count, log2 of
// the mean horizon, the test family (0 rectangles and circles, 1 the
// point-in-polygon rectangle test, 2 outlines) and log2 of the scene count
// (0 for single scenes, so batches are tuned apart from them).
std::array<int, 4> size_class(const mhc_scene *scenes, int n);

mhc_status ensure_device(mhc_ctx *ctx, size_t bytes);
// Copies the results of the n scenes of layout L (device workspace dbase,
// written on stream s) to the callers' host buffers res[0..n) and waits for
// them.
mhc_status download_results(mhc_ctx *ctx, const mhc::Layout &L, int n, const char *dbase, const mhc_result *res,
                            hipStream_t s);
mhc_status batch_run(mhc_ctx *ctx, int n, const mhc_scene *scenes, mhc_result *res);
