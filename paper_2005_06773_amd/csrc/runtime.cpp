// Host runtime behind the C ABI: scene ingest (validation, pair list, work
// list), packing of the scene image, device memory, launches, and the plain,
// asynchronous, plan and batched entry points.
#include "runtime.h"

#include <algorithm>
#include <functional>
#include <queue>
#include <cmath>
#include <numeric>
#include <cstdio>
#include <cstdint>
#include <climits>
#include <cstring>
#include <string>
#include <vector>

namespace mhc {

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int pair_class(int ka, int kb, int overlap, bool outline_a, bool outline_b)
{
    if (outline_a || outline_b) {
        // a polygon on either side: vehicles are polygons (rectangles by their corners)
        if (ka == KIND_VEHICLE && kb == KIND_VEHICLE) return overlap == MHC_OVERLAP_PIP ? CLS_GG_PIP : CLS_GG;
        if (ka == KIND_VEHICLE) return CLS_GC;
        return CLS_CG;
    }
    if (overlap == MHC_OVERLAP_PIP) return CLS_VV_PIP;  // validated: vehicles only
    if (ka == KIND_VEHICLE && kb == KIND_VEHICLE) return CLS_VV;
    if (ka == KIND_VEHICLE) return CLS_VP;
    if (kb == KIND_VEHICLE) return CLS_PV;
    return CLS_PP;
}

bool scene_has_outline(const mhc_scene *s)
{
    for (int a = 0; a < s->n_objects; ++a)
        if (s->objects[a].n_vertices > 0) return true;
    return false;
}

int scene_family(const mhc_scene *s)
{
    if (scene_has_outline(s)) return FAM_POLY;
    return s->overlap == MHC_OVERLAP_PIP ? FAM_PIP : FAM_PLAIN;
}

// Relative VALU cost of one check per class, for longest-first ordering; the
// polygon classes scale with the vertex counts (class_cost).
static const double kClsCost[N_CLS] = {25.0, 12.0, 12.0, 6.4, 60.0, 0.0, 0.0, 0.0, 0.0};

double class_cost(int cls, int k_a, int k_b)
{
    switch (cls) {
    case CLS_GG:
    case CLS_GG_PIP: return 14.0 + 4.0 * (k_a + k_b) + 6.0 * k_a * k_b;
    case CLS_GC: return 8.0 + 13.0 * k_a;
    case CLS_CG: return 8.0 + 13.0 * k_b;
    default: return kClsCost[cls];
    }
}

// Padded vertex count of an object's polygon in a polygon pair (4 for a
// rectangle, 4 or 8 for an outline).
static int padded_vertices(int n) { return n <= 4 ? 4 : MAX_VERTICES; }
static int poly_vertices(const mhc_object &o) { return padded_vertices(o.n_vertices > 0 ? o.n_vertices : 4); }
// Per-unit cost outside the step loop (setup, result stores), same units.
static const double kUnitOverhead = 120.0;
// From this many work units per collision wave on, waves take contiguous
// stretches of the unit sequence instead of individually packed units.
static const int kContiguousUnitsPerWave = 8;
// Below this many work units per resident collision wave, units are split in
// time (up to S = 8 parts side by side in a wave) to get more, shorter
// units. Around one unit per wave the split costs more than it balances
// (measured on the 11-object scene: 40.5 us with S = 2 against 37.0 us).
static const double kSplitBelowUnitsPerWave = 0.75;

// Collision units of a pair with time split 2^tshift (E = 64 >> tshift items
// per unit): E consecutive items of the row-major item grid (bshift = 0), or
// blocks of E >> bshift item rows by 2^bshift item columns.
static int64_t pair_units(const DPair &pr, int tshift, int bshift)
{
    const int64_t per = WAVE >> tshift;
    if (bshift == 0) return ((int64_t)pr.n_ig * pr.n_jg + per - 1) / per;
    const int64_t rows = per >> bshift, cols = (int64_t)1 << bshift;
    return ((pr.n_ig + rows - 1) / rows) * ((pr.n_jg + cols - 1) / cols);
}

// Unit shape of a pair. A row-major unit reads, at every step, the poses of
// one or two a-items and of E b-items; a block of 8 x 8 items reads 8 of each,
// about a third of the cache lines, which matters once the scene's poses no
// longer fit in an XCD's L2. Blocks are taken where they add at most 1/32 of
// idle lanes (grids whose sides are near multiples of the block's).
static int unit_shape(const DPair &pr, int tshift)
{
    const int64_t lin = pair_units(pr, tshift, 0);
    int best = 0;
    int64_t best_u = 0;
    for (int bs = 3; bs <= 4; ++bs) {  // 8 or 16 item columns
        if (((WAVE >> tshift) >> bs) < 1) break;
        const int64_t u = pair_units(pr, tshift, bs);
        if (u * 32 <= lin * 33 && (best == 0 || u < best_u)) {
            best = bs;
            best_u = u;
        }
    }
    return best;
}

// Steps per part of a unit with time split 2^tshift: ceil(H / S).
static int split_chunk(int H, int tshift) { return (H + (1 << tshift) - 1) >> tshift; }

// A split fits a horizon when every part has a step and the parts' overlap
// (S * ceil(H / S) - H steps tested twice) is at most an eighth of H.
static bool split_fits(int H, int tshift)
{
    const int S = 1 << tshift;
    return S <= H && 8 * (S * split_chunk(H, tshift) - H) <= H;
}

static bool finite(double v) { return std::isfinite(v); }

// ---------------------------------------------------------------------------
// Ingest: validation. Every rule here is checked before anything is launched.
// ---------------------------------------------------------------------------

// A vehicle outline: finite, strictly convex and counter-clockwise (every
// turn to the left), each interior angle at least 45 degrees (so that a
// vertex outside another polygon by more than the test tolerance is outside
// one of its edge lines by a comparable distance).
bool outline_ok(int k, const double *v)
{
    for (int e = 0; e < 2 * k; ++e)
        if (!finite(v[e])) return false;
    const double cos45 = std::sqrt(0.5);
    for (int e = 0; e < k; ++e) {
        const int p = (e + k - 1) % k, q = (e + 1) % k;
        const double ax = v[2 * e] - v[2 * p], ay = v[2 * e + 1] - v[2 * p + 1];   // incoming edge
        const double bx = v[2 * q] - v[2 * e], by = v[2 * q + 1] - v[2 * e + 1];   // outgoing edge
        if (!(ax * by - ay * bx > 0.0)) return false;                              // left turn
        // interior angle between -a and b
        const double la = std::hypot(ax, ay), lb = std::hypot(bx, by);
        if (!(la > 0.0) || !(lb > 0.0)) return false;
        const double cosint = (-ax * bx - ay * by) / (la * lb);
        if (cosint > cos45) return false;
    }
    return true;
}
bool validate_scene(const mhc_scene *s, std::string &err, int scene_index)
{
    char buf[256];
    auto fail = [&](const char *fmt, int a) {
        if (scene_index >= 0) {
            char b2[200];
            snprintf(b2, sizeof b2, fmt, a);
            snprintf(buf, sizeof buf, "scene %d: %s", scene_index, b2);
        } else {
            snprintf(buf, sizeof buf, fmt, a);
        }
        err = buf;
        return false;
    };
    if (!s) return fail("scene is NULL%.0d", 0);
    if (s->n_objects < 2) return fail("n_objects must be >= 2 (got %d)", s->n_objects);
    if (s->n_objects > kMaxObjects) return fail("n_objects must be <= %d", kMaxObjects);
    if (!s->objects) return fail("objects is NULL%.0d", 0);
    if (s->horizon < 1 || s->horizon > 32767) return fail("horizon must be in [1, 32767] (got %d)", s->horizon);
    if (!finite(s->dt) || !(s->dt > 0.0)) return fail("dt must be finite and > 0%.0d", 0);
    if (s->pairs != MHC_PAIRS_ALL && s->pairs != MHC_PAIRS_EGO) return fail("pairs must be 0 or 1 (got %d)", s->pairs);
    if (s->overlap != MHC_OVERLAP_EXACT && s->overlap != MHC_OVERLAP_PIP)
        return fail("overlap must be 0 or 1 (got %d)", s->overlap);
    if (s->risk != MHC_RISK_EXCLUSIVE && s->risk != MHC_RISK_INDEPENDENT)
        return fail("risk must be 0 or 1 (got %d)", s->risk);
    if (s->timeline != 0 && s->timeline != 1) return fail("timeline must be 0 or 1 (got %d)", s->timeline);
    if (s->timeline && s->n_objects > kMaxTimelineObjects)
        return fail("a time-resolved scene has at most %d objects", kMaxTimelineObjects);
    for (int a = 0; a < s->n_objects; ++a) {
        const mhc_object &o = s->objects[a];
        if (o.kind != MHC_VEHICLE && o.kind != MHC_PEDESTRIAN) return fail("object %d: kind must be 0 or 1", a);
        if (!finite(o.x) || !finite(o.y) || !finite(o.heading) || !finite(o.speed))
            return fail("object %d: state must be finite", a);
        if (!(o.speed >= 0.0)) return fail("object %d: speed must be >= 0", a);
        if (o.model != MHC_MODEL_KINEMATIC && o.model != MHC_MODEL_PED_ACCEL && o.model != MHC_MODEL_ONE_TRACK)
            return fail("object %d: model must be 0, 1 or 2", a);
        if (o.model == MHC_MODEL_PED_ACCEL) {
            if (o.kind != MHC_PEDESTRIAN) return fail("object %d: the acceleration model is for pedestrians", a);
            if (!finite(o.params[0]) || !(o.params[0] > 0.0)) return fail("object %d: v_max must be finite and > 0", a);
        }
        if (o.model == MHC_MODEL_ONE_TRACK) {
            if (o.kind != MHC_VEHICLE) return fail("object %d: the one-track model is for vehicles", a);
            for (int k = 0; k < 6; ++k)
                if (!finite(o.params[k]) || !(o.params[k] > 0.0))
                    return fail("object %d: one-track parameters must be finite and > 0", a);
            if (o.params[3] * o.params[1] < o.params[2] * o.params[0])
                return fail("object %d: the one-track parameters must understeer (l_r c_r >= l_f c_f)", a);
        }
        if (o.n_vertices != 0) {
            if (o.kind != MHC_VEHICLE) return fail("object %d: only vehicles take an outline", a);
            if (o.n_vertices < 3 || o.n_vertices > MHC_MAX_VERTICES)
                return fail("object %d: an outline has 3 to 8 vertices", a);
            if (!o.vertices) return fail("object %d: outline vertices must not be NULL", a);
            if (!outline_ok(o.n_vertices, o.vertices))
                return fail("object %d: the outline must be finite, strictly convex, counter-clockwise, "
                            "with interior angles >= 45 degrees", a);
        } else if (o.kind == MHC_VEHICLE) {
            if (!finite(o.length) || !(o.length > 0.0) || !finite(o.width) || !(o.width > 0.0))
                return fail("object %d: vehicle length and width must be finite and > 0", a);
        } else {
            if (!finite(o.radius) || !(o.radius > 0.0)) return fail("object %d: pedestrian radius must be finite and > 0", a);
        }
        if (o.n_u < 1 || o.n_w < 1) return fail("object %d: n_u and n_w must be >= 1", a);
        if ((int64_t)o.n_u * o.n_w > kMaxTraj) return fail("object %d: n_u*n_w exceeds the trajectory limit", a);
        if ((int64_t)o.n_u * o.n_w * s->horizon > kMaxPosesPerObject)
            return fail("object %d: horizon * n_u * n_w exceeds the per-object pose limit (2^27)", a);
        if (!o.u || !o.w) return fail("object %d: control grids u and w must not be NULL", a);
        for (int k = 0; k < o.n_u; ++k)
            if (!finite(o.u[k])) return fail("object %d: control grid u must be finite", a);
        for (int k = 0; k < o.n_w; ++k)
            if (!finite(o.w[k])) return fail("object %d: control grid w must be finite", a);
        if (o.score) {
            double l1 = 0.0;
            const int T = o.n_u * o.n_w;
            for (int k = 0; k < T; ++k) {
                if (!finite(o.score[k]) || !(o.score[k] >= 0.0)) return fail("object %d: scores must be finite and >= 0", a);
                l1 += o.score[k];
            }
            if (!(l1 > 0.0) || !finite(l1)) return fail("object %d: scores must have a positive finite sum", a);
        }
    }
    if (s->objects[0].kind != MHC_VEHICLE && s->pairs == MHC_PAIRS_EGO)
        return fail("EGO pair mode needs object 0 to be a vehicle%.0d", 0);
    if (s->overlap == MHC_OVERLAP_PIP)
        for (int a = 0; a < s->n_objects; ++a)
            if (s->objects[a].kind != MHC_VEHICLE)
                return fail("object %d: the point-in-polygon overlap test needs every object to be a vehicle", a);
    return true;
}

bool validate_outputs(const mhc_scene *s, const mhc_result *r, std::string &err, int scene_index)
{
    if (!r || s->timeline) return true;
    if (r->crit_t || r->traj_crit_t || r->attrib || r->traj_attrib) {
        err = (scene_index >= 0 ? "scene " + std::to_string(scene_index) + ": " : std::string()) +
              "crit_t, traj_crit_t, attrib and traj_attrib need a scene with timeline = 1";
        return false;
    }
    return true;
}

// ---------------------------------------------------------------------------
// Ingest: pair list, work list and the packed scene image.
// ---------------------------------------------------------------------------
static void pair_list(const mhc_scene *s, std::vector<std::pair<int, int>> &out)
{
    out.clear();
    for (int a = 0; a < s->n_objects; ++a)
        for (int b = a + 1; b < s->n_objects; ++b)
            if (s->pairs == MHC_PAIRS_ALL || a == 0) out.emplace_back(a, b);
}

// Empties a layout for the next build. Its tables keep their storage: a
// batch's tables span megabytes, and freshly allocated ones would be paged in
// again on every launch (about half of the host time of a 64-scene launch).
static void reset_layout(Layout &L)
{
    Layout fresh;
    auto keep = [](auto &to, auto &from) {
        to = std::move(from);
        to.clear();
    };
    keep(fresh.objs, L.objs);
    keep(fresh.vals, L.vals);
    keep(fresh.pairs, L.pairs);
    keep(fresh.work, L.work);
    keep(fresh.bins, L.bins);
    keep(fresh.polys, L.polys);
    keep(fresh.sc, L.sc);
    keep(fresh.k1_rows, L.k1_rows);
    L = std::move(fresh);
}

static void build_layout_once(const mhc_scene *scenes, int n_scenes, int variant, int max_waves, Layout &L,
                              bool with_hits, int max_tshift);

void build_layout(const mhc_scene *scenes, int n_scenes, int variant, int max_waves, Layout &L, bool with_hits,
                  int max_waves_staged, int max_tshift)
{
    max_tshift = std::min(std::max(max_tshift, 0), MAX_TSHIFT);
    build_layout_once(scenes, n_scenes, variant, max_waves, L, with_hits, max_tshift);
    const bool stage = L.family == FAM_PLAIN && !L.timeline && max_waves > 0 && L.staged_share >= 0.5;
    if (stage && max_waves_staged > 0 && max_waves_staged != max_waves)
        build_layout_once(scenes, n_scenes, variant, max_waves_staged, L, with_hits, max_tshift);
    L.stage = stage;
}

static void build_layout_once(const mhc_scene *scenes, int n_scenes, int variant, int max_waves, Layout &L,
                              bool with_hits, int max_tshift)
{
    reset_layout(L);
    L.variant = variant;
    L.with_hits = with_hits;
    struct PairCost {
        double c;        // cost of one of the pair's work units
        int32_t pidx;
        int32_t n_units;
    };
    std::vector<PairCost> costs;
    std::vector<std::pair<int, int>> plist;
    std::vector<int> pair_vertices;   // per pair: polygon vertex counts of a and b
    for (int k = 0; k < n_scenes; ++k) {
        const mhc_scene &s = scenes[k];
        const int n = s.n_objects;
        SceneExt ext{};
        ext.n_obj = n;
        ext.H = s.horizon;
        ext.obj0 = L.n_obj;
        ext.traj0 = L.n_traj;
        ext.hit0 = L.n_hits;
        ext.q0 = L.n_q;
        ext.timeline = s.timeline != 0;
        ext.tl_obj0 = L.n_tl_obj;
        ext.tl_traj0 = L.n_tl_traj;
        ext.tl_att0 = L.n_tl_att;
        L.timeline |= ext.timeline;
        const int obj_base = (int)L.objs.size();
        int64_t toff = 0;
        for (int a = 0; a < n; ++a) {
            const mhc_object &o = s.objects[a];
            DObj d{};
            d.kind = o.kind;
            d.n_u = o.n_u;
            d.n_w = o.n_w;
            d.T = o.n_u * o.n_w;
            d.has_score = o.score != nullptr;
            d.H = s.horizon;
            d.local = a;
            d.n_scene_obj = n;
            d.risk = s.risk;
            d.timeline = s.timeline;
            d.model = o.model;
            L.one_track |= o.model == MHC_MODEL_ONE_TRACK;
            if (s.timeline) {
                int W = 1;
                while (W < n) W <<= 1;
                d.tl_w = W;
                d.hist_off = L.n_hist;
                d.tl_traj = L.n_tl_traj;
                d.tl_obj = L.n_tl_obj;
                d.tl_att = L.n_tl_att;
                L.n_hist += (int64_t)W * s.horizon * d.T;
                L.k3t_x = std::max<int64_t>(L.k3t_x, ((int64_t)d.T * W + WAVE - 1) / WAVE);
                L.k4t_y = std::max(L.k4t_y, s.horizon + n);
                L.n_tl_traj += (int64_t)s.horizon * d.T;
                L.n_tl_obj += s.horizon;
                L.n_tl_att += n;
            }
            d.traj_off = L.n_traj + toff;
            d.q_row = L.n_q + toff * n;
            d.pose_off = (int64_t)L.pose_bytes;
            L.pose_bytes += align256((size_t)s.horizon * d.T * (o.kind == MHC_VEHICLE ? 16 : 8));
            d.frame_off = -1;
            if (o.kind == MHC_VEHICLE) {
                d.frame_off = (int64_t)L.pose_bytes;
                L.pose_bytes += align256((size_t)s.horizon * d.T * 16);
            }
            d.u_off = (int64_t)L.vals.size();
            d.w_off = d.u_off + o.n_u;
            d.score_off = d.w_off + o.n_w;
            L.vals.resize(L.vals.size() + o.n_u + o.n_w + (o.score ? d.T : 0));
            d.obj_out = L.n_obj + a;
            L.k3_x = std::max(L.k3_x, (d.T + WG - 1) / WG);
            L.objs.push_back(d);
            toff += d.T;
        }
        // polygons: with an outline anywhere in the scene, every vehicle of the
        // scene gets one (its rectangle's corners if it has no outline)
        std::vector<int32_t> poly_of(n, -1);
        if (scene_has_outline(&s))
            for (int a = 0; a < n; ++a)
                if (s.objects[a].kind == MHC_VEHICLE) {
                    poly_of[a] = (int32_t)L.polys.size();
                    L.polys.push_back(DPoly{});
                }
        pair_list(&s, plist);
        int64_t hoff = 0;
        for (auto &ab : plist) {
            const int a = ab.first, b = ab.second;
            const mhc_object &oa = s.objects[a], &ob = s.objects[b];
            DPair pr{};
            pr.a = obj_base + a;
            pr.b = obj_base + b;
            pr.cls = pair_class(oa.kind, ob.kind, s.overlap, oa.n_vertices > 0, ob.n_vertices > 0);
            pr.poly_a = poly_of[a];
            pr.poly_b = poly_of[b];
            pair_vertices.push_back(poly_vertices(oa));
            pair_vertices.push_back(poly_vertices(ob));
            L.family = std::max(L.family, class_family(pr.cls));
            pr.H = s.horizon;
            pr.Ta = oa.n_u * oa.n_w;
            pr.Tb = ob.n_u * ob.n_w;
            const TileShape ts = kTiles[variant][pr.cls];
            pr.n_ig = (pr.Ta + ts.ri - 1) / ts.ri;
            pr.n_jg = (pr.Tb + ts.rj - 1) / ts.rj;
            pr.hit_off = L.n_hits + hoff;
            // the rectangle-rectangle tests take b's pose in b's frame, the
            // rectangle-circle tests the rectangle's (frame blocks)
            const bool frame_a = pr.cls == CLS_VP;
            const bool frame_b = pr.cls == CLS_VV || pr.cls == CLS_VV_PIP || pr.cls == CLS_PV;
            pr.pose_a = frame_a ? L.objs[obj_base + a].frame_off : L.objs[obj_base + a].pose_off;
            pr.pose_b = frame_b ? L.objs[obj_base + b].frame_off : L.objs[obj_base + b].pose_off;
            pr.qn = n;
            pr.qa0 = L.objs[obj_base + a].q_row + b;
            pr.qb0 = L.objs[obj_base + b].q_row + a;
            pr.pa_off = L.objs[obj_base + a].traj_off;
            pr.pb_off = L.objs[obj_base + b].traj_off;
            pr.timeline = s.timeline;
            if (s.timeline) {
                pr.hwa = L.objs[obj_base + a].tl_w;
                pr.hwb = L.objs[obj_base + b].tl_w;
                pr.ha0 = L.objs[obj_base + a].hist_off + b;
                pr.hb0 = L.objs[obj_base + b].hist_off + a;
            }
            L.pairs.push_back(pr);
            hoff += (int64_t)pr.Ta * pr.Tb;
            ext.checks += (int64_t)pr.Ta * pr.Tb * s.horizon;
        }
        ext.n_traj = toff;
        ext.n_hits = hoff;
        ext.n_pairs = (int64_t)plist.size();
        L.sc.push_back(ext);
        L.n_traj += toff;
        L.n_hits += hoff;
        L.n_q += toff * n;
        L.n_obj += n;
        L.n_checks += ext.checks;
    }
    // Trajectory kernel grid. An object takes a normalisation block and a
    // block per K1_TPB trajectories. With objects of one size the grid is
    // (blocks, objects); otherwise rows of as many blocks as the smallest
    // object has, each row a stretch of one object's blocks (the row table),
    // so that no workgroup of a large object's extent is launched for a small
    // one (empty workgroups cost dispatch time).
    {
        int bmin = INT_MAX, bmax = 0;
        for (const DObj &d : L.objs) {
            const int b = (d.T + K1_TPB - 1) / K1_TPB + 1;
            bmin = std::min(bmin, b);
            bmax = std::max(bmax, b);
        }
        L.k1_x = bmax;
        L.k1_nrows = (int)L.objs.size();
        if (bmin < bmax) {
            int B = bmin;
            auto rows_of = [&](int w) {
                int64_t r = 0;
                for (const DObj &d : L.objs) r += ((d.T + K1_TPB - 1) / K1_TPB + 1 + w - 1) / w;
                return r;
            };
            while (rows_of(B) > 65535) B *= 2;  // the grid's y extent
            for (int a = 0; a < (int)L.objs.size(); ++a) {
                const int b = (L.objs[a].T + K1_TPB - 1) / K1_TPB + 1;
                for (int s0 = 0; s0 < b; s0 += B) {
                    L.k1_rows.push_back(a);
                    L.k1_rows.push_back(s0);
                }
            }
            L.k1_x = B;
            L.k1_nrows = (int)(L.k1_rows.size() / 2);
        }
    }
    // Time split. With few units for the resident waves, a unit's steps are
    // cut into S parts that run side by side in one wave (64/S items,
    // ceil(H/S) steps per lane): S times as many, S times shorter units, which
    // the packing below can spread evenly and which fill the GPU. S is the
    // smallest of 1, 2, 4, 8 that gives enough units (the largest allowed for
    // the size bound, max_waves = 0), lowered per pair until it fits the
    // horizon (split_fits).
    int want = max_tshift;
    if (max_waves > 0) {
        for (want = 0; want < max_tshift; ++want) {
            int64_t u = 0;
            for (const DPair &pr : L.pairs) u += pair_units(pr, want, 0);
            if ((double)u >= kSplitBelowUnitsPerWave * max_waves) break;
        }
    }
    for (size_t pidx = 0; pidx < L.pairs.size(); ++pidx) {
        DPair &pr = L.pairs[pidx];
        int sh = want;
        while (sh > 0 && !split_fits(pr.H, sh)) --sh;
        pr.tshift = sh;
        pr.bshift = unit_shape(pr, sh);
        const TileShape ts = kTiles[variant][pr.cls];
        const int ka = pr.poly_a >= 0 ? pair_vertices[2 * pidx] : 0, kb = pr.poly_b >= 0 ? pair_vertices[2 * pidx + 1] : 0;
        // a wave executes every step of every test of a unit, whether or
        // not all of its lanes hold an item
        // (rectangle-rectangle and rectangle-circle tests: 25 and 12 VALU each,
        // the rectangle's frame read ready from its frame block)
        const double per_test = class_cost(pr.cls, ka, kb);
        const double unit_cost = (double)ts.ri * ts.rj * split_chunk(pr.H, sh) * per_test + kUnitOverhead;
        costs.push_back(PairCost{unit_cost, (int32_t)pidx, (int32_t)pair_units(pr, sh, pr.bshift)});
    }

    // Collision plan: every wave slot gets a list of segments of work units.
    int64_t n_units = 0;
    double total_cost = 0.0, staged_cost = 0.0;
    for (const PairCost &pc : costs) {
        n_units += pc.n_units;
        total_cost += pc.c * pc.n_units;
        const DPair &pr = L.pairs[pc.pidx];
        if (pr.bshift == 3 && pr.tshift == 0) staged_cost += pc.c * pc.n_units;
    }
    L.staged_share = total_cost > 0.0 ? staged_cost / total_cost : 0.0;
    const int n_bins = (int)std::max<int64_t>(1, std::min<int64_t>(n_units, max_waves > 0 ? max_waves : n_units));
    L.work.clear();
    L.bins.assign(n_bins + 1, 0);
    L.contiguous = n_units >= (int64_t)kContiguousUnitsPerWave * n_bins;
    if (L.contiguous) {
        // Many units per wave: each slot takes the next stretch of the unit
        // sequence (pairs in scene order) worth total/n_bins of cost, so the
        // plan is O(pairs + waves) and neighbouring slots, which sit on one
        // XCD, work on neighbouring pairs.
        const double per_slot = total_cost / n_bins;
        size_t p = 0;
        int32_t u = 0;
        double acc = 0.0;
        for (int sl = 0; sl < n_bins; ++sl) {
            L.bins[sl] = (int32_t)L.work.size();
            const double goal = (sl + 1) * per_slot;
            while (p < costs.size()) {
                const PairCost &pc = costs[p];
                const int32_t left = pc.n_units - u;
                int32_t k = left;
                if (sl < n_bins - 1) {
                    const double want = std::floor((goal - acc) / pc.c + 0.5);
                    k = (int32_t)std::max(0.0, std::min((double)left, want));
                }
                if (k > 0) {
                    L.work.push_back(WorkItem{pc.pidx, u * (WAVE >> L.pairs[pc.pidx].tshift), k, 0});
                    acc += pc.c * k;
                    u += k;
                }
                if (u == pc.n_units) {
                    ++p;
                    u = 0;
                } else {
                    break;
                }
            }
        }
    } else {
        // Few units per wave: longest first, each to the least-loaded wave.
        // Units of one pair shape cost the same, so the list splits into a
        // few groups of equal cost: unit g of a group goes to the wave at
        // position g mod n_bins of the (load, index) order, i.e. every wave
        // once per full round and the remainder to the least-loaded ones.
        std::vector<PairCost> sorted(costs);
        std::stable_sort(sorted.begin(), sorted.end(), [](const PairCost &x, const PairCost &y) { return x.c > y.c; });
        std::vector<WorkItem> units((size_t)n_units);
        std::vector<int32_t> unit_bin((size_t)n_units);
        std::vector<double> load((size_t)n_bins, 0.0);
        std::vector<int32_t> order((size_t)n_bins), merged((size_t)n_bins);
        for (int b = 0; b < n_bins; ++b) order[b] = b;
        auto before = [&](int32_t x, int32_t y) { return load[x] < load[y] || (load[x] == load[y] && x < y); };
        int64_t k = 0;
        size_t p0 = 0;
        while (p0 < sorted.size()) {
            size_t p1 = p0;
            int64_t m_total = 0;
            while (p1 < sorted.size() && sorted[p1].c == sorted[p0].c) m_total += sorted[p1++].n_units;
            const double c = sorted[p0].c;
            const int64_t full = m_total / n_bins, rem = m_total % n_bins;
            int pos = 0;
            for (size_t pp = p0; pp < p1; ++pp)
                for (int32_t u = 0; u < sorted[pp].n_units; ++u, ++k) {
                    units[k] = WorkItem{sorted[pp].pidx, u * (WAVE >> L.pairs[sorted[pp].pidx].tshift), 1, 0};
                    unit_bin[k] = order[pos];
                    if (++pos == n_bins) pos = 0;
                }
            for (int b = 0; b < n_bins; ++b) load[b] += c * full;
            for (int64_t i = 0; i < rem; ++i) load[order[i]] += c;
            if (rem > 0) {
                // the first `rem` waves stay sorted among themselves after the
                // increment, so one merge restores the order
                std::merge(order.begin() + rem, order.end(), order.begin(), order.begin() + rem, merged.begin(), before);
                order.swap(merged);
            }
            p0 = p1;
        }
        // group the units by wave (longest first inside each wave)
        for (int64_t i = 0; i < n_units; ++i) ++L.bins[unit_bin[i] + 1];
        for (int b = 0; b < n_bins; ++b) L.bins[b + 1] += L.bins[b];
        L.work.resize((size_t)n_units);
        std::vector<int32_t> fill(L.bins.begin(), L.bins.end() - 1);
        for (int64_t i = 0; i < n_units; ++i) L.work[fill[unit_bin[i]]++] = units[i];
    }
    L.bins[n_bins] = (int32_t)L.work.size();

    size_t off = 0;
    auto put = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    // the tables fill_values rewrites come first, the collision plan (which
    // depends on the shapes only) last
    L.o_objs = put(L.objs.size() * sizeof(DObj));
    L.o_vals = put(L.vals.size() * sizeof(double));
    L.o_pairs = put(L.pairs.size() * sizeof(DPair));
    L.o_polys = put(L.polys.size() * sizeof(DPoly));
    L.value_bytes = off;
    L.o_work = put(L.work.size() * sizeof(WorkItem));
    L.o_bins = put(L.bins.size() * sizeof(int32_t));
    L.o_k1rows = put(L.k1_rows.size() * sizeof(int32_t));
    L.image_bytes = off;
    L.o_poses = put(L.pose_bytes);
    L.o_pfix = put((size_t)L.n_traj * sizeof(unsigned long long));
    L.o_qacc = put((size_t)L.n_q * sizeof(unsigned long long));
    L.o_done = put((size_t)L.n_obj * sizeof(unsigned long long));
    // the outputs most calls ask for are neighbours, so they come down together
    L.o_p = put((size_t)L.n_traj * sizeof(double));
    L.o_tc = put((size_t)L.n_traj * sizeof(double));
    L.o_oc = put((size_t)L.n_obj * sizeof(double));
    L.o_q = put((size_t)L.n_q * sizeof(double));
    L.o_hits = put(with_hits ? (size_t)L.n_hits * sizeof(int16_t) : 0);
    const size_t tq = L.timeline ? (size_t)L.n_q : 0;
    L.o_hist = put((size_t)L.n_hist * sizeof(unsigned long long));
    L.o_attw = put(tq * sizeof(double));
    L.o_ctw = put((size_t)L.n_tl_traj * sizeof(double));
    L.o_ct = put((size_t)L.n_tl_obj * sizeof(double));
    L.o_tct = put((size_t)L.n_tl_traj * sizeof(double));
    L.o_at = put((size_t)L.n_tl_att * sizeof(double));
    L.o_tat = put(tq * sizeof(double));
    L.total_bytes = off;
    fill_values(scenes, n_scenes, L);
}

// The value part of a layout: states, control grids, scores and extents.
// Everything else in a layout depends only on the scene shapes.
// The test constants of a vehicle's polygon: its outline, or the corners of
// its rectangle, counter-clockwise in the body frame (FP64, then FP32).
static void fill_poly(const mhc_object &o, DPoly &g)
{
    double vx[MAX_VERTICES], vy[MAX_VERTICES];
    int k;
    if (o.n_vertices > 0) {
        k = o.n_vertices;
        for (int e = 0; e < k; ++e) {
            vx[e] = o.vertices[2 * e];
            vy[e] = o.vertices[2 * e + 1];
        }
    } else {
        const double l = o.length / 2.0, w = o.width / 2.0;
        k = 4;
        const double cx[4] = {l, l, -l, -l}, cy[4] = {-w, w, w, -w};
        for (int e = 0; e < 4; ++e) {
            vx[e] = cx[e];
            vy[e] = cy[e];
        }
    }
    g = DPoly{};
    g.k = padded_vertices(k);
    for (int e = 0; e < g.k; ++e) {
        if (e >= k) {  // padding: copies of vertex 0 and of edge 0
            g.vx[e] = g.vx[0];
            g.vy[e] = g.vy[0];
            g.nx[e] = g.nx[0];
            g.ny[e] = g.ny[0];
            g.h[e] = g.h[0];
            g.ex[e] = g.ex[0];
            g.ey[e] = g.ey[0];
            g.il[e] = g.il[0];
            continue;
        }
        const int f = (e + 1) % k;
        const double ex = vx[f] - vx[e], ey = vy[f] - vy[e];
        const double len = std::hypot(ex, ey);
        const double nx = ey / len, ny = -ex / len;   // outward for a CCW polygon
        g.vx[e] = (float)vx[e];
        g.vy[e] = (float)vy[e];
        g.nx[e] = (float)nx;
        g.ny[e] = (float)ny;
        g.h[e] = (float)(nx * vx[e] + ny * vy[e]);
        g.ex[e] = (float)ex;
        g.ey[e] = (float)ey;
        g.il[e] = (float)(1.0 / (ex * ex + ey * ey));
    }
}

// The origin a scene's positions are taken relative to before the GPU sees
// them: the middle of the box of the initial positions, rounded to a multiple
// of kOriginGrid metres. The overlap tests are invariant under a shift of the
// whole scene, but their FP32 rounding grows with the coordinates; relative
// to this origin a scene far from (0, 0) is tested with the precision of one
// near it. The subtraction costs at most one FP64 rounding (1e-12 m at
// 10 km), and a scene whose box is centred within 128 m of (0, 0) keeps its
// coordinates unchanged.
static const double kOriginGrid = 256.0;

void scene_origin(const mhc_scene &s, double *ox, double *oy)
{
    double x0 = s.objects[0].x, x1 = x0, y0 = s.objects[0].y, y1 = y0;
    for (int a = 1; a < s.n_objects; ++a) {
        x0 = std::min(x0, s.objects[a].x);
        x1 = std::max(x1, s.objects[a].x);
        y0 = std::min(y0, s.objects[a].y);
        y1 = std::max(y1, s.objects[a].y);
    }
    *ox = kOriginGrid * std::nearbyint((x0 / 2.0 + x1 / 2.0) / kOriginGrid);
    *oy = kOriginGrid * std::nearbyint((y0 / 2.0 + y1 / 2.0) / kOriginGrid);
}

void fill_values(const mhc_scene *scenes, int n_scenes, Layout &L)
{
    size_t oi = 0, pi = 0, gi = 0;
    std::vector<std::pair<int, int>> plist;
    for (int k = 0; k < n_scenes; ++k) {
        const mhc_scene &s = scenes[k];
        double ox, oy;
        scene_origin(s, &ox, &oy);
        for (int a = 0; a < s.n_objects; ++a, ++oi) {
            const mhc_object &o = s.objects[a];
            DObj &d = L.objs[oi];
            d.x = o.x - ox;
            d.y = o.y - oy;
            d.heading = o.heading;
            d.speed = o.speed;
            d.tau = s.dt;
            for (int k = 0; k < 6; ++k) d.params[k] = o.params[k];
            std::copy(o.u, o.u + o.n_u, L.vals.begin() + d.u_off);
            std::copy(o.w, o.w + o.n_w, L.vals.begin() + d.w_off);
            if (o.score) std::copy(o.score, o.score + d.T, L.vals.begin() + d.score_off);
        }
        if (scene_has_outline(&s))
            for (int a = 0; a < s.n_objects; ++a)
                if (s.objects[a].kind == MHC_VEHICLE) fill_poly(s.objects[a], L.polys[gi++]);
        pair_list(&s, plist);
        for (auto &ab : plist) {
            const mhc_object &oa = s.objects[ab.first], &ob = s.objects[ab.second];
            DPair &pr = L.pairs[pi++];
            pr.la = (float)(oa.length / 2.0);
            pr.wa = (float)(oa.width / 2.0);
            pr.lb = (float)(ob.length / 2.0);
            pr.wb = (float)(ob.width / 2.0);
            pr.rr = 0.0f;
            if (pr.cls == CLS_VP || pr.cls == CLS_GC) pr.rr = (float)(ob.radius * ob.radius);
            else if (pr.cls == CLS_PV || pr.cls == CLS_CG) pr.rr = (float)(oa.radius * oa.radius);
            else if (pr.cls == CLS_PP) pr.rr = (float)((oa.radius + ob.radius) * (oa.radius + ob.radius));
        }
    }
}

void pack_image(const Layout &L, char *dst, bool values_only)
{
    // each table, then zeros up to the next one (the image is written once)
    auto cp = [&](size_t o, const void *src, size_t bytes, size_t next) {
        if (bytes) std::memcpy(dst + o, src, bytes);
        std::memset(dst + o + bytes, 0, next - o - bytes);
    };
    cp(L.o_objs, L.objs.data(), L.objs.size() * sizeof(DObj), L.o_vals);
    cp(L.o_vals, L.vals.data(), L.vals.size() * sizeof(double), L.o_pairs);
    cp(L.o_pairs, L.pairs.data(), L.pairs.size() * sizeof(DPair), L.o_polys);
    cp(L.o_polys, L.polys.data(), L.polys.size() * sizeof(DPoly), L.value_bytes);
    if (values_only) return;
    cp(L.o_work, L.work.data(), L.work.size() * sizeof(WorkItem), L.o_bins);
    cp(L.o_bins, L.bins.data(), L.bins.size() * sizeof(int32_t), L.o_k1rows);
    cp(L.o_k1rows, L.k1_rows.data(), L.k1_rows.size() * sizeof(int32_t), L.image_bytes);
}

Launch make_launch(const Layout &L, char *base, const mhc_result *dev_out, bool keep_hits, int n_cu)
{
    Launch X{};
    X.objs = reinterpret_cast<const DObj *>(base + L.o_objs);
    X.vals = reinterpret_cast<const double *>(base + L.o_vals);
    X.pairs = reinterpret_cast<const DPair *>(base + L.o_pairs);
    X.work = reinterpret_cast<const WorkItem *>(base + L.o_work);
    X.poses = base + L.o_poses;
    X.pfix = reinterpret_cast<unsigned long long *>(base + L.o_pfix);
    X.qacc = reinterpret_cast<unsigned long long *>(base + L.o_qacc);
    X.done = reinterpret_cast<unsigned long long *>(base + L.o_done);
    X.bins = reinterpret_cast<const int32_t *>(base + L.o_bins);
    X.k1_rows = L.k1_rows.empty() ? nullptr : reinterpret_cast<const int2 *>(base + L.o_k1rows);
    X.k1_nrows = L.k1_nrows;
    X.polys = reinterpret_cast<const DPoly *>(base + L.o_polys);
    X.p = reinterpret_cast<double *>(base + L.o_p);
    X.hits = reinterpret_cast<int16_t *>(base + L.o_hits);
    X.q = reinterpret_cast<double *>(base + L.o_q);
    X.traj_crit = reinterpret_cast<double *>(base + L.o_tc);
    X.obj_crit = reinterpret_cast<double *>(base + L.o_oc);
    if (!keep_hits || !L.with_hits) X.hits = nullptr;
    X.timeline = L.timeline ? 1 : 0;
    X.one_track = L.one_track ? 1 : 0;
    X.stage = L.stage ? 1 : 0;
    if (L.timeline) {
        X.hist = reinterpret_cast<unsigned long long *>(base + L.o_hist);
        X.att_w = reinterpret_cast<double *>(base + L.o_attw);
        X.ct_w = reinterpret_cast<double *>(base + L.o_ctw);
        X.crit_t = reinterpret_cast<double *>(base + L.o_ct);
        X.traj_crit_t = reinterpret_cast<double *>(base + L.o_tct);
        X.attrib = reinterpret_cast<double *>(base + L.o_at);
        X.traj_attrib = reinterpret_cast<double *>(base + L.o_tat);
    }
    if (dev_out) {
        if (dev_out->traj_prob) X.p = dev_out->traj_prob;
        if (dev_out->first_hit) X.hits = dev_out->first_hit;
        if (dev_out->q) X.q = dev_out->q;
        if (dev_out->traj_crit) X.traj_crit = dev_out->traj_crit;
        if (dev_out->object_crit) X.obj_crit = dev_out->object_crit;
        if (L.timeline) {
            if (dev_out->crit_t) X.crit_t = dev_out->crit_t;
            if (dev_out->traj_crit_t) X.traj_crit_t = dev_out->traj_crit_t;
            if (dev_out->attrib) X.attrib = dev_out->attrib;
            if (dev_out->traj_attrib) X.traj_attrib = dev_out->traj_attrib;
        }
    }
    X.n_obj = (int)L.objs.size();
    X.n_pairs = (int)L.pairs.size();
    X.n_work = (int)L.work.size();
    X.k1_x = L.k1_x;
    X.k3_x = L.k3_x;
    X.k3t_x = (int)L.k3t_x;
    X.k4t_y = L.k4t_y;
    X.variant = L.variant;
    X.family = L.family;
    X.n_bins = (int)L.bins.size() - 1;
    X.xcd_major = L.contiguous ? 1 : 0;
    (void)n_cu;
    return X;
}

hipError_t launch_all(const Launch &X, hipStream_t s)
{
    hipError_t e = launch_trajgen(X, s);
    if (e == hipSuccess) e = launch_collide(X, s);
    if (e == hipSuccess) e = launch_risk(X, s);
    return e;
}

}  // namespace mhc

using namespace mhc;

// ===========================================================================
// Context
// ===========================================================================

static mhc_status dev_err(mhc_ctx *ctx, hipError_t e, const char *what)
{
    if (ctx) ctx->err = std::string(what) + ": " + hipGetErrorString(e);
    return MHC_E_DEVICE;
}

#define HIPC(call)                                          \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return dev_err(ctx, e_, #call); \
    } while (0)

extern "C" mhc_status mhc_create(int device, size_t hbm_budget_bytes, mhc_ctx **out)
{
    if (!out) return MHC_E_INVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return MHC_E_DEVICE;
    if (device < 0 || device >= n) return MHC_E_INVAL;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return MHC_E_DEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return MHC_E_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return MHC_E_DEVICE;
    mhc_ctx *ctx = new mhc_ctx();
    ctx->device = device;
    ctx->budget = hbm_budget_bytes;
    ctx->n_cu = prop.multiProcessorCount;
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->staging_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->noalloc_ev, hipEventDisableTiming) != hipSuccess ||
        noalloc_scratch_address(device, &ctx->scratch) != hipSuccess) {
        if (ctx->noalloc_ev) (void)hipEventDestroy(ctx->noalloc_ev);
        if (ctx->staging_ev) (void)hipEventDestroy(ctx->staging_ev);
        if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
        delete ctx;
        return MHC_E_DEVICE;
    }
    *out = ctx;
    return MHC_OK;
}

extern "C" void mhc_destroy(mhc_ctx *ctx)
{
    if (!ctx) return;
    hipSetDevice(ctx->device);
    hipStreamSynchronize(ctx->stream);
    ctx->batch_graphs.clear();
    hipEventSynchronize(ctx->staging_ev);
    if (ctx->dbuf) hipFree(ctx->dbuf);
    if (ctx->staging) hipHostFree(ctx->staging);
    if (ctx->res_pin) hipHostFree(ctx->res_pin);
    hipEventSynchronize(ctx->noalloc_ev);
    hipEventDestroy(ctx->staging_ev);
    hipEventDestroy(ctx->noalloc_ev);
    hipStreamDestroy(ctx->stream);
    delete ctx;
}

int mhc_ctx::max_waves(int v, const mhc_scene *scenes, int n)
{
    int fam = 0, tl = 0;
    for (int k = 0; k < n; ++k) {
        fam = std::max(fam, scene_family(&scenes[k]));
        tl |= scenes[k].timeline != 0;
    }
    return max_waves_of(v, fam, tl != 0);
}

int mhc_ctx::max_waves_staged(int v, const mhc_scene *scenes, int n)
{
    for (int k = 0; k < n; ++k)
        if (scene_family(&scenes[k]) != FAM_PLAIN || scenes[k].timeline) return 0;
    return max_waves_of(v, FAM_PLAIN, false, true);
}

int mhc_ctx::max_waves_of(int v, int fam, bool tl, bool stage)
{
    if (v < 0 || v >= N_VARIANTS) v = 0;
    stage = stage && fam == FAM_PLAIN && !tl;
    int &w = waves_cache[v][fam][tl ? 1 : 0][stage ? 1 : 0];
    if (!w) w = n_cu * collide_blocks_per_cu(v, fam, tl, stage) * (WG / WAVE);
    return w;
}

extern "C" const char *mhc_last_error(const mhc_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

extern "C" mhc_status mhc_query_sizes(const mhc_scene *scene, mhc_sizes *out)
{
    if (!out) return MHC_E_INVAL;
    std::string err;
    if (!validate_scene(scene, err)) return MHC_E_INVAL;
    // The workspace size depends on the micro-tile variant and on how many
    // waves the GPU holds; report the largest over all variants with one
    // wave per work unit, which bounds every actual layout.
    size_t bytes = 0;
    Layout L;
    for (int v = 0; v < N_VARIANTS; ++v) {
        build_layout(scene, 1, v, 0, L, true);
        bytes = std::max(bytes, L.total_bytes);
    }
    out->n_traj = L.n_traj;
    out->n_pairs = (int64_t)L.pairs.size();
    out->n_traj_pairs = L.n_hits;
    out->n_checks = L.n_checks;
    out->device_bytes = bytes;
    return MHC_OK;
}

// Walks a collision plan the way k2_collide decodes it: wave slot -> segments
// -> units -> lanes -> items -> trajectory pairs and steps, counting how often
// each item is tested and every index that leaves its pair.
static void walk_plan(const Layout &L, mhc_plan_info &info)
{
    std::vector<int64_t> item_base(L.pairs.size() + 1, 0);
    for (size_t p = 0; p < L.pairs.size(); ++p)
        item_base[p + 1] = item_base[p] + (int64_t)L.pairs[p].n_ig * L.pairs[p].n_jg;
    std::vector<uint8_t> seen((size_t)item_base.back(), 0);
    const int n_bins = (int)L.bins.size() - 1;
    int64_t bad = 0, units = 0;
    int32_t time_split = 1;
    if (n_bins < 1 || L.bins[0] != 0 || L.bins[n_bins] != (int32_t)L.work.size()) ++bad;
    for (int b = 0; b < n_bins && !bad; ++b) {
        if (L.bins[b + 1] < L.bins[b]) {
            ++bad;
            break;
        }
        for (int32_t wi = L.bins[b]; wi < L.bins[b + 1]; ++wi) {
            const WorkItem &w = L.work[wi];
            if (w.pair < 0 || w.pair >= (int32_t)L.pairs.size() || w.n_units < 0) {
                ++bad;
                continue;
            }
            const DPair &pr = L.pairs[w.pair];
            const int per = WAVE >> pr.tshift;
            const int chunk = split_chunk(pr.H, pr.tshift);
            const TileShape ts = kTiles[L.variant][pr.cls];
            const int ri = ts.ri, rj = ts.rj;
            if (pr.tshift < 0 || pr.tshift > MAX_TSHIFT || w.item0 % per != 0) ++bad;
            // the parts' step ranges: inside [0, H), the first from 0, the
            // last to H, each starting at or before the end of the one before
            for (int part = 0, end = 0; part < (1 << pr.tshift); ++part) {
                const int t0 = std::min(part * chunk, pr.H - chunk);
                if (t0 < 0 || t0 > end || t0 + chunk > pr.H) ++bad;
                end = t0 + chunk;
                if (part == (1 << pr.tshift) - 1 && end != pr.H) ++bad;
            }
            time_split = std::max(time_split, 1 << pr.tshift);
            const int64_t n_units = pair_units(pr, pr.tshift, pr.bshift);
            for (int32_t u = 0; u < w.n_units; ++u) {
                ++units;
                const int64_t item0 = (int64_t)w.item0 + (int64_t)u * per;
                const int64_t v = item0 / per;
                if (v >= n_units) ++bad;
                for (int lane = 0; lane < WAVE; ++lane) {
                    const int part = lane >> (6 - pr.tshift);
                    const int e = lane & (per - 1);
                    int64_t ig, jg;
                    if (pr.bshift == 0) {
                        const int64_t f = item0 + e;
                        if (f >= (int64_t)pr.n_ig * pr.n_jg) continue;
                        ig = f / pr.n_jg;
                        jg = f - ig * pr.n_jg;
                    } else {
                        const int bs = pr.bshift;
                        const int64_t nb = (pr.n_jg + (1 << bs) - 1) >> bs;
                        const int64_t bi = v / nb;
                        ig = ((bi << (6 - pr.tshift)) >> bs) + (e >> bs);
                        jg = ((v - bi * nb) << bs) + (e & ((1 << bs) - 1));
                        if (ig >= pr.n_ig || jg >= pr.n_jg) continue;
                    }
                    if (ig < 0 || jg < 0) {
                        ++bad;
                        continue;
                    }
                    for (int r = 0; r < ri; ++r)
                        for (int sidx = 0; sidx < rj; ++sidx) {
                            const int64_t i = ig + (int64_t)r * pr.n_ig, j = jg + (int64_t)sidx * pr.n_jg;
                            if (i >= pr.Ta || j >= pr.Tb) continue;  // idle tile slot
                            const int64_t h = pr.hit_off + i * pr.Tb + j;
                            if (h < 0 || h >= L.n_hits) ++bad;
                            if (pr.qa0 + i * pr.qn >= L.n_q || pr.qb0 + j * pr.qn >= L.n_q) ++bad;
                        }
                    if (part == 0) {
                        uint8_t &c = seen[(size_t)(item_base[w.pair] + ig * pr.n_jg + jg)];
                        if (c < 255) ++c;
                    }
                }
            }
        }
    }
    int64_t uncovered = 0, repeated = 0;
    for (uint8_t c : seen) {
        uncovered += c == 0;
        repeated += c > 1;
    }
    // the trajectory kernel's grid: every block of every object (its
    // normalisation block and one per K1_TPB trajectories) taken by exactly
    // one workgroup, as the kernel maps (row, x) to (object, block)
    {
        const int n_obj = (int)L.objs.size();
        std::vector<int64_t> first(n_obj + 1, 0);
        for (int a = 0; a < n_obj; ++a) first[a + 1] = first[a] + (L.objs[a].T + K1_TPB - 1) / K1_TPB + 1;
        std::vector<uint8_t> took((size_t)first[n_obj], 0);
        const bool table = !L.k1_rows.empty();
        if (table ? (int64_t)L.k1_rows.size() != 2LL * L.k1_nrows : L.k1_nrows != n_obj) ++bad;
        for (int r = 0; r < L.k1_nrows && !bad; ++r) {
            const int obj = table ? L.k1_rows[2 * r] : r, b0 = table ? L.k1_rows[2 * r + 1] : 0;
            if (obj < 0 || obj >= n_obj || b0 < 0) {
                ++bad;
                break;
            }
            for (int x = 0; x < L.k1_x; ++x)
                if (first[obj] + b0 + x < first[obj + 1]) {
                    uint8_t &c = took[(size_t)(first[obj] + b0 + x)];
                    if (c < 255) ++c;
                }
        }
        for (uint8_t c : took) bad += c != 1;
    }
    int64_t blocked = 0;
    for (const DPair &pr : L.pairs) blocked += pr.bshift != 0;
    info.n_units = units;
    info.n_waves = n_bins;
    info.blocked_pairs = blocked;
    info.uncovered = uncovered;
    info.repeated = repeated;
    info.out_of_range = bad;
    info.contiguous = L.contiguous ? 1 : 0;
    info.time_split = time_split;
}

extern "C" mhc_status mhc_plan_check(int32_t n_scenes, const mhc_scene *scenes, int32_t variant, int32_t max_waves,
                                     mhc_plan_info *info)
{
    if (n_scenes < 1 || !scenes || !info || variant < 0 || variant >= N_VARIANTS || max_waves < 0)
        return MHC_E_INVAL;
    std::string err;
    int64_t total_objects = 0;
    for (int k = 0; k < n_scenes; ++k) {
        if (!validate_scene(&scenes[k], err, k)) return MHC_E_INVAL;
        total_objects += scenes[k].n_objects;
    }
    if (total_objects > kMaxObjectsPerLaunch) return MHC_E_INVAL;
    Layout L;
    build_layout(scenes, n_scenes, variant, max_waves, L, true);
    walk_plan(L, *info);
    return info->uncovered == 0 && info->repeated == 0 && info->out_of_range == 0 ? MHC_OK : MHC_E_INVAL;
}

extern "C" mhc_status mhc_anticipation_time(int32_t n_frames, const double *crit, double frame_dt, double threshold,
                                            int32_t event_frame, double *out_seconds)
{
    if (!crit || !out_seconds || n_frames < 1 || event_frame < 1 || event_frame > n_frames) return MHC_E_INVAL;
    if (!std::isfinite(frame_dt) || !(frame_dt > 0.0) || !std::isfinite(threshold)) return MHC_E_INVAL;
    for (int32_t f = 0; f < event_frame; ++f)
        if (!std::isfinite(crit[f])) return MHC_E_INVAL;
    // walk back from the last frame before the event while the criticality
    // stays at or above the threshold
    int32_t first = event_frame;
    while (first > 0 && crit[first - 1] >= threshold) --first;
    *out_seconds = (double)(event_frame - first) * frame_dt;
    return MHC_OK;
}

std::vector<int32_t> mhc::shape_of(const mhc_scene *s)
{
    std::vector<int32_t> v{s->n_objects, s->horizon, s->pairs, s->overlap, s->risk, s->timeline};
    for (int a = 0; a < s->n_objects; ++a) {
        v.push_back(s->objects[a].kind);
        v.push_back(s->objects[a].n_u);
        v.push_back(s->objects[a].n_w);
        v.push_back(s->objects[a].score != nullptr);
        v.push_back(s->objects[a].n_vertices);
        v.push_back(s->objects[a].model);
    }
    return v;
}

// Layout of `scene` for this context: the shape-dependent tables of the
// previous call are reused when the shape (and the tile variant) repeats.
static bool layout_for(mhc_ctx *ctx, const mhc_scene *scene, Layout &L, bool with_hits)
{
    const int v = ctx->variant_for(scene, 1);
    std::vector<int32_t> shape = shape_of(scene);
    shape.push_back(v);
    shape.push_back(ctx->max_waves(v, scene, 1));
    shape.push_back(with_hits);
    if (!L.objs.empty() && shape == ctx->layout_shape) {
        fill_values(scene, 1, L);
        return true;
    }
    build_layout(scene, 1, v, ctx->max_waves(v, scene, 1), L, with_hits, ctx->max_waves_staged(v, scene, 1));
    ctx->layout_shape = std::move(shape);
    return false;
}

// Pinned staging for the scene image. The previous upload from it must have
// left the host buffer before it is rewritten.
static mhc_status stage_image(mhc_ctx *ctx, const Layout &L, char **host, bool values_only = false)
{
    HIPC(hipEventSynchronize(ctx->staging_ev));
    if (ctx->staging_bytes < L.image_bytes) {
        if (ctx->staging) HIPC(hipHostFree(ctx->staging));
        ctx->staging = nullptr;
        ctx->staging_bytes = 0;
        size_t want = std::max<size_t>(L.image_bytes, 1 << 20);
        HIPC(hipHostMalloc(reinterpret_cast<void **>(&ctx->staging), want, hipHostMallocDefault));
        ctx->staging_bytes = want;
    }
    pack_image(L, ctx->staging, values_only);
    *host = ctx->staging;
    return MHC_OK;
}

mhc_status ensure_device(mhc_ctx *ctx, size_t bytes)
{
    if (ctx->budget && bytes > ctx->budget) {
        ctx->err = "scene needs " + std::to_string(bytes) + " device bytes, above the context budget";
        return MHC_E_NOMEM;
    }
    if (ctx->dbuf_bytes >= bytes) return MHC_OK;
    HIPC(hipStreamSynchronize(ctx->stream));
    ctx->batch_graphs.clear();  // their launches point into the old workspace
    ctx->resident_image.clear();
    if (ctx->dbuf) HIPC(hipFree(ctx->dbuf));
    ctx->dbuf = nullptr;
    ctx->dbuf_bytes = 0;
    size_t want = align256(bytes + bytes / 4);
    if (ctx->budget) want = std::min(want, ctx->budget);
    hipError_t e = hipMalloc(&ctx->dbuf, want);
    if (e != hipSuccess) {
        ctx->err = std::string("hipMalloc of the context workspace failed: ") + hipGetErrorString(e);
        return MHC_E_NOMEM;
    }
    ctx->dbuf_bytes = want;
    return MHC_OK;
}

static mhc_status upload_and_launch(mhc_ctx *ctx, const Layout &L, char *dbase, const mhc_result *dev_out,
                                    bool keep_hits, hipStream_t s)
{
    char *host = nullptr;
    mhc_status st = stage_image(ctx, L, &host);
    if (st != MHC_OK) return st;
    HIPC(hipMemcpyAsync(dbase, host, L.image_bytes, hipMemcpyHostToDevice, s));
    HIPC(hipEventRecord(ctx->staging_ev, s));
    Launch X = make_launch(L, dbase, dev_out, keep_hits, ctx->n_cu);
    HIPC(launch_all(X, s));
    return MHC_OK;
}

// Upload + trajectory/collision/risk launches of a context-owned layout,
// replayed as one graph per shape key (the scene image's values change from
// call to call, its layout and every launch argument do not). A key's first
// launch is direct (GraphCache::repeated): capturing costs more than it saves
// for a shape that does not come back soon.
static mhc_status graph_upload_and_launch(mhc_ctx *ctx, const Layout &L, char *dbase, bool keep_hits,
                                          std::vector<int64_t> key, hipStream_t s, bool values_only = false)
{
    char *host = nullptr;
    mhc_status st = stage_image(ctx, L, &host, values_only);
    if (st != MHC_OK) return st;
    const size_t up = values_only ? L.value_bytes : L.image_bytes;
    key.push_back((int64_t)(uintptr_t)dbase);
    key.push_back((int64_t)(uintptr_t)host);
    key.push_back(keep_hits);
    key.push_back((int64_t)L.image_bytes);
    key.push_back((int64_t)up);
    Launch X = make_launch(L, dbase, nullptr, keep_hits, ctx->n_cu);
    if (ctx->batch_graphs.repeated(key)) {
        hipGraphExec_t exec = nullptr;
        HIPC(ctx->batch_graphs.get(key, [&](hipStream_t cs) {
            hipError_t e = hipMemcpyAsync(dbase, host, up, hipMemcpyHostToDevice, cs);
            return e == hipSuccess ? launch_all(X, cs) : e;
        }, &exec));
        HIPC(hipGraphLaunch(exec, s));
    } else {
        HIPC(hipMemcpyAsync(dbase, host, up, hipMemcpyHostToDevice, s));
        HIPC(launch_all(X, s));
    }
    HIPC(hipEventRecord(ctx->staging_ev, s));
    return MHC_OK;
}

// Every output is one region of the workspace in which scene k's part starts
// at a known offset, so each requested output of all scenes comes down in one
// transfer into pinned host memory (one DMA instead of one staged copy into
// pageable memory per scene and output), and the host then copies each
// scene's part to its buffer. Unless every output is to be staged, regions
// above kResultStageMax (the first hits of large scenes), and the largest
// ones while the staged total exceeds kResultStageTotal, are copied per scene
// straight to the callers' buffers.
static const size_t kResultStageMax = size_t(64) << 20;
static const size_t kResultStageTotal = size_t(256) << 20;
// Staged outputs at most this far apart in the workspace share one transfer
// (the bytes between them come along).
static const size_t kResultMergeGap = size_t(64) << 10;

namespace mhc {

// Output f (RESULT order, then the time-resolved ones) of scene k: its host
// buffer (NULL when not asked for) and its bytes in the workspace.
static void result_part(const Layout &L, const mhc_result *res, int f, int k, void **dst, size_t *off,
                        size_t *bytes)
{
    const SceneExt &e = L.sc[k];
    const mhc_result &r = res[k];
    const size_t H = (size_t)e.H, nq = (size_t)e.n_traj * e.n_obj;
    switch (f) {
    case 0: *dst = r.object_crit; *off = L.o_oc + e.obj0 * 8; *bytes = (size_t)e.n_obj * 8; break;
    case 1: *dst = r.traj_crit; *off = L.o_tc + e.traj0 * 8; *bytes = (size_t)e.n_traj * 8; break;
    case 2: *dst = r.traj_prob; *off = L.o_p + e.traj0 * 8; *bytes = (size_t)e.n_traj * 8; break;
    case 3: *dst = r.q; *off = L.o_q + e.q0 * 8; *bytes = nq * 8; break;
    case 4: *dst = r.first_hit; *off = L.o_hits + e.hit0 * 2; *bytes = (size_t)e.n_hits * 2; break;
    case 5: *dst = e.timeline ? r.crit_t : nullptr; *off = L.o_ct + e.tl_obj0 * 8; *bytes = (size_t)e.n_obj * H * 8; break;
    case 6: *dst = e.timeline ? r.traj_crit_t : nullptr; *off = L.o_tct + e.tl_traj0 * 8; *bytes = (size_t)e.n_traj * H * 8; break;
    case 7: *dst = e.timeline ? r.attrib : nullptr; *off = L.o_at + e.tl_att0 * 8; *bytes = (size_t)e.n_obj * e.n_obj * 8; break;
    default: *dst = e.timeline ? r.traj_attrib : nullptr; *off = L.o_tat + e.q0 * 8; *bytes = nq * 8; break;
    }
    if (!*bytes) *dst = nullptr;
}

ResultPlan plan_results(const Layout &L, int n, const mhc_result *res, bool stage_all)
{
    ResultPlan R;
    size_t total = 0;
    for (int f = 0; f < ResultPlan::kOutputs; ++f) {
        R.lo[f] = SIZE_MAX;
        R.hi[f] = 0;
        for (int k = 0; k < n; ++k) {
            void *dst;
            size_t off, bytes;
            result_part(L, res, f, k, &dst, &off, &bytes);
            if (!dst) continue;
            R.lo[f] = std::min(R.lo[f], off);
            R.hi[f] = std::max(R.hi[f], off + bytes);
        }
        R.stage[f] = R.hi[f] > R.lo[f] && (stage_all || R.hi[f] - R.lo[f] <= kResultStageMax);
        if (R.stage[f]) total += R.hi[f] - R.lo[f];
    }
    while (!stage_all && total > kResultStageTotal) {
        int big = -1;
        for (int f = 0; f < ResultPlan::kOutputs; ++f)
            if (R.stage[f] && (big < 0 || R.hi[f] - R.lo[f] > R.hi[big] - R.lo[big])) big = f;
        R.stage[big] = false;
        total -= R.hi[big] - R.lo[big];
    }
    // staged outputs in workspace order; one transfer for each run of them
    // separated by at most kResultMergeGap bytes
    int ord[ResultPlan::kOutputs], m = 0;
    for (int f = 0; f < ResultPlan::kOutputs; ++f)
        if (R.stage[f]) ord[m++] = f;
    std::sort(ord, ord + m, [&](int x, int y) { return R.lo[x] < R.lo[y]; });
    R.staged = 0;
    R.n_copies = 0;
    for (int i = 0; i < m; ++i) {
        const int f = ord[i];
        if (R.n_copies > 0 && R.lo[f] <= R.copy_hi[R.n_copies - 1] + kResultMergeGap) {
            R.copy_hi[R.n_copies - 1] = std::max(R.copy_hi[R.n_copies - 1], R.hi[f]);
        } else {
            R.copy_lo[R.n_copies] = R.lo[f];
            R.copy_hi[R.n_copies] = R.hi[f];
            ++R.n_copies;
        }
    }
    for (int c = 0; c < R.n_copies; ++c) {
        R.copy_at[c] = R.staged;
        R.staged += (R.copy_hi[c] - R.copy_lo[c] + 255) & ~size_t(255);
    }
    for (int i = 0; i < m; ++i) {
        const int f = ord[i];
        int c = 0;
        while (!(R.copy_lo[c] <= R.lo[f] && R.hi[f] <= R.copy_hi[c])) ++c;
        R.at[f] = R.copy_at[c] + (R.lo[f] - R.copy_lo[c]);
    }
    return R;
}

hipError_t enqueue_results(const ResultPlan &R, const Layout &L, int n, const char *dbase, char *pinned,
                           const mhc_result *res, hipStream_t s)
{
    for (int c = 0; c < R.n_copies; ++c) {
        const hipError_t e = hipMemcpyAsync(pinned + R.copy_at[c], dbase + R.copy_lo[c],
                                            R.copy_hi[c] - R.copy_lo[c], hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
    }
    for (int f = 0; f < ResultPlan::kOutputs; ++f) {
        if (R.hi[f] <= R.lo[f] || R.stage[f]) continue;
        for (int k = 0; k < n; ++k) {
            void *dst;
            size_t off, bytes;
            result_part(L, res, f, k, &dst, &off, &bytes);
            if (!dst) continue;
            const hipError_t e = hipMemcpyAsync(dst, dbase + off, bytes, hipMemcpyDeviceToHost, s);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

void scatter_results(const ResultPlan &R, const Layout &L, int n, const char *pinned, const mhc_result *res)
{
    for (int f = 0; f < ResultPlan::kOutputs; ++f) {
        if (!R.stage[f]) continue;
        for (int k = 0; k < n; ++k) {
            void *dst;
            size_t off, bytes;
            result_part(L, res, f, k, &dst, &off, &bytes);
            if (dst) std::memcpy(dst, pinned + R.at[f] + (off - R.lo[f]), bytes);
        }
    }
}

}  // namespace mhc

mhc_status download_results(mhc_ctx *ctx, const Layout &L, int n, const char *dbase, const mhc_result *res,
                            hipStream_t s)
{
    const ResultPlan R = plan_results(L, n, res, false);
    if (R.staged > ctx->res_pin_bytes) {
        if (ctx->res_pin) HIPC(hipHostFree(ctx->res_pin));
        ctx->res_pin = nullptr;
        ctx->res_pin_bytes = 0;
        const size_t want = std::max(R.staged, size_t(1) << 20);
        HIPC(hipHostMalloc(reinterpret_cast<void **>(&ctx->res_pin), want, hipHostMallocDefault));
        ctx->res_pin_bytes = want;
    }
    HIPC(enqueue_results(R, L, n, dbase, ctx->res_pin, res, s));
    HIPC(hipStreamSynchronize(s));
    scatter_results(R, L, n, ctx->res_pin, res);
    return MHC_OK;
}

extern "C" mhc_status mhc_evaluate(mhc_ctx *ctx, const mhc_scene *scene, mhc_result *res)
{
    if (!ctx) return MHC_E_INVAL;
    if (!res || !res->object_crit) {
        ctx->err = "result and result->object_crit must not be NULL";
        return MHC_E_INVAL;
    }
    if (!validate_scene(scene, ctx->err) || !validate_outputs(scene, res, ctx->err)) return MHC_E_INVAL;
    HIPC(hipSetDevice(ctx->device));
    Layout &L = ctx->layout;
    const bool reused = layout_for(ctx, scene, L, res->first_hit != nullptr);
    mhc_status st = ensure_device(ctx, L.total_bytes);
    if (st != MHC_OK) return st;
    char *dbase = static_cast<char *>(ctx->dbuf);
    std::vector<int64_t> key(ctx->layout_shape.begin(), ctx->layout_shape.end());
    key.push_back(-1);  // single scene
    // When the previous launch in this workspace was this shape's, its
    // collision plan is still there and only the image's value part goes up.
    std::vector<int64_t> resident = key;
    resident.push_back((int64_t)(uintptr_t)dbase);
    const bool values_only = reused && ctx->resident_image == resident;
    ctx->resident_image.clear();
    st = graph_upload_and_launch(ctx, L, dbase, res->first_hit != nullptr, key, ctx->stream, values_only);
    if (st != MHC_OK) return st;
    ctx->resident_image = std::move(resident);
    return download_results(ctx, L, 1, dbase, res, ctx->stream);
}

extern "C" mhc_status mhc_evaluate_async(mhc_ctx *ctx, const mhc_scene *scene, void *dev_workspace,
                                         size_t workspace_bytes, const mhc_result *dev_out, void *hip_stream)
{
    if (!ctx) return MHC_E_INVAL;
    if (!dev_out || !dev_out->object_crit || !dev_workspace) {
        ctx->err = "dev_workspace, dev_out and dev_out->object_crit must not be NULL";
        return MHC_E_INVAL;
    }
    if (reinterpret_cast<uintptr_t>(dev_workspace) % 256 != 0) {
        ctx->err = "dev_workspace must be 256-byte aligned";
        return MHC_E_INVAL;
    }
    if (!validate_scene(scene, ctx->err) || !validate_outputs(scene, dev_out, ctx->err)) return MHC_E_INVAL;
    Layout L;
    const int v = ctx->variant_for(scene, 1);
    build_layout(scene, 1, v, ctx->max_waves(v, scene, 1), L, true, ctx->max_waves_staged(v, scene, 1));
    if (workspace_bytes < L.total_bytes) {
        ctx->err = "workspace too small: need " + std::to_string(L.total_bytes) + " bytes";
        return MHC_E_INVAL;
    }
    HIPC(hipSetDevice(ctx->device));
    return upload_and_launch(ctx, L, static_cast<char *>(dev_workspace), dev_out, false,
                             static_cast<hipStream_t>(hip_stream));
}

extern "C" mhc_status mhc_evaluate_noalloc(mhc_ctx *ctx, const mhc_scene *scene, const mhc_result *dev_out,
                                           void *hip_stream)
{
    if (!ctx) return MHC_E_INVAL;
    if (!dev_out || !dev_out->object_crit) {
        ctx->err = "dev_out and dev_out->object_crit must not be NULL";
        return MHC_E_INVAL;
    }
    if (!validate_scene(scene, ctx->err) || !validate_outputs(scene, dev_out, ctx->err)) return MHC_E_INVAL;
    HIPC(hipSetDevice(ctx->device));
    if (!ctx->scratch) {
        ctx->err = "the allocation-free workspace of this device was not found";
        return MHC_E_DEVICE;
    }
    // the first hits go to dev_out->first_hit only, so the array holds none
    Layout &L = ctx->noalloc_layout;
    const int v = ctx->variant_for(scene, 1);
    build_layout(scene, 1, v, ctx->max_waves(v, scene, 1), L, false, ctx->max_waves_staged(v, scene, 1));
    if (L.total_bytes > kNoallocBytes) {
        ctx->err = "scene needs " + std::to_string(L.total_bytes) + " workspace bytes, above MHC_NOALLOC_MAX_BYTES (" +
                   std::to_string(kNoallocBytes) + ")";
        return MHC_E_NOMEM;
    }
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    // the previous call's upload must have left the host image before it is
    // rewritten
    HIPC(hipEventSynchronize(ctx->noalloc_ev));
    if (ctx->noalloc_image.size() < L.image_bytes) ctx->noalloc_image.resize(L.image_bytes);
    pack_image(L, ctx->noalloc_image.data());
    HIPC(hipMemcpyAsync(ctx->scratch, ctx->noalloc_image.data(), L.image_bytes, hipMemcpyHostToDevice, s));
    HIPC(hipEventRecord(ctx->noalloc_ev, s));
    Launch X = make_launch(L, ctx->scratch, dev_out, false, ctx->n_cu);
    HIPC(launch_all(X, s));
    return MHC_OK;
}

// ===========================================================================
// Graph cache: one instantiated HIP graph per key, captured from a launch
// sequence on a private stream (capture does not execute anything).
// ===========================================================================

GraphCache::~GraphCache() { clear(); }

void GraphCache::clear()
{
    for (auto &kv : graphs) hipGraphExecDestroy(kv.second);
    graphs.clear();
    order.clear();
    seen.clear();
    if (capture) hipStreamDestroy(capture);
    capture = nullptr;
}

bool GraphCache::repeated(const std::vector<int64_t> &key)
{
    ++uses;
    if (graphs.count(key)) return true;
    for (auto it = seen.begin(); it != seen.end(); ++it)
        if (it->first == key) {
            if (uses - it->second <= (int64_t)kMaxGraphs) {
                seen.erase(it);
                return true;
            }
            it->second = uses;
            return false;
        }
    if (seen.size() >= kMaxSeen) seen.pop_front();
    seen.emplace_back(key, uses);
    return false;
}

hipError_t GraphCache::get(const std::vector<int64_t> &key, const std::function<hipError_t(hipStream_t)> &enqueue,
                           hipGraphExec_t *out)
{
    auto it = graphs.find(key);
    if (it != graphs.end()) {
        *out = it->second;
        return hipSuccess;
    }
    hipError_t e = hipSuccess;
    if (!capture) e = hipStreamCreateWithFlags(&capture, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t le = enqueue(capture);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(capture, &g);
    if (le != hipSuccess) {
        if (g) hipGraphDestroy(g);
        return le;
    }
    if (e != hipSuccess) return e;
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) return e;
    if (graphs.size() >= kMaxGraphs) {  // drop the oldest
        auto old = graphs.find(order.front());
        if (old != graphs.end()) {
            hipGraphExecDestroy(old->second);
            graphs.erase(old);
        }
        order.erase(order.begin());
    }
    graphs[key] = ex;
    order.push_back(key);
    *out = ex;
    return hipSuccess;
}

// ===========================================================================
// Plans: inputs resident in device memory, launched repeatedly.
// ===========================================================================

struct mhc_plan {
    mhc_ctx *ctx = nullptr;
    Layout L;
    mhc_scene flags{};            // pair mode, overlap, risk and timeline of the planned scene
    char *dbuf = nullptr;
    std::vector<int32_t> shape;   // kinds, grid sizes, horizon, pair mode
    GraphCache graphs;            // K1 -> K2 -> K3 per set of output pointers
    bool use_graphs = false;
};


extern "C" mhc_status mhc_plan_create(mhc_ctx *ctx, const mhc_scene *scene, mhc_plan **out)
{
    if (!ctx || !out) return MHC_E_INVAL;
    *out = nullptr;
    if (!validate_scene(scene, ctx->err)) return MHC_E_INVAL;
    HIPC(hipSetDevice(ctx->device));
    mhc_plan *pl = new mhc_plan();
    pl->ctx = ctx;
    const int v = ctx->variant_for(scene, 1);
    build_layout(scene, 1, v, ctx->max_waves(v, scene, 1), pl->L, true, ctx->max_waves_staged(v, scene, 1));
    pl->shape = shape_of(scene);
    pl->flags = *scene;
    pl->flags.objects = nullptr;
    if (ctx->budget && pl->L.total_bytes > ctx->budget) {
        ctx->err = "plan needs more device memory than the context budget";
        delete pl;
        return MHC_E_NOMEM;
    }
    if (hipMalloc(reinterpret_cast<void **>(&pl->dbuf), pl->L.total_bytes) != hipSuccess) {
        ctx->err = "hipMalloc for the plan failed";
        delete pl;
        return MHC_E_NOMEM;
    }
    std::vector<char> img(pl->L.image_bytes);
    pack_image(pl->L, img.data());
    hipError_t e = hipMemcpy(pl->dbuf, img.data(), pl->L.image_bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(pl->dbuf);
        delete pl;
        return dev_err(ctx, e, "plan upload");
    }
    *out = pl;
    return MHC_OK;
}

extern "C" mhc_status mhc_plan_update(mhc_plan *pl, const mhc_scene *scene)
{
    if (!pl) return MHC_E_INVAL;
    mhc_ctx *ctx = pl->ctx;
    if (!validate_scene(scene, ctx->err)) return MHC_E_INVAL;
    if (shape_of(scene) != pl->shape) {
        ctx->err = "mhc_plan_update: scene shape differs from the plan";
        return MHC_E_INVAL;
    }
    HIPC(hipSetDevice(ctx->device));
    Layout L;
    build_layout(scene, 1, pl->L.variant, ctx->max_waves(pl->L.variant, scene, 1), L, true,
                 ctx->max_waves_staged(pl->L.variant, scene, 1));
    std::vector<char> img(L.image_bytes);
    pack_image(L, img.data());
    HIPC(hipDeviceSynchronize());
    HIPC(hipMemcpy(pl->dbuf, img.data(), L.image_bytes, hipMemcpyHostToDevice));
    pl->L = std::move(L);
    pl->flags = *scene;
    pl->flags.objects = nullptr;
    return MHC_OK;
}

extern "C" mhc_status mhc_plan_execute(mhc_plan *pl, const mhc_result *dev_out, void *hip_stream)
{
    if (!pl) return MHC_E_INVAL;
    mhc_ctx *ctx = pl->ctx;
    if (!validate_outputs(&pl->flags, dev_out, ctx->err)) return MHC_E_INVAL;
    HIPC(hipSetDevice(ctx->device));
    Launch X = make_launch(pl->L, pl->dbuf, dev_out, true, ctx->n_cu);
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (!pl->use_graphs) {
        HIPC(launch_all(X, s));
        return MHC_OK;
    }
    // The launch sequence depends only on the plan and the output pointers:
    // it is captured once per pointer set and replayed as one graph.
    std::vector<int64_t> key{(int64_t)(uintptr_t)pl->dbuf};
    if (dev_out)
        for (const void *ptr : {(const void *)dev_out->object_crit, (const void *)dev_out->traj_crit,
                                (const void *)dev_out->traj_prob, (const void *)dev_out->q,
                                (const void *)dev_out->first_hit, (const void *)dev_out->crit_t,
                                (const void *)dev_out->traj_crit_t, (const void *)dev_out->attrib,
                                (const void *)dev_out->traj_attrib})
            key.push_back((int64_t)(uintptr_t)ptr);
    hipGraphExec_t exec = nullptr;
    HIPC(pl->graphs.get(key, [&](hipStream_t cs) { return launch_all(X, cs); }, &exec));
    HIPC(hipGraphLaunch(exec, s));
    return MHC_OK;
}

extern "C" mhc_status mhc_plan_execute_stages(mhc_plan *pl, const mhc_result *dev_out, void *hip_stream,
                                              uint32_t stages)
{
    if (!pl) return MHC_E_INVAL;
    mhc_ctx *ctx = pl->ctx;
    if (stages == 0 || stages > MHC_STAGE_ALL) {
        ctx->err = "stages must be a non-empty combination of MHC_STAGE_* bits";
        return MHC_E_INVAL;
    }
    if (!validate_outputs(&pl->flags, dev_out, ctx->err)) return MHC_E_INVAL;
    HIPC(hipSetDevice(ctx->device));
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    Launch X = make_launch(pl->L, pl->dbuf, dev_out, true, ctx->n_cu);
    if (stages & MHC_STAGE_TRAJ) HIPC(launch_trajgen(X, s));
    if (stages & MHC_STAGE_COLLIDE) HIPC(launch_collide(X, s));
    if (stages & MHC_STAGE_RISK) HIPC(launch_risk(X, s));
    return MHC_OK;
}

extern "C" mhc_status mhc_plan_set_graph(mhc_plan *pl, int32_t enable)
{
    if (!pl || (enable != 0 && enable != 1)) return MHC_E_INVAL;
    pl->use_graphs = enable == 1;
    return MHC_OK;
}

extern "C" mhc_status mhc_plan_download(mhc_plan *pl, mhc_result *host_out)
{
    if (!pl || !host_out) return MHC_E_INVAL;
    mhc_ctx *ctx = pl->ctx;
    if (!validate_outputs(&pl->flags, host_out, ctx->err)) return MHC_E_INVAL;
    HIPC(hipSetDevice(ctx->device));
    HIPC(hipDeviceSynchronize());
    return download_results(ctx, pl->L, 1, static_cast<const char *>(pl->dbuf), host_out, ctx->stream);
}

extern "C" void mhc_plan_destroy(mhc_plan *pl)
{
    if (!pl) return;
    hipSetDevice(pl->ctx->device);
    hipDeviceSynchronize();
    pl->graphs.clear();
    if (pl->dbuf) hipFree(pl->dbuf);
    delete pl;
}

// ===========================================================================
// Batched
// ===========================================================================

extern "C" mhc_status mhc_evaluate_batch(mhc_ctx *ctx, int32_t n, const mhc_scene *scenes, mhc_result *res)
{
    if (!ctx) return MHC_E_INVAL;
    if (n < 1 || !scenes || !res) {
        ctx->err = "batch needs n >= 1, scenes and results";
        return MHC_E_INVAL;
    }
    int64_t total_objects = 0;
    for (int k = 0; k < n; ++k) {
        if (!validate_scene(&scenes[k], ctx->err, k)) return MHC_E_INVAL;
        total_objects += scenes[k].n_objects;
        if (total_objects > kMaxObjectsPerLaunch) {
            ctx->err = "batch holds more than 65535 objects";
            return MHC_E_INVAL;
        }
        if (!res[k].object_crit) {
            ctx->err = "result " + std::to_string(k) + ": object_crit must not be NULL";
            return MHC_E_INVAL;
        }
        if (!validate_outputs(&scenes[k], &res[k], ctx->err, k)) return MHC_E_INVAL;
    }
    HIPC(hipSetDevice(ctx->device));
    return batch_run(ctx, n, scenes, res);
}

// Batched form: all scenes share one scene image, one trajectory launch, one
// collision launch over a longest-first work list and one risk launch.
mhc_status batch_run(mhc_ctx *ctx, int n, const mhc_scene *scenes, mhc_result *res)
{
    Layout &L = ctx->layout;
    bool keep = false;
    for (int k = 0; k < n; ++k) keep |= res[k].first_hit != nullptr;
    const int v = ctx->variant_for(scenes, n);
    const int waves = ctx->max_waves(v, scenes, n);
    std::vector<int64_t> key{v, waves, n};
    // the layout's shape: a batch marker (a single scene's shape starts with
    // its object count), the key and whether first hits are kept
    std::vector<int32_t> shape{-2, v, waves, n, keep};
    for (int k = 0; k < n; ++k) {
        const std::vector<int32_t> sh = shape_of(&scenes[k]);
        key.insert(key.end(), sh.begin(), sh.end());
        shape.insert(shape.end(), sh.begin(), sh.end());
    }
    // A batch of the previous call's shapes keeps its layout (pairs, plan,
    // offsets) and only takes the new values, and when the workspace still
    // holds that layout's image only the value part goes up.
    const bool reused = !L.objs.empty() && shape == ctx->layout_shape;
    if (reused) {
        fill_values(scenes, n, L);
    } else {
        build_layout(scenes, n, v, waves, L, keep, ctx->max_waves_staged(v, scenes, n));
        ctx->layout_shape = std::move(shape);
    }
    mhc_status st = ensure_device(ctx, L.total_bytes);
    if (st != MHC_OK) return st;
    char *dbase = static_cast<char *>(ctx->dbuf);
    std::vector<int64_t> resident = key;
    resident.push_back(keep);
    resident.push_back((int64_t)(uintptr_t)dbase);
    const bool values_only = reused && ctx->resident_image == resident;
    ctx->resident_image.clear();
    st = graph_upload_and_launch(ctx, L, dbase, keep, key, ctx->stream, values_only);
    if (st != MHC_OK) return st;
    ctx->resident_image = std::move(resident);
    return download_results(ctx, L, n, dbase, res, ctx->stream);
}
