// Internal device-side layouts shared by the host runtime and the kernels.
//
// A packed "scene image" (built on the host during ingest, copied to HBM in
// one transfer) holds these tables; the kernels read nothing else besides the
// pose buffer they produce and the result buffers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mhc {

enum Kind : int32_t { KIND_VEHICLE = 0, KIND_PEDESTRIAN = 1 };
enum Model : int32_t { MODEL_KINEMATIC = 0, MODEL_PED_ACCEL = 1, MODEL_ONE_TRACK = 2 };

// Shape class of an object pair: which overlap test applies and which side
// holds the rectangle or polygon.
// CLS_VV_PIP: two rectangles under the point-in-polygon test.
// CLS_GG, CLS_GG_PIP: two convex polygons (at least one a vehicle outline, a
//   rectangle otherwise by its corners), separating axes / point-in-polygon.
// CLS_GC, CLS_CG: polygon and circle (polygon first / second).
enum PairClass : int32_t {
    CLS_VV = 0, CLS_VP = 1, CLS_PV = 2, CLS_PP = 3, CLS_VV_PIP = 4,
    CLS_GG = 5, CLS_GG_PIP = 6, CLS_GC = 7, CLS_CG = 8, N_CLS = 9
};
// Families of test classes, each carried by its own collision-kernel
// instances (a family includes the ones before it).
enum ClassFamily : int32_t { FAM_PLAIN = 0, FAM_PIP = 1, FAM_POLY = 2 };
constexpr int class_family(int cls) { return cls >= CLS_GG ? FAM_POLY : (cls == CLS_VV_PIP ? FAM_PIP : FAM_PLAIN); }

constexpr int MAX_VERTICES = 8;

// Convex polygon of a vehicle in a polygon pair, body frame, CCW, as FP32
// test constants: vertices, unit outward edge normals and offsets (a point
// is inside iff nx*x + ny*y <= h on every edge), and for the circle test the
// edge vectors (vertex e to e+1) with 1 / |edge|^2. k is 4 or 8: a polygon
// of fewer vertices is padded with copies of vertex 0 and of edge 0, which
// change none of the tests.
struct DPoly {
    int32_t k, pad0, pad1, pad2;
    float vx[MAX_VERTICES], vy[MAX_VERTICES];
    float nx[MAX_VERTICES], ny[MAX_VERTICES], h[MAX_VERTICES];
    float ex[MAX_VERTICES], ey[MAX_VERTICES], il[MAX_VERTICES];
};

// Reading of the conditional-probability approximation (mhc.h MHC_RISK_*).
enum RiskModel : int32_t { RISK_EXCLUSIVE = 0, RISK_INDEPENDENT = 1 };

// One object of one scene. Offsets are global across all scenes of a launch.
struct DObj {
    int32_t kind, n_u, n_w, T;
    int32_t has_score, H;
    int32_t local, n_scene_obj;   // index within its scene, object count of the scene
    int32_t risk, timeline;       // RiskModel of its scene; 1: time-resolved risk
    int32_t tl_w;                 // time-resolved: lanes per trajectory, the power of two >= n_scene_obj
    int32_t model;                // motion model (mhc.h MHC_MODEL_*)
    int64_t traj_off;             // index of trajectory 0 in the p / traj_crit arrays
    int64_t q_row;                // q index of (this object, i = 0, b = 0)
    int64_t pose_off;             // byte offset of the pose block [H][T]
    int64_t frame_off;            // vehicles: byte offset of the block [H][T] of the same poses in
                                  // their own frame, (K_x, K_y, cos, sin) with K = c in that frame
    int64_t u_off, w_off, score_off;  // offsets (doubles) into the value array
    int64_t obj_out;              // index in the object_crit array
    // time-resolved risk (timeline scenes only)
    int64_t hist_off;             // slot sums [s][i][b < tl_w]: index of (s = 0, i = 0, b = 0)
    int64_t tl_traj;              // [s][i] criticality over time, and traj_crit_t (i, s): index of i = 0, s = 0
    int64_t tl_obj;               // crit_t index of (this object, s = 0)
    int64_t tl_att;               // attrib index of (this object, b = 0)
    double x, y, heading, speed;  // position relative to the scene origin (scene_origin)
    double tau;
    double params[6];             // motion-model parameters
};

// One object pair (a < b within its scene). The collision kernel covers the
// T_a x T_b trajectory pairs as a flat list of n_ig * n_jg "items": item f is
// the micro-tile ig = f / n_jg, jg = f % n_jg, holding trajectories
// i = ig + r*n_ig (r < RI) and j = jg + s*n_jg (s < RJ).
struct DPair {
    int32_t a, b;                 // global object indices
    int32_t cls, H;
    int32_t Ta, Tb;
    int32_t n_ig, n_jg;
    int64_t hit_off;              // first-hit entry of (i = 0, j = 0)
    int64_t pose_a, pose_b;       // byte offsets of the two pose blocks (a rectangle whose tests take
                                  // its pose in its own frame: the object's frame block)
    float la, wa, lb, wb;         // half length / half width of vehicles
    float rr;                     // squared test radius: r_Q^2 (rect-circle), (r_P + r_Q)^2 (circle-circle)
    int32_t qn;                   // q row stride: object count of the scene
    int32_t tshift;               // time split S = 2^tshift (S <= H): a unit's steps run in S parts
    int64_t qa0;                  // q index of (a, i = 0, b)
    int64_t qb0;                  // q index of (b, j = 0, a)
    int64_t pa_off, pb_off;       // trajectory index of (a, 0) and (b, 0)
    int32_t timeline;             // 1: q sums go to the per-slot sums below
    int32_t hwa, hwb;             // lanes per trajectory of a's and of b's per-slot sums
    int32_t poly_a, poly_b;       // DPoly of a and of b (polygon classes), else -1
    int32_t bshift;               // unit shape: 0 = E consecutive items of the row-major item grid;
                                  // else blocks of (E >> bshift) item rows x 2^bshift item columns
    int64_t ha0;                  // slot-sum index of (a: s = 0, i = 0, b); slot s, trajectory i at + (s*Ta + i)*hwa
    int64_t hb0;                  // slot-sum index of (b: s = 0, j = 0, a); + (s*Tb + j)*hwb
};

// A run of collision work for one wave: n_units consecutive units of a pair.
// A pair's items (ig, jg) form an n_ig x n_jg grid; with time split S a unit
// holds E = 64 / S of them, and lane l takes item l % E of unit item0 / E + u
// and the c = ceil(H/S) steps from min(p*c, H - c) of part p = l / E, so the
// S parts of an item run side by side in one wave and cover every step (the
// last part overlaps its neighbour where S does not divide H). With bshift = 0 the items of unit v are
// E*v .. E*v + E-1 in row-major order; otherwise unit v is the block
// (v / nb, v % nb) of the grid cut into blocks of E / 2^bshift rows and
// 2^bshift columns (nb blocks per block row), so that a wave reads few
// distinct poses of either object per step. Items past the grid are idle
// lanes. The host assigns every wave of the collision kernel a range of
// segments.
struct WorkItem {
    int32_t pair;
    int32_t item0;
    int32_t n_units;
    int32_t pad;
};

constexpr int WG = 256;           // threads per workgroup, all kernels
constexpr int WAVE = 64;          // wavefront size
constexpr int MAX_TSHIFT = 3;     // time split of a collision unit: S <= 8
constexpr int N_XCD = 8;          // accelerator complex dies; workgroups are dealt to them in turn
constexpr int K1_TPB = WG / 64;   // trajectories per trajectory workgroup (one wave each)
// q sums are accumulated exactly as integers. EXCLUSIVE reading: p scaled by
// 2^62 and rounded (sum <= 1). INDEPENDENT reading: -log(1 - p), capped at 64,
// scaled by 2^56 and rounded; over one object's trajectories (sum p = 1) the
// sum stays below 66 * 2^56 < 2^63.
constexpr double kQScale = 4611686018427387904.0;        // 2^62
constexpr double kQInvScale = 2.168404344971009e-19;     // 2^-62
constexpr double kLScale = 72057594037927936.0;          // 2^56
constexpr double kLInvScale = 1.3877787807814457e-17;    // 2^-56
constexpr double kLCap = 64.0;                           // exp(-64) rounds 1 - q to 0

// Micro-tile shape per class, selected by a kernel variant id.
struct TileShape {
    int ri, rj;
};
constexpr int N_VARIANTS = 4;
// variant -> shape per class {VV, VP, PV, PP, VV_PIP, GG, GG_PIP, GC, CG}.
// The shapes keep the VALU cost of one work unit similar across classes (25,
// 12, 6 and 58 VALU per rect-rect, rect-circle, circle-circle and
// point-in-polygon test; 100-500 for polygon pairs) and the loads per test
// low: a rectangle-circle tile pairs each rectangle pose (read in its own
// frame) with 4 or 8 circles. Variants 2 and 3 cut the work into more,
// smaller units for scenes with few of them.
// Polygon-polygon pairs always take one test per thread (their tests are
// long, and the kernel has one code path per padded vertex-count pair).
constexpr TileShape kTiles[N_VARIANTS][N_CLS] = {
    {{4, 2}, {2, 4}, {4, 2}, {4, 4}, {4, 2}, {1, 1}, {1, 1}, {4, 1}, {1, 4}},
    {{4, 2}, {2, 8}, {8, 2}, {4, 4}, {4, 2}, {1, 1}, {1, 1}, {4, 1}, {1, 4}},
    {{2, 2}, {2, 4}, {4, 2}, {4, 4}, {2, 1}, {1, 1}, {1, 1}, {2, 2}, {2, 2}},
    {{2, 1}, {1, 4}, {4, 1}, {4, 2}, {1, 1}, {1, 1}, {1, 1}, {1, 1}, {1, 1}},
};
static_assert(kTiles[0][CLS_GG].ri == 1 && kTiles[1][CLS_GG].ri == 1 && kTiles[2][CLS_GG].ri == 1 &&
                  kTiles[3][CLS_GG].ri == 1 && kTiles[0][CLS_GG].rj == 1 && kTiles[1][CLS_GG].rj == 1 &&
                  kTiles[2][CLS_GG].rj == 1 && kTiles[3][CLS_GG].rj == 1,
              "polygon-polygon tiles are 1 x 1");
static_assert(kTiles[0][CLS_GG_PIP].ri == 1 && kTiles[1][CLS_GG_PIP].ri == 1 && kTiles[2][CLS_GG_PIP].ri == 1 &&
                  kTiles[3][CLS_GG_PIP].ri == 1 && kTiles[0][CLS_GG_PIP].rj == 1 && kTiles[1][CLS_GG_PIP].rj == 1 &&
                  kTiles[2][CLS_GG_PIP].rj == 1 && kTiles[3][CLS_GG_PIP].rj == 1,
              "polygon-polygon tiles are 1 x 1");

// Launch entry points (kernels.hip).
struct Launch {
    const DObj *objs;
    const double *vals;
    const DPair *pairs;
    const WorkItem *work;
    char *poses;
    unsigned long long *pfix;     // p * 2^62, per trajectory
    unsigned long long *qacc;     // integer q sums [n_q]
    const int32_t *bins;          // [n_bins+1] segment range of each collision wave slot
    const DPoly *polys;           // polygons of the polygon pairs
    double *p;
    int16_t *hits;
    double *q;
    double *traj_crit;
    double *obj_crit;
    int n_obj, n_pairs, n_work, n_bins;
    int k1_x;                     // trajectory kernel grid x: blocks of a row
    int k1_nrows;                 // trajectory kernel grid y: rows (objects, or k1_rows entries)
    const int2 *k1_rows;          // per row: object and its first block; null when row = object
    int k3_x;                     // risk kernel grid x: 256-trajectory chunks of the largest object
    unsigned long long *done;     // per object: risk chunks finished (bits 56..63) and their
                                  // criticality sum in units of 2^-55 (bits 0..55)
    // time-resolved risk (null / 0 when no scene of the launch asks for it)
    int timeline;
    int k3t_x, k4t_y;             // time-resolved kernel grids: a wave of lanes of the largest object per workgroup; rows
    unsigned long long *hist;     // per-slot integer q sums
    double *att_w;                // attribution [b][i] per object
    double *ct_w;                 // criticality over time [s][i] per object
    double *crit_t, *traj_crit_t, *attrib, *traj_attrib;
    int xcd_major;                // plan of contiguous stretches: number the slots XCD-major
    int collide_parts;            // the collision plan runs as this many launches (0 or 1: one)
    int collide_only;             // 0: launch every part; k > 0: launch only part k - 1
    int one_track;                // some object follows the one-track model (heavier trajectory kernel)
    int stage;                    // collision instance that stages 8 x 8 item blocks in LDS
    int variant;
    int family;                   // ClassFamily covering every pair of the launch
};

hipError_t launch_trajgen(const Launch &L, hipStream_t s);
hipError_t launch_collide(const Launch &L, hipStream_t s);
// risk: the time-resolved kernels (timeline launches) and the risk kernel
hipError_t launch_risk(const Launch &L, hipStream_t s);
// Bytes of the allocation-free entry point's device array (mhc.h
// MHC_NOALLOC_MAX_BYTES) and the most GPUs whose copy of it is looked up.
constexpr size_t kNoallocBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
// This GPU's address of that array (the device must be current on the
// calling thread); looked up once per device, then cached.
hipError_t noalloc_scratch_address(int device, char **out);
// resident workgroups per CU of the collision kernel for a variant, class
// family, with or without the per-slot sums, with or without LDS-staged blocks
int collide_blocks_per_cu(int variant, int family, bool timeline, bool stage);

}  // namespace mhc
