// HIP kernels for gfx950 (CDNA4): trajectory generation, collision
// recognition and risk assessment of the multi-hypothesis criticality method
// (Sanchez Morales et al., IEEE IV 2019, Fig. 1: the three modules after
// street data processing, run in that order, each data-parallel inside).
#include "mhc_internal.h"

#include <math.h>

namespace mhc {

// ===========================================================================
// K1: trajectory generation (Sec. IV-B) and probability normalisation
// (Sec. IV-D.1).
//
// Vehicles follow the Euler pose update of Sec. IV-B.1 with side slip 0 and
// no yaw acceleration; the constant acceleration of trajectory i acts inside
// each step and is cut so that the speed stops at 0. The time loop of one
// trajectory is sequential (Sec. IV-B.4), but the heading of step n is
// psi0 + n*w*tau, so the FP64 sine/cosine of a chunk of steps are computed by
// all 256 threads first and the 16 trajectories of the block then integrate
// through the chunk from LDS. Positions are integrated in FP64 and stored as
// FP32 (x, y, cos psi, sin psi), one float4 per pose, layout [t][i].
// Pedestrians (Sec. IV-B.3) walk at constant speed along a fixed heading:
// one thread per trajectory, float2 (x, y) poses.
// ===========================================================================

__device__ void normalise_probabilities(const DObj &o, const double *__restrict__ vals, double *__restrict__ p)
{
    __shared__ double red[WG];
    const int tid = threadIdx.x;
    double part = 0.0;
    if (o.has_score) {
        for (int k = tid; k < o.T; k += WG) part += vals[o.score_off + k];
    }
    red[tid] = part;
    __syncthreads();
    for (int s = WG / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    const double total = red[0];
    for (int k = tid; k < o.T; k += WG)
        p[o.traj_off + k] = o.has_score ? vals[o.score_off + k] / total : 1.0 / (double)o.T;
}

__global__ __launch_bounds__(WG) void k1_trajgen(const DObj *__restrict__ objs, const double *__restrict__ vals,
                                                 const K1Block *__restrict__ blocks, char *__restrict__ poses,
                                                 double *__restrict__ p)
{
    const K1Block blk = blocks[blockIdx.x];
    const DObj o = objs[blk.obj];
    const int tid = threadIdx.x;
    const double tau = o.tau;
    const int H = o.H;

    if (o.kind == KIND_VEHICLE) {
        __shared__ double s_c[K1_VT][K1_CH + 1];
        __shared__ double s_s[K1_VT][K1_CH + 1];
        const int lt = tid % K1_VT;
        const int helper = tid / K1_VT;
        const int i = blk.i0 + lt;
        const bool valid = i < o.T;
        const int ic = valid ? i : o.T - 1;
        const int k = ic / o.n_w, l = ic - (ic / o.n_w) * o.n_w;
        const double accel = vals[o.u_off + k];
        const double omega = vals[o.w_off + l];
        const double half_tau2 = tau * tau / 2.0;
        double x = o.x, y = o.y, v = o.speed;
        float4 *out = reinterpret_cast<float4 *>(poses + o.pose_off);
        for (int n0 = 0; n0 < H; n0 += K1_CH) {
            const int nn = min(K1_CH, H - n0);
            for (int q = helper; q <= nn; q += WG / K1_VT) {
                const double psi = o.heading + (double)(n0 + q) * (omega * tau);
                double sv, cv;
                sincos(psi, &sv, &cv);
                s_c[lt][q] = cv;
                s_s[lt][q] = sv;
            }
            __syncthreads();
            if (helper == 0 && valid) {
                for (int q = 0; q < nn; ++q) {
                    const double c = s_c[lt][q], s = s_s[lt][q];
                    double vdot = accel;
                    double v_next = v + vdot * tau;
                    if (v_next < 0.0) {
                        vdot = -v / tau;
                        v_next = 0.0;
                    }
                    const double ax = vdot;
                    const double ay = v * omega;
                    const double xn = x + c * v * tau + c * ax * half_tau2 - s * ay * half_tau2;
                    const double yn = y + s * v * tau + s * ax * half_tau2 + c * ay * half_tau2;
                    x = xn;
                    y = yn;
                    v = v_next;
                    out[(size_t)(n0 + q) * o.T + i] =
                        make_float4((float)x, (float)y, (float)s_c[lt][q + 1], (float)s_s[lt][q + 1]);
                }
            }
            __syncthreads();
        }
    } else {
        const int i = blk.i0 + tid;
        if (i < o.T) {
            const int k = i / o.n_w, l = i - (i / o.n_w) * o.n_w;
            const double speed = vals[o.u_off + k];
            const double psi = o.heading + vals[o.w_off + l];
            double sv, cv;
            sincos(psi, &sv, &cv);
            double x = o.x, y = o.y;
            float2 *out = reinterpret_cast<float2 *>(poses + o.pose_off);
            for (int n = 0; n < H; ++n) {
                x = x + cv * speed * tau;
                y = y + sv * speed * tau;
                out[(size_t)n * o.T + i] = make_float2((float)x, (float)y);
            }
        }
    }
    if (blk.i0 == 0) {
        __syncthreads();
        normalise_probabilities(o, vals, p);
    }
}

// ===========================================================================
// K2: collision recognition (Sec. IV-C).
//
// Every trajectory pair of every object pair is tested at every step. A
// thread owns an RI x RJ micro-tile of trajectory pairs, walks the steps from
// the last to the first and records the step of each overlap, so the value
// left at the end is the earliest colliding step (or -1). Tests are exact
// closed-shape tests in FP32:
//   rectangle-rectangle: separating axes u_P, v_P, u_Q, v_Q; the projected
//     half extents use |cos(psi_Q - psi_P)| and |sin(psi_Q - psi_P)|;
//   rectangle-circle: distance from the centre to the rectangle <= r;
//   circle-circle: centre distance <= r_P + r_Q.
// ===========================================================================

struct CheckVV {
    float lP, wP, lQ, wQ;
    __device__ __forceinline__ bool operator()(const float4 P, const float4 Q) const
    {
        const float dx = Q.x - P.x;
        const float dy = Q.y - P.y;
        const float C = fmaf(P.z, Q.z, P.w * Q.w);    // u_P . u_Q = v_P . v_Q
        const float S = fmaf(P.z, Q.w, -(P.w * Q.z)); // v_P . u_Q = -u_P . v_Q
        const float aC = fabsf(C), aS = fabsf(S);
        const float p1 = fmaf(dx, P.z, dy * P.w);     // d . u_P
        const float p2 = fmaf(dy, P.z, -(dx * P.w));  // d . v_P
        const float p3 = fmaf(dx, Q.z, dy * Q.w);     // d . u_Q
        const float p4 = fmaf(dy, Q.z, -(dx * Q.w));  // d . v_Q
        const float r1 = fmaf(lQ, aC, fmaf(wQ, aS, lP));
        const float r2 = fmaf(lQ, aS, fmaf(wQ, aC, wP));
        const float r3 = fmaf(lP, aC, fmaf(wP, aS, lQ));
        const float r4 = fmaf(lP, aS, fmaf(wP, aC, wQ));
        return (fabsf(p1) <= r1) & (fabsf(p2) <= r2) & (fabsf(p3) <= r3) & (fabsf(p4) <= r4);
    }
};

__device__ __forceinline__ bool rect_circle(const float4 P, const float2 Q, float lP, float wP, float rr)
{
    const float dx = Q.x - P.x;
    const float dy = Q.y - P.y;
    const float lam = fmaf(dx, P.z, dy * P.w);
    const float mu = fmaf(dy, P.z, -(dx * P.w));
    const float ex = fmaxf(fabsf(lam) - lP, 0.0f);
    const float ey = fmaxf(fabsf(mu) - wP, 0.0f);
    return fmaf(ex, ex, ey * ey) <= rr;
}

struct CheckVP {
    float lP, wP, rr;
    __device__ __forceinline__ bool operator()(const float4 P, const float2 Q) const { return rect_circle(P, Q, lP, wP, rr); }
};

struct CheckPV {
    float lQ, wQ, rr;
    __device__ __forceinline__ bool operator()(const float2 P, const float4 Q) const { return rect_circle(Q, P, lQ, wQ, rr); }
};

struct CheckPP {
    float rr;
    __device__ __forceinline__ bool operator()(const float2 P, const float2 Q) const
    {
        const float dx = Q.x - P.x;
        const float dy = Q.y - P.y;
        return fmaf(dx, dx, dy * dy) <= rr;
    }
};

template <int RI, int RJ, class PA, class PB, class Check>
__device__ __forceinline__ void collide_items(const DPair &pr, int item0, const char *__restrict__ poses,
                                              int16_t *__restrict__ hits, const Check chk)
{
    const int n_ig = pr.n_ig, n_jg = pr.n_jg;
    const int f = item0 + (int)threadIdx.x;
    if (f >= n_ig * n_jg) return;
    const int ig = f / n_jg;
    const int jg = f - ig * n_jg;
    const int Ta = pr.Ta, Tb = pr.Tb;
    int ia[RI], jb[RJ];
#pragma unroll
    for (int r = 0; r < RI; ++r) ia[r] = min(ig + r * n_ig, Ta - 1);
#pragma unroll
    for (int s = 0; s < RJ; ++s) jb[s] = min(jg + s * n_jg, Tb - 1);
    const PA *__restrict__ A = reinterpret_cast<const PA *>(poses + pr.pose_a);
    const PB *__restrict__ B = reinterpret_cast<const PB *>(poses + pr.pose_b);
    int first[RI][RJ];
#pragma unroll
    for (int r = 0; r < RI; ++r)
#pragma unroll
        for (int s = 0; s < RJ; ++s) first[r][s] = -1;

    for (int t = pr.H - 1; t >= 0; --t) {
        const PA *__restrict__ At = A + (size_t)t * Ta;
        const PB *__restrict__ Bt = B + (size_t)t * Tb;
        PA a[RI];
        PB b[RJ];
#pragma unroll
        for (int r = 0; r < RI; ++r) a[r] = At[ia[r]];
#pragma unroll
        for (int s = 0; s < RJ; ++s) b[s] = Bt[jb[s]];
#pragma unroll
        for (int r = 0; r < RI; ++r)
#pragma unroll
            for (int s = 0; s < RJ; ++s)
                if (chk(a[r], b[s])) first[r][s] = t;
    }
#pragma unroll
    for (int r = 0; r < RI; ++r) {
        const int i = ig + r * n_ig;
#pragma unroll
        for (int s = 0; s < RJ; ++s) {
            const int j = jg + s * n_jg;
            if (i < Ta && j < Tb) hits[pr.hit_off + (int64_t)i * Tb + j] = (int16_t)first[r][s];
        }
    }
}

template <int V>
__device__ __forceinline__ void collide_work(const DPair &pr, int item0, const char *__restrict__ poses,
                                             int16_t *__restrict__ hits)
{
    switch (pr.cls) {
    case CLS_VV:
        collide_items<kTiles[V][CLS_VV].ri, kTiles[V][CLS_VV].rj, float4, float4>(
            pr, item0, poses, hits, CheckVV{pr.la, pr.wa, pr.lb, pr.wb});
        break;
    case CLS_VP:
        collide_items<kTiles[V][CLS_VP].ri, kTiles[V][CLS_VP].rj, float4, float2>(
            pr, item0, poses, hits, CheckVP{pr.la, pr.wa, pr.rr});
        break;
    case CLS_PV:
        collide_items<kTiles[V][CLS_PV].ri, kTiles[V][CLS_PV].rj, float2, float4>(
            pr, item0, poses, hits, CheckPV{pr.lb, pr.wb, pr.rr});
        break;
    default:
        collide_items<kTiles[V][CLS_PP].ri, kTiles[V][CLS_PP].rj, float2, float2>(
            pr, item0, poses, hits, CheckPP{pr.rr});
        break;
    }
}

template <int V>
__global__ __launch_bounds__(WG) void k2_collide(const DPair *__restrict__ pairs, const WorkItem *__restrict__ work,
                                                 const char *__restrict__ poses, int16_t *__restrict__ hits)
{
    const WorkItem w = work[blockIdx.x];
    const DPair pr = pairs[w.pair];
    collide_work<V>(pr, w.item0, poses, hits);
}

// ===========================================================================
// K3: risk assessment (Sec. IV-D, IV-D.2).
//
// q_{a,i;b} = sum_j [first_hit >= 0] p_{b,j} for both directions of every
// pair (rows: one wave per trajectory i of a, lanes over j; columns: one
// thread per trajectory j of b, sequential over i), then per trajectory
// crit = 1 - prod_{b != a} (1 - q_{a,i;b}) in ascending b and per object
// C_a = sum_i p_{a,i} crit_{a,i}. Every sum runs in a fixed order that does
// not depend on how the collision kernel was tiled, so results are identical
// for any tiling and any batch.
// ===========================================================================

__global__ __launch_bounds__(WG) void k3_qsum(const DObj *__restrict__ objs, const DPair *__restrict__ pairs,
                                              const K3Item *__restrict__ items, const int16_t *__restrict__ hits,
                                              const double *__restrict__ p, double *__restrict__ q)
{
    const K3Item it = items[blockIdx.x];
    const DPair pr = pairs[it.pair];
    const DObj oa = objs[pr.a];
    const DObj ob = objs[pr.b];
    const int16_t *__restrict__ h = hits + pr.hit_off;
    if (it.kind == 0) {
        const int lane = threadIdx.x & 63;
        const int i = it.start + (int)(threadIdx.x >> 6);
        if (i >= pr.Ta) return;
        const double *__restrict__ pb = p + ob.traj_off;
        double acc = 0.0;
        for (int j = lane; j < pr.Tb; j += 64)
            if (h[(int64_t)i * pr.Tb + j] >= 0) acc += pb[j];
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m, 64);
        if (lane == 0) q[oa.q_row + (int64_t)i * oa.n_scene_obj + ob.local] = fmin(acc, 1.0);
    } else {
        const int j = it.start + (int)threadIdx.x;
        if (j >= pr.Tb) return;
        const double *__restrict__ pa = p + oa.traj_off;
        double acc = 0.0;
        for (int i = 0; i < pr.Ta; ++i)
            if (h[(int64_t)i * pr.Tb + j] >= 0) acc += pa[i];
        q[ob.q_row + (int64_t)j * ob.n_scene_obj + oa.local] = fmin(acc, 1.0);
    }
}

__global__ __launch_bounds__(WG) void k3_crit(const DObj *__restrict__ objs, const int32_t *__restrict__ pairmap,
                                              const double *__restrict__ p, double *__restrict__ q,
                                              double *__restrict__ traj_crit, double *__restrict__ obj_crit)
{
    __shared__ double red[WG];
    const DObj o = objs[blockIdx.x];
    const int n = o.n_scene_obj;
    const int32_t *__restrict__ pm = pairmap + o.pairmap_off;
    const int tid = threadIdx.x;
    double part = 0.0;
    for (int i = tid; i < o.T; i += WG) {
        double *__restrict__ qi = q + o.q_row + (int64_t)i * n;
        double no_collision = 1.0;
        for (int b = 0; b < n; ++b) {
            if (pm[b] < 0) {
                qi[b] = 0.0;
            } else {
                no_collision *= 1.0 - qi[b];
            }
        }
        const double crit = 1.0 - no_collision;
        traj_crit[o.traj_off + i] = crit;
        part += p[o.traj_off + i] * crit;
    }
    red[tid] = part;
    __syncthreads();
    for (int s = WG / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) obj_crit[o.obj_out] = red[0];
}

// ===========================================================================
// Launchers
// ===========================================================================

hipError_t launch_trajgen(const Launch &L, hipStream_t s)
{
    if (L.n_k1 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k1_trajgen, dim3(L.n_k1), dim3(WG), 0, s, L.objs, L.vals, L.k1, L.poses, L.p);
    return hipGetLastError();
}

hipError_t launch_collide(const Launch &L, hipStream_t s)
{
    if (L.n_work <= 0) return hipSuccess;
    switch (L.variant) {
    case 0: hipLaunchKernelGGL(k2_collide<0>, dim3(L.n_work), dim3(WG), 0, s, L.pairs, L.work, L.poses, L.hits); break;
    case 1: hipLaunchKernelGGL(k2_collide<1>, dim3(L.n_work), dim3(WG), 0, s, L.pairs, L.work, L.poses, L.hits); break;
    case 2: hipLaunchKernelGGL(k2_collide<2>, dim3(L.n_work), dim3(WG), 0, s, L.pairs, L.work, L.poses, L.hits); break;
    case 3: hipLaunchKernelGGL(k2_collide<3>, dim3(L.n_work), dim3(WG), 0, s, L.pairs, L.work, L.poses, L.hits); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_risk(const Launch &L, hipStream_t s)
{
    if (L.n_k3 > 0) {
        hipLaunchKernelGGL(k3_qsum, dim3(L.n_k3), dim3(WG), 0, s, L.objs, L.pairs, L.k3, L.hits, L.p, L.q);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (L.n_obj > 0) {
        hipLaunchKernelGGL(k3_crit, dim3(L.n_obj), dim3(WG), 0, s, L.objs, L.pairmap, L.p, L.q, L.traj_crit, L.obj_crit);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace mhc
