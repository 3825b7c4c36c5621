// HIP kernels for gfx950 (CDNA4): trajectory generation, collision
// recognition and risk assessment of the multi-hypothesis criticality method
// (Sanchez Morales et al., IEEE IV 2019, Fig. 1: the three modules after
// street data processing, run in that order, each data-parallel inside).
#include "mhc_internal.h"

#include <climits>
#include <math.h>
#include <mutex>

// The overlap tests combine their comparisons with bitwise & and | on bools
// on purpose: every comparison is evaluated and the results are merged as
// lane masks, with no branch per comparison.
#pragma clang diagnostic ignored "-Wbitwise-instead-of-logical"

namespace mhc {

// ===========================================================================
// K1: trajectory generation (Sec. IV-B) and probability normalisation
// (Sec. IV-D.1).
//
// Vehicles follow the Euler pose update of Sec. IV-B.1 with side slip 0 and
// no yaw acceleration: in step n the speed v_n, heading psi_n = psi0 + n*w*tau
// and acceleration give the displacement
//   dx_n = c(psi_n) v_n tau + c(psi_n) a_x tau^2/2 - s(psi_n) a_y tau^2/2
//   dy_n = s(psi_n) v_n tau + s(psi_n) a_x tau^2/2 + c(psi_n) a_y tau^2/2
// with a_x the acceleration cut so that the speed stops at 0 and
// a_y = v_n w. The speed of a constant acceleration with a stop at 0 has the
// closed form max(0, v0 + n a tau), so every step's displacement is
// independent: one wave integrates one trajectory, lane q computing step
// n0 + q (FP64, including its own sine/cosine), and the positions are the
// running sums of the displacements, formed by a wave-wide scan and carried
// from one 64-step chunk to the next. Pedestrians (Sec. IV-B.3) move by the
// constant displacement of their speed and heading each step.
// Poses are stored as FP32: float4 (x, y, cos psi, sin psi) for vehicles,
// float2 (x, y) for pedestrians, layout [t][i], slot t = step t+1.
// ===========================================================================

// The integer summand of one colliding combination of probability p: p itself
// in units of 2^-62 (EXCLUSIVE reading: an object's trajectories exclude one
// another, so the q of an object is a sum of p), or -log(1 - p), capped at
// 64, in units of 2^-56 (INDEPENDENT reading: q = 1 - prod(1 - p) =
// 1 - exp(-sum of -log(1 - p))).
__device__ __forceinline__ unsigned long long fixed_term(int risk, double p)
{
    if (risk == RISK_EXCLUSIVE) return __double2ull_rn(p * kQScale);
    return __double2ull_rn(fmin(-log1p(-p), kLCap) * kLScale);
}

// q from its integer sum, under the object's reading.
__device__ __forceinline__ double q_of(int risk, unsigned long long v)
{
    if (risk == RISK_EXCLUSIVE) return fmin((double)v * kQInvScale, 1.0);
    return -expm1(-(double)v * kLInvScale);
}

// A double moved across lanes by the DPP control CTRL in the rows of
// ROW_MASK; a lane without a source (or outside those rows) gets `old`.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double x, double old)
{
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(x), CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(x), CTRL, ROW_MASK, 0xF, false);
    return __hiloint2double(hi, lo);
}

// The steps of a wave-wide inclusive scan over 64 lanes without LDS: shifts
// by 1, 2, 4 and 8 lanes within each row of 16 (row_shr), then lane 15 of
// rows 0 and 2 into rows 1 and 3 (row_bcast:15), then lane 31 into rows 2 and
// 3 (row_bcast:31). After step k every lane holds the combination of the
// lanes below it up to the step's reach, so after the six it holds lanes
// 0..l. DPP controls of the GFX9 family.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143, kDppWaveShr1 = 0x138;

// Inclusive prefix sum over the 64 lanes of a wave (lane l gets the sum of
// lanes 0..l).
__device__ __forceinline__ double scan_add(double v, int lane)
{
    (void)lane;
    v += dpp_move<kDppRowShr1, 0xF>(v, 0.0);
    v += dpp_move<kDppRowShr2, 0xF>(v, 0.0);
    v += dpp_move<kDppRowShr4, 0xF>(v, 0.0);
    v += dpp_move<kDppRowShr8, 0xF>(v, 0.0);
    v += dpp_move<kDppRowBcast15, 0xA>(v, 0.0);
    v += dpp_move<kDppRowBcast31, 0xC>(v, 0.0);
    return v;
}

// The value of the lane below (lane 0 gets `first`).
__device__ __forceinline__ double lane_below(double x, double first) { return dpp_move<kDppWaveShr1, 0xF>(x, first); }

// The sum of v over a workgroup of WG threads, in a fixed order: each wave's
// sum by the DPP scan (its lane 63), then the waves' sums in wave order. Every
// thread of the workgroup must call it; the result is valid in every thread.
__device__ __forceinline__ double block_sum(double v, double *ws)
{
    const int lane = (int)(threadIdx.x & (WAVE - 1)), w = (int)(threadIdx.x / WAVE);
    v = scan_add(v, lane);
    if (lane == WAVE - 1) ws[w] = v;
    __syncthreads();
    double s = ws[0];
#pragma unroll
    for (int k = 1; k < WG / WAVE; ++k) s += ws[k];
    return s;
}

// Thread tid adds the scores tid, tid + 256, ... in ascending order, eight
// loads in flight at a time, then the workgroup adds the 256 partial sums in a
// fixed order (block_sum): the order depends on T only.
__device__ void normalise_probabilities(const DObj &o, int obj, const double *__restrict__ vals,
                                        double *__restrict__ p, unsigned long long *__restrict__ pfix,
                                        unsigned long long *__restrict__ done)
{
    __shared__ double red[WG / WAVE];
    const int tid = threadIdx.x;
    const double *__restrict__ sc = vals + o.score_off;
    double part = 0.0;
    if (o.has_score) {
        for (int base = 0; base < o.T; base += 8 * WG) {
            double v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int idx = base + k * WG + tid;
                v[k] = idx < o.T ? sc[idx] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (base + k * WG + tid < o.T) part += v[k];
        }
    }
    const double total = block_sum(part, red);
    for (int base = 0; base < o.T; base += 8 * WG) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int idx = base + k * WG + tid;
            v[k] = (o.has_score && idx < o.T) ? sc[idx] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int idx = base + k * WG + tid;
            if (idx < o.T) {
                const double pk = o.has_score ? v[k] / total : 1.0 / (double)o.T;
                p[o.traj_off + idx] = pk;
                pfix[o.traj_off + idx] = fixed_term(o.risk, pk);
            }
        }
    }
    // the object's completion counter of the risk kernel starts from zero
    // (each trajectory's wave clears its row of the q accumulators)
    if (tid == 0) done[obj] = 0ull;
}

// A vehicle pose (x, y, cos, sin) in its own frame: K = (x cos + y sin,
// y cos - x sin) is its centre there, and (K_x, K_y, cos, sin) is what the
// rectangle tests take for the rectangle they measure in its frame. The
// trajectory kernel writes it beside the pose (the object's frame block), in
// FP32 from the stored FP32 pose, so that no test prepares it again.
__device__ __forceinline__ float4 rect_frame(const float4 P)
{
    return make_float4(fmaf(P.x, P.z, P.y * P.w), fmaf(P.y, P.z, -(P.x * P.w)), P.z, P.w);
}

// Stores vehicle pose n of trajectory i and its frame form.
__device__ __forceinline__ void store_vehicle_pose(char *__restrict__ poses, const DObj &o, int n, int i, const float4 P)
{
    const size_t k = (size_t)n * o.T + i;
    reinterpret_cast<float4 *>(poses + o.pose_off)[k] = P;
    reinterpret_cast<float4 *>(poses + o.frame_off)[k] = rect_frame(P);
}

// Vehicle trajectory i on the linear one-track model (Sec. IV-B.1): side slip
// beta and yaw rate r obey
//   beta' = -(cf+cr)/(m v) beta + ((cr lr - cf lf)/(m v^2) - 1) r + cf/(m v) delta
//   r'    = (cr lr - cf lf)/Iz beta - (cf lf^2 + cr lr^2)/(Iz v) r + cf lf/Iz delta
// for the constant steering angle delta = w[l], integrated with the paper's
// Euler pose update (accelerations a_x, a_y in the vehicle frame from step
// n, the speed stopping at 0). Where the explicit step is unstable (an
// eigenvalue of I + tau A(v_n) of modulus >= 1, tested by the Jury
// conditions) the lateral state takes the steady state at v_{n+1} instead:
//   r = v delta / (L (1 + K v^2)), beta = delta (lr/L - m lf v^2/(cr L^2)) / (1 + K v^2),
// L = lf + lr, K = m (lr cr - lf cf) / (L^2 cf cr). FP64; poses stored as
// FP32 (x, y, cos psi, sin psi), [t][i].
//
// Evaluation: one wave per trajectory, a lane per step, chunks of 64 steps
// with the state carried across chunks. The speed has a closed form,
// v_n = max(v_0 + n a tau, 0), and it alone decides each step's
// update of s = (beta, r): an explicit Euler step s_{n+1} = M_n s_n + c_n
// where that step is stable, else the steady state of the speed reached,
// s_{n+1} = s*(v_{n+1}) (M_n = 0). These affine maps compose, so an
// inclusive scan over the lanes gives every s_n of the chunk at once; the
// rates of step n follow from s_n and s_{n+1} as in the serial update, and
// the heading and the position are prefix sums of the per-step increments.
// Only the order of the additions differs from the serial recursion.


__device__ void one_track_wave(const DObj &o, const double *__restrict__ vals, char *__restrict__ poses, int i,
                               int lane)
{
    const double cf = o.params[0], cr = o.params[1], lf = o.params[2], lr = o.params[3];
    const double m = o.params[4], Iz = o.params[5];
    const double L = lf + lr;
    const double K = m * (lr * cr - lf * cf) / (L * L * cf * cr);
    const double cd = cr * lr - cf * lf;
    const double cq = cf * lf * lf + cr * lr * lr;
    // the model's coefficients without their speed factors
    const double kb = (cf + cr) / m, kc = cd / m, kf = cf / m;       // beta'
    const double kcz = cd / Iz, kq = cq / Iz, kfz = cf * lf / Iz;   // r'
    const double lr_L = lr / L, mlf_crL2 = m * lf / (cr * L * L);    // steady state
    const int k = i / o.n_w, l = i - (i / o.n_w) * o.n_w;
    const double accel = vals[o.u_off + k];
    const double delta = vals[o.w_off + l];
    const double tau = o.tau, h2 = tau * tau / 2.0, at = accel * tau;
    // state at the chunk's first step
    double cx = o.x, cy = o.y, cpsi = o.heading, cbeta = 0.0, crate = 0.0, csp, ccp;
    sincos(cpsi, &csp, &ccp);
    for (int n0 = 0; n0 < o.H; n0 += 64) {
        const int n = n0 + lane;
        const bool active = n < o.H;
        const double v = fmax(o.speed + (double)n * at, 0.0);
        double vdot = accel, v1 = v + at;
        if (v1 < 0.0) {
            vdot = -v / tau;
            v1 = 0.0;
        }
        bool stable = false;
        const double iv = v > 0.0 ? 1.0 / v : 0.0;
        double a11 = 1.0, a12 = 0.0, a21 = 0.0, a22 = 1.0, b1 = 0.0, b2 = 0.0;  // identity past the horizon
        if (active) {
            if (v > 0.0) {
                const double m11 = 1.0 - tau * kb * iv, m12 = tau * (kc * iv * iv - 1.0);
                const double m21 = tau * kcz, m22 = 1.0 - tau * kq * iv;
                const double tr = m11 + m22, det = m11 * m22 - m12 * m21;
                stable = det < 1.0 && tr < 1.0 + det && tr > -(1.0 + det);
                if (stable) {
                    a11 = m11;
                    a12 = m12;
                    a21 = m21;
                    a22 = m22;
                    b1 = tau * kf * iv * delta;
                    b2 = tau * kfz * delta;
                }
            }
            if (!stable) {
                const double g = 1.0 + K * v1 * v1;
                a11 = a12 = a21 = a22 = 0.0;
                b1 = delta * (lr_L - mlf_crL2 * v1 * v1) / g;
                b2 = v1 * delta / (L * g);
            }
        }
        // lane n: the composition f_n o ... o f_{n0}; (A, b) o (P, q) = (AP, Aq + b),
        // in the steps of scan_add (a lane without a source composes with the
        // identity, which leaves its map as it is)
        auto compose = [&](double p11, double p12, double p21, double p22, double q1, double q2) {
            const double n11 = a11 * p11 + a12 * p21, n12 = a11 * p12 + a12 * p22;
            const double n21 = a21 * p11 + a22 * p21, n22 = a21 * p12 + a22 * p22;
            const double nb1 = a11 * q1 + a12 * q2 + b1, nb2 = a21 * q1 + a22 * q2 + b2;
            a11 = n11;
            a12 = n12;
            a21 = n21;
            a22 = n22;
            b1 = nb1;
            b2 = nb2;
        };
#define MHC_COMPOSE_STEP(CTRL, ROWS)                                                                           \
    compose(dpp_move<CTRL, ROWS>(a11, 1.0), dpp_move<CTRL, ROWS>(a12, 0.0), dpp_move<CTRL, ROWS>(a21, 0.0), \
            dpp_move<CTRL, ROWS>(a22, 1.0), dpp_move<CTRL, ROWS>(b1, 0.0), dpp_move<CTRL, ROWS>(b2, 0.0))
        MHC_COMPOSE_STEP(kDppRowShr1, 0xF);
        MHC_COMPOSE_STEP(kDppRowShr2, 0xF);
        MHC_COMPOSE_STEP(kDppRowShr4, 0xF);
        MHC_COMPOSE_STEP(kDppRowShr8, 0xF);
        MHC_COMPOSE_STEP(kDppRowBcast15, 0xA);
        MHC_COMPOSE_STEP(kDppRowBcast31, 0xC);
#undef MHC_COMPOSE_STEP
        // (beta, r) after step n, and before it (the previous lane's, or the carry)
        const double beta1 = a11 * cbeta + a12 * crate + b1;
        const double r1 = a21 * cbeta + a22 * crate + b2;
        const double beta = lane_below(beta1, cbeta), r = lane_below(r1, crate);
        double beta_dot, r_dot;
        if (stable) {
            beta_dot = -kb * iv * beta + (kc * iv * iv - 1.0) * r + kf * iv * delta;
            r_dot = kcz * beta - kq * iv * r + kfz * delta;
        } else {
            beta_dot = (beta1 - beta) / tau;
            r_dot = (r1 - r) / tau;
        }
        // heading after step n; the step itself turns with the heading before it
        const double psi1 = cpsi + scan_add(active ? r * tau + r_dot * h2 : 0.0, lane);
        double sp1, cp1;
        sincos(psi1, &sp1, &cp1);
        const double sp = lane_below(sp1, csp), cp = lane_below(cp1, ccp);
        double sb, cb;
        sincos(beta, &sb, &cb);
        const double spb = sp * cb + cp * sb, cpb = cp * cb - sp * sb;   // psi + beta
        const double ax = cb * vdot - sb * v * (beta_dot + r);
        const double ay = sb * vdot + cb * v * (beta_dot + r);
        const double x1 = cx + scan_add(active ? cpb * v * tau + cp * ax * h2 - sp * ay * h2 : 0.0, lane);
        const double y1 = cy + scan_add(active ? spb * v * tau + sp * ax * h2 + cp * ay * h2 : 0.0, lane);
        if (active) store_vehicle_pose(poses, o, n, i, make_float4((float)x1, (float)y1, (float)cp1, (float)sp1));
        cx = __shfl(x1, 63, 64);
        cy = __shfl(y1, 63, 64);
        cpsi = __shfl(psi1, 63, 64);
        csp = __shfl(sp1, 63, 64);
        ccp = __shfl(cp1, 63, 64);
        cbeta = __shfl(beta1, 63, 64);
        crate = __shfl(r1, 63, 64);
    }
}

// Grid: y = object; x = 0 is the object's probability normalisation (the
// longest block for large T, so it is dispatched first), x >= 1 are
// trajectory blocks of K1_TPB trajectories, one wave each.
// ONE_TRACK: whether the instance carries the one-track model's scan, whose
// FP64 state needs far more registers (130 VGPRs against the kinematic
// instance's); launches without one-track vehicles use the lighter instance,
// which also fits beside a running collision kernel on a shared GPU.
// For time-resolved scenes, trajectory block c also zeroes the c-th stretch
// of K1_TPB * W * H entries of the object's per-slot q sums.
template <bool ONE_TRACK>
__global__ __launch_bounds__(WG) void k1_trajgen(const DObj *__restrict__ objs, const double *__restrict__ vals,
                                                 char *__restrict__ poses, double *__restrict__ p,
                                                 unsigned long long *__restrict__ pfix,
                                                 unsigned long long *__restrict__ qacc, unsigned long long *__restrict__ done,
                                                 unsigned long long *__restrict__ hist, const int2 *__restrict__ rows)
{
    // the row's object and the block of that object this workgroup is
    int obj = (int)blockIdx.y, xb = (int)blockIdx.x;
    if (rows) {
        const int2 r = rows[blockIdx.y];
        obj = r.x;
        xb += r.y;
    }
    const DObj o = objs[obj];
    if (xb == 0) {
        normalise_probabilities(o, obj, vals, p, pfix, done);
        return;
    }
    if (o.timeline) {
        const int64_t per = (int64_t)K1_TPB * o.tl_w * o.H;
        const int64_t total = (int64_t)o.T * o.tl_w * o.H;
        const int64_t lo = ((int64_t)xb - 1) * per;
        const int64_t hi = min(total, lo + per);
        // 16-byte stores: hist_off, the stretch and the total are even
        ulonglong2 *h2 = reinterpret_cast<ulonglong2 *>(hist + o.hist_off);
        for (int64_t k = lo / 2 + (int64_t)threadIdx.x; k < hi / 2; k += WG) h2[k] = make_ulonglong2(0ull, 0ull);
    }
    const int lane = threadIdx.x & 63;
    const int i = (xb - 1) * K1_TPB + (int)(threadIdx.x >> 6);
    if (i >= o.T) return;  // whole wave
    // this trajectory's row of the integer q accumulators starts from zero
    for (int k = lane; k < o.n_scene_obj; k += 64) qacc[o.q_row + (int64_t)i * o.n_scene_obj + k] = 0ull;
    if constexpr (ONE_TRACK) {
        if (o.model == MODEL_ONE_TRACK) {
            one_track_wave(o, vals, poses, i, lane);
            return;
        }
    }
    const int k = i / o.n_w, l = i - (i / o.n_w) * o.n_w;
    const double tau = o.tau;
    const double half_tau2 = tau * tau / 2.0;
    const int H = o.H;
    const bool vehicle = o.kind == KIND_VEHICLE;
    const double u = vals[o.u_off + k];
    const double w = vals[o.w_off + l];
    // pedestrians: kinematic model (speed u, heading offset w) or the
    // acceleration model (acceleration u, absolute heading w, speed clamped
    // to [0, v_max]: after the first step v_n = clamp(v_1 + (n-1) u tau))
    const bool ped_accel = o.model == MODEL_PED_ACCEL;
    double ped_c = 0.0, ped_s = 0.0;
    if (!vehicle) sincos(ped_accel ? w : o.heading + w, &ped_s, &ped_c);
    const double v_max = o.params[0];
    const double v_first = ped_accel ? fmin(fmax(o.speed + u * tau, 0.0), v_max) : 0.0;
    double cx = o.x, cy = o.y;
    for (int n0 = 0; n0 < H; n0 += 64) {
        const int n = n0 + lane;
        const bool active = n < H;
        double dx = 0.0, dy = 0.0;
        float c_next = 0.f, s_next = 0.f;
        if (active) {
            if (vehicle) {
                const double wt = w * tau;
                double sn, cn, s1, c1;
                sincos(o.heading + (double)n * wt, &sn, &cn);
                sincos(o.heading + (double)(n + 1) * wt, &s1, &c1);
                const double at = u * tau;
                double v = o.speed + (double)n * at;
                const double v_next = o.speed + (double)(n + 1) * at;
                double ax = u;
                if (v_next < 0.0) {
                    if (v <= 0.0) {
                        v = 0.0;
                        ax = 0.0;
                    } else {
                        ax = -v / tau;
                    }
                }
                const double ay = v * w;
                dx = cn * v * tau + cn * ax * half_tau2 - sn * ay * half_tau2;
                dy = sn * v * tau + sn * ax * half_tau2 + cn * ay * half_tau2;
                c_next = (float)c1;
                s_next = (float)s1;
            } else if (ped_accel) {
                // step n -> n+1 moves by the mean of the two speeds
                const double vn = n == 0 ? o.speed : fmin(fmax(v_first + (double)(n - 1) * u * tau, 0.0), v_max);
                const double vn1 = fmin(fmax(v_first + (double)n * u * tau, 0.0), v_max);
                const double dist = (vn + vn1) * (tau / 2.0);
                dx = ped_c * dist;
                dy = ped_s * dist;
            } else {
                dx = ped_c * u * tau;
                dy = ped_s * u * tau;
            }
        }
        dx = scan_add(dx, lane);
        dy = scan_add(dy, lane);
        const double x = cx + dx, y = cy + dy;
        if (active) {
            if (vehicle)
                store_vehicle_pose(poses, o, n, i, make_float4((float)x, (float)y, c_next, s_next));
            else
                reinterpret_cast<float2 *>(poses + o.pose_off)[(size_t)n * o.T + i] = make_float2((float)x, (float)y);
        }
        cx = __shfl(x, 63, 64);
        cy = __shfl(y, 63, 64);
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
// The point-in-polygon mode instead tests the four corners of each rectangle
// against the other rectangle (the paper's test, both ways).
// ===========================================================================


// Rectangle-rectangle (separating axes). With C = u_P.u_Q and S = v_P.u_Q
// (so u_P = C u_Q - S v_Q, v_P = S u_Q + C v_Q) and d = c_Q - c_P, the
// rectangles overlap iff
//   |d.u_P| <= lP + lQ|C| + wQ|S|,   |d.v_P| <= wP + lQ|S| + wQ|C|,
//   |d.u_Q| <= lQ + lP|C| + wP|S|,   |d.v_Q| <= wQ + lP|S| + wP|C|.
// Q's pose comes in its own frame (its object's frame block: K = c_Q there),
// so d.u_Q = K.x - (x_P cos_Q + y_P sin_Q) and d.v_Q = K.y - (y_P cos_Q - x_P
// sin_Q) are two FMA chains each, and d.u_P, d.v_P follow from them by the
// rotation (C, S): 25 VALU per test.
struct CheckVV {
    float lP, wP, lQ, wQ;
    __device__ __forceinline__ bool operator()(const float4 P, const float4 Qk) const
    {
        const float C = fmaf(P.z, Qk.z, P.w * Qk.w);    // u_P . u_Q = v_P . v_Q
        const float S = fmaf(P.z, Qk.w, -(P.w * Qk.z)); // v_P . u_Q = -u_P . v_Q
        const float aC = fabsf(C), aS = fabsf(S);
        const float p3 = fmaf(-P.x, Qk.z, fmaf(-P.y, Qk.w, Qk.x));  // d . u_Q
        const float p4 = fmaf(-P.y, Qk.z, fmaf(P.x, Qk.w, Qk.y));   // d . v_Q
        const float p1 = fmaf(C, p3, -(S * p4));                     // d . u_P
        const float p2 = fmaf(S, p3, C * p4);                        // d . v_P
        const float r1 = fmaf(lQ, aC, fmaf(wQ, aS, lP));
        const float r2 = fmaf(lQ, aS, fmaf(wQ, aC, wP));
        const float r3 = fmaf(lP, aC, fmaf(wP, aS, lQ));
        const float r4 = fmaf(lP, aS, fmaf(wP, aC, wQ));
        return (fabsf(p1) <= r1) & (fabsf(p2) <= r2) & (fabsf(p3) <= r3) & (fabsf(p4) <= r4);
    }
};

// Point-in-polygon both ways for two rectangles. A corner of Q is
// c_Q + al*lQ*u_Q + be*wQ*v_Q (al, be = +-1); in P's frame it sits at
//   x = d.u_P + al*lQ*C - be*wQ*S,   y = d.v_P + al*lQ*S + be*wQ*C
// (C = u_P.u_Q, S = v_P.u_Q, d = c_Q - c_P) and lies in the closed P iff
// |x| <= lP and |y| <= wP. The corners of P in Q's frame follow with the roles
// swapped; flipping both signs of a corner leaves |x| and |y| unchanged, so
// they are (d.u_Q + al*lP*C + be*wP*S, d.v_Q - al*lP*S + be*wP*C).
// Q's pose comes in its own frame and the projections are formed as in the
// separating-axes test.
struct CheckVVPip {
    float lP, wP, lQ, wQ;
    __device__ __forceinline__ bool operator()(const float4 P, const float4 Qk) const
    {
        const float C = fmaf(P.z, Qk.z, P.w * Qk.w);
        const float S = fmaf(P.z, Qk.w, -(P.w * Qk.z));
        const float p3 = fmaf(-P.x, Qk.z, fmaf(-P.y, Qk.w, Qk.x));  // d . u_Q
        const float p4 = fmaf(-P.y, Qk.z, fmaf(P.x, Qk.w, Qk.y));   // d . v_Q
        const float p1 = fmaf(C, p3, -(S * p4));                     // d . u_P
        const float p2 = fmaf(S, p3, C * p4);                        // d . v_P
        // Q's corners in P: (p1 +- g, p2 +- k) and (p1 +- h, p2 +- m), signs paired
        const float wQS = wQ * S, wQC = wQ * C;
        const float g = fmaf(lQ, C, -wQS), h = fmaf(lQ, C, wQS);
        const float k = fmaf(lQ, S, wQC), m = fmaf(lQ, S, -wQC);
        const bool q_in_p = ((fabsf(p1 + g) <= lP) & (fabsf(p2 + k) <= wP)) |
                            ((fabsf(p1 - g) <= lP) & (fabsf(p2 - k) <= wP)) |
                            ((fabsf(p1 + h) <= lP) & (fabsf(p2 + m) <= wP)) |
                            ((fabsf(p1 - h) <= lP) & (fabsf(p2 - m) <= wP));
        // P's corners in Q: (p3 +- g2, p4 -+ k2) and (p3 +- h2, p4 -+ m2)
        const float wPS = wP * S, wPC = wP * C;
        const float g2 = fmaf(lP, C, wPS), h2 = fmaf(lP, C, -wPS);
        const float k2 = fmaf(lP, S, -wPC), m2 = fmaf(lP, S, wPC);
        const bool p_in_q = ((fabsf(p3 + g2) <= lQ) & (fabsf(p4 - k2) <= wQ)) |
                            ((fabsf(p3 - g2) <= lQ) & (fabsf(p4 + k2) <= wQ)) |
                            ((fabsf(p3 + h2) <= lQ) & (fabsf(p4 - m2) <= wQ)) |
                            ((fabsf(p3 - h2) <= lQ) & (fabsf(p4 + m2) <= wQ));
        return q_in_p | p_in_q;
    }
};

// Rectangle-circle: the circle centre Q in P's frame is (lam, mu) =
// ((Q - c_P) . u_P, (Q - c_P) . v_P), and the two overlap iff the distance
// from Q to the rectangle, sqrt(max(|lam| - l, 0)^2 + max(|mu| - w, 0)^2), is
// at most r. The rectangle's pose comes in its own frame (its object's frame
// block): K = (x_P cos + y_P sin, y_P cos - x_P sin) is c_P there, so
//   (lam, mu) = (x_Q cos + y_Q sin - K.x, y_Q cos - x_Q sin - K.y)
// (two FMA chains each) without the difference Q - c_P: 12 VALU per test.
// Every tile computes each test with the same operations, so results do not
// depend on the tile.
__device__ __forceinline__ bool rect_circle(const float4 Pk, const float2 Q, float lP, float wP, float rr)
{
    const float lam = fmaf(Q.x, Pk.z, fmaf(Q.y, Pk.w, -Pk.x));
    const float mu = fmaf(Q.y, Pk.z, fmaf(-Q.x, Pk.w, -Pk.y));
    const float ex = fmaxf(fabsf(lam) - lP, 0.0f);
    const float ey = fmaxf(fabsf(mu) - wP, 0.0f);
    return fmaf(ex, ex, ey * ey) <= rr;
}

struct CheckVP {  // a: the rectangle, in its own frame
    float lP, wP, rr;
    __device__ __forceinline__ bool operator()(const float4 Pk, const float2 Q) const { return rect_circle(Pk, Q, lP, wP, rr); }
};

struct CheckPV {  // b: the rectangle, in its own frame
    float lQ, wQ, rr;
    __device__ __forceinline__ bool operator()(const float2 P, const float4 Qk) const { return rect_circle(Qk, P, lQ, wQ, rr); }
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

// General convex polygons (vehicle outlines; Sec. IV-C.1 allows polygons of
// any complexity). Q's vertices in P's frame are c + v_x (C, S) + v_y (-S, C) with
// c = (d.u_P, d.v_P); P's in Q's frame are c' + v_x (C, -S) + v_y (S, C)
// with c' = (-d.u_Q, -d.v_Q). With the unit outward edge normals n_e and
// offsets h_e of a polygon, a point x is inside iff n_e.x <= h_e for all e.
//   separating axes: disjoint iff for some edge of either polygon every
//     vertex of the other has n_e.x > h_e;
//   point-in-polygon (the paper's test, both ways): a hit iff some vertex of
//     one has n_e.x <= h_e for every edge of the other.
// Both read the same vertex-edge values. Polygons come padded to KP, KQ = 4
// or 8 vertices (repeated vertices and edges change none of the tests), so
// the loops are straight-line code; their constants are read from the wave's
// copy of the two polygons in LDS.
template <int KP, int KQ, bool PIPMODE>
struct CheckGG {
    const DPoly *P, *Q;   // LDS
    __device__ __forceinline__ bool operator()(const float4 a, const float4 b) const
    {
        const float dx = b.x - a.x;
        const float dy = b.y - a.y;
        const float C = fmaf(a.z, b.z, a.w * b.w);       // u_P . u_Q
        const float S = fmaf(a.z, b.w, -(a.w * b.z));    // v_P . u_Q
        const float lam = fmaf(dx, a.z, dy * a.w);       // d . u_P
        const float mu = fmaf(dy, a.z, -(dx * a.w));     // d . v_P
        const float lam2 = -fmaf(dx, b.z, dy * b.w);     // -d . u_Q
        const float mu2 = -fmaf(dy, b.z, -(dx * b.w));   // -d . v_Q
        float qx[KQ], qy[KQ], px[KP], py[KP];
#pragma unroll
        for (int v = 0; v < KQ; ++v) {
            qx[v] = fmaf(Q->vx[v], C, fmaf(-Q->vy[v], S, lam));
            qy[v] = fmaf(Q->vx[v], S, fmaf(Q->vy[v], C, mu));
        }
#pragma unroll
        for (int v = 0; v < KP; ++v) {
            px[v] = fmaf(P->vx[v], C, fmaf(P->vy[v], S, lam2));
            py[v] = fmaf(-P->vx[v], S, fmaf(P->vy[v], C, mu2));
        }
        if constexpr (!PIPMODE) {
            bool sep = false;
#pragma unroll
            for (int e = 0; e < KP; ++e) {
                const float nx = P->nx[e], ny = P->ny[e], h = P->h[e];
                bool out = true;
#pragma unroll
                for (int v = 0; v < KQ; ++v) out &= fmaf(nx, qx[v], ny * qy[v]) > h;
                sep |= out;
            }
#pragma unroll
            for (int e = 0; e < KQ; ++e) {
                const float nx = Q->nx[e], ny = Q->ny[e], h = Q->h[e];
                bool out = true;
#pragma unroll
                for (int v = 0; v < KP; ++v) out &= fmaf(nx, px[v], ny * py[v]) > h;
                sep |= out;
            }
            return !sep;
        } else {
            bool in_q[KQ], in_p[KP];
#pragma unroll
            for (int v = 0; v < KQ; ++v) in_q[v] = true;
#pragma unroll
            for (int v = 0; v < KP; ++v) in_p[v] = true;
#pragma unroll
            for (int e = 0; e < KP; ++e) {
                const float nx = P->nx[e], ny = P->ny[e], h = P->h[e];
#pragma unroll
                for (int v = 0; v < KQ; ++v) in_q[v] &= fmaf(nx, qx[v], ny * qy[v]) <= h;
            }
#pragma unroll
            for (int e = 0; e < KQ; ++e) {
                const float nx = Q->nx[e], ny = Q->ny[e], h = Q->h[e];
#pragma unroll
                for (int v = 0; v < KP; ++v) in_p[v] &= fmaf(nx, px[v], ny * py[v]) <= h;
            }
            bool hit = false;
#pragma unroll
            for (int v = 0; v < KQ; ++v) hit |= in_q[v];
#pragma unroll
            for (int v = 0; v < KP; ++v) hit |= in_p[v];
            return hit;
        }
    }
};

// Convex polygon G (K vertices, padded) and circle (centre c, squared radius
// rr): c in G's frame; a hit iff c is inside or its squared distance to some
// edge segment is at most rr.
template <int K>
__device__ __forceinline__ bool poly_circle(const float4 P, const float2 c, const DPoly *G, float rr)
{
    const float dx = c.x - P.x;
    const float dy = c.y - P.y;
    const float lam = fmaf(dx, P.z, dy * P.w);
    const float mu = fmaf(dy, P.z, -(dx * P.w));
    bool inside = true;
    float best = 3.0e38f;
#pragma unroll
    for (int e = 0; e < K; ++e) {
        inside &= fmaf(G->nx[e], lam, G->ny[e] * mu) <= G->h[e];
        const float ax = lam - G->vx[e], ay = mu - G->vy[e];
        const float t = fminf(fmaxf(fmaf(ax, G->ex[e], ay * G->ey[e]) * G->il[e], 0.0f), 1.0f);
        const float cx = fmaf(-t, G->ex[e], ax), cy = fmaf(-t, G->ey[e], ay);
        best = fminf(best, fmaf(cx, cx, cy * cy));
    }
    return inside | (best <= rr);
}

template <int K>
struct CheckGC {
    const DPoly *G;   // LDS
    float rr;
    __device__ __forceinline__ bool operator()(const float4 P, const float2 Q) const { return poly_circle<K>(P, Q, G, rr); }
};

template <int K>
struct CheckCG {
    const DPoly *G;   // LDS
    float rr;
    __device__ __forceinline__ bool operator()(const float2 P, const float4 Q) const { return poly_circle<K>(Q, P, G, rr); }
};

// Raw buffer descriptor (CDNA: dword3 = 0x00020000) over `bytes` bytes.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t pose_rsrc(const char *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(base), (short)0, (int)bytes, 0x00020000);
}

template <class P>
__device__ __forceinline__ P load_pose(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);

template <>
__device__ __forceinline__ float4 load_pose<float4>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
}

template <>
__device__ __forceinline__ float2 load_pose<float2>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}

// The minimum of v over the lanes l ^ E, l ^ 2E, ... (E = 64 >> tshift, the
// lanes of one item's parts), moved without LDS: lane l ^ 8 by a rotation of
// its row of 16 by 8 (DPP row_ror), l ^ 16 and l ^ 32 by the gfx950 lane-half
// swaps, whose two results hold each lane's own value and its partner's.
__device__ __forceinline__ int min_over_parts(int v, int tshift)
{
    if (tshift >= 3) v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x128, 0xF, 0xF, false));
    if (tshift >= 2) {
        const auto h = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        v = min((int)h[0], (int)h[1]);
    }
    const auto w = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return min((int)w[0], (int)w[1]);
}

// STAGE: the instance stages the poses of 8 x 8 item blocks in LDS (units of
// 2-D blocks without a time split): per step, the wave loads each distinct
// pose of its block once (lane k the k-th pose of either object) into LDS,
// and every lane then reads its tile's poses from there. The tests and
// their results are those of the unstaged loop; only where the poses come
// from differs. Each step's loads are issued before the previous step's tests.
template <int RI, int RJ, bool TL, class PA, class PB, class Check, bool STAGE = false>
__device__ __forceinline__ void collide_items(const DPair &pr, int item0, const char *__restrict__ poses,
                                              int16_t *__restrict__ hits, const unsigned long long *__restrict__ pfix,
                                              unsigned long long *__restrict__ qacc,
                                              unsigned long long *__restrict__ hist, const Check chk)
{
    const int n_ig = pr.n_ig, n_jg = pr.n_jg;
    // time split: E = 64 >> tshift items per unit; part p of the steps per
    // lane, chunk = ceil(H / S) steps from min(p * chunk, H - chunk), so the
    // last part ends at H (overlapping its neighbour when S does not divide H)
    const int lane = (int)(threadIdx.x & (WAVE - 1));
    const int tshift = pr.tshift;
    const int per = WAVE >> tshift;
    const int part = lane >> (6 - tshift);
    const int chunk = (pr.H + (1 << tshift) - 1) >> tshift;
    const int e = lane & (per - 1);
    // Item of this lane. Row-major units (bshift = 0) hold the items
    // item0 .. item0 + E-1; a block unit v is the block (v / nb, v % nb) of
    // E / 2^bshift rows and 2^bshift columns, which is the same as the
    // row-major decode of item (first row of the block) * n_jg + first column
    // + (e / 2^bshift) * n_jg + e % 2^bshift.
    const int bs = pr.bshift;
    int f;
    if (bs == 0) {
        f = item0 + e;
    } else {
        const int v = item0 >> (6 - tshift);
        const int nb = (n_jg + (1 << bs) - 1) >> bs;
        const int bi = v / nb;
        const int c0 = (v - bi * nb) << bs;                // first column of the block
        const int col = c0 + (e & ((1 << bs) - 1));
        // a column past the grid's edge is an idle lane
        f = col < n_jg ? (((bi << (6 - tshift)) >> bs) + (e >> bs)) * n_jg + col : INT_MAX;
    }
    const bool stage = STAGE && bs == 3 && tshift == 0;
    int ig, jg;
    bool live = true;  // the lane's item lies in the grid (staged blocks keep every lane to the end)
    int ig0 = 0, jg0 = 0;
    if (stage) {
        const int v = item0 >> 6;
        const int nb = (n_jg + 7) >> 3;
        const int bi = v / nb;
        ig0 = bi << 3;              // the block's first item row and column
        jg0 = (v - bi * nb) << 3;
        ig = ig0 + (e >> 3);
        jg = jg0 + (e & 7);
        live = ig < n_ig && jg < n_jg;
    } else {
        if (f >= n_ig * n_jg) return;  // every part of an item leaves together
        ig = f / n_jg;
        jg = f - ig * n_jg;
    }
    const int Ta = pr.Ta, Tb = pr.Tb;
    int ia[RI], jb[RJ];
#pragma unroll
    for (int r = 0; r < RI; ++r) ia[r] = min(ig + r * n_ig, Ta - 1);
#pragma unroll
    for (int s = 0; s < RJ; ++s) jb[s] = min(jg + s * n_jg, Tb - 1);
    // Poses are read with buffer loads: the step's offset t * T * sizeof(pose)
    // lives in a scalar register and the lane offsets are loop-invariant, so
    // no vector instruction is spent on addressing.
    const __amdgpu_buffer_rsrc_t A = pose_rsrc(poses + pr.pose_a, (uint32_t)((size_t)pr.H * Ta * sizeof(PA)));
    const __amdgpu_buffer_rsrc_t B = pose_rsrc(poses + pr.pose_b, (uint32_t)((size_t)pr.H * Tb * sizeof(PB)));
    const uint32_t strideA = (uint32_t)Ta * (uint32_t)sizeof(PA), strideB = (uint32_t)Tb * (uint32_t)sizeof(PB);
    // lane offsets: the trajectory and the first step of this lane's part
    const uint32_t t0 = (uint32_t)min(part * chunk, pr.H - chunk);
    int first[RI][RJ];
#pragma unroll
    for (int r = 0; r < RI; ++r)
#pragma unroll
        for (int s = 0; s < RJ; ++s) first[r][s] = -1;

    if constexpr (STAGE) {
        if (stage) {
            // the block's 8 item rows give 8 * RI trajectories of a (entry
            // r * 8 + row), its 8 columns 8 * RJ of b (entry s * 8 + column)
            constexpr int NA = 8 * RI, NB = 8 * RJ;
            __shared__ PA stage_a[WG / WAVE][NA];
            __shared__ PB stage_b[WG / WAVE][NB];
            const int w = (int)(threadIdx.x / WAVE);
            const int ka = lane % NA, kb = lane % NB;
            const uint32_t la = (uint32_t)min(ig0 + (ka & 7) + (ka >> 3) * n_ig, Ta - 1) * (uint32_t)sizeof(PA);
            const uint32_t lb = (uint32_t)min(jg0 + (kb & 7) + (kb >> 3) * n_jg, Tb - 1) * (uint32_t)sizeof(PB);
            const int row = e >> 3, col = e & 7;
            PA ga = load_pose<PA>(A, la, (uint32_t)(chunk - 1) * strideA);
            PB gb = load_pose<PB>(B, lb, (uint32_t)(chunk - 1) * strideB);
            for (int t = chunk - 1; t >= 0; --t) {
                if (lane < NA) stage_a[w][lane] = ga;
                if (lane < NB) stage_b[w][lane] = gb;
                // a wave's LDS operations complete in order; keep the
                // compiler from moving the reads above the writes
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (t > 0) {
                    ga = load_pose<PA>(A, la, (uint32_t)(t - 1) * strideA);
                    gb = load_pose<PB>(B, lb, (uint32_t)(t - 1) * strideB);
                }
                PA a[RI];
                PB b[RJ];
#pragma unroll
                for (int r = 0; r < RI; ++r) a[r] = stage_a[w][r * 8 + row];
#pragma unroll
                for (int s = 0; s < RJ; ++s) b[s] = stage_b[w][s * 8 + col];
#pragma unroll
                for (int r = 0; r < RI; ++r)
#pragma unroll
                    for (int s = 0; s < RJ; ++s)
                        if (chk(a[r], b[s])) first[r][s] = t;
                // and the next step's writes below this step's reads
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            if (!live) return;
        }
    }
    if (!stage) {
        uint32_t oa[RI], ob[RJ];
#pragma unroll
        for (int r = 0; r < RI; ++r) oa[r] = (uint32_t)ia[r] * (uint32_t)sizeof(PA) + t0 * strideA;
#pragma unroll
        for (int s = 0; s < RJ; ++s) ob[s] = (uint32_t)jb[s] * (uint32_t)sizeof(PB) + t0 * strideB;
        for (int t = chunk - 1; t >= 0; --t) {
            const uint32_t sa = (uint32_t)t * strideA, sb = (uint32_t)t * strideB;
            PA a[RI];
            PB b[RJ];
#pragma unroll
            for (int r = 0; r < RI; ++r) a[r] = load_pose<PA>(A, oa[r], sa);
#pragma unroll
            for (int s = 0; s < RJ; ++s) b[s] = load_pose<PB>(B, ob[s], sb);
#pragma unroll
            for (int r = 0; r < RI; ++r)
#pragma unroll
                for (int s = 0; s < RJ; ++s)
                    if (chk(a[r], b[s])) first[r][s] = t;
        }
    }
    if (tshift) {
        // the earliest hit over the parts: their step ranges cover [0, H), so
        // it is the smallest step found by any part (lanes l ^ E, l ^ 2E, ...;
        // the parts of an item are active together)
#pragma unroll
        for (int r = 0; r < RI; ++r)
#pragma unroll
            for (int s = 0; s < RJ; ++s) {
                const int v = first[r][s] >= 0 ? first[r][s] + (int)t0 : INT_MAX;
                const int m = min_over_parts(v, tshift);
                first[r][s] = m == INT_MAX ? -1 : m;
            }
        if (part != 0) return;
    }
    // Results: the first hits, and this thread's share of the q sums. A
    // colliding trajectory pair (i, j) adds p_{b,j} to q_{a,i;b} and p_{a,i}
    // to q_{b,j;a}; sums are exact integers (p * 2^62), so their value does
    // not depend on the order in which threads add them.
    bool any = false;
#pragma unroll
    for (int r = 0; r < RI; ++r) {
        const int i = ig + r * n_ig;
#pragma unroll
        for (int s = 0; s < RJ; ++s) {
            const int j = jg + s * n_jg;
            const bool valid = i < Ta && j < Tb;
            if (!valid) first[r][s] = -1;
            if (hits && valid) hits[pr.hit_off + (int64_t)i * Tb + j] = (int16_t)first[r][s];
            any |= first[r][s] >= 0;
        }
    }
    if (any) {
        unsigned long long pa[RI], pb[RJ];
#pragma unroll
        for (int r = 0; r < RI; ++r) pa[r] = pfix[pr.pa_off + ia[r]];
#pragma unroll
        for (int s = 0; s < RJ; ++s) pb[s] = pfix[pr.pb_off + jb[s]];
        if (TL && pr.timeline) {
            // time-resolved: each colliding pair adds to the sums of its
            // first colliding slot
#pragma unroll
            for (int r = 0; r < RI; ++r)
#pragma unroll
                for (int s = 0; s < RJ; ++s)
                    if (first[r][s] >= 0) {
                        const int64_t k = first[r][s];
                        atomicAdd(&hist[pr.ha0 + (k * Ta + (ig + r * n_ig)) * pr.hwa], pb[s]);
                        atomicAdd(&hist[pr.hb0 + (k * Tb + (jg + s * n_jg)) * pr.hwb], pa[r]);
                    }
            return;
        }
#pragma unroll
        for (int r = 0; r < RI; ++r) {
            unsigned long long row = 0;
#pragma unroll
            for (int s = 0; s < RJ; ++s)
                if (first[r][s] >= 0) row += pb[s];
            if (row) atomicAdd(&qacc[pr.qa0 + (int64_t)(ig + r * n_ig) * pr.qn], row);
        }
#pragma unroll
        for (int s = 0; s < RJ; ++s) {
            unsigned long long col = 0;
#pragma unroll
            for (int r = 0; r < RI; ++r)
                if (first[r][s] >= 0) col += pa[r];
            if (col) atomicAdd(&qacc[pr.qb0 + (int64_t)(jg + s * n_jg) * pr.qn], col);
        }
    }
}

// EXT: whether this kernel instance carries the extended classes (the
// point-in-polygon rectangle test and the polygon classes). Their larger
// code and tiles need more registers, which would lower the occupancy of the
// plain classes; launches without such pairs use the instance without them.
// TL: whether it can add to per-slot sums (time-resolved scenes); likewise
// kept out of the instances that launches without such scenes use.
// Copies the two polygons of a polygon pair into this wave's LDS slot (each
// lane a few words), so that their constants reach the tests as vector
// registers instead of competing for scalar ones.
__device__ __forceinline__ void stage_polygons(DPoly *slot, const DPoly *__restrict__ polys, const DPair &pr)
{
    constexpr int words = (int)(sizeof(DPoly) / sizeof(int32_t));
    const int lane = (int)(threadIdx.x & (WAVE - 1));
    int32_t *dst = reinterpret_cast<int32_t *>(slot);
    const int32_t *pa = reinterpret_cast<const int32_t *>(polys + (pr.poly_a >= 0 ? pr.poly_a : pr.poly_b));
    const int32_t *pb = reinterpret_cast<const int32_t *>(polys + (pr.poly_b >= 0 ? pr.poly_b : pr.poly_a));
    for (int k = lane; k < words; k += WAVE) {
        dst[k] = pa[k];
        dst[words + k] = pb[k];
    }
    // the wave's LDS operations complete in order; keep the compiler from
    // moving the reads above the writes
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// FAM: the test classes this kernel instance carries. FAM_PLAIN: rectangles
// and circles; FAM_PIP: also the point-in-polygon rectangle test; FAM_POLY:
// also the polygon classes. The larger code and tiles of the later families
// need more registers, which would lower the occupancy of the earlier ones;
// a launch uses the smallest family that covers its pairs.
// TL: whether it can add to per-slot sums (time-resolved scenes); likewise
// kept out of the instances that launches without such scenes use.
template <int V, int FAM, bool TL, bool STAGE = false>
__device__ __forceinline__ void collide_work(const DPair &pr, int item0, const char *__restrict__ poses,
                                             int16_t *__restrict__ hits, const unsigned long long *__restrict__ pfix,
                                             unsigned long long *__restrict__ qacc,
                                             unsigned long long *__restrict__ hist, const DPoly *lp)
{
    if constexpr (FAM >= FAM_PIP) {
        if (pr.cls == CLS_VV_PIP) {
            collide_items<kTiles[V][CLS_VV_PIP].ri, kTiles[V][CLS_VV_PIP].rj, TL, float4, float4>(
                pr, item0, poses, hits, pfix, qacc, hist, CheckVVPip{pr.la, pr.wa, pr.lb, pr.wb});
            return;
        }
    }
    if constexpr (FAM >= FAM_POLY) {
        const DPoly *P = lp, *Q = lp + 1;  // the pair's polygons (staged)
        switch (pr.cls) {
        case CLS_GG:
        case CLS_GG_PIP: {
            const int shape = (P->k == 8 ? 2 : 0) + (Q->k == 8 ? 1 : 0) + (pr.cls == CLS_GG_PIP ? 4 : 0);
            switch (shape) {
#define MHC_GG(S, KP, KQ, PIPM)                                                                                      \
    case S:                                                                                                          \
        collide_items<1, 1, TL, float4, float4>(pr, item0, poses, hits, pfix, qacc, hist, CheckGG<KP, KQ, PIPM>{P, Q}); \
        return;
                MHC_GG(0, 4, 4, false)
                MHC_GG(1, 4, 8, false)
                MHC_GG(2, 8, 4, false)
                MHC_GG(3, 8, 8, false)
                MHC_GG(4, 4, 4, true)
                MHC_GG(5, 4, 8, true)
                MHC_GG(6, 8, 4, true)
                MHC_GG(7, 8, 8, true)
#undef MHC_GG
            }
            return;
        }
        case CLS_GC:
            if (P->k == 8)
                collide_items<kTiles[V][CLS_GC].ri, kTiles[V][CLS_GC].rj, TL, float4, float2>(
                    pr, item0, poses, hits, pfix, qacc, hist, CheckGC<8>{P, pr.rr});
            else
                collide_items<kTiles[V][CLS_GC].ri, kTiles[V][CLS_GC].rj, TL, float4, float2>(
                    pr, item0, poses, hits, pfix, qacc, hist, CheckGC<4>{P, pr.rr});
            return;
        case CLS_CG:
            if (P->k == 8)
                collide_items<kTiles[V][CLS_CG].ri, kTiles[V][CLS_CG].rj, TL, float2, float4>(
                    pr, item0, poses, hits, pfix, qacc, hist, CheckCG<8>{P, pr.rr});
            else
                collide_items<kTiles[V][CLS_CG].ri, kTiles[V][CLS_CG].rj, TL, float2, float4>(
                    pr, item0, poses, hits, pfix, qacc, hist, CheckCG<4>{P, pr.rr});
            return;
        default:
            break;
        }
    }
    switch (pr.cls) {
    case CLS_VV:
        collide_items<kTiles[V][CLS_VV].ri, kTiles[V][CLS_VV].rj, TL, float4, float4, CheckVV, STAGE>(
            pr, item0, poses, hits, pfix, qacc, hist, CheckVV{pr.la, pr.wa, pr.lb, pr.wb});
        break;
    case CLS_VP:
        collide_items<kTiles[V][CLS_VP].ri, kTiles[V][CLS_VP].rj, TL, float4, float2, CheckVP, STAGE>(
            pr, item0, poses, hits, pfix, qacc, hist, CheckVP{pr.la, pr.wa, pr.rr});
        break;
    case CLS_PV:
        collide_items<kTiles[V][CLS_PV].ri, kTiles[V][CLS_PV].rj, TL, float2, float4, CheckPV, STAGE>(
            pr, item0, poses, hits, pfix, qacc, hist, CheckPV{pr.lb, pr.wb, pr.rr});
        break;
    default:
        collide_items<kTiles[V][CLS_PP].ri, kTiles[V][CLS_PP].rj, TL, float2, float2, CheckPP, STAGE>(
            pr, item0, poses, hits, pfix, qacc, hist, CheckPP{pr.rr});
        break;
    }
}

// Collision kernel: every wave owns one slot of the host-built plan and runs
// its segments. For plans of contiguous stretches (large scenes) the slots
// are numbered XCD-major (workgroups are dealt to the XCDs in turn), so the
// pairs one XCD works on stay together in its L2; for individually packed
// plans neighbouring slots are spread over the XCDs and CUs, which mixes the
// load-heavy and arithmetic-heavy test classes on every CU. The host
// balances the slots by the exact instruction cost of the work, so every
// SIMD finishes together without any cross-XCD atomics.
// The plain-class instances are held to at least 5 waves per SIMD and the
// point-in-polygon ones to 4: with fewer the vector ALU idles on pose loads,
// and without the bound the compiler's occupancy heuristic may trade a wave
// for registers it does not need.
template <int FAM>
constexpr int kCollideMinWaves = FAM == FAM_PLAIN ? 5 : FAM == FAM_PIP ? 4 : 1;

// A launch may run one part of the plan (part of n_parts): every wave then
// takes only its units [U part / n_parts, U (part + 1) / n_parts) of the U
// units of its segments, so that n_parts launches cover each unit once.
template <int V, int FAM, bool TL, bool STAGE>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(kCollideMinWaves<FAM>))) void k2_collide(const DPair *__restrict__ pairs, const WorkItem *__restrict__ work,
                                                 const int32_t *__restrict__ bins, int n_bins, int xcd_major,
                                                 const char *__restrict__ poses, int16_t *__restrict__ hits,
                                                 const unsigned long long *__restrict__ pfix,
                                                 unsigned long long *__restrict__ qacc,
                                                 unsigned long long *__restrict__ hist, const DPoly *__restrict__ polys,
                                                 int part, int n_parts)
{
    const int wave_in_block = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const int blocks = (int)gridDim.x;
    const int xcd = (int)blockIdx.x % N_XCD, round = (int)blockIdx.x / N_XCD;
    const int per_xcd = (blocks / N_XCD) * (WG / WAVE);
    int slot;
    if (xcd_major && (int)blockIdx.x < (blocks / N_XCD) * N_XCD)
        slot = xcd * per_xcd + round * (WG / WAVE) + wave_in_block;
    else
        slot = (int)blockIdx.x * (WG / WAVE) + wave_in_block;  // grid not a multiple of the XCD count
    if (slot >= n_bins) return;
    // per wave: the two polygons of its current polygon pair
    constexpr bool poly = FAM >= FAM_POLY;
    __shared__ DPoly lds_polys[poly ? 2 * (WG / WAVE) : 1];
    DPoly *lp = lds_polys + (poly ? 2 * wave_in_block : 0);
    const int s0 = bins[slot], s1 = bins[slot + 1];
    int lo = 0, hi = INT_MAX;   // this launch's units of the wave
    if (n_parts > 1) {
        int units = 0;
        for (int k = s0; k < s1; ++k) units += work[k].n_units;
        lo = (int)((int64_t)units * part / n_parts);
        hi = (int)((int64_t)units * (part + 1) / n_parts);
    }
    int base = 0;   // units of the wave's segments before segment k
    for (int k = s0; k < s1 && base < hi; ++k) {
        const WorkItem w = work[k];
        const int u0 = max(lo - base, 0), u1 = min(hi - base, w.n_units);
        base += w.n_units;
        if (u0 >= u1) continue;
        const DPair pr = pairs[w.pair];
        if (poly && pr.cls >= CLS_GG) stage_polygons(lp, polys, pr);
        const int per = WAVE >> pr.tshift;
        for (int u = u0; u < u1; ++u)
            collide_work<V, FAM, TL, STAGE>(pr, w.item0 + u * per, poses, hits, pfix, qacc, hist, lp);
    }
}

// ===========================================================================
// K3: risk assessment (Sec. IV-D, IV-D.2).
//
// The collision kernel has left the q_{a,i;b} as exact integer sums (p in
// units of 2^-62, or -log(1 - p) in units of 2^-56 for the INDEPENDENT
// reading; for time-resolved scenes the k3_timeline kernel has added up the
// per-slot sums into the same accumulators). Grid: y = object, x = chunk of 256
// trajectories; thread tid of chunk c takes trajectory i = 256 c + tid,
// converts its sums (rounding once), clamps to 1, writes q and forms
//   crit_{a,i} = 1 - prod_{b != a} (1 - q_{a,i;b})     (ascending b).
// The workgroup adds p_{a,i} crit_{a,i} over its chunk in a fixed order. An
// object of one chunk writes C_a directly; otherwise the chunks add their
// sums in fixed point into a per-object word (zeroed by the trajectory
// kernel) that also counts them, and the chunk that completes the count
// writes C_a. Nothing depends on how the collision work was tiled or
// batched, or on which chunk ends last, so every result is identical for any
// tiling and any batch.
// ===========================================================================

constexpr int K3_LOADS = 16;
constexpr unsigned long long kChunkOne = 1ull << 56;  // one finished chunk in the per-object word
constexpr double kCritScale = 0x1p55, kCritInvScale = 0x1p-55;

__global__ __launch_bounds__(WG) void k3_crit(const DObj *__restrict__ objs,
                                              const unsigned long long *__restrict__ qacc,
                                              const double *__restrict__ p, double *__restrict__ q,
                                              double *__restrict__ traj_crit, double *__restrict__ obj_crit,
                                              unsigned long long *__restrict__ done)
{
    __shared__ double red[WG / WAVE];
    const int obj = (int)blockIdx.y;
    const DObj o = objs[obj];
    const int chunks = (o.T + WG - 1) / WG;
    const int c = (int)blockIdx.x;
    if (c >= chunks) return;  // whole workgroup
    const int n = o.n_scene_obj;
    const int tid = threadIdx.x;
    double acc = 0.0;
    const int i = c * WG + tid;
    if (i < o.T) {
        // The trajectory kernel zeroed all n accumulators of this trajectory,
        // so b == a and objects outside the pair set read as q = 0. Loads are
        // issued sixteen at a time (scenes of up to 16 objects in one round),
        // ahead of the dependent product.
        const unsigned long long *__restrict__ qa = qacc + o.q_row + (int64_t)i * n;
        double *__restrict__ qi = q ? q + o.q_row + (int64_t)i * n : nullptr;
        const double pi = p[o.traj_off + i];
        double no_collision = 1.0;
        for (int b0 = 0; b0 < n; b0 += K3_LOADS) {
            unsigned long long v[K3_LOADS];
#pragma unroll
            for (int k = 0; k < K3_LOADS; ++k) v[k] = b0 + k < n ? qa[b0 + k] : 0ull;
#pragma unroll
            for (int k = 0; k < K3_LOADS; ++k) {
                if (b0 + k < n) {
                    const double qv = q_of(o.risk, v[k]);
                    if (qi) qi[b0 + k] = qv;
                    no_collision *= 1.0 - qv;
                }
            }
        }
        const double crit = 1.0 - no_collision;
        traj_crit[o.traj_off + i] = crit;
        acc = pi * crit;
    }
    const double chunk_sum = block_sum(acc, red);
    if (chunks == 1) {
        if (tid == 0) obj_crit[o.obj_out] = chunk_sum;
        return;
    }
    if (tid != 0) return;
    // One atomic per chunk adds the chunk's sum in fixed point (units of
    // 2^-55; an object's sum is at most 1, so it stays below 2^56) together
    // with a count of one at bit 56 (at most 128 chunks). The chunk whose add
    // completes the count has the whole sum in the value it gets back; the
    // sum is exact in integers, so it does not depend on which chunk ends
    // last, and nothing else is shared between the chunks.
    const unsigned long long mine = kChunkOne + __double2ull_rn(chunk_sum * kCritScale);
    const unsigned long long before = atomicAdd(&done[obj], mine);
    if ((before >> 56) != (unsigned long long)(chunks - 1)) return;
    obj_crit[o.obj_out] = (double)((before + mine) & (kChunkOne - 1)) * kCritInvScale;
    done[obj] = 0ull;  // the risk stage may run again on the same sums
}

// ===========================================================================
// Time-resolved risk (Sec. IV-D.2 over the horizon; the criticality curve the
// anticipation time of Sec. IV-D / VI-A is read from).
//
// For time-resolved scenes the collision kernel adds the summand of every
// colliding trajectory pair to the sums of its first colliding slot s:
// hist_a[s][i][b] (object a's block, b padded to W = the power of two >= n,
// so the W sums of one trajectory and slot are contiguous). For trajectory
// (a, i) with running sums Q_b(s) = sum_{s' <= s} hist_a[s'][i][b] and
// no-collision factors f_b(s) = 1 - q(Q_b(s)), the combinations are taken
// slot by slot, ascending b within a slot; the probability that the first
// collision happens with b at slot s is
//   (f_b(s-1) - f_b(s)) * prod_{b' < b} f_{b'}(s) * prod_{b' > b} f_{b'}(s-1)
// Adding these up over slots gives the attribution A_{a,i;b}, and
// crit_{a,i}(s) = 1 - prod_b f_b(s).
// ===========================================================================

constexpr int K3T_SLOTS = 8;  // slots processed together: loads one group ahead, scans interleaved

// A double from the lane d below (UP) or above (!UP) in the same row of 16
// lanes (DPP row shift; lanes whose source lies outside the row get 0).
template <int D, bool UP>
__device__ __forceinline__ double row_shift(double x)
{
    constexpr int ctrl = (UP ? 0x110 : 0x100) | D;  // row_shr:D / row_shl:D
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), ctrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// One step of the segmented inclusive products: lo over lanes b' <= b,
// hi over lanes b' >= b, for every slot of the group.
template <int D>
__device__ __forceinline__ void scan_step_row(double (&lo)[K3T_SLOTS], double (&hi)[K3T_SLOTS], int b, int W)
{
#pragma unroll
    for (int k = 0; k < K3T_SLOTS; ++k) {
        const double tl = row_shift<D, true>(lo[k]);
        const double th = row_shift<D, false>(hi[k]);
        if (b >= D) lo[k] *= tl;
        if (b + D < W) hi[k] *= th;
    }
}

// The running product of one trajectory's factors over its slots, for one
// risk reading (a template parameter, so the slot loop has no branch on it).
template <int RISK>
__device__ __forceinline__ double keep_of(unsigned long long v)
{
    if constexpr (RISK == RISK_EXCLUSIVE) return 1.0 - fmin((double)v * kQInvScale, 1.0);
    else return 1.0 + expm1(-(double)v * kLInvScale);
}

// Inclusive product over the lanes b' <= b of each trajectory's segment of W
// lanes (DPP row shifts for W <= 16, lane permutes for W = 32, 64).
__device__ __forceinline__ double segment_product(double x, int b, int W)
{
    if (W <= 16) {
        double t;
        if (W > 1) { t = row_shift<1, true>(x); if (b >= 1) x *= t; }
        if (W > 2) { t = row_shift<2, true>(x); if (b >= 2) x *= t; }
        if (W > 4) { t = row_shift<4, true>(x); if (b >= 4) x *= t; }
        if (W > 8) { t = row_shift<8, true>(x); if (b >= 8) x *= t; }
        return x;
    }
    for (int d = 1; d < W; d <<= 1) {
        const double t = __shfl_up(x, d, W);
        if (b >= d) x *= t;
    }
    return x;
}

// Slots [s_begin, s_end) of trajectory (a, i), lane b, from the running sum
// Q of all slots before s_begin (the last lane of the segment also gets
// all_carry = prod_b f_b(s_begin - 1)). Writes the criticality of these
// slots and returns this lane's attribution terms over them; the sums of
// each group of slots are loaded one group ahead of their use.
template <int RISK>
__device__ __forceinline__ double timeline_chunk(const DObj &o, const unsigned long long *__restrict__ hist,
                                                 double *__restrict__ ct_w, double *__restrict__ traj_crit_t, int i,
                                                 int b, int W, int s_begin, int s_end, unsigned long long Q,
                                                 double all_carry)
{
    const int H = o.H;
    const int64_t T = o.T;
    const bool valid = i < o.T && b < o.n_scene_obj;
    const bool writer = b == W - 1 && i < o.T;
    const int64_t slot_stride = T * W;
    if (s_begin >= s_end) return 0.0;
    // every lane loads (padding lanes b >= n hold zeros; lanes past the last
    // trajectory read trajectory 0 and slots past the chunk read its last
    // slot), and the values that do not belong to the lane are masked: no
    // branch per load
    const unsigned long long *__restrict__ h = hist + o.hist_off + (int64_t)(i < o.T ? i : 0) * W + b;
    double f_carry = valid ? keep_of<RISK>(Q) : 1.0, A = 0.0;
    const int last = s_end - 1;
    unsigned long long v[K3T_SLOTS];
#pragma unroll
    for (int k = 0; k < K3T_SLOTS; ++k) v[k] = h[(int64_t)min(s_begin + k, last) * slot_stride];
    for (int s0 = s_begin; s0 < s_end; s0 += K3T_SLOTS) {
        unsigned long long vn[K3T_SLOTS];
#pragma unroll
        for (int k = 0; k < K3T_SLOTS; ++k) vn[k] = h[(int64_t)min(s0 + K3T_SLOTS + k, last) * slot_stride];
        bool change = false;
#pragma unroll
        for (int k = 0; k < K3T_SLOTS; ++k) change |= valid && s0 + k < s_end && v[k] != 0ull;
        if (!__any(change)) {
            // no first hit in these slots for any trajectory of the wave: the
            // factors, the attribution and the criticality stay as they are
            if (writer) {
#pragma unroll
                for (int k = 0; k < K3T_SLOTS; ++k) {
                    const int s = s0 + k;
                    if (s < s_end) {
                        ct_w[o.tl_traj + (int64_t)s * T + i] = 1.0 - all_carry;
                        if (traj_crit_t) traj_crit_t[o.tl_traj + (int64_t)i * H + s] = 1.0 - all_carry;
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < K3T_SLOTS; ++k) v[k] = vn[k];
            continue;
        }
        // factors after (g) and before (f) each slot; slots past the chunk repeat the last
        double g[K3T_SLOTS], f[K3T_SLOTS];
#pragma unroll
        for (int k = 0; k < K3T_SLOTS; ++k) {
            f[k] = k == 0 ? f_carry : g[k - 1];
            Q += (valid && s0 + k < s_end) ? v[k] : 0ull;
            g[k] = valid ? keep_of<RISK>(Q) : 1.0;
        }
        f_carry = g[K3T_SLOTS - 1];
        double lo[K3T_SLOTS], hi[K3T_SLOTS];
#pragma unroll
        for (int k = 0; k < K3T_SLOTS; ++k) {
            lo[k] = g[k];
            hi[k] = f[k];
        }
        double below[K3T_SLOTS], above[K3T_SLOTS];
        if (W <= 16) {
            if (W > 1) scan_step_row<1>(lo, hi, b, W);
            if (W > 2) scan_step_row<2>(lo, hi, b, W);
            if (W > 4) scan_step_row<4>(lo, hi, b, W);
            if (W > 8) scan_step_row<8>(lo, hi, b, W);
#pragma unroll
            for (int k = 0; k < K3T_SLOTS; ++k) {
                below[k] = row_shift<1, true>(lo[k]);
                above[k] = row_shift<1, false>(hi[k]);
            }
        } else {
            for (int d = 1; d < W; d <<= 1) {
#pragma unroll
                for (int k = 0; k < K3T_SLOTS; ++k) {
                    const double tl = __shfl_up(lo[k], d, W);
                    const double th = __shfl_down(hi[k], d, W);
                    if (b >= d) lo[k] *= tl;
                    if (b + d < W) hi[k] *= th;
                }
            }
#pragma unroll
            for (int k = 0; k < K3T_SLOTS; ++k) {
                below[k] = __shfl_up(lo[k], 1, W);
                above[k] = __shfl_down(hi[k], 1, W);
            }
        }
#pragma unroll
        for (int k = 0; k < K3T_SLOTS; ++k) {
            const double bl = b > 0 ? below[k] : 1.0;      // inclusive -> exclusive
            const double ab = b + 1 < W ? above[k] : 1.0;
            A += (f[k] - g[k]) * bl * ab;                   // 0 past the chunk: f == g there
        }
        if (writer) {  // lo at the last lane = prod_b f_b(s)
#pragma unroll
            for (int k = 0; k < K3T_SLOTS; ++k) {
                const int s = s0 + k;
                if (s < s_end) {
                    ct_w[o.tl_traj + (int64_t)s * T + i] = 1.0 - lo[k];
                    if (traj_crit_t) traj_crit_t[o.tl_traj + (int64_t)i * H + s] = 1.0 - lo[k];
                }
            }
        }
        all_carry = lo[K3T_SLOTS - 1];
#pragma unroll
        for (int k = 0; k < K3T_SLOTS; ++k) v[k] = vn[k];
    }
    return A;
}

// K3t: grid y = object, x = group of 64 / W trajectories, lane = (trajectory,
// b); the four waves of a workgroup take the same lanes and split the slots
// into four consecutive chunks, so that every trajectory's slots are walked
// by four waves side by side. Wave c first adds up the per-slot sums of its
// chunk (one load per slot and lane); after a barrier it starts from the sums
// of the chunks before it (added in chunk order), their factors and, in the
// segment's last lane, their product, and walks its chunk: slots go in
// groups of K3T_SLOTS, the lanes load the group's sums (one group ahead),
// form the running sums and factors, and the segment of W lanes of every
// trajectory forms, for all slots of the group at once (independent chains,
// so their latencies overlap), the products of the factors below b (new) and
// above b (old): DPP row shifts for W <= 16, lane permutes for W = 32, 64.
// Lane b then adds its attribution terms; the last lane of the segment holds
// prod_b f_b(s). After a second barrier wave 0 adds the four chunks'
// attribution terms in chunk order. Writes the criticality over time as
// [s][i] scratch (and traj_crit_t (i, s) if asked for), the attribution as
// [b][i] scratch (and (i, b) if asked for), and the total sums of every b
// into the integer accumulators k3_crit reads. Timeline scenes have at most
// 64 objects.
__global__ __launch_bounds__(WG) void k3_timeline(const DObj *__restrict__ objs,
                                                  const unsigned long long *__restrict__ hist,
                                                  unsigned long long *__restrict__ qacc, double *__restrict__ att_w,
                                                  double *__restrict__ ct_w, double *__restrict__ traj_crit_t,
                                                  double *__restrict__ traj_attrib)
{
    constexpr int CHUNKS = WG / WAVE;
    __shared__ unsigned long long chunk_sum[CHUNKS][WAVE];
    __shared__ double chunk_att[CHUNKS][WAVE];
    const DObj o = objs[blockIdx.y];
    if (!o.timeline) return;  // whole workgroup
    const int W = o.tl_w;
    const int lane = (int)(threadIdx.x & (WAVE - 1));
    const int c = (int)(threadIdx.x / WAVE);
    const int per_wave = WAVE / W;
    const int first_i = (int)blockIdx.x * per_wave;
    if (first_i >= o.T) return;  // whole workgroup: every lane below takes part in the exchanges
    const int i = first_i + lane / W;
    const int b = lane & (W - 1);
    const bool valid = i < o.T && b < o.n_scene_obj;
    const int H = o.H;
    const int len = (H + CHUNKS - 1) / CHUNKS;
    const int s_begin = min(c * len, H), s_end = min(s_begin + len, H);
    // this chunk's sums, eight loads in flight at a time
    const unsigned long long *__restrict__ h = hist + o.hist_off + (int64_t)(i < o.T ? i : 0) * W + b;
    const int64_t slot_stride = (int64_t)o.T * W;
    unsigned long long sum = 0ull;
    for (int s0 = s_begin; s0 < s_end; s0 += 8) {
        unsigned long long v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = h[(int64_t)min(s0 + k, s_end - 1) * slot_stride];
#pragma unroll
        for (int k = 0; k < 8; ++k) sum += s0 + k < s_end ? v[k] : 0ull;
    }
    chunk_sum[c][lane] = valid ? sum : 0ull;
    __syncthreads();
    unsigned long long Q = 0ull;
    for (int k = 0; k < c; ++k) Q += chunk_sum[k][lane];
    const double f0 =
        valid ? (o.risk == RISK_EXCLUSIVE ? keep_of<RISK_EXCLUSIVE>(Q) : keep_of<RISK_INDEPENDENT>(Q)) : 1.0;
    const double all_carry = segment_product(f0, b, W);
    const double A = o.risk == RISK_EXCLUSIVE
                         ? timeline_chunk<RISK_EXCLUSIVE>(o, hist, ct_w, traj_crit_t, i, b, W, s_begin, s_end, Q,
                                                          all_carry)
                         : timeline_chunk<RISK_INDEPENDENT>(o, hist, ct_w, traj_crit_t, i, b, W, s_begin, s_end, Q,
                                                            all_carry);
    chunk_att[c][lane] = A;
    __syncthreads();
    if (c != 0 || !valid) return;
    double At = 0.0;
    unsigned long long Qt = 0ull;
    for (int k = 0; k < CHUNKS; ++k) {
        At += chunk_att[k][lane];
        Qt += chunk_sum[k][lane];
    }
    const int n = o.n_scene_obj;
    qacc[o.q_row + (int64_t)i * n + b] = Qt;
    att_w[o.q_row + (int64_t)b * o.T + i] = At;
    if (traj_attrib) traj_attrib[o.q_row + (int64_t)i * n + b] = At;
}

// Sum of a double over the 64 lanes of a wave in a fixed butterfly order.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

// K4t: grid x = object, y = row: rows 0..H-1 are the slots (C_a(s)), rows
// H..H+n-1 the collision objects (A_{a,b}). Thread t adds p_{a,i} times the
// trajectory value over i = t, t + 256, ... in ascending order (loads four
// ahead), and the workgroup adds the 256 partial sums in a fixed order
// (block_sum): every sum has a fixed order.
__global__ __launch_bounds__(WG) void k4_timeline(const DObj *__restrict__ objs, const double *__restrict__ p,
                                                  const double *__restrict__ ct_w, const double *__restrict__ att_w,
                                                  double *__restrict__ crit_t, double *__restrict__ attrib)
{
    __shared__ double red[WG / WAVE];
    const DObj o = objs[blockIdx.x];
    if (!o.timeline) return;
    const int row = (int)blockIdx.y;
    const int n = o.n_scene_obj, H = o.H, T = o.T;
    if (row >= H + n) return;  // whole workgroup
    const int tid = (int)threadIdx.x;
    const double *__restrict__ pp = p + o.traj_off;
    const double *__restrict__ r =
        row < H ? ct_w + o.tl_traj + (int64_t)row * T : att_w + o.q_row + (int64_t)(row - H) * T;
    double acc = 0.0;
    for (int base = 0; base < T; base += 4 * WG) {
        double x[4], w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int idx = base + k * WG + tid;
            x[k] = idx < T ? r[idx] : 0.0;
            w[k] = idx < T ? pp[idx] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (base + k * WG + tid < T) acc += w[k] * x[k];
    }
    const double total = block_sum(acc, red);
    if (tid != 0) return;
    if (row < H)
        crit_t[o.tl_obj + row] = total;
    else
        attrib[o.tl_att + (row - H)] = total;
}

// ===========================================================================
// Launchers
// ===========================================================================

hipError_t launch_trajgen(const Launch &L, hipStream_t s)
{
    if (L.n_obj <= 0) return hipSuccess;
    if (L.one_track)
        hipLaunchKernelGGL(k1_trajgen<true>, dim3(L.k1_x, L.k1_nrows), dim3(WG), 0, s, L.objs, L.vals, L.poses, L.p,
                           L.pfix, L.qacc, L.done, L.hist, L.k1_rows);
    else
        hipLaunchKernelGGL(k1_trajgen<false>, dim3(L.k1_x, L.k1_nrows), dim3(WG), 0, s, L.objs, L.vals, L.poses, L.p,
                           L.pfix, L.qacc, L.done, L.hist, L.k1_rows);
    return hipGetLastError();
}

template <int V, int FAM, bool TL, bool STAGE>
static hipError_t launch_k2(const Launch &L, hipStream_t s)
{
    const int blocks = (L.n_bins + WG / WAVE - 1) / (WG / WAVE);
    const int parts = L.collide_parts > 1 ? L.collide_parts : 1;
    const int first = L.collide_only > 0 ? L.collide_only - 1 : 0;
    const int last = L.collide_only > 0 ? L.collide_only : parts;
    if (first >= parts) return hipErrorInvalidValue;
    for (int part = first; part < last; ++part) {
        hipLaunchKernelGGL((k2_collide<V, FAM, TL, STAGE>), dim3(blocks), dim3(WG), 0, s, L.pairs, L.work, L.bins,
                           L.n_bins, L.xcd_major, L.poses, L.hits, L.pfix, L.qacc, L.hist, L.polys, part, parts);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int V, int FAM, bool TL, bool STAGE>
static int k2_resident_blocks()
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k2_collide<V, FAM, TL, STAGE>, WG, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return per_cu;
}

// The kernel instance of (variant, class family, per-slot sums, LDS-staged
// blocks): F::run<V, FAM, TL, STAGE>() is called for the instance. Staged
// instances exist for the plain family without per-slot sums only.
template <int FAM, bool TL, bool STAGE, class F>
static auto with_variant(int variant, const F &f)
{
    switch (variant) {
    case 0: return f.template run<0, FAM, TL, STAGE>();
    case 1: return f.template run<1, FAM, TL, STAGE>();
    case 2: return f.template run<2, FAM, TL, STAGE>();
    default: return f.template run<3, FAM, TL, STAGE>();
    }
}

template <int FAM, class F>
static auto with_timeline(int variant, bool tl, const F &f)
{
    return tl ? with_variant<FAM, true, false>(variant, f) : with_variant<FAM, false, false>(variant, f);
}

template <class F>
static auto with_instance(int variant, int family, bool tl, bool stage, const F &f)
{
    switch (family) {
    case FAM_PLAIN:
        if (stage && !tl) return with_variant<FAM_PLAIN, false, true>(variant, f);
        return with_timeline<FAM_PLAIN>(variant, tl, f);
    case FAM_PIP: return with_timeline<FAM_PIP>(variant, tl, f);
    default: return with_timeline<FAM_POLY>(variant, tl, f);
    }
}

struct LaunchK2 {
    const Launch &L;
    hipStream_t s;
    template <int V, int FAM, bool TL, bool STAGE>
    hipError_t run() const { return launch_k2<V, FAM, TL, STAGE>(L, s); }
};

struct ResidentK2 {
    template <int V, int FAM, bool TL, bool STAGE>
    int run() const { return k2_resident_blocks<V, FAM, TL, STAGE>(); }
};

hipError_t launch_collide(const Launch &L, hipStream_t s)
{
    if (L.n_work <= 0) return hipSuccess;
    if (L.variant < 0 || L.variant >= N_VARIANTS || L.family < FAM_PLAIN || L.family > FAM_POLY)
        return hipErrorInvalidValue;
    return with_instance(L.variant, L.family, L.timeline != 0, L.stage != 0, LaunchK2{L, s});
}

int collide_blocks_per_cu(int variant, int family, bool timeline, bool stage)
{
    return with_instance(variant, family, timeline, stage, ResidentK2{});
}

// ===========================================================================
// Workspace of the allocation-free entry point (mhc_evaluate_noalloc): a
// file-scope device array, one copy on every GPU, held until the process
// ends. Host code must not pass its name to a kernel (on the host it is a
// stand-in, not a device address); noalloc_scratch_address looks up this
// GPU's address once, with the device current, and every later use goes
// through that address.
// ===========================================================================

static __device__ __align__(256) char noalloc_scratch[kNoallocBytes];

hipError_t noalloc_scratch_address(int device, char **out)
{
    static std::mutex mu;
    static char *addr[kMaxDevices] = {};
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
        if (e != hipSuccess) return e;
        if (!p || reinterpret_cast<uintptr_t>(p) % 256 != 0) return hipErrorInvalidSymbol;
        addr[device] = static_cast<char *>(p);
    }
    *out = addr[device];
    return hipSuccess;
}

hipError_t launch_risk(const Launch &L, hipStream_t s)
{
    if (L.n_obj <= 0) return hipSuccess;
    if (L.timeline) {
        hipLaunchKernelGGL(k3_timeline, dim3(L.k3t_x, L.n_obj), dim3(WG), 0, s, L.objs, L.hist, L.qacc, L.att_w,
                           L.ct_w, L.traj_crit_t, L.traj_attrib);
        hipLaunchKernelGGL(k4_timeline, dim3(L.n_obj, L.k4t_y), dim3(WG), 0, s, L.objs, L.p, L.ct_w, L.att_w,
                           L.crit_t, L.attrib);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k3_crit, dim3(L.k3_x, L.n_obj), dim3(WG), 0, s, L.objs, L.qacc, L.p, L.q, L.traj_crit,
                       L.obj_crit, L.done);
    return hipGetLastError();
}

}  // namespace mhc
