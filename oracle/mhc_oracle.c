/*
 * mhc_oracle.c -- plain FP64 CPU oracle for the multi-hypothesis criticality
 * method of Sanchez Morales et al., "Parallel Multi-Hypothesis Algorithm for
 * Criticality Estimation in Traffic and Collision Avoidance" (IEEE IV 2019).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library. It shares no code, header,
 * table or constant with the GPU library, and it is deliberately slow and
 * literal: every result is computed from its definition, in double precision,
 * one trajectory pair and one time step at a time, with no blocking, no
 * culling and no fast-math.
 *
 * Pipeline (Fig. 1 of the paper, street module dropped):
 *   probabilities  (Sec. IV-D.1, L1 normalisation of trajectory scores)
 *   trajectories   (Sec. IV-B.1 Euler pose update; Sec. IV-B.3 pedestrians)
 *   pairs          (Sec. IV-C.1; all unordered pairs, or EGO-CO only)
 *   overlap margin (Sec. IV-C.1; exact closed-shape intersection, or the
 *                   paper's point-in-polygon test both ways)
 *   first hit      (earliest colliding step of each trajectory pair)
 *   risk           (Sec. IV-D p_cra double sum, Sec. IV-D.2 chronological
 *                   scaling of the conditional probabilities)
 *
 * Readings of the paper that this file takes (the paper is silent or
 * ambiguous on each):
 *   - vehicles move on the kinematic special case of the Euler update with
 *     side slip beta = 0 and yaw acceleration 0; the longitudinal
 *     acceleration of step n acts within step n (no one-step lag) and the
 *     speed is clamped at zero, the acceleration that step being the one that
 *     stops the vehicle;
 *   - vehicles are rectangles, or convex polygons when given an outline (at
 *     most 8 vertices in the body frame), pedestrians circles; touching
 *     counts as a collision (margin <= 0). The default overlap test is the
 *     exact intersection of the closed shapes; the paper's point-in-polygon
 *     test, run both ways, is the second mode (vehicles only), with a vertex
 *     on the other polygon's boundary counting as inside;
 *   - poses are predicted for n = 1..H and stored at slot n-1; the measured
 *     state (n = 0) is never checked;
 *   - the chronological scaling is read as: collision objects independent of
 *     one another, the trajectories of one object mutually exclusive, all
 *     conditioned on the trajectory of the object being assessed. The product
 *     of "no collision" factors then telescopes, so no ordering is needed for
 *     the totals (ORC_RISK_EXCLUSIVE, the default). The second reading takes
 *     every combination of the assessed trajectory with one trajectory of
 *     another object as an independent event (ORC_RISK_INDEPENDENT);
 *   - combinations that collide at the same step are taken in ascending order
 *     of the other object's index, then of its trajectory index; only the
 *     attribution of criticality to collision objects depends on this.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_VEHICLE 0
#define ORC_PEDESTRIAN 1

/* overlap test of the collision recognition */
#define ORC_OVERLAP_EXACT 0   /* closed shapes intersect */
#define ORC_OVERLAP_PIP 1     /* a vertex of one polygon lies in the other (both ways) */

/* reading of the conditional-probability approximation (Sec. IV-D.2) */
#define ORC_RISK_EXCLUSIVE 0   /* one object's trajectories exclusive, objects independent */
#define ORC_RISK_INDEPENDENT 1 /* every trajectory combination an independent event */

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2

/* ------------------------------------------------------------------------ */
/* Probabilities: Sec. IV-D.1. The scores of one object are normalised with  */
/* respect to the L1 norm; without scores every trajectory is equally likely.*/
/* ------------------------------------------------------------------------ */
int orc_probabilities(int n, const double *score, double *p)
{
    if (n < 1) return ORC_EINVAL;
    if (score == NULL) {
        for (int i = 0; i < n; ++i) p[i] = 1.0 / (double)n;
        return ORC_OK;
    }
    double l1 = 0.0;
    for (int i = 0; i < n; ++i) {
        if (!(score[i] >= 0.0) || !isfinite(score[i])) return ORC_EINVAL;
        l1 += fabs(score[i]);
    }
    if (!(l1 > 0.0) || !isfinite(l1)) return ORC_EINVAL;
    for (int i = 0; i < n; ++i) p[i] = score[i] / l1;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Trajectories. Output arrays are [H][n_u*n_w], slot t holding the pose of  */
/* step n = t+1. Trajectory index i = k*n_w + l.                             */
/* ------------------------------------------------------------------------ */

/* Vehicle: Euler pose update of Sec. IV-B.1 with beta = beta_dot = 0 and
 * psi_ddot = 0, driven by a constant acceleration u[k] and a constant yaw
 * rate w[l]:
 *   v_{n+1}   = v_n + vdot_n tau            (vdot_n clamped so v >= 0)
 *   psi_{n+1} = psi_n + psi_dot tau
 *   a_x,n = vdot_n,  a_y,n = v_n psi_dot     (vehicle frame)
 *   x_{n+1} = x_n + c(psi_n) v_n tau + c(psi_n) a_x,n tau^2/2 - s(psi_n) a_y,n tau^2/2
 *   y_{n+1} = y_n + s(psi_n) v_n tau + s(psi_n) a_x,n tau^2/2 + c(psi_n) a_y,n tau^2/2
 */
static void vehicle_trajectory(double x0, double y0, double psi0, double v0,
                               double accel, double yaw_rate, int H, double tau,
                               int T, int i, double *ox, double *oy, double *opsi)
{
    double x = x0, y = y0, psi = psi0, v = v0;
    for (int n = 0; n < H; ++n) {
        double vdot = accel;
        double v_next = v + vdot * tau;
        if (v_next < 0.0) {          /* the vehicle stops inside this step */
            vdot = -v / tau;
            v_next = 0.0;
        }
        double ax = vdot;
        double ay = v * yaw_rate;
        double c = cos(psi), s = sin(psi);
        double x_next = x + c * v * tau + c * ax * (tau * tau / 2.0) - s * ay * (tau * tau / 2.0);
        double y_next = y + s * v * tau + s * ax * (tau * tau / 2.0) + c * ay * (tau * tau / 2.0);
        double psi_next = psi + yaw_rate * tau;
        x = x_next;
        y = y_next;
        psi = psi_next;
        v = v_next;
        ox[(size_t)n * T + i] = x;
        oy[(size_t)n * T + i] = y;
        opsi[(size_t)n * T + i] = psi;
    }
}

/* Pedestrian: kinematic model of Sec. IV-B.3 with a constant speed u[k]
 * (vdot_P = 0) along the heading psi0 + w[l]:
 *   x_{n+1} = x_n + c(psi_P) v_P tau,  y_{n+1} = y_n + s(psi_P) v_P tau. */
static void pedestrian_trajectory(double x0, double y0, double psi0,
                                  double speed, double heading_offset, int H, double tau,
                                  int T, int i, double *ox, double *oy, double *opsi)
{
    double psi = psi0 + heading_offset;
    double c = cos(psi), s = sin(psi);
    double x = x0, y = y0;
    for (int n = 0; n < H; ++n) {
        x = x + c * speed * tau;
        y = y + s * speed * tau;
        ox[(size_t)n * T + i] = x;
        oy[(size_t)n * T + i] = y;
        opsi[(size_t)n * T + i] = psi;
    }
}

/* Pedestrian with the acceleration grid of Sec. IV-B.3: the heading psi_P
 * is a sample of [0, 360) degrees (absolute), the acceleration vdot_P a
 * sample of its range, and the speed is limited to [0, v_max]:
 *   v_{n+1} = v_n + vdot_n tau, vdot_n cut so that 0 <= v_{n+1} <= v_max,
 *   x_{n+1} = x_n + c(psi_P) v_n tau + c(psi_P) vdot_n tau^2/2   (same for y, s). */
static void pedestrian_accel_trajectory(double x0, double y0, double v0, double accel, double heading,
                                        double v_max, int H, double tau, int T, int i,
                                        double *ox, double *oy, double *opsi)
{
    double c = cos(heading), s = sin(heading);
    double x = x0, y = y0, v = v0;
    for (int n = 0; n < H; ++n) {
        double vdot = accel;
        double v_next = v + vdot * tau;
        if (v_next > v_max) { vdot = (v_max - v) / tau; v_next = v_max; }
        if (v_next < 0.0) { vdot = -v / tau; v_next = 0.0; }
        x = x + c * v * tau + c * vdot * (tau * tau / 2.0);
        y = y + s * v * tau + s * vdot * (tau * tau / 2.0);
        v = v_next;
        ox[(size_t)n * T + i] = x;
        oy[(size_t)n * T + i] = y;
        opsi[(size_t)n * T + i] = heading;
    }
}

/* Vehicle on the linear one-track model of Sec. IV-B.1 (the model the paper
 * uses for the collision objects):
 *   beta_dot  = -(cf + cr)/(m v) beta + ((cr lr - cf lf)/(m v^2) - 1) psi_dot + cf/(m v) delta
 *   psi_ddot  = (cr lr - cf lf)/Iz beta - (cf lf^2 + cr lr^2)/(Iz v) psi_dot + cf lf/Iz delta
 * with a constant front steering angle delta (the lateral controller needs
 * lanes, which are not modelled) and a constant acceleration vdot (the
 * speed stopping at 0 as for the kinematic model), integrated with the Euler
 * update of Sec. IV-B.1:
 *   v_{n+1} = v_n + vdot_n tau,  beta_{n+1} = beta_n + beta_dot_n tau,
 *   psi_{n+1} = psi_n + psi_dot_n tau + psi_ddot_n tau^2/2,
 *   a_x = c(beta) vdot - s(beta) v (beta_dot + psi_dot),
 *   a_y = s(beta) vdot + c(beta) v (beta_dot + psi_dot),
 *   x_{n+1} = x_n + c(psi + beta) v tau + c(psi) a_x tau^2/2 - s(psi) a_y tau^2/2 (y likewise),
 * all from step n (no one-step lag, as for the kinematic model). The explicit
 * Euler step is unstable at low speed (the model's time constants scale with
 * v); where the step matrix I + tau A(v_n) has an eigenvalue of modulus >= 1
 * the lateral state is instead set to the model's steady state at v_{n+1}:
 *   psi_dot = v delta / (L (1 + K v^2)),
 *   beta    = delta (lr / L - m lf v^2 / (cr L^2)) / (1 + K v^2),
 * L = lf + lr, K = m (lr cr - lf cf) / (L^2 cf cr) >= 0 (understeer), and
 * beta_dot, psi_ddot of that step are the differences over tau. The state
 * starts at beta = psi_dot = 0. p = {cf, cr, lf, lr, m, Iz}. */
static void one_track_steady(const double *p, double v, double delta, double *beta, double *psi_dot)
{
    double cf = p[0], cr = p[1], lf = p[2], lr = p[3], m = p[4];
    double L = lf + lr;
    double K = m * (lr * cr - lf * cf) / (L * L * cf * cr);
    double g = 1.0 + K * v * v;
    *psi_dot = v * delta / (L * g);
    *beta = delta * (lr / L - m * lf * v * v / (cr * L * L)) / g;
}

static int one_track_euler_stable(const double *p, double v, double tau)
{
    if (!(v > 0.0)) return 0;
    double cf = p[0], cr = p[1], lf = p[2], lr = p[3], m = p[4], Iz = p[5];
    double a11 = -(cf + cr) / (m * v), a12 = (cr * lr - cf * lf) / (m * v * v) - 1.0;
    double a21 = (cr * lr - cf * lf) / Iz, a22 = -(cf * lf * lf + cr * lr * lr) / (Iz * v);
    /* M = I + tau A; both eigenvalues inside the unit circle (Jury): */
    double m11 = 1.0 + tau * a11, m12 = tau * a12, m21 = tau * a21, m22 = 1.0 + tau * a22;
    double tr = m11 + m22, det = m11 * m22 - m12 * m21;
    return det < 1.0 && tr < 1.0 + det && tr > -(1.0 + det);
}

static void one_track_trajectory(double x0, double y0, double psi0, double v0, double accel, double delta,
                                 const double *p, int H, double tau, int T, int i,
                                 double *ox, double *oy, double *opsi)
{
    double cf = p[0], cr = p[1], lf = p[2], lr = p[3], m = p[4], Iz = p[5];
    double x = x0, y = y0, psi = psi0, v = v0, beta = 0.0, r = 0.0;   /* r = psi_dot */
    for (int n = 0; n < H; ++n) {
        double vdot = accel;
        double v_next = v + vdot * tau;
        if (v_next < 0.0) { vdot = -v / tau; v_next = 0.0; }
        double beta_next, r_next, beta_dot, r_dot;
        if (one_track_euler_stable(p, v, tau)) {
            beta_dot = -(cf + cr) / (m * v) * beta + ((cr * lr - cf * lf) / (m * v * v) - 1.0) * r + cf / (m * v) * delta;
            r_dot = (cr * lr - cf * lf) / Iz * beta - (cf * lf * lf + cr * lr * lr) / (Iz * v) * r + cf * lf / Iz * delta;
            beta_next = beta + beta_dot * tau;
            r_next = r + r_dot * tau;
        } else {
            one_track_steady(p, v_next, delta, &beta_next, &r_next);
            beta_dot = (beta_next - beta) / tau;
            r_dot = (r_next - r) / tau;
        }
        double ax = cos(beta) * vdot - sin(beta) * v * (beta_dot + r);
        double ay = sin(beta) * vdot + cos(beta) * v * (beta_dot + r);
        double h2 = tau * tau / 2.0;
        double x_next = x + cos(psi + beta) * v * tau + cos(psi) * ax * h2 - sin(psi) * ay * h2;
        double y_next = y + sin(psi + beta) * v * tau + sin(psi) * ax * h2 + cos(psi) * ay * h2;
        double psi_next = psi + r * tau + r_dot * h2;
        x = x_next;
        y = y_next;
        psi = psi_next;
        v = v_next;
        beta = beta_next;
        r = r_next;
        ox[(size_t)n * T + i] = x;
        oy[(size_t)n * T + i] = y;
        opsi[(size_t)n * T + i] = psi;
    }
}

/* Motion models of an object (per object):
 *   ORC_MODEL_KINEMATIC:  vehicles acceleration x yaw rate, pedestrians speed
 *                         x heading offset (the readings above);
 *   ORC_MODEL_PED_ACCEL:  pedestrians acceleration x absolute heading with
 *                         params[0] = v_max;
 *   ORC_MODEL_ONE_TRACK:  vehicles acceleration x front steering angle on the
 *                         one-track model, params = {cf, cr, lf, lr, m, Iz}. */
#define ORC_MODEL_KINEMATIC 0
#define ORC_MODEL_PED_ACCEL 1
#define ORC_MODEL_ONE_TRACK 2

int orc_trajectories_model(int kind, int model, const double *params, double x0, double y0, double psi0,
                           double v0, int n_u, const double *u, int n_w, const double *w,
                           int H, double tau, double *ox, double *oy, double *opsi)
{
    if (n_u < 1 || n_w < 1 || H < 1 || !(tau > 0.0)) return ORC_EINVAL;
    if (model == ORC_MODEL_PED_ACCEL && (kind != ORC_PEDESTRIAN || !(params[0] > 0.0))) return ORC_EINVAL;
    if (model == ORC_MODEL_ONE_TRACK) {
        if (kind != ORC_VEHICLE) return ORC_EINVAL;
        for (int k = 0; k < 6; ++k)
            if (!(params[k] > 0.0) || !isfinite(params[k])) return ORC_EINVAL;
        if (params[3] * params[1] < params[2] * params[0]) return ORC_EINVAL;   /* understeer */
    }
    if (model < ORC_MODEL_KINEMATIC || model > ORC_MODEL_ONE_TRACK) return ORC_EINVAL;
    int T = n_u * n_w;
    for (int k = 0; k < n_u; ++k)
        for (int l = 0; l < n_w; ++l) {
            int i = k * n_w + l;
            if (model == ORC_MODEL_PED_ACCEL)
                pedestrian_accel_trajectory(x0, y0, v0, u[k], w[l], params[0], H, tau, T, i, ox, oy, opsi);
            else if (model == ORC_MODEL_ONE_TRACK)
                one_track_trajectory(x0, y0, psi0, v0, u[k], w[l], params, H, tau, T, i, ox, oy, opsi);
            else if (kind == ORC_VEHICLE)
                vehicle_trajectory(x0, y0, psi0, v0, u[k], w[l], H, tau, T, i, ox, oy, opsi);
            else if (kind == ORC_PEDESTRIAN)
                pedestrian_trajectory(x0, y0, psi0, u[k], w[l], H, tau, T, i, ox, oy, opsi);
            else
                return ORC_EINVAL;
        }
    return ORC_OK;
}

int orc_trajectories(int kind, double x0, double y0, double psi0, double v0,
                     int n_u, const double *u, int n_w, const double *w,
                     int H, double tau, double *ox, double *oy, double *opsi)
{
    const double none[6] = {0, 0, 0, 0, 0, 0};
    return orc_trajectories_model(kind, ORC_MODEL_KINEMATIC, none, x0, y0, psi0, v0, n_u, u, n_w, w, H, tau,
                                  ox, oy, opsi);
}

/* ------------------------------------------------------------------------ */
/* Overlap margin: Sec. IV-C.1. At one time step two objects collide when    */
/* their (closed) shapes intersect. The margin is <= 0 exactly then.         */
/* ------------------------------------------------------------------------ */

/* Corners of a rectangle centred at (x, y), heading psi, full length L along
 * the heading and full width W across it. */
static void rect_corners(double x, double y, double psi, double L, double W, double cx[4], double cy[4])
{
    double ux = cos(psi), uy = sin(psi);       /* along the heading */
    double vx = -uy, vy = ux;                  /* across the heading */
    const double sl[4] = {+1, +1, -1, -1};
    const double sw[4] = {+1, -1, -1, +1};
    for (int k = 0; k < 4; ++k) {
        cx[k] = x + sl[k] * (L / 2.0) * ux + sw[k] * (W / 2.0) * vx;
        cy[k] = y + sl[k] * (L / 2.0) * uy + sw[k] * (W / 2.0) * vy;
    }
}

/* Two convex polygons are disjoint iff their projections on some edge normal
 * are disjoint (separating axis theorem). For rectangles the edge normals are
 * the two heading axes of each. The margin is the largest gap between the
 * projected intervals over those four axes; a negative gap on every axis
 * means the closed rectangles intersect. */
double orc_margin_rect_rect(double xP, double yP, double psiP, double LP, double WP,
                            double xQ, double yQ, double psiQ, double LQ, double WQ)
{
    double px[4], py[4], qx[4], qy[4];
    rect_corners(xP, yP, psiP, LP, WP, px, py);
    rect_corners(xQ, yQ, psiQ, LQ, WQ, qx, qy);
    double axes[4][2] = {
        {cos(psiP), sin(psiP)}, {-sin(psiP), cos(psiP)},
        {cos(psiQ), sin(psiQ)}, {-sin(psiQ), cos(psiQ)},
    };
    double margin = -INFINITY;
    for (int a = 0; a < 4; ++a) {
        double nx = axes[a][0], ny = axes[a][1];
        double pmin = INFINITY, pmax = -INFINITY, qmin = INFINITY, qmax = -INFINITY;
        for (int k = 0; k < 4; ++k) {
            double sp = px[k] * nx + py[k] * ny;
            double sq = qx[k] * nx + qy[k] * ny;
            if (sp < pmin) pmin = sp;
            if (sp > pmax) pmax = sp;
            if (sq < qmin) qmin = sq;
            if (sq > qmax) qmax = sq;
        }
        double gap = fmax(qmin - pmax, pmin - qmax);
        if (gap > margin) margin = gap;
    }
    return margin;
}

/* Rectangle P and circle Q intersect iff the distance from Q's centre to the
 * closest point of P is at most r_Q. The closest point is found in P's frame
 * by clamping the centre's local coordinates to the half extents. */
double orc_margin_rect_circle(double xP, double yP, double psiP, double LP, double WP,
                              double xQ, double yQ, double rQ)
{
    double dx = xQ - xP, dy = yQ - yP;
    double lam = dx * cos(psiP) + dy * sin(psiP);     /* along P's heading */
    double mu = -dx * sin(psiP) + dy * cos(psiP);     /* across P's heading */
    double cl = fmin(fmax(lam, -LP / 2.0), LP / 2.0);
    double cm = fmin(fmax(mu, -WP / 2.0), WP / 2.0);
    double dist = hypot(lam - cl, mu - cm);
    return dist - rQ;
}

double orc_margin_circle_circle(double xP, double yP, double rP, double xQ, double yQ, double rQ)
{
    return hypot(xQ - xP, yQ - yP) - (rP + rQ);
}

/* ------------------------------------------------------------------------ */
/* Point-in-polygon overlap, the paper's own test (Sec. IV-C.1). Both        */
/* objects are polygons, and at each step the vertices of each are tested     */
/* against the other with a point-in-polygon test, once in each direction.    */
/* The margin is the smallest signed distance of any vertex of one polygon   */
/* to the boundary of the other: negative when the vertex lies inside (sign   */
/* from the crossing-number test), positive outside, so the margin is <= 0    */
/* exactly when some vertex lies in the other closed polygon. Two convex     */
/* shapes can overlap with no vertex of either inside the other (two bars    */
/* crossing like a plus sign); this test misses such an overlap by design.   */
/* ------------------------------------------------------------------------ */

int orc_point_in_polygon(double x, double y, int n, const double *vx, const double *vy);

static double point_segment_distance(double x, double y, double ax, double ay, double bx, double by)
{
    double ex = bx - ax, ey = by - ay;
    double len2 = ex * ex + ey * ey;
    double t = len2 > 0.0 ? ((x - ax) * ex + (y - ay) * ey) / len2 : 0.0;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    return hypot(x - (ax + t * ex), y - (ay + t * ey));
}

/* Signed distance of (x, y) to the boundary of the polygon (vx, vy)[n]. */
static double signed_boundary_distance(double x, double y, int n, const double *vx, const double *vy)
{
    double d = INFINITY;
    for (int k = 0, l = n - 1; k < n; l = k++) {
        double dk = point_segment_distance(x, y, vx[l], vy[l], vx[k], vy[k]);
        if (dk < d) d = dk;
    }
    return orc_point_in_polygon(x, y, n, vx, vy) ? -d : d;
}

double orc_margin_pip(int nP, const double *px, const double *py, int nQ, const double *qx, const double *qy)
{
    double m = INFINITY;
    for (int k = 0; k < nP; ++k) {            /* P over Q */
        double d = signed_boundary_distance(px[k], py[k], nQ, qx, qy);
        if (d < m) m = d;
    }
    for (int k = 0; k < nQ; ++k) {            /* Q over P */
        double d = signed_boundary_distance(qx[k], qy[k], nP, px, py);
        if (d < m) m = d;
    }
    return m;
}

double orc_margin_rect_rect_pip(double xP, double yP, double psiP, double LP, double WP,
                                     double xQ, double yQ, double psiQ, double LQ, double WQ)
{
    double px[4], py[4], qx[4], qy[4];
    rect_corners(xP, yP, psiP, LP, WP, px, py);
    rect_corners(xQ, yQ, psiQ, LQ, WQ, qx, qy);
    return orc_margin_pip(4, px, py, 4, qx, qy);
}

/* ------------------------------------------------------------------------ */
/* General convex polygons (Sec. IV-C.1 allows any complexity). A           */
/* vehicle may carry an outline: the vertices of a convex polygon in its     */
/* body frame (x along the heading, y to the left), counter-clockwise, at    */
/* most ORC_MAX_VERTICES. Polygons below are in world coordinates, CCW.      */
/* ------------------------------------------------------------------------ */
#define ORC_MAX_VERTICES 8

/* Vertices of an outline placed at pose (x, y, psi). */
static void place_outline(int n, const double *bx, const double *by, double x, double y, double psi,
                          double *wx, double *wy)
{
    double c = cos(psi), s = sin(psi);
    for (int k = 0; k < n; ++k) {
        wx[k] = x + c * bx[k] - s * by[k];
        wy[k] = y + s * bx[k] + c * by[k];
    }
}

/* Separating axis theorem for two convex polygons: they are disjoint iff
 * the other polygon lies strictly outside the supporting line of some edge
 * of one of them. With unit outward edge normals n_e and edge starts a_e the
 * margin is max over all edges e of min over the other polygon's vertices v
 * of n_e . (v - a_e): the largest gap along an edge normal; <= 0 exactly when
 * the closed polygons intersect. For rectangles it is orc_margin_rect_rect. */
static double edge_gap(int nP, const double *px, const double *py, int nQ, const double *qx, const double *qy)
{
    double best = -INFINITY;
    for (int e = 0; e < nP; ++e) {
        int f = (e + 1) % nP;
        double ex = px[f] - px[e], ey = py[f] - py[e];
        double len = hypot(ex, ey);
        double nx = ey / len, ny = -ex / len;   /* outward for a CCW polygon */
        double lo = INFINITY;
        for (int k = 0; k < nQ; ++k) {
            double v = nx * (qx[k] - px[e]) + ny * (qy[k] - py[e]);
            if (v < lo) lo = v;
        }
        if (lo > best) best = lo;
    }
    return best;
}

double orc_margin_poly_poly(int nP, const double *px, const double *py, int nQ, const double *qx, const double *qy)
{
    return fmax(edge_gap(nP, px, py, nQ, qx, qy), edge_gap(nQ, qx, qy, nP, px, py));
}

/* Convex polygon P and circle (c, r): the distance from c to the closed
 * polygon (0 inside) minus r. */
double orc_margin_poly_circle(int nP, const double *px, const double *py, double cx, double cy, double r)
{
    int inside = 1;
    double d = INFINITY;
    for (int e = 0; e < nP; ++e) {
        int f = (e + 1) % nP;
        double ex = px[f] - px[e], ey = py[f] - py[e];
        if (ex * (cy - py[e]) - ey * (cx - px[e]) < 0.0) inside = 0;   /* right of a CCW edge */
        double de = point_segment_distance(cx, cy, px[e], py[e], px[f], py[f]);
        if (de < d) d = de;
    }
    return (inside ? 0.0 : d) - r;
}

/* Shape of an object at one pose, as a polygon (vehicles) or a circle. */
typedef struct {
    int kind, n;                      /* n > 0: polygon of n vertices */
    double x[ORC_MAX_VERTICES], y[ORC_MAX_VERTICES];
    double cx, cy, r;
} orc_shape;

static void shape_at(orc_shape *sh, int kind, int nv, const double *bx, const double *by, double L, double W,
                     double r, double x, double y, double psi)
{
    sh->kind = kind;
    sh->cx = x;
    sh->cy = y;
    sh->r = r;
    sh->n = 0;
    if (kind != ORC_VEHICLE) return;
    if (nv > 0) {
        sh->n = nv;
        place_outline(nv, bx, by, x, y, psi, sh->x, sh->y);
    } else {
        /* rect_corners lists the corners clockwise; polygons here are CCW */
        double cx[4], cy[4];
        rect_corners(x, y, psi, L, W, cx, cy);
        sh->n = 4;
        for (int k = 0; k < 4; ++k) {
            sh->x[k] = cx[3 - k];
            sh->y[k] = cy[3 - k];
        }
    }
}

static double margin_at(int overlap, int kindP, double xP, double yP, double psiP, double LP, double WP, double rP,
                        int nvP, const double *bxP, const double *byP,
                        int kindQ, double xQ, double yQ, double psiQ, double LQ, double WQ, double rQ,
                        int nvQ, const double *bxQ, const double *byQ)
{
    if (nvP == 0 && nvQ == 0) {
        /* rectangles and circles */
        if (overlap == ORC_OVERLAP_PIP)
            return orc_margin_rect_rect_pip(xP, yP, psiP, LP, WP, xQ, yQ, psiQ, LQ, WQ);
        if (kindP == ORC_VEHICLE && kindQ == ORC_VEHICLE)
            return orc_margin_rect_rect(xP, yP, psiP, LP, WP, xQ, yQ, psiQ, LQ, WQ);
        if (kindP == ORC_VEHICLE)
            return orc_margin_rect_circle(xP, yP, psiP, LP, WP, xQ, yQ, rQ);
        if (kindQ == ORC_VEHICLE)
            return orc_margin_rect_circle(xQ, yQ, psiQ, LQ, WQ, xP, yP, rP);
        return orc_margin_circle_circle(xP, yP, rP, xQ, yQ, rQ);
    }
    /* at least one outline: every vehicle is a polygon (a rectangle by its
     * four corners) */
    orc_shape P, Q;
    shape_at(&P, kindP, nvP, bxP, byP, LP, WP, rP, xP, yP, psiP);
    shape_at(&Q, kindQ, nvQ, bxQ, byQ, LQ, WQ, rQ, xQ, yQ, psiQ);
    if (overlap == ORC_OVERLAP_PIP) return orc_margin_pip(P.n, P.x, P.y, Q.n, Q.x, Q.y);
    if (P.n && Q.n) return orc_margin_poly_poly(P.n, P.x, P.y, Q.n, Q.x, Q.y);
    if (P.n) return orc_margin_poly_circle(P.n, P.x, P.y, Q.cx, Q.cy, Q.r);
    if (Q.n) return orc_margin_poly_circle(Q.n, Q.x, Q.y, P.cx, P.cy, P.r);
    return orc_margin_circle_circle(xP, yP, rP, xQ, yQ, rQ);
}

/* ------------------------------------------------------------------------ */
/* Pairs: Sec. IV-C.1 checks EGO (object 0) against every collision object   */
/* only; the all-pairs mode checks every unordered pair a < b. Pairs are     */
/* listed in lexicographic order.                                            */
/* ------------------------------------------------------------------------ */
int orc_pairs(int n_objects, int ego_only, int32_t *pa, int32_t *pb)
{
    int n = 0;
    for (int a = 0; a < n_objects; ++a)
        for (int b = a + 1; b < n_objects; ++b) {
            if (ego_only && a != 0) continue;
            if (pa) pa[n] = a;
            if (pb) pb[n] = b;
            ++n;
        }
    return n;
}

/* Trajectory-generation thread count r_tra of Sec. IV-B.4 and the collision
 * combination count r_col of Sec. IV-C.2, as plain sums over the scene. */
int64_t orc_count_trajectories(int n_objects, const int32_t *T)
{
    int64_t s = 0;
    for (int a = 0; a < n_objects; ++a) s += T[a];
    return s;
}

int64_t orc_count_combinations(int n_objects, const int32_t *T, int ego_only)
{
    int64_t s = 0;
    for (int a = 0; a < n_objects; ++a)
        for (int b = a + 1; b < n_objects; ++b)
            if (!ego_only || a == 0) s += (int64_t)T[a] * (int64_t)T[b];
    return s;
}

/* ------------------------------------------------------------------------ */
/* First hits.                                                                */
/*                                                                            */
/* Poses of all objects are concatenated: object a's block starts at          */
/* H * sum_{c<a} T_c and is laid out [t][i]. For every listed pair (a, b),    */
/* trajectory i of a, trajectory j of b, entry e = pair_offset + i*T_b + j:    */
/*   k64[e]     = min{ t : m(t) <= 0 }, else -1                              */
/*   kstrict[e] = min{ t : m(t) <= -eps }, else -1                           */
/*   loose[e*W + t/64]  bit t%64 set iff m(t) <= +eps   (W = ceil(H/64))    */
/*   strict[e*W + t/64] bit t%64 set iff m(t) <= -eps                       */
/* Vehicle a with n_vertices[a] > 0 has the outline (outline_x, outline_y)   */
/* [a * 8 ...] (body frame, CCW) instead of its rectangle; n_vertices may be */
/* NULL (no outlines).                                                        */
/* Any output pointer may be NULL. eps is the tolerance band within which an */
/* FP32 evaluation of the same test may legitimately decide either way.      */
/* ------------------------------------------------------------------------ */
int orc_first_hits(int overlap, int n_objects, const int32_t *kind, const double *length, const double *width,
                   const double *radius, const int32_t *n_vertices, const double *outline_x,
                   const double *outline_y, const int32_t *T, int H,
                   const double *px, const double *py, const double *ppsi,
                   int n_pairs, const int32_t *pair_a, const int32_t *pair_b,
                   double eps, int threads,
                   int32_t *k64, int32_t *kstrict, uint64_t *loose, uint64_t *strict)
{
    if (n_objects < 1 || H < 1 || n_pairs < 0) return ORC_EINVAL;
    if (overlap != ORC_OVERLAP_EXACT && overlap != ORC_OVERLAP_PIP) return ORC_EINVAL;
    if (overlap == ORC_OVERLAP_PIP)          /* polygons: vehicles only */
        for (int a = 0; a < n_objects; ++a)
            if (kind[a] != ORC_VEHICLE) return ORC_EINVAL;
    if (n_vertices)
        for (int a = 0; a < n_objects; ++a)
            if (n_vertices[a] < 0 || n_vertices[a] > ORC_MAX_VERTICES || (n_vertices[a] && kind[a] != ORC_VEHICLE))
                return ORC_EINVAL;
    int W = (H + 63) / 64;
    int64_t *obj_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_objects + 1));
    int64_t *pair_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_pairs + 1));
    if (!obj_off || !pair_off) { free(obj_off); free(pair_off); return ORC_ENOMEM; }
    obj_off[0] = 0;
    for (int a = 0; a < n_objects; ++a) obj_off[a + 1] = obj_off[a] + (int64_t)H * T[a];
    pair_off[0] = 0;
    for (int p = 0; p < n_pairs; ++p) {
        int a = pair_a[p], b = pair_b[p];
        if (a < 0 || b < 0 || a >= n_objects || b >= n_objects || a == b) {
            free(obj_off); free(pair_off); return ORC_EINVAL;
        }
        pair_off[p + 1] = pair_off[p] + (int64_t)T[a] * T[b];
    }
    /* rows = (pair, i), the unit of work that threads may share */
    int64_t *row_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_pairs + 1));
    if (!row_off) { free(obj_off); free(pair_off); return ORC_ENOMEM; }
    row_off[0] = 0;
    for (int p = 0; p < n_pairs; ++p) row_off[p + 1] = row_off[p] + T[pair_a[p]];
    int64_t n_rows = row_off[n_pairs];

#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t r = 0; r < n_rows; ++r) {
        int p = 0;
        while (row_off[p + 1] <= r) ++p;
        int a = pair_a[p], b = pair_b[p];
        int i = (int)(r - row_off[p]);
        int Ta = T[a], Tb = T[b];
        for (int j = 0; j < Tb; ++j) {
            int64_t e = pair_off[p] + (int64_t)i * Tb + j;
            int32_t first = -1, first_strict = -1;
            if (loose) for (int wd = 0; wd < W; ++wd) loose[e * W + wd] = 0;
            if (strict) for (int wd = 0; wd < W; ++wd) strict[e * W + wd] = 0;
            for (int t = 0; t < H; ++t) {
                size_t ia = (size_t)(obj_off[a] + (int64_t)t * Ta + i);
                size_t ib = (size_t)(obj_off[b] + (int64_t)t * Tb + j);
                int nva = n_vertices ? n_vertices[a] : 0, nvb = n_vertices ? n_vertices[b] : 0;
                double m = margin_at(overlap, kind[a], px[ia], py[ia], ppsi[ia], length[a], width[a], radius[a],
                                     nva, outline_x + a * ORC_MAX_VERTICES, outline_y + a * ORC_MAX_VERTICES,
                                     kind[b], px[ib], py[ib], ppsi[ib], length[b], width[b], radius[b],
                                     nvb, outline_x + b * ORC_MAX_VERTICES, outline_y + b * ORC_MAX_VERTICES);
                if (m <= 0.0 && first < 0) first = t;
                if (m <= -eps && first_strict < 0) first_strict = t;
                if (loose && m <= eps) loose[e * W + t / 64] |= (uint64_t)1 << (t % 64);
                if (strict && m <= -eps) strict[e * W + t / 64] |= (uint64_t)1 << (t % 64);
            }
            if (k64) k64[e] = first;
            if (kstrict) kstrict[e] = first_strict;
        }
    }
    free(row_off);
    free(obj_off);
    free(pair_off);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Risk: Sec. IV-D and Sec. IV-D.2.                                           */
/*                                                                            */
/* hit[e] (entry layout as above) says whether trajectory pair e collides.    */
/* For object a, trajectory i and another object b, the probability that the */
/* collision with b happens along trajectory i is                             */
/*   EXCLUSIVE:   q[a,i;b] = sum_j hit(a,i;b,j) p_{b,j}                       */
/*                (b follows exactly one of its trajectories)                */
/*   INDEPENDENT: q[a,i;b] = 1 - prod_j (1 - hit(a,i;b,j) p_{b,j})            */
/*                (every combination occurs independently)                   */
/* Under the chronological scaling the collision with b only counts when no  */
/* other object has collided first; with the objects independent, the        */
/* probability that some collision happens along trajectory i is             */
/*   crit[a,i]  = 1 - prod_{b != a} (1 - q[a,i;b])                           */
/* and the criticality of object a weights its trajectories by probability:  */
/*   C[a]       = sum_i p_{a,i} crit[a,i]                                    */
/* With a single collision object and the exclusive reading C[0] is the      */
/* double sum p_cra of Sec. IV-D.                                            */
/* q is [sum T][n_objects] (nullable); traj_crit [sum T]; obj_crit [n].       */
/* Pairs not listed contribute q = 0.                                         */
/* ------------------------------------------------------------------------ */
static double combine_q(int model, double acc, double p)
{
    /* fold one colliding combination of probability p into q */
    return model == ORC_RISK_EXCLUSIVE ? acc + p : 1.0 - (1.0 - acc) * (1.0 - p);
}

int orc_risk(int model, int n_objects, const int32_t *T, const double *p,
             int n_pairs, const int32_t *pair_a, const int32_t *pair_b,
             const uint8_t *hit, double *q_out, double *traj_crit, double *obj_crit)
{
    if (n_objects < 1 || n_pairs < 0) return ORC_EINVAL;
    if (model != ORC_RISK_EXCLUSIVE && model != ORC_RISK_INDEPENDENT) return ORC_EINVAL;
    int64_t *toff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_objects + 1));
    if (!toff) return ORC_ENOMEM;
    toff[0] = 0;
    for (int a = 0; a < n_objects; ++a) toff[a + 1] = toff[a] + T[a];
    int64_t n_traj = toff[n_objects];
    double *q = (double *)calloc((size_t)n_traj * (size_t)n_objects, sizeof(double));
    if (!q) { free(toff); return ORC_ENOMEM; }

    int64_t e0 = 0;
    for (int pr = 0; pr < n_pairs; ++pr) {
        int a = pair_a[pr], b = pair_b[pr];
        int Ta = T[a], Tb = T[b];
        for (int i = 0; i < Ta; ++i) {
            double s = 0.0;
            for (int j = 0; j < Tb; ++j)
                if (hit[e0 + (int64_t)i * Tb + j]) s = combine_q(model, s, p[toff[b] + j]);
            q[(toff[a] + i) * n_objects + b] = fmin(s, 1.0);
        }
        for (int j = 0; j < Tb; ++j) {
            double s = 0.0;
            for (int i = 0; i < Ta; ++i)
                if (hit[e0 + (int64_t)i * Tb + j]) s = combine_q(model, s, p[toff[a] + i]);
            q[(toff[b] + j) * n_objects + a] = fmin(s, 1.0);
        }
        e0 += (int64_t)Ta * Tb;
    }
    for (int a = 0; a < n_objects; ++a) {
        double C = 0.0;
        for (int i = 0; i < T[a]; ++i) {
            double no_collision = 1.0;
            for (int b = 0; b < n_objects; ++b)
                if (b != a) no_collision *= 1.0 - q[(toff[a] + i) * n_objects + b];
            double crit = 1.0 - no_collision;
            if (traj_crit) traj_crit[toff[a] + i] = crit;
            C += p[toff[a] + i] * crit;
        }
        if (obj_crit) obj_crit[a] = C;
    }
    if (q_out) memcpy(q_out, q, sizeof(double) * (size_t)n_traj * (size_t)n_objects);
    free(q);
    free(toff);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Risk over time: the chronological scaling of Sec. IV-D.2, step by step,    */
/* and the time-resolved criticality behind the anticipation time of          */
/* Sec. IV-D / Sec. VI-A.                                                     */
/*                                                                            */
/* k[e] is the earliest colliding slot of entry e (layout as above), or -1.  */
/* For object a and trajectory i, every colliding combination with a        */
/* trajectory j of another object b is an event (slot k, b, j) of            */
/* probability p_{b,j}. The events are taken in time order (ties: ascending  */
/* b, then j). The first keeps its probability; each later one counts only  */
/* if no collision has happened before it:                                   */
/*   EXCLUSIVE:   scaled = p_{b,j} * prod_{b' != b} (1 - Q_{b'})             */
/*                where Q_{b'} sums p over the events of b' taken so far     */
/*                (b's own earlier events exclude this one: b follows one    */
/*                trajectory), then Q_b += p_{b,j};                          */
/*   INDEPENDENT: scaled = p_{b,j} * prod over all earlier events of (1 - p) */
/*                (the paper's P(C and not B and not A) = P(~A) P(~B) P(C)). */
/* The scaled probabilities of the events up to slot s add up to             */
/*   crit_t[a,i][s]  the probability of a collision at or before slot s,     */
/* and those of b's events to                                                */
/*   attrib[a,i][b]  the probability that the first collision is with b;    */
/* sum_b attrib[a,i][b] = crit_t[a,i][H-1] = crit[a,i] of orc_risk.          */
/* Object level: C_t[a][s] = sum_i p_{a,i} crit_t[a,i][s] and                */
/* A[a][b] = sum_i p_{a,i} attrib[a,i][b].                                    */
/* Outputs (each nullable): traj_crit_t [sum T][H], obj_crit_t [n][H],        */
/* traj_attrib [sum T][n], obj_attrib [n][n].                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t k, b, j;
    double p;
} orc_event;

static int event_order(const void *x, const void *y)
{
    const orc_event *e = (const orc_event *)x, *f = (const orc_event *)y;
    if (e->k != f->k) return e->k < f->k ? -1 : 1;
    if (e->b != f->b) return e->b < f->b ? -1 : 1;
    if (e->j != f->j) return e->j < f->j ? -1 : 1;
    return 0;
}

int orc_risk_timeline(int model, int n_objects, const int32_t *T, const double *p, int H,
                      int n_pairs, const int32_t *pair_a, const int32_t *pair_b, const int32_t *k,
                      double *traj_crit_t, double *obj_crit_t, double *traj_attrib, double *obj_attrib)
{
    if (n_objects < 1 || n_pairs < 0 || H < 1) return ORC_EINVAL;
    if (model != ORC_RISK_EXCLUSIVE && model != ORC_RISK_INDEPENDENT) return ORC_EINVAL;
    int64_t *toff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_objects + 1));
    int64_t *poff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_pairs + 1));
    if (!toff || !poff) { free(toff); free(poff); return ORC_ENOMEM; }
    toff[0] = 0;
    for (int a = 0; a < n_objects; ++a) toff[a + 1] = toff[a] + T[a];
    poff[0] = 0;
    int64_t max_events = 0;
    for (int pr = 0; pr < n_pairs; ++pr) {
        poff[pr + 1] = poff[pr] + (int64_t)T[pair_a[pr]] * T[pair_b[pr]];
        max_events += T[pair_a[pr]] > T[pair_b[pr]] ? T[pair_a[pr]] : T[pair_b[pr]];
    }
    orc_event *ev = (orc_event *)malloc(sizeof(orc_event) * (size_t)(max_events + 1));
    double *Q = (double *)malloc(sizeof(double) * (size_t)n_objects);
    double *A = (double *)malloc(sizeof(double) * (size_t)n_objects);
    double *ct = (double *)malloc(sizeof(double) * (size_t)H);
    if (!ev || !Q || !A || !ct) {
        free(toff); free(poff); free(ev); free(Q); free(A); free(ct);
        return ORC_ENOMEM;
    }
    if (obj_crit_t) memset(obj_crit_t, 0, sizeof(double) * (size_t)n_objects * (size_t)H);
    if (obj_attrib) memset(obj_attrib, 0, sizeof(double) * (size_t)n_objects * (size_t)n_objects);

    for (int a = 0; a < n_objects; ++a) {
        for (int i = 0; i < T[a]; ++i) {
            /* gather the colliding combinations of trajectory (a, i) */
            int64_t m = 0;
            for (int pr = 0; pr < n_pairs; ++pr) {
                int pa = pair_a[pr], pb = pair_b[pr];
                if (pa == a) {
                    for (int j = 0; j < T[pb]; ++j) {
                        int32_t kk = k[poff[pr] + (int64_t)i * T[pb] + j];
                        if (kk >= 0) ev[m++] = (orc_event){kk, pb, j, p[toff[pb] + j]};
                    }
                } else if (pb == a) {
                    for (int j = 0; j < T[pa]; ++j) {
                        int32_t kk = k[poff[pr] + (int64_t)j * T[a] + i];
                        if (kk >= 0) ev[m++] = (orc_event){kk, pa, j, p[toff[pa] + j]};
                    }
                }
            }
            qsort(ev, (size_t)m, sizeof(orc_event), event_order);
            for (int b = 0; b < n_objects; ++b) { Q[b] = 0.0; A[b] = 0.0; }
            double crit = 0.0, survive = 1.0;
            int64_t e = 0;
            for (int s = 0; s < H; ++s) {
                for (; e < m && ev[e].k == s; ++e) {
                    int b = ev[e].b;
                    double scaled;
                    if (model == ORC_RISK_EXCLUSIVE) {
                        double keep = 1.0;
                        for (int c = 0; c < n_objects; ++c)
                            if (c != b && c != a) keep *= 1.0 - fmin(Q[c], 1.0);
                        scaled = ev[e].p * keep;
                        Q[b] += ev[e].p;
                    } else {
                        scaled = ev[e].p * survive;
                        survive *= 1.0 - ev[e].p;
                    }
                    A[b] += scaled;
                    crit += scaled;
                }
                ct[s] = crit;
            }
            double pi = p[toff[a] + i];
            if (traj_crit_t) memcpy(traj_crit_t + (toff[a] + i) * H, ct, sizeof(double) * (size_t)H);
            if (obj_crit_t)
                for (int s = 0; s < H; ++s) obj_crit_t[(int64_t)a * H + s] += pi * ct[s];
            if (traj_attrib) memcpy(traj_attrib + (toff[a] + i) * n_objects, A, sizeof(double) * (size_t)n_objects);
            if (obj_attrib)
                for (int b = 0; b < n_objects; ++b) obj_attrib[(int64_t)a * n_objects + b] += pi * A[b];
        }
    }
    free(toff); free(poff); free(ev); free(Q); free(A); free(ct);
    return ORC_OK;
}

/* Point-in-polygon test (crossing number) for a convex or concave polygon,
 * the per-vertex test the paper runs in both directions (Sec. IV-C.1). It
 * gives the sign of the point-in-polygon overlap margin above; a point on an
 * edge may fall either way, which the margin's magnitude (zero there) makes
 * irrelevant. */
int orc_point_in_polygon(double x, double y, int n, const double *vx, const double *vy)
{
    int inside = 0;
    for (int k = 0, l = n - 1; k < n; l = k++) {
        if (((vy[k] > y) != (vy[l] > y)) &&
            (x < (vx[l] - vx[k]) * (y - vy[k]) / (vy[l] - vy[k]) + vx[k]))
            inside = !inside;
    }
    return inside;
}

int orc_rect_corners(double x, double y, double psi, double L, double W, double *cx, double *cy)
{
    rect_corners(x, y, psi, L, W, cx, cy);
    return ORC_OK;
}
