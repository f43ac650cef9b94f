/*
 * cpf_oracle.c -- plain, slow, FP64 CPU oracle for the CppFlow refinement
 * path (arXiv 2309.09102).  TEST INFRASTRUCTURE ONLY: the product path never
 * calls, links or includes this file; only the tests, the smoke check and the
 * benchmark's CPU-baseline leg do.
 *
 * Everything is IEEE double, built with -O2 -ffp-contract=off (no fused
 * multiply-add, no fast-math) so every operation rounds exactly as written.
 * The notation follows the paper with the build's names: T waypoints, n
 * joints, K candidate plans per waypoint.
 *
 * Contents and the passages they follow:
 *   or_fk          forward kinematics FK(q) : R^n -> SE(3)          Sec. II
 *                  (standard distal Denavit-Hartenberg chain of revolute
 *                  and prismatic joints, Sec. IV's Fetch.Full torso lift)
 *                  and the geometric (kinematic) Jacobian J_fk      Sec. III-C
 *   or_log_so3     rotation vector of a rotation matrix; its norm is the
 *                  geodesic rotation error used as the validity metric Sec. II
 *   or_cost        pose residual + differencing residual, squared   Sec. III-C,
 *                  and weighted                                      Fig. (residual)
 *   or_dp          layered-graph search minimising the maximum joint angle
 *                  change (mjac) with the joint-limit penalty        Sec. III-B
 *   or_btd_solve   the LM normal equations (J^T J + lambda I) step   Sec. III-C
 *                  for the block-tridiagonal system that the pose and
 *                  differencing residuals give (their Jacobians are
 *                  per-waypoint blocks and +-I)
 *   or_lm          Levenberg-Marquardt with clamping to joint limits Sec. III-C
 *   or_plan        search, then LM from the searched seed            Sec. III
 *
 * Readings where the paper is silent or garbled (each listed with its reason
 * in the design notes):
 *   - rotation residual = Log(R(q) R*^T) (world frame) rather than a roll /
 *     pitch / yaw difference; its norm is the paper's geodesic error;
 *   - LM step (J^T W J + lambda I) delta = -J^T W r (transpose and sign of the
 *     printed update restored), pure Levenberg damping lambda*I;
 *   - weights multiply squared norms: C = w_p/2 sum|r_t|^2 + w_s/2 sum|dq|^2;
 *   - lambda schedule: Nielsen's gain-ratio rule (H.B. Nielsen, IMM-REP-1999-05;
 *     Madsen, Nielsen & Tingleff 2004, Sec. 3.2);
 *   - penalties enter the search on the edge into the penalised node; ties
 *     are broken by the key (value, edge change, predecessor index);
 *   - a prismatic joint's value adds to its link's offset d and its Jacobian
 *     column is [z; 0]; its limit margin is 3 cm and its validity step 2 cm,
 *     while edge costs and mjac keep the printed formula over all joints.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXN 16
#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Small dense helpers (row-major)                                           */
/* ------------------------------------------------------------------------ */

/* 4x4 homogeneous transform as a 3x4 row-major block [R | p]. */
static void tf_identity(double M[12]) {
    memset(M, 0, 12 * sizeof(double));
    M[0] = 1.0; M[5] = 1.0; M[10] = 1.0;
}

/* Standard DH link transform Rz(theta) Tz(d) Tx(a) Rx(alpha). */
static void dh_link(double theta, double d, double a, double alpha, double A[12]) {
    double ct = cos(theta), st = sin(theta);
    double ca = cos(alpha), sa = sin(alpha);
    A[0] = ct;  A[1] = -st * ca; A[2]  = st * sa;  A[3]  = a * ct;
    A[4] = st;  A[5] = ct * ca;  A[6]  = -ct * sa; A[7]  = a * st;
    A[8] = 0.0; A[9] = sa;       A[10] = ca;       A[11] = d;
}

/* C = A * B for 3x4 homogeneous blocks. */
static void tf_mul(const double A[12], const double B[12], double C[12]) {
    double out[12];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 4; ++c) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[r * 4 + k] * B[k * 4 + c];
            if (c == 3) s += A[r * 4 + 3];
            out[r * 4 + c] = s;
        }
    }
    memcpy(C, out, sizeof(out));
}

/* ------------------------------------------------------------------------ */
/* Forward kinematics and geometric Jacobian (Sec. II, Sec. III-C)           */
/* ------------------------------------------------------------------------ */

/*
 * pose[12] = (x, y, z, R00, R01, R02, R10, ..., R22) of the end effector.
 * J (optional) is 6 x n row-major: rows vx, vy, vz, wx, wy, wz; column i is
 * z_{i-1} x (p - o_{i-1}) over z_{i-1}, the axis and origin of joint i, for
 * a revolute joint and z_{i-1} over 0 for a prismatic one.
 * jtype (optional, NULL = all revolute): 1 marks a prismatic joint, whose
 * value is added to the link's offset d while its angle stays at theta_off;
 * a revolute joint's value is added to theta_off.
 */
static int prismatic(const int32_t *jtype, int i) { return jtype && jtype[i] == 1; }

/* DH angle and offset of link i at joint value qi. */
static void joint_dh(const int32_t *jtype, const double *d, const double *theta_off, int i, double qi,
                     double *th, double *di) {
    double off = theta_off ? theta_off[i] : 0.0;
    if (prismatic(jtype, i)) { *th = off; *di = d[i] + qi; }
    else { *th = qi + off; *di = d[i]; }
}

void or_fk(int n, const double *a, const double *d, const double *alpha,
           const double *theta_off, const int32_t *jtype, const double *q, double *pose, double *J) {
    double M[12], A[12];
    double z[OR_MAXN][3], o[OR_MAXN][3];
    tf_identity(M);
    for (int i = 0; i < n; ++i) {
        z[i][0] = M[2]; z[i][1] = M[6]; z[i][2] = M[10];
        o[i][0] = M[3]; o[i][1] = M[7]; o[i][2] = M[11];
        double th, di;
        joint_dh(jtype, d, theta_off, i, q[i], &th, &di);
        dh_link(th, di, a[i], alpha[i], A);
        tf_mul(M, A, M);
    }
    pose[0] = M[3]; pose[1] = M[7]; pose[2] = M[11];
    pose[3] = M[0]; pose[4] = M[1]; pose[5] = M[2];
    pose[6] = M[4]; pose[7] = M[5]; pose[8] = M[6];
    pose[9] = M[8]; pose[10] = M[9]; pose[11] = M[10];
    if (J) {
        for (int i = 0; i < n; ++i) {
            if (prismatic(jtype, i)) {
                J[0 * n + i] = z[i][0];
                J[1 * n + i] = z[i][1];
                J[2 * n + i] = z[i][2];
                J[3 * n + i] = 0.0;
                J[4 * n + i] = 0.0;
                J[5 * n + i] = 0.0;
                continue;
            }
            double dx = pose[0] - o[i][0], dy = pose[1] - o[i][1], dz = pose[2] - o[i][2];
            J[0 * n + i] = z[i][1] * dz - z[i][2] * dy;
            J[1 * n + i] = z[i][2] * dx - z[i][0] * dz;
            J[2 * n + i] = z[i][0] * dy - z[i][1] * dx;
            J[3 * n + i] = z[i][0];
            J[4 * n + i] = z[i][1];
            J[5 * n + i] = z[i][2];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Rotation vector (log map of SO(3))                                        */
/* ------------------------------------------------------------------------ */

/*
 * phi = theta * u with R = exp([phi]x).  theta = atan2(|v|, (tr R - 1)/2),
 * v = vee(R - R^T)/2.  Near theta = 0 the factor theta/sin(theta) is its
 * Taylor series; near theta = pi the axis comes from the symmetric part
 * (R + R^T)/2 - cos(theta) I = (1 - cos theta) u u^T.
 */
void or_log_so3(const double *R, double *phi) {
    double v0 = 0.5 * (R[7] - R[5]);
    double v1 = 0.5 * (R[2] - R[6]);
    double v2 = 0.5 * (R[3] - R[1]);
    double s = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
    double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
    double th = atan2(s, c);
    if (th < 1e-4) {
        double k = 1.0 + th * th / 6.0;
        phi[0] = k * v0; phi[1] = k * v1; phi[2] = k * v2;
        return;
    }
    if (th > OR_PI - 1e-6) {
        double B[9];
        for (int r = 0; r < 3; ++r)
            for (int cc = 0; cc < 3; ++cc)
                B[r * 3 + cc] = 0.5 * (R[r * 3 + cc] + R[cc * 3 + r]) - (r == cc ? c : 0.0);
        int i = 0;
        if (B[4] > B[i * 4]) i = 1;
        if (B[8] > B[i * 4]) i = 2;
        double omc = 1.0 - c;
        double ui = sqrt(B[i * 4] / omc);
        double u[3];
        for (int j = 0; j < 3; ++j) u[j] = B[i * 3 + j] / (omc * ui);
        u[i] = ui;
        double dotv = u[0] * v0 + u[1] * v1 + u[2] * v2;
        if (dotv < 0.0) { u[0] = -u[0]; u[1] = -u[1]; u[2] = -u[2]; }
        phi[0] = th * u[0]; phi[1] = th * u[1]; phi[2] = th * u[2];
        return;
    }
    double k = th / s;
    phi[0] = k * v0; phi[1] = k * v1; phi[2] = k * v2;
}

/* Geodesic angle between two rotations: angle of A B^T. */
static double rot_angle(const double *A, const double *B) {
    double M[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            M[r * 3 + c] = A[r * 3 + 0] * B[c * 3 + 0] + A[r * 3 + 1] * B[c * 3 + 1] +
                           A[r * 3 + 2] * B[c * 3 + 2];
    double v0 = 0.5 * (M[7] - M[5]), v1 = 0.5 * (M[2] - M[6]), v2 = 0.5 * (M[3] - M[1]);
    double s = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
    double c = 0.5 * (M[0] + M[4] + M[8] - 1.0);
    return atan2(s, c);
}

/* ------------------------------------------------------------------------ */
/* Residual and cost (Sec. III-C, residual figure)                           */
/* ------------------------------------------------------------------------ */

/* ------------------------------------------------------------------------ */
/* Collision geometry (Sec. II collision avoidance; Sec. III-C robot-robot   */
/* and robot-environment distances)                                          */
/* ------------------------------------------------------------------------ */

/*
 * A capsule on every link: a segment between two points fixed in the frame
 * after link i, and a radius.  Obstacles are cuboids: a frame (origin, then
 * the rotation row-major, its columns the cuboid's axes) and the corners
 * p_min, p_max in that frame.  Flat description (NULL: no geometry):
 *   spec[0] margin m of the residual max(0, m - d), spec[1] weight w_c of the
 *   collision residuals, spec[2] search penalty of a colliding configuration,
 *   spec[3] number of obstacles n_obs, then n x 7 capsule values
 *   (p0 xyz, p1 xyz, radius), then n_obs x 18 obstacle values
 *   (origin xyz, R row-major, p_min xyz, p_max xyz).
 */
typedef struct {
    double margin, w_c, penalty;
    int nobs;
    const double *caps, *obs;
} or_coll;

static void coll_parse(int n, const double *spec, or_coll *c) {
    c->margin = spec[0];
    c->w_c = spec[1];
    c->penalty = spec[2];
    c->nobs = (int)spec[3];
    c->caps = spec + 4;
    c->obs = spec + 4 + 7 * n;
}

typedef struct {
    int n;
    const double *a, *d, *alpha, *theta_off;
    const int32_t *jtype;  /* NULL: all revolute */
    const double *lo, *hi;
    const or_coll *coll;   /* NULL: no collision geometry */
} or_robot;

/* r[6] = [p(q) - p*; Log(R(q) R*^T)] for one waypoint; J6 optional (6 x n). */
static void pose_residual(const or_robot *rb, const double *q, const double *target,
                          double *r, double *J6) {
    double pose[12];
    or_fk(rb->n, rb->a, rb->d, rb->alpha, rb->theta_off, rb->jtype, q, pose, J6);
    r[0] = pose[0] - target[0];
    r[1] = pose[1] - target[1];
    r[2] = pose[2] - target[2];
    const double *R = pose + 3, *Rt = target + 3;
    double E[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            E[i * 3 + j] = R[i * 3 + 0] * Rt[j * 3 + 0] + R[i * 3 + 1] * Rt[j * 3 + 1] +
                           R[i * 3 + 2] * Rt[j * 3 + 2];
    or_log_so3(E, r + 3);
}

/*
 * Squared distance of the segments p(s) = P0 + s (P1 - P0) and
 * q(t) = Q0 + t (Q1 - Q0), s, t in [0, 1] (the robot-robot QP of Sec.
 * III-C).  f(s, t) = |r + s d1 - t d2|^2 is convex, so its minimum over the
 * square is the interior stationary point (when it exists and lies inside)
 * or the smallest of the four edge minima, each a clamped 1-D quadratic.
 * Candidates are compared in the order interior, s = 0, s = 1, t = 0, t = 1;
 * the first of equal values wins.
 */
static double seg_seg(const double P0[3], const double P1[3], const double Q0[3], const double Q1[3],
                      double *s_out, double *t_out) {
    double d1[3], d2[3], r[3];
    for (int k = 0; k < 3; ++k) {
        d1[k] = P1[k] - P0[k];
        d2[k] = Q1[k] - Q0[k];
        r[k] = P0[k] - Q0[k];
    }
    double a = 0, b = 0, e = 0, c = 0, f = 0;
    for (int k = 0; k < 3; ++k) {
        a += d1[k] * d1[k];
        b += d1[k] * d2[k];
        e += d2[k] * d2[k];
        c += d1[k] * r[k];
        f += d2[k] * r[k];
    }
    double cs[5], ct[5];
    int nc = 0;
    double det = a * e - b * b;
    if (det > 1e-12 * a * e && det > 0.0) {
        double s = (b * f - c * e) / det, t = (a * f - b * c) / det;
        if (s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0) { cs[nc] = s; ct[nc] = t; ++nc; }
    }
    for (int side = 0; side < 2; ++side) {          /* s fixed */
        double s = side, t = e > 0.0 ? (b * s + f) / e : 0.0;
        t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
        cs[nc] = s; ct[nc] = t; ++nc;
    }
    for (int side = 0; side < 2; ++side) {          /* t fixed */
        double t = side, s = a > 0.0 ? (b * t - c) / a : 0.0;
        s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
        cs[nc] = s; ct[nc] = t; ++nc;
    }
    double best = INFINITY;
    for (int i = 0; i < nc; ++i) {
        double v = 0.0;
        for (int k = 0; k < 3; ++k) {
            double w = r[k] + cs[i] * d1[k] - ct[i] * d2[k];
            v += w * w;
        }
        if (v < best) { best = v; *s_out = cs[i]; *t_out = ct[i]; }
    }
    return best;
}

/* Squared distance from x to the interval [lo, hi] (one axis of a cuboid). */
static double axis_gap2(double x, double lo, double hi) {
    if (x < lo) return (lo - x) * (lo - x);
    if (x > hi) return (x - hi) * (x - hi);
    return 0.0;
}

/*
 * Squared distance of the segment x(s) = A + s D (cuboid frame) to the box
 * [pmin, pmax] (the robot-environment QP of Sec. III-C, minimised over the
 * box point in closed form).  f(s) = sum_k gap_k(x_k(s))^2 is convex and
 * quadratic between the points where some x_k crosses pmin_k or pmax_k, so
 * its minimum is at an end of such a piece or at the vertex of the piece's
 * quadratic.  All those candidates are evaluated; the first smallest wins.
 */
static double seg_box(const double A[3], const double D[3], const double pmin[3], const double pmax[3],
                      double *s_out) {
    double br[8];
    int nb = 0;
    br[nb++] = 0.0;
    br[nb++] = 1.0;
    for (int k = 0; k < 3; ++k) {
        if (D[k] == 0.0) continue;
        double sa = (pmin[k] - A[k]) / D[k], sb = (pmax[k] - A[k]) / D[k];
        if (sa > 0.0 && sa < 1.0 && nb < 8) br[nb++] = sa;
        if (sb > 0.0 && sb < 1.0 && nb < 8) br[nb++] = sb;
    }
    for (int i = 1; i < nb; ++i)   /* insertion sort */
        for (int j = i; j > 0 && br[j] < br[j - 1]; --j) { double tmp = br[j]; br[j] = br[j - 1]; br[j - 1] = tmp; }
    double cand[16];
    int nc = 0;
    for (int i = 0; i < nb; ++i) cand[nc++] = br[i];
    for (int i = 0; i + 1 < nb; ++i) {
        double mid = 0.5 * (br[i] + br[i + 1]);
        /* the piece's quadratic: sum over axes outside the box at mid */
        double qa = 0.0, qb = 0.0;
        for (int k = 0; k < 3; ++k) {
            double x = A[k] + mid * D[k];
            double edge = x < pmin[k] ? pmin[k] : (x > pmax[k] ? pmax[k] : x);
            if (x < pmin[k] || x > pmax[k]) {   /* (A + s D - edge)^2 */
                qa += D[k] * D[k];
                qb += 2.0 * D[k] * (A[k] - edge);
            }
        }
        if (qa > 0.0) {
            double v = -qb / (2.0 * qa);
            if (v > br[i] && v < br[i + 1]) cand[nc++] = v;
        }
    }
    double best = INFINITY;
    for (int i = 0; i < nc; ++i) {
        double v = 0.0;
        for (int k = 0; k < 3; ++k) v += axis_gap2(A[k] + cand[i] * D[k], pmin[k], pmax[k]);
        if (v < best) { best = v; *s_out = cand[i]; }
    }
    return best;
}

/* Test entry points of the two distance QPs: out = {squared distance, s, t}
 * (t = 0 for the box; the box is given in its own frame). */
void or_seg_seg(const double *P0, const double *P1, const double *Q0, const double *Q1, double *out) {
    out[0] = seg_seg(P0, P1, Q0, Q1, &out[1], &out[2]);
}
void or_seg_box(const double *A, const double *D, const double *pmin, const double *pmax, double *out) {
    out[0] = seg_box(A, D, pmin, pmax, &out[1]);
    out[2] = 0.0;
}

/* Joint axes z[i], origins o[i] (before link i) and the frame F[i] after
 * link i (3x4), for i = 0..n-1. */
static void link_frames(const or_robot *rb, const double *q, double z[][3], double o[][3], double F[][12]) {
    double M[12], A[12];
    tf_identity(M);
    for (int i = 0; i < rb->n; ++i) {
        z[i][0] = M[2]; z[i][1] = M[6]; z[i][2] = M[10];
        o[i][0] = M[3]; o[i][1] = M[7]; o[i][2] = M[11];
        double th, di;
        joint_dh(rb->jtype, rb->d, rb->theta_off, i, q[i], &th, &di);
        dh_link(th, di, rb->a[i], rb->alpha[i], A);
        tf_mul(M, A, M);
        memcpy(F[i], M, sizeof(M));
    }
}

/* World point of a point fixed in frame F. */
static void frame_point(const double F[12], const double p[3], double w[3]) {
    for (int r = 0; r < 3; ++r) w[r] = F[r * 4 + 0] * p[0] + F[r * 4 + 1] * p[1] + F[r * 4 + 2] * p[2] + F[r * 4 + 3];
}

/* Gradient contribution of moving the point w, carried by link `lnk`:
 * g[k] += sgn * u . (z_k x (w - o_k)) for the revolute joints k <= lnk and
 * sgn * u . z_k for the prismatic ones (the point's velocity per unit of
 * joint k). */
static void point_grad(const int32_t *jtype, const double z[][3], const double o[][3], int lnk, const double w[3],
                       const double u[3], double sgn, double *g) {
    for (int k = 0; k <= lnk; ++k) {
        if (prismatic(jtype, k)) {
            g[k] += sgn * (u[0] * z[k][0] + u[1] * z[k][1] + u[2] * z[k][2]);
            continue;
        }
        double v[3] = {w[0] - o[k][0], w[1] - o[k][1], w[2] - o[k][2]};
        double c0 = z[k][1] * v[2] - z[k][2] * v[1];
        double c1 = z[k][2] * v[0] - z[k][0] * v[2];
        double c2 = z[k][0] * v[1] - z[k][1] * v[0];
        g[k] += sgn * (u[0] * c0 + u[1] * c1 + u[2] * c2);
    }
}

/*
 * Collision distances of configuration q: dmin[0] = min over capsule pairs
 * of links at least three apart in the chain (i, j >= i + 3; nearer links
 * meet at the joints between them, so their checks are left out, as the
 * paper leaves out pairs that cannot collide) of |p_i - p_j| - r_i - r_j,
 * dmin[1] =
 * min over capsules and cuboids of |p - box| - r, with the closest points of
 * the QPs (the distance is the square root of the QP's optimum less the
 * radii); +inf where nothing is checked.  grad (optional, [2][n]): the
 * gradient of each minimum with respect to q through its closest points
 * (the points move with their links; derivative of a minimum over the QP's
 * variables taken at the optimum), zero where the closest points are less
 * than OR_CONTACT_EPS apart (cores touching or crossing: the distance is at
 * its floor minus the radii and the direction between the points is only
 * rounding).
 */
#define OR_CONTACT_EPS 1e-9
static void coll_eval(const or_robot *rb, const double *q, double dmin[2], double *grad) {
    const int n = rb->n;
    const or_coll *c = rb->coll;
    double z[OR_MAXN][3], o[OR_MAXN][3], F[OR_MAXN][12];
    double P0[OR_MAXN][3], P1[OR_MAXN][3];
    link_frames(rb, q, z, o, F);
    for (int i = 0; i < n; ++i) {
        frame_point(F[i], c->caps + 7 * i, P0[i]);
        frame_point(F[i], c->caps + 7 * i + 3, P1[i]);
    }
    dmin[0] = INFINITY;
    dmin[1] = INFINITY;
    if (grad) memset(grad, 0, sizeof(double) * 2 * n);
    int bi = -1, bj = -1;
    double bs = 0, bt = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i + 3; j < n; ++j) {
            double s, t;
            double d2 = seg_seg(P0[i], P1[i], P0[j], P1[j], &s, &t);
            double d = sqrt(d2) - c->caps[7 * i + 6] - c->caps[7 * j + 6];
            if (d < dmin[0]) { dmin[0] = d; bi = i; bj = j; bs = s; bt = t; }
        }
    if (grad && bi >= 0) {
        double pa[3], pb[3], u[3], nrm = 0.0;
        for (int k = 0; k < 3; ++k) {
            pa[k] = P0[bi][k] + bs * (P1[bi][k] - P0[bi][k]);
            pb[k] = P0[bj][k] + bt * (P1[bj][k] - P0[bj][k]);
            u[k] = pa[k] - pb[k];
            nrm += u[k] * u[k];
        }
        nrm = sqrt(nrm);
        if (nrm > OR_CONTACT_EPS) {
            for (int k = 0; k < 3; ++k) u[k] /= nrm;
            point_grad(rb->jtype, z, o, bi, pa, u, 1.0, grad);
            point_grad(rb->jtype, z, o, bj, pb, u, -1.0, grad);
        }
    }
    int li = -1, ob = -1;
    double ls = 0;
    for (int i = 0; i < n; ++i)
        for (int m = 0; m < c->nobs; ++m) {
            const double *B = c->obs + 18 * m, *R = B + 3;
            double A[3], D[3];
            for (int r = 0; r < 3; ++r) {   /* R^T (P0 - origin), R^T (P1 - P0) */
                A[r] = R[0 * 3 + r] * (P0[i][0] - B[0]) + R[1 * 3 + r] * (P0[i][1] - B[1]) +
                       R[2 * 3 + r] * (P0[i][2] - B[2]);
                D[r] = R[0 * 3 + r] * (P1[i][0] - P0[i][0]) + R[1 * 3 + r] * (P1[i][1] - P0[i][1]) +
                       R[2 * 3 + r] * (P1[i][2] - P0[i][2]);
            }
            double s;
            double d2 = seg_box(A, D, B + 12, B + 15, &s);
            double d = sqrt(d2) - c->caps[7 * i + 6];
            if (d < dmin[1]) { dmin[1] = d; li = i; ob = m; ls = s; }
        }
    if (grad && li >= 0) {
        const double *B = c->obs + 18 * ob, *R = B + 3;
        double pa[3], x[3], pb[3], u[3], nrm = 0.0;
        for (int k = 0; k < 3; ++k) pa[k] = P0[li][k] + ls * (P1[li][k] - P0[li][k]);
        for (int r = 0; r < 3; ++r) {
            double v = R[0 * 3 + r] * (pa[0] - B[0]) + R[1 * 3 + r] * (pa[1] - B[1]) + R[2 * 3 + r] * (pa[2] - B[2]);
            x[r] = v < B[12 + r] ? B[12 + r] : (v > B[15 + r] ? B[15 + r] : v);
        }
        for (int k = 0; k < 3; ++k) {
            pb[k] = B[k] + R[k * 3 + 0] * x[0] + R[k * 3 + 1] * x[1] + R[k * 3 + 2] * x[2];
            u[k] = pa[k] - pb[k];
            nrm += u[k] * u[k];
        }
        nrm = sqrt(nrm);
        if (nrm > OR_CONTACT_EPS) {
            for (int k = 0; k < 3; ++k) u[k] /= nrm;
            point_grad(rb->jtype, z, o, li, pa, u, 1.0, grad + n);
        }
    }
}

/* The two collision residuals of a waypoint, max(0, m - dmin), and (J
 * optional, [2][n]) their Jacobians (minus the distance gradients where the
 * residual is positive). */
static void coll_residual(const or_robot *rb, const double *q, double rc[2], double *J) {
    double dmin[2], g[2 * OR_MAXN];
    coll_eval(rb, q, dmin, J ? g : NULL);
    for (int h = 0; h < 2; ++h) {
        double r = rb->coll->margin - dmin[h];
        rc[h] = r > 0.0 ? r : 0.0;
        if (J)
            for (int k = 0; k < rb->n; ++k) J[h * rb->n + k] = r > 0.0 ? -g[h * rb->n + k] : 0.0;
    }
}

/* C(xi) = w_p/2 sum_t |r_t|^2 + w_s/2 sum_{t<T-1} |xi_{t+1} - xi_t|^2
 * + w_c/2 sum_t (r_self,t^2 + r_env,t^2) (xi is [T][n]; the collision terms
 * only with collision geometry). */
static double cost_of(const or_robot *rb, int T, const double *xi, const double *targets,
                      double w_p, double w_s, double w_c) {
    int n = rb->n;
    double pose_sum = 0.0, diff_sum = 0.0, coll_sum = 0.0;
    for (int t = 0; t < T; ++t) {
        double r[6];
        pose_residual(rb, xi + (size_t)t * n, targets + (size_t)t * 12, r, NULL);
        for (int i = 0; i < 6; ++i) pose_sum += r[i] * r[i];
    }
    for (int t = 0; t + 1 < T; ++t)
        for (int j = 0; j < n; ++j) {
            double dq = xi[(size_t)(t + 1) * n + j] - xi[(size_t)t * n + j];
            diff_sum += dq * dq;
        }
    if (rb->coll && w_c != 0.0)
        for (int t = 0; t < T; ++t) {
            double rc[2];
            coll_residual(rb, xi + (size_t)t * n, rc, NULL);
            coll_sum += rc[0] * rc[0] + rc[1] * rc[1];
        }
    return 0.5 * w_p * pose_sum + 0.5 * w_s * diff_sum + 0.5 * w_c * coll_sum;
}

double or_cost(int n, const double *a, const double *d, const double *alpha,
               const double *theta_off, const int32_t *jtype, int T, const double *xi, const double *targets,
               double w_p, double w_s, const double *coll) {
    or_coll cg;
    or_robot rb = {n, a, d, alpha, theta_off, jtype, NULL, NULL, NULL};
    if (coll) { coll_parse(n, coll, &cg); rb.coll = &cg; }
    return cost_of(&rb, T, xi, targets, w_p, w_s, rb.coll ? cg.w_c : 0.0);
}

/* Collision distances of M configurations q[M][n]: out[M][2] (self, env)
 * and optionally their gradients grad[M][2][n] (see coll_eval). */
void or_coll_eval(int n, const double *a, const double *d, const double *alpha,
                  const double *theta_off, const int32_t *jtype, const double *coll, long M, const double *q,
                  double *out, double *grad) {
    or_coll cg;
    coll_parse(n, coll, &cg);
    or_robot rb = {n, a, d, alpha, theta_off, jtype, NULL, NULL, &cg};
    for (long m = 0; m < M; ++m)
        coll_eval(&rb, q + (size_t)m * n, out + 2 * m, grad ? grad + (size_t)2 * n * m : NULL);
}

/* ------------------------------------------------------------------------ */
/* Global discrete search (Sec. III-B)                                       */
/* ------------------------------------------------------------------------ */

/* Penalty of candidate k at waypoint t: joint-limit margin (margin for a
 * revolute joint, margin_m for a prismatic one) plus caller extra. */
static double node_penalty(int n, const int32_t *jtype, const double *q, const double *lo, const double *hi,
                           double margin, double margin_m, double penalty, double extra) {
    int near = 0;
    for (int j = 0; j < n; ++j) {
        double m = prismatic(jtype, j) ? margin_m : margin;
        if (q[j] <= lo[j] + m || q[j] >= hi[j] - m) near = 1;
    }
    return (near ? penalty : 0.0) + extra;
}

static double coll_pen(const or_robot *rb, const double *q) {
    double dmin[2];
    coll_eval(rb, q, dmin, NULL);
    return (dmin[0] < 0.0 || dmin[1] < 0.0) ? rb->coll->penalty : 0.0;
}

/*
 * cand is [K][T][n].  B_0(k) = pen_0(k);
 * B_t(k) = min over k' of max(B_{t-1}(k'), e_t(k',k) + pen_t(k)),
 * e_t(k',k) = max_j |q_t^k[j] - q_{t-1}^{k'}[j]|; the minimising k' is the
 * smallest under the key (value, e_t(k',k), k').  The end node is the
 * smallest under (B_{T-1}(k), k); backtracking gives path[T].
 * Optional outputs: B_all[T][K], bp_all[T][K] (bp_all[0][*] = -1).
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int or_dp(int T, int K, int n, const double *cand, const double *lo, const double *hi,
          double margin, double margin_m, double penalty, const double *extra, int32_t *path,
          double *best_out, double *B_all, int32_t *bp_all, const double *a, const double *d,
          const double *alpha, const double *theta_off, const int32_t *jtype, const double *coll) {
    if (T < 1 || K < 1 || n < 1 || n > OR_MAXN) return -1;
    or_coll cg;
    or_robot rb = {n, a, d, alpha, theta_off, jtype, lo, hi, NULL};
    if (coll) { coll_parse(n, coll, &cg); rb.coll = &cg; }
    /* a configuration in collision (some distance below zero) costs the
     * collision penalty on top (Sec. III-B) */
#define COLL_PEN(q) (rb.coll ? coll_pen(&rb, (q)) : 0.0)
    double *Bp = (double *)malloc(sizeof(double) * K);
    double *Bc = (double *)malloc(sizeof(double) * K);
    int32_t *bp = (int32_t *)malloc(sizeof(int32_t) * (size_t)T * K);
    if (!Bp || !Bc || !bp) { free(Bp); free(Bc); free(bp); return -1; }
#define CAND(k, t) (cand + ((size_t)(k) * T + (t)) * n)
    for (int k = 0; k < K; ++k) {
        Bp[k] = node_penalty(n, jtype, CAND(k, 0), lo, hi, margin, margin_m, penalty, extra ? extra[k] : 0.0) +
                COLL_PEN(CAND(k, 0));
        bp[k] = -1;
    }
    if (B_all) memcpy(B_all, Bp, sizeof(double) * K);
    for (int t = 1; t < T; ++t) {
        for (int k = 0; k < K; ++k) {
            const double *qk = CAND(k, t);
            double pen = node_penalty(n, jtype, qk, lo, hi, margin, margin_m, penalty,
                                      extra ? extra[(size_t)t * K + k] : 0.0) +
                         COLL_PEN(qk);
            double bv = INFINITY, be = INFINITY;
            int bk = -1;
            for (int kp = 0; kp < K; ++kp) {
                const double *qp = CAND(kp, t - 1);
                double e = 0.0;
                for (int j = 0; j < n; ++j) {
                    double dq = fabs(qk[j] - qp[j]);
                    if (dq > e) e = dq;
                }
                double v = e + pen;
                if (Bp[kp] > v) v = Bp[kp];
                if (v < bv || (v == bv && e < be)) { bv = v; be = e; bk = kp; }
            }
            Bc[k] = bv;
            bp[(size_t)t * K + k] = bk;
        }
        if (B_all) memcpy(B_all + (size_t)t * K, Bc, sizeof(double) * K);
        double *tmp = Bp; Bp = Bc; Bc = tmp;
    }
    int kend = 0;
    for (int k = 1; k < K; ++k)
        if (Bp[k] < Bp[kend]) kend = k;
    if (best_out) *best_out = Bp[kend];
    path[T - 1] = kend;
    for (int t = T - 1; t > 0; --t) path[t - 1] = bp[(size_t)t * K + path[t]];
    if (bp_all) memcpy(bp_all, bp, sizeof(int32_t) * (size_t)T * K);
#undef CAND
#undef COLL_PEN
    free(Bp); free(Bc); free(bp);
    return 0;
}

/* Maximum joint-angle change along xi ([T][n]); 0 when T < 2. */
double or_mjac(int T, int n, const double *xi) {
    double m = 0.0;
    for (int t = 0; t + 1 < T; ++t)
        for (int j = 0; j < n; ++j) {
            double dq = fabs(xi[(size_t)(t + 1) * n + j] - xi[(size_t)t * n + j]);
            if (dq > m) m = dq;
        }
    return m;
}

/* ------------------------------------------------------------------------ */
/* Block-tridiagonal symmetric positive definite solve                       */
/* ------------------------------------------------------------------------ */

/* In-place lower Cholesky of an n x n row-major SPD matrix; -1 if not SPD. */
static int chol(int n, double *A) {
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
        if (!(s > 0.0)) return -1;
        double ljj = sqrt(s);
        A[j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double u = A[i * n + j];
            for (int k = 0; k < j; ++k) u -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = u / ljj;
        }
        for (int i = 0; i < j; ++i) A[i * n + j] = 0.0;
    }
    return 0;
}

/* x = L^{-1} b (forward substitution). */
static void lsolve(int n, const double *L, const double *b, double *x) {
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i * n + k] * x[k];
        x[i] = s / L[i * n + i];
    }
}

/* x = L^{-T} b (backward substitution). */
static void ltsolve(int n, const double *L, const double *b, double *x) {
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * x[k];
        x[i] = s / L[i * n + i];
    }
}

/*
 * Solve H x = b for H with diagonal blocks D_t ([T][n][n], symmetric) and
 * off-diagonal blocks -w I, by block Cholesky H = L L^T with L block lower
 * bidiagonal: diagonal blocks L_t with L_t L_t^T = S_t,
 * S_0 = D_0, S_t = D_t - w^2 S_{t-1}^{-1}; sub-diagonal blocks -w L_{t-1}^{-T}.
 * Returns 0, or -1 (a pivot was not positive), -2 (allocation).
 */
int or_btd_solve(int T, int n, const double *D, double w, const double *b, double *x) {
    if (T < 1 || n < 1 || n > OR_MAXN) return -2;
    size_t nn = (size_t)n * n;
    double *L = (double *)malloc(sizeof(double) * nn * T);
    double *z = (double *)malloc(sizeof(double) * (size_t)n * T);
    if (!L || !z) { free(L); free(z); return -2; }
    double col[OR_MAXN], tmp[OR_MAXN], inv[OR_MAXN * OR_MAXN];
    int rc = 0;
    for (int t = 0; t < T; ++t) {
        double *Lt = L + nn * t;
        memcpy(Lt, D + nn * t, sizeof(double) * nn);
        if (t > 0) {
            const double *Lp = L + nn * (t - 1);
            /* inv = S_{t-1}^{-1}, column by column. */
            for (int c = 0; c < n; ++c) {
                for (int i = 0; i < n; ++i) col[i] = (i == c) ? 1.0 : 0.0;
                lsolve(n, Lp, col, tmp);
                ltsolve(n, Lp, tmp, col);
                for (int i = 0; i < n; ++i) inv[i * n + c] = col[i];
            }
            for (size_t e = 0; e < nn; ++e) Lt[e] -= w * w * inv[e];
        }
        if (chol(n, Lt) != 0) { rc = -1; break; }
    }
    if (rc == 0) {
        /* Forward: L_t z_t = b_t + w L_{t-1}^{-T} z_{t-1}. */
        for (int t = 0; t < T; ++t) {
            double rhs[OR_MAXN];
            for (int i = 0; i < n; ++i) rhs[i] = b[(size_t)t * n + i];
            if (t > 0) {
                ltsolve(n, L + nn * (t - 1), z + (size_t)(t - 1) * n, tmp);
                for (int i = 0; i < n; ++i) rhs[i] += w * tmp[i];
            }
            lsolve(n, L + nn * t, rhs, z + (size_t)t * n);
        }
        /* Backward: L_t^T x_t = z_t + w L_t^{-1} x_{t+1}. */
        for (int t = T - 1; t >= 0; --t) {
            double rhs[OR_MAXN];
            for (int i = 0; i < n; ++i) rhs[i] = z[(size_t)t * n + i];
            if (t < T - 1) {
                lsolve(n, L + nn * t, x + (size_t)(t + 1) * n, tmp);
                for (int i = 0; i < n; ++i) rhs[i] += w * tmp[i];
            }
            ltsolve(n, L + nn * t, rhs, x + (size_t)t * n);
        }
    }
    free(L); free(z);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Levenberg-Marquardt (Sec. III-C)                                          */
/* ------------------------------------------------------------------------ */

/*
 * Linearise at xi ([T][n]): per waypoint A_t = w_p J_t^T J_t ([T][n][n]) and
 * gradient g_t = w_p J_t^T r_t + w_s (c_t xi_t - xi_{t-1} - xi_{t+1}), with
 * c_t the number of neighbours of t (the differencing residual's Jacobian is
 * +I on q_{t+1} and -I on q_t); with collision geometry also
 * w_c sum_h (J_h^T J_h, J_h^T r_h) of the two collision residuals.
 */
static void linearise(const or_robot *rb, int T, const double *xi, const double *targets,
                      double w_p, double w_s, double w_c, double *A, double *g) {
    int n = rb->n;
    double J6[6 * OR_MAXN], r[6];
    for (int t = 0; t < T; ++t) {
        const double *q = xi + (size_t)t * n;
        pose_residual(rb, q, targets + (size_t)t * 12, r, J6);
        double *At = A + (size_t)t * n * n;
        double *gt = g + (size_t)t * n;
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int k = 0; k < 6; ++k) s += J6[k * n + i] * J6[k * n + j];
                At[i * n + j] = w_p * s;
            }
            double s = 0.0;
            for (int k = 0; k < 6; ++k) s += J6[k * n + i] * r[k];
            gt[i] = w_p * s;
        }
        for (int j = 0; j < n; ++j) {
            double sm = 0.0;
            if (t > 0) sm += q[j] - xi[(size_t)(t - 1) * n + j];
            if (t + 1 < T) sm += q[j] - xi[(size_t)(t + 1) * n + j];
            gt[j] += w_s * sm;
        }
        if (rb->coll && w_c != 0.0) {
            double rc[2], Jc[2 * OR_MAXN];
            coll_residual(rb, q, rc, Jc);
            for (int h = 0; h < 2; ++h)
                for (int i = 0; i < n; ++i) {
                    for (int j = 0; j < n; ++j) At[i * n + j] += w_c * Jc[h * n + i] * Jc[h * n + j];
                    gt[i] += w_c * Jc[h * n + i] * rc[h];
                }
        }
    }
}

/* Solve (A + w_s L (x) I + lambda I) delta = -g; returns or_btd_solve's code. */
static int lm_solve(int T, int n, const double *A, const double *g, double w_s,
                    double lambda, double *delta, double *Dbuf, double *rhs) {
    size_t nn = (size_t)n * n;
    for (int t = 0; t < T; ++t) {
        int ct = (t > 0) + (t + 1 < T);
        memcpy(Dbuf + nn * t, A + nn * t, sizeof(double) * nn);
        for (int i = 0; i < n; ++i) Dbuf[nn * t + (size_t)i * n + i] += w_s * ct + lambda;
        for (int i = 0; i < n; ++i) rhs[(size_t)t * n + i] = -g[(size_t)t * n + i];
    }
    return or_btd_solve(T, n, Dbuf, w_s, rhs, delta);
}

/*
 * One damped Gauss-Newton step at xi without accepting it: writes the step
 * delta ([T][n]) and optionally the gradient g ([T][n]).  Returns 0 or the
 * solve's error code.
 */
int or_lm_step(int n, const double *a, const double *d, const double *alpha,
               const double *theta_off, const int32_t *jtype, int T, const double *xi, const double *targets,
               double w_p, double w_s, double lambda, double *delta, double *g_out,
               const double *coll, double w_c) {
    or_coll cg;
    or_robot rb = {n, a, d, alpha, theta_off, jtype, NULL, NULL, NULL};
    if (coll) { coll_parse(n, coll, &cg); rb.coll = &cg; }
    size_t nn = (size_t)n * n;
    double *A = (double *)malloc(sizeof(double) * nn * T);
    double *g = (double *)malloc(sizeof(double) * (size_t)n * T);
    double *Db = (double *)malloc(sizeof(double) * nn * T);
    double *rhs = (double *)malloc(sizeof(double) * (size_t)n * T);
    int rc = -2;
    if (A && g && Db && rhs) {
        linearise(&rb, T, xi, targets, w_p, w_s, w_c, A, g);
        rc = lm_solve(T, n, A, g, w_s, lambda, delta, Db, rhs);
        if (g_out) memcpy(g_out, g, sizeof(double) * (size_t)n * T);
    }
    free(A); free(g); free(Db); free(rhs);
    return rc;
}

typedef struct {
    double w_pose, w_smooth, lambda0, lambda_min, lambda_max;
} or_lm_opts;

/*
 * Levenberg-Marquardt from xi ([T][n], overwritten with the result).
 * Start: xi <- clamp(xi), lambda <- lambda0, nu <- 2.  Each of `iters`
 * iterations: linearise at xi (reused after a rejected trial), solve for
 * delta, trial xi' = clamp(xi + delta), C' = C(xi'); predicted reduction
 * pred = delta^T (lambda delta - g) / 2 (unclamped delta), gain rho =
 * (C - C')/pred.  Accept iff C' < C: xi <- xi', lambda *= max(1/3,
 * 1 - (2 rho - 1)^3), nu <- 2; else lambda *= nu, nu *= 2.  lambda is kept in
 * [lambda_min, lambda_max].  No early exit.
 * Histories (optional, length iters): cost after the iteration, lambda used
 * by the iteration, accept flag.  Returns 0, -1 (non-positive pivot: xi left
 * at the last accepted iterate), -2 (allocation).
 */
int or_lm(int n, const double *a, const double *d, const double *alpha,
          const double *theta_off, const int32_t *jtype, const double *lo, const double *hi, int T,
          double *xi, const double *targets, const double *opts5, int iters,
          double *cost_hist, double *lambda_hist, int32_t *acc_hist, double *cost0_out,
          const double *coll) {
    or_coll cg;
    or_robot rb = {n, a, d, alpha, theta_off, jtype, lo, hi, NULL};
    if (coll) { coll_parse(n, coll, &cg); rb.coll = &cg; }
    const double w_c = rb.coll ? cg.w_c : 0.0;
    or_lm_opts o = {opts5[0], opts5[1], opts5[2], opts5[3], opts5[4]};
    size_t nn = (size_t)n * n, nT = (size_t)n * T;
    double *A = (double *)malloc(sizeof(double) * nn * T);
    double *g = (double *)malloc(sizeof(double) * nT);
    double *Db = (double *)malloc(sizeof(double) * nn * T);
    double *rhs = (double *)malloc(sizeof(double) * nT);
    double *delta = (double *)malloc(sizeof(double) * nT);
    double *trial = (double *)malloc(sizeof(double) * nT);
    int rc = 0;
    if (!A || !g || !Db || !rhs || !delta || !trial) { rc = -2; goto done; }
    for (int t = 0; t < T; ++t)
        for (int j = 0; j < n; ++j) {
            double v = xi[(size_t)t * n + j];
            if (v < lo[j]) v = lo[j];
            if (v > hi[j]) v = hi[j];
            xi[(size_t)t * n + j] = v;
        }
    double lambda = o.lambda0, nu = 2.0;
    double C = cost_of(&rb, T, xi, targets, o.w_pose, o.w_smooth, w_c);
    if (cost0_out) *cost0_out = C;
    int need_lin = 1;
    for (int it = 0; it < iters; ++it) {
        if (need_lin) linearise(&rb, T, xi, targets, o.w_pose, o.w_smooth, w_c, A, g);
        if (lambda_hist) lambda_hist[it] = lambda;
        if (lm_solve(T, n, A, g, o.w_smooth, lambda, delta, Db, rhs) != 0) { rc = -1; break; }
        for (int t = 0; t < T; ++t)
            for (int j = 0; j < n; ++j) {
                size_t e = (size_t)t * n + j;
                double v = xi[e] + delta[e];
                if (v < lo[j]) v = lo[j];
                if (v > hi[j]) v = hi[j];
                trial[e] = v;
            }
        double Cn = cost_of(&rb, T, trial, targets, o.w_pose, o.w_smooth, w_c);
        double pred = 0.0;
        for (size_t e = 0; e < nT; ++e) pred += delta[e] * (lambda * delta[e] - g[e]);
        pred *= 0.5;
        int acc = Cn < C;
        if (acc) {
            double rho = (C - Cn) / pred;
            double u = 2.0 * rho - 1.0;
            double f = 1.0 - u * u * u;
            if (f < 1.0 / 3.0) f = 1.0 / 3.0;
            lambda *= f;
            nu = 2.0;
            memcpy(xi, trial, sizeof(double) * nT);
            C = Cn;
            need_lin = 1;
        } else {
            lambda *= nu;
            nu *= 2.0;
            need_lin = 0;
        }
        if (lambda < o.lambda_min) lambda = o.lambda_min;
        if (lambda > o.lambda_max) lambda = o.lambda_max;
        if (cost_hist) cost_hist[it] = C;
        if (acc_hist) acc_hist[it] = acc;
    }
done:
    free(A); free(g); free(Db); free(rhs); free(delta); free(trial);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Whole plan and evaluator                                                  */
/* ------------------------------------------------------------------------ */

/*
 * Search (or_dp) over cand [K][T][n], seed xi_out[T][n] with the chosen
 * candidates, then `iters` LM iterations.  Returns 0 or a negative code.
 */
int or_plan(int n, const double *a, const double *d, const double *alpha,
            const double *theta_off, const int32_t *jtype, const double *lo, const double *hi, int T, int K,
            const double *cand, const double *targets, const double *extra, double margin,
            double margin_m, double penalty, const double *opts5, int iters, int32_t *path, double *best,
            double *xi_out, double *cost_out, const double *coll) {
    int rc = or_dp(T, K, n, cand, lo, hi, margin, margin_m, penalty, extra, path, best, NULL, NULL, a, d, alpha,
                   theta_off, jtype, coll);
    if (rc) return rc;
    for (int t = 0; t < T; ++t)
        memcpy(xi_out + (size_t)t * n, cand + ((size_t)path[t] * T + t) * n, sizeof(double) * n);
    double *hist = (double *)malloc(sizeof(double) * (iters > 0 ? iters : 1));
    if (!hist) return -2;
    double c0 = 0.0;
    rc = or_lm(n, a, d, alpha, theta_off, jtype, lo, hi, T, xi_out, targets, opts5, iters, hist, NULL,
               NULL, &c0, coll);
    if (cost_out) *cost_out = iters > 0 ? hist[iters - 1] : c0;
    free(hist);
    return rc;
}

/*
 * Pose agreement of two trajectories under this oracle's FK:
 * out[0] = max_t |p_a - p_b| (m), out[1] = max_t angle(R_a R_b^T) (rad).
 * With xi_b == NULL the second pose comes from targets[T][12] instead.
 */
void or_pose_compare(int n, const double *a, const double *d, const double *alpha,
                     const double *theta_off, const int32_t *jtype, int T, const double *xi_a, const double *xi_b,
                     const double *targets, double *out) {
    double pa[12], pb[12], mp = 0.0, mr = 0.0;
    for (int t = 0; t < T; ++t) {
        or_fk(n, a, d, alpha, theta_off, jtype, xi_a + (size_t)t * n, pa, NULL);
        if (xi_b) or_fk(n, a, d, alpha, theta_off, jtype, xi_b + (size_t)t * n, pb, NULL);
        else memcpy(pb, targets + (size_t)t * 12, sizeof(pb));
        double dx = pa[0] - pb[0], dy = pa[1] - pb[1], dz = pa[2] - pb[2];
        double ep = sqrt(dx * dx + dy * dy + dz * dz);
        double er = rot_angle(pa + 3, pb + 3);
        if (ep > mp) mp = ep;
        if (er > mr) mr = er;
    }
    out[0] = mp; out[1] = mr;
}

/*
 * Non-stationary objective with anytime validity (Sec. III-C: the optimiser
 * alternates between the pose residual alone and the differencing residual,
 * and keeps the latest valid solution; validity thresholds of Sec. II).
 * Before every iteration, and once after the last, the current trajectory is
 * checked: position error <= tol[0] (m) and geodesic rotation error <=
 * tol[1] (rad) at every waypoint, and no revolute joint changing by more
 * than tol[2] (rad) and no prismatic joint by more than tol[3] (m) between
 * consecutive waypoints (joint limits hold by clamping), and
 * with collision geometry no capsule distance below zero (Sec. II collision
 * avoidance).  A trajectory that passes is kept in xi_valid.  A trajectory
 * whose pose errors are within the thresholds then takes one LM step on the
 * differencing residual, with the collision residuals (w_pose = 0); any
 * other takes one LM step on the pose residual alone (w_smooth = w_c = 0).  The pose objective's damping
 * (lambda, nu) follows the same Nielsen rule as or_lm.  The differencing
 * step keeps the fixed damping lambda0: its objective is quadratic, so its
 * gain ratio is 1 up to clamping and the rule would only shrink lambda
 * towards its floor, after which one step would collapse the whole path
 * onto a constant configuration.  A step is accepted iff it lowers its own
 * objective.
 * info[0] = checks passed, info[1] = iteration of the first pass (-1: none;
 * iters: only after the last iteration), info[2] = trajectory length of the
 * latest valid trajectory (sum over steps and joints of |change|), info[3] =
 * pose steps taken, info[4] = differencing steps taken.
 */
int or_lm_schedule(int n, const double *a, const double *d, const double *alpha,
                   const double *theta_off, const int32_t *jtype, const double *lo, const double *hi, int T,
                   double *xi, const double *targets, const double *opts5, const double *tol, int iters,
                   double *xi_valid, double *info, const double *coll) {
    or_coll cg;
    or_robot rb = {n, a, d, alpha, theta_off, jtype, lo, hi, NULL};
    if (coll) { coll_parse(n, coll, &cg); rb.coll = &cg; }
    or_lm_opts o = {opts5[0], opts5[1], opts5[2], opts5[3], opts5[4]};
    size_t nn = (size_t)n * n, nT = (size_t)n * T;
    double *A = (double *)malloc(sizeof(double) * nn * T);
    double *g = (double *)malloc(sizeof(double) * nT);
    double *Db = (double *)malloc(sizeof(double) * nn * T);
    double *rhs = (double *)malloc(sizeof(double) * nT);
    double *delta = (double *)malloc(sizeof(double) * nT);
    double *trial = (double *)malloc(sizeof(double) * nT);
    int rc = 0;
    info[0] = 0; info[1] = -1; info[2] = 0; info[3] = 0; info[4] = 0;
    if (!A || !g || !Db || !rhs || !delta || !trial) { rc = -2; goto done; }
    for (size_t e = 0; e < nT; ++e) {
        int j = (int)(e % (size_t)n);
        if (xi[e] < lo[j]) xi[e] = lo[j];
        if (xi[e] > hi[j]) xi[e] = hi[j];
    }
    double lam = o.lambda0, nu = 2.0;   /* pose objective */
    for (int it = 0; it <= iters; ++it) {
        double err[2];
        or_pose_compare(n, a, d, alpha, theta_off, jtype, T, xi, NULL, targets, err);
        int pose_ok = err[0] <= tol[0] && err[1] <= tol[1];
        int steps_ok = 1;
        for (int t = 0; t + 1 < T; ++t)
            for (int j = 0; j < n; ++j)
                if (fabs(xi[(size_t)(t + 1) * n + j] - xi[(size_t)t * n + j]) > tol[prismatic(jtype, j) ? 3 : 2])
                    steps_ok = 0;
        int coll_ok = 1;
        if (rb.coll)
            for (int t = 0; t < T; ++t) {
                double dmin[2];
                coll_eval(&rb, xi + (size_t)t * n, dmin, NULL);
                if (dmin[0] < 0.0 || dmin[1] < 0.0) coll_ok = 0;
            }
        if (pose_ok && steps_ok && coll_ok) {
            memcpy(xi_valid, xi, sizeof(double) * nT);
            info[0] += 1;
            if (info[1] < 0) info[1] = it;
            double len = 0.0;
            for (int t = 0; t + 1 < T; ++t)
                for (int j = 0; j < n; ++j) len += fabs(xi[(size_t)(t + 1) * n + j] - xi[(size_t)t * n + j]);
            info[2] = len;
        }
        if (it == iters) break;
        const int m = pose_ok ? 1 : 0;   /* 0: pose step, 1: differencing step */
        const double wp = m ? 0.0 : o.w_pose, ws = m ? o.w_smooth : 0.0;
        const double wc = (m && rb.coll) ? cg.w_c : 0.0;
        const double l = m ? o.lambda0 : lam;
        info[3 + m] += 1;
        const double C = cost_of(&rb, T, xi, targets, wp, ws, wc);
        linearise(&rb, T, xi, targets, wp, ws, wc, A, g);
        if (lm_solve(T, n, A, g, ws, l, delta, Db, rhs) != 0) { rc = -1; break; }
        for (size_t e = 0; e < nT; ++e) {
            int j = (int)(e % (size_t)n);
            double v = xi[e] + delta[e];
            if (v < lo[j]) v = lo[j];
            if (v > hi[j]) v = hi[j];
            trial[e] = v;
        }
        const double Cn = cost_of(&rb, T, trial, targets, wp, ws, wc);
        const int acc = Cn < C;
        if (acc) memcpy(xi, trial, sizeof(double) * nT);
        if (m == 0) {
            double pred = 0.0;
            for (size_t e = 0; e < nT; ++e) pred += delta[e] * (lam * delta[e] - g[e]);
            pred *= 0.5;
            if (acc) {
                double rho = (C - Cn) / pred;
                double u = 2.0 * rho - 1.0;
                double f = 1.0 - u * u * u;
                if (f < 1.0 / 3.0) f = 1.0 / 3.0;
                lam *= f;
                nu = 2.0;
            } else {
                lam *= nu;
                nu *= 2.0;
            }
            if (lam < o.lambda_min) lam = o.lambda_min;
            if (lam > o.lambda_max) lam = o.lambda_max;
        }
    }
done:
    free(A); free(g); free(Db); free(rhs); free(delta); free(trial);
    return rc;
}

/* FK of M configurations q[M][n] -> pose[M][12] (and J[M][6][n] if non-NULL). */
void or_fk_many(int n, const double *a, const double *d, const double *alpha,
                const double *theta_off, const int32_t *jtype, long M, const double *q, double *pose, double *J) {
    for (long m = 0; m < M; ++m)
        or_fk(n, a, d, alpha, theta_off, jtype, q + (size_t)m * n, pose + (size_t)m * 12,
              J ? J + (size_t)m * 6 * n : NULL);
}
