// cpf_device.h -- per-lane math of the CppFlow refinement path (arXiv
// 2309.09102) on gfx950 for a chain of CPF_NJ joints.  Every kernel source
// is compiled once per chain length (CPF_NJ = 7 or 8); each compilation puts
// its kernels, launchers and helpers in its own namespace, cpf::j7 or
// cpf::j8, beside the shared plan descriptor of cpf_plan.h.
#pragma once

#include "cpf_plan.h"

#if !defined(CPF_NJ)
#error "CPF_NJ (the number of joints the kernels are built for) must be defined"
#elif CPF_NJ == 7
#define CPF_JNS j7
#elif CPF_NJ == 8
#define CPF_JNS j8
#else
#error "kernels are built for chains of 7 or 8 joints"
#endif

namespace cpf {
namespace CPF_JNS {

constexpr int NJ = CPF_NJ;                 // joints
constexpr int NTRI = NJ * (NJ + 1) / 2;    // packed lower triangle of an NJ x NJ block
constexpr int NBLK = NJ * NJ;              // full NJ x NJ block
static_assert(NJ <= NJMAX, "descriptor rows");

template <typename S>
struct RobotT {
    S a[NJ], d[NJ], ca[NJ], sa[NJ], off[NJ];
    uint32_t prism;   // bit i set: joint i is prismatic
};

// The plan's robot in precision S.  PRISM false: a chain known to be all
// revolute (the plans with collision capsules, which cannot hold a
// prismatic joint); the joint-type mask is then neither loaded nor used, and
// the chain functions below compile their revolute-only form.
template <typename S> struct RobotRows;
template <> struct RobotRows<double> {
    static __device__ __forceinline__ void get(const DevPlan &P, RobotT<double> &r) {
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            r.a[i] = P.a[i]; r.d[i] = P.d[i]; r.ca[i] = P.ca[i]; r.sa[i] = P.sa[i]; r.off[i] = P.off[i];
        }
    }
};
template <> struct RobotRows<float> {
    static __device__ __forceinline__ void get(const DevPlan &P, RobotT<float> &r) {
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            r.a[i] = P.af[i]; r.d[i] = P.df[i]; r.ca[i] = P.caf[i]; r.sa[i] = P.saf[i]; r.off[i] = P.offf[i];
        }
    }
};

template <typename S, bool PRISM = true>
__device__ __forceinline__ RobotT<S> load_robot(const DevPlan &P) {
    RobotT<S> r;
    RobotRows<S>::get(P, r);
    if constexpr (PRISM) r.prism = (uint32_t)P.prism;
    return r;
}

__device__ __forceinline__ void dev_sincos(float x, float *s, float *c) { sincosf(x, s, c); }
__device__ __forceinline__ void dev_sincos(double x, double *s, double *c) { sincos(x, s, c); }

// Kinematic chain of the standard DH convention, kept in registers.
// Frame columns X, Y, Z and origin p start at the identity; link i maps
//   X' = c X + s Y,  W = c Y - s X,  Y' = ca W + sa Z,  Z' = ca Z - sa W,
//   p' = p + a X' + d Z,
// which is the product with Rz(theta) Tz(d) Tx(a) Rx(alpha) written per
// column; theta = q + offset and d fixed for a revolute joint, theta = offset
// and d + q for a prismatic one.  With FRAMES the axis Z and origin p of
// joint i (before link i) are kept for the geometric Jacobian.
template <typename S>
__device__ __forceinline__ void chain_start(S X[3], S Y[3], S Z[3], S p[3]) {
    X[0] = 1; X[1] = 0; X[2] = 0;
    Y[0] = 0; Y[1] = 1; Y[2] = 0;
    Z[0] = 0; Z[1] = 0; Z[2] = 1;
    p[0] = 0; p[1] = 0; p[2] = 0;
}

// Link i of the chain: the frame before it becomes the frame after it.
// PRISM false: every joint revolute (the mask is not read).
template <typename S, bool PRISM = true>
__device__ __forceinline__ void dh_step(const RobotT<S> &rb, int i, S qi, S X[3], S Y[3], S Z[3], S p[3]) {
    if constexpr (!PRISM) {
        S s, c;
        dev_sincos(qi + rb.off[i], &s, &c);
        S nx[3], w[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            nx[r] = c * X[r] + s * Y[r];
            w[r] = c * Y[r] - s * X[r];
        }
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            p[r] = p[r] + rb.a[i] * nx[r] + rb.d[i] * Z[r];
            Y[r] = rb.ca[i] * w[r] + rb.sa[i] * Z[r];
            Z[r] = rb.ca[i] * Z[r] - rb.sa[i] * w[r];
            X[r] = nx[r];
        }
        return;
    }
    const bool pr = is_prismatic(rb.prism, i);
    S s, c;
    dev_sincos(pr ? rb.off[i] : qi + rb.off[i], &s, &c);
    const S di = pr ? rb.d[i] + qi : rb.d[i];
    S nx[3], w[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        nx[r] = c * X[r] + s * Y[r];
        w[r] = c * Y[r] - s * X[r];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        p[r] = p[r] + rb.a[i] * nx[r] + di * Z[r];
        Y[r] = rb.ca[i] * w[r] + rb.sa[i] * Z[r];
        Z[r] = rb.ca[i] * Z[r] - rb.sa[i] * w[r];
        X[r] = nx[r];
    }
}

// Column i of the geometric Jacobian at end-effector position p: a revolute
// joint gives [z x (p - o); z], a prismatic one [z; 0].
template <typename S>
__device__ __forceinline__ void jac_column(uint32_t prism, int i, const S z[3], const S o[3], const S p[3],
                                           S col[6]) {
    const bool pr = is_prismatic(prism, i);
    const S dx = p[0] - o[0], dy = p[1] - o[1], dz = p[2] - o[2];
    col[0] = pr ? z[0] : z[1] * dz - z[2] * dy;
    col[1] = pr ? z[1] : z[2] * dx - z[0] * dz;
    col[2] = pr ? z[2] : z[0] * dy - z[1] * dx;
    col[3] = pr ? S(0) : z[0];
    col[4] = pr ? S(0) : z[1];
    col[5] = pr ? S(0) : z[2];
}

template <typename S, bool FRAMES, bool PRISM = true>
__device__ __forceinline__ void chain(const RobotT<S> &rb, const S *q, S X[3], S Y[3], S Z[3],
                                      S p[3], S Zs[NJ][3], S Os[NJ][3]) {
    chain_start(X, Y, Z, p);
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        if (FRAMES) {
#pragma unroll
            for (int r = 0; r < 3; ++r) { Zs[i][r] = Z[r]; Os[i][r] = p[r]; }
        }
        dh_step<S, PRISM>(rb, i, q[i], X, Y, Z, p);
    }
}

template <typename S> __device__ __forceinline__ S dev_atan2(S y, S x);
template <> __device__ __forceinline__ float dev_atan2<float>(float y, float x) { return atan2f(y, x); }
template <> __device__ __forceinline__ double dev_atan2<double>(double y, double x) { return atan2(y, x); }

// Rotation vector of E (row-major 3x3): angle atan2(|v|, (tr E - 1)/2) with
// v = vee(E - E^T)/2; series for the small-angle factor, and the axis of the
// symmetric part near pi.
template <typename S>
__device__ __forceinline__ void log_rot(const S E[9], S phi[3]) {
    const S v0 = S(0.5) * (E[7] - E[5]);
    const S v1 = S(0.5) * (E[2] - E[6]);
    const S v2 = S(0.5) * (E[3] - E[1]);
    const S sn = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
    const S cs = S(0.5) * (E[0] + E[4] + E[8] - S(1));
    const S th = dev_atan2<S>(sn, cs);
    if (th < S(1e-4)) {
        const S k = S(1) + th * th / S(6);
        phi[0] = k * v0; phi[1] = k * v1; phi[2] = k * v2;
        return;
    }
    if (th > S(3.14159265358979323846) - S(1e-6)) {
        S B[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                B[r][c] = S(0.5) * (E[r * 3 + c] + E[c * 3 + r]) - (r == c ? cs : S(0));
        int i = 0;
        if (B[1][1] > B[i][i]) i = 1;
        if (B[2][2] > B[i][i]) i = 2;
        const S omc = S(1) - cs;
        const S ui = sqrt(B[i][i] / omc);
        S u[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) u[j] = B[i][j] / (omc * ui);
        u[i] = ui;
        if (u[0] * v0 + u[1] * v1 + u[2] * v2 < S(0)) { u[0] = -u[0]; u[1] = -u[1]; u[2] = -u[2]; }
        phi[0] = th * u[0]; phi[1] = th * u[1]; phi[2] = th * u[2];
        return;
    }
    const S k = th / sn;
    phi[0] = k * v0; phi[1] = k * v1; phi[2] = k * v2;
}

// Pose residual r = [p - p*; Log(R R*^T)] of one waypoint; R has columns
// X, Y, Z.  tgt is x y z then R* row-major (already in S).
template <typename S>
__device__ __forceinline__ void pose_residual(const S X[3], const S Y[3], const S Z[3], const S p[3],
                                              const S tgt[12], S r[6]) {
    r[0] = p[0] - tgt[0];
    r[1] = p[1] - tgt[1];
    r[2] = p[2] - tgt[2];
    S E[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)   // (R R*^T)_ij = sum_k R_ik R*_jk, R_ik = column k row i
            E[i * 3 + j] = X[i] * tgt[3 + j * 3 + 0] + Y[i] * tgt[3 + j * 3 + 1] + Z[i] * tgt[3 + j * 3 + 2];
    log_rot<S>(E, r + 3);
}

}  // namespace CPF_JNS
}  // namespace cpf
