// coll_device.h -- capsule distances on the device (Sec. II collision
// avoidance; Sec. III-C robot-robot and robot-environment distances).
//
// Every link carries a capsule: a segment between two points fixed in the
// frame after the link, and a radius.  Obstacles are cuboids given by a frame
// (origin, rotation row-major with the cuboid's axes as columns) and the
// corners p_min, p_max in that frame.  A distance is the square root of the
// QP's optimum less the radii:
//   robot-robot:        min over s, t in [0, 1] of |p(s) - q(t)|
//   robot-environment:  min over s in [0, 1], x in [p_min, p_max] of |x - p(s)|
//                       (cuboid frame).
// Self pairs are the links at least three apart in the chain (nearer links
// meet at the joints between them).  Gradients follow the closest points,
// each carried by its link: d dist / d q_k = u . (z_k x (w - o_k)) for the
// joints k up to that link, u the unit vector between the closest points,
// and zero where the points are closer than contact_eps (cores touching or
// crossing: the distance sits at its floor minus the radii, and the
// direction between the points is only rounding).
#pragma once

#include "cpf_device.h"

namespace cpf {
namespace CPF_JNS {

template <typename S> __device__ __forceinline__ S contact_eps();
template <> __device__ __forceinline__ double contact_eps<double>() { return 1e-9; }
template <> __device__ __forceinline__ float contact_eps<float>() { return 1e-6f; }

// A pair is skipped when a lower bound on its distance (bounding spheres of
// the segments and of the cuboid) exceeds the smallest distance found so far
// by more than this slack, which covers the bound's rounding: a skipped pair
// is strictly farther than the minimum, so the minimum and its pair are those
// of the full enumeration.
template <typename S> __device__ __forceinline__ S cull_slack();
template <> __device__ __forceinline__ double cull_slack<double>() { return 1e-9; }
template <> __device__ __forceinline__ float cull_slack<float>() { return 1e-5f; }

template <typename S>
__device__ __forceinline__ S clamp01(S v) {
    return v < S(0) ? S(0) : (v > S(1) ? S(1) : v);
}

// Chain with the capsules: world endpoints P0[i], P1[i] of capsule i and the
// axis Zs[i] and origin Os[i] of joint i (before link i).
template <typename S, typename C, bool PRISM = true>
__device__ __forceinline__ void capsule_chain(const RobotT<S> &rb, const C cap[NJ][7], const S *q,
                                              S Zs[NJ][3], S Os[NJ][3], S P0[NJ][3], S P1[NJ][3]) {
    S X[3], Y[3], Z[3], p[3];
    chain_start(X, Y, Z, p);
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
#pragma unroll
        for (int r = 0; r < 3; ++r) { Zs[i][r] = Z[r]; Os[i][r] = p[r]; }
        dh_step<S, PRISM>(rb, i, q[i], X, Y, Z, p);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            P0[i][r] = p[r] + X[r] * (S)cap[i][0] + Y[r] * (S)cap[i][1] + Z[r] * (S)cap[i][2];
            P1[i][r] = p[r] + X[r] * (S)cap[i][3] + Y[r] * (S)cap[i][4] + Z[r] * (S)cap[i][5];
        }
    }
}

// Closest points of two segments, the convex QP on the unit square solved by
// clamping (the line parameter s of the first segment from the unconstrained
// optimum, t from s, and s again from a clamped t), as in Ericson,
// Real-Time Collision Detection, Sec. 5.1.9.  Returns the squared distance.
template <typename S>
__device__ __forceinline__ S seg_seg_d2(const S P0[3], const S P1[3], const S Q0[3], const S Q1[3], S &s, S &t) {
    S d1[3], d2[3], r[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        d1[k] = P1[k] - P0[k];
        d2[k] = Q1[k] - Q0[k];
        r[k] = P0[k] - Q0[k];
    }
    const S a = d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2];
    const S e = d2[0] * d2[0] + d2[1] * d2[1] + d2[2] * d2[2];
    const S f = d2[0] * r[0] + d2[1] * r[1] + d2[2] * r[2];
    const S c = d1[0] * r[0] + d1[1] * r[1] + d1[2] * r[2];
    const S b = d1[0] * d2[0] + d1[1] * d2[1] + d1[2] * d2[2];
    if (a <= S(0) && e <= S(0)) {
        s = S(0);
        t = S(0);
    } else if (a <= S(0)) {
        s = S(0);
        t = clamp01(f / e);
    } else if (e <= S(0)) {
        t = S(0);
        s = clamp01(-c / a);
    } else {
        const S den = a * e - b * b;
        s = den > S(0) ? clamp01((b * f - c * e) / den) : S(0);
        t = (b * s + f) / e;
        if (t < S(0)) {
            t = S(0);
            s = clamp01(-c / a);
        } else if (t > S(1)) {
            t = S(1);
            s = clamp01((b - c) / a);
        }
    }
    S d2s = S(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const S w = r[k] + s * d1[k] - t * d2[k];
        d2s += w * w;
    }
    return d2s;
}

template <typename S>
__device__ __forceinline__ S box_gap2(const S x[3], const S lo[3], const S hi[3]) {
    S v = S(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const S g = x[k] < lo[k] ? lo[k] - x[k] : (x[k] > hi[k] ? x[k] - hi[k] : S(0));
        v += g * g;
    }
    return v;
}

// Squared distance of x(s) = A + s D (cuboid frame) to [lo, hi] over s in
// [0, 1].  The function is convex and quadratic between the parameters where
// a coordinate crosses a face plane; the minimum is at one of those
// parameters, the ends, or the vertex of one piece's quadratic.
template <typename S>
__device__ __forceinline__ S seg_box_d2(const S A[3], const S D[3], const S lo[3], const S hi[3], S &s_best) {
    S br[8];
    br[0] = S(0);
    int nb = 1;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (D[k] != S(0)) {
            const S u = (lo[k] - A[k]) / D[k], v = (hi[k] - A[k]) / D[k];
            if (u > S(0) && u < S(1)) br[nb++] = u;
            if (v > S(0) && v < S(1)) br[nb++] = v;
        }
    }
    br[nb++] = S(1);
    // sort the inner parameters (at most 6)
    for (int i = 2; i < nb - 1; ++i)
        for (int j = i; j > 1 && br[j] < br[j - 1]; --j) {
            const S tmp = br[j];
            br[j] = br[j - 1];
            br[j - 1] = tmp;
        }
    S best = S(0);
    s_best = S(0);
    {
        S x[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) x[k] = A[k];
        best = box_gap2(x, lo, hi);
    }
    for (int i = 1; i < nb; ++i) {
        // end of the piece [br[i-1], br[i]] and the vertex of its quadratic
        const S mid = S(0.5) * (br[i - 1] + br[i]);
        S qa = S(0), qb = S(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const S x = A[k] + mid * D[k];
            const S face = x < lo[k] ? lo[k] : hi[k];
            if (x < lo[k] || x > hi[k]) {
                qa += D[k] * D[k];
                qb += D[k] * (A[k] - face);
            }
        }
        S cand[2] = {br[i], br[i]};
        if (qa > S(0)) {
            const S v = -qb / qa;
            if (v > br[i - 1] && v < br[i]) cand[1] = v;
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            S x[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) x[k] = A[k] + cand[c] * D[k];
            const S v = box_gap2(x, lo, hi);
            if (v < best) {
                best = v;
                s_best = cand[c];
            }
        }
    }
    return best;
}

// Gradient of a distance through a closest point w carried by link lnk: the
// point's velocity for joint k is z_k x (w - o_k) (revolute) or z_k
// (prismatic).  PRISM false: every joint revolute (prism is not read).
template <typename S, bool PRISM = true>
__device__ __forceinline__ void point_gradient(uint32_t prism, const S Zs[NJ][3], const S Os[NJ][3], int lnk,
                                               const S w[3], const S u[3], S sgn, S g[NJ]) {
    if constexpr (!PRISM) {
#pragma unroll
        for (int k = 0; k < NJ; ++k) {
            if (k <= lnk) {
                const S v0 = w[0] - Os[k][0], v1 = w[1] - Os[k][1], v2 = w[2] - Os[k][2];
                const S c0 = Zs[k][1] * v2 - Zs[k][2] * v1;
                const S c1 = Zs[k][2] * v0 - Zs[k][0] * v2;
                const S c2 = Zs[k][0] * v1 - Zs[k][1] * v0;
                g[k] += sgn * (u[0] * c0 + u[1] * c1 + u[2] * c2);
            }
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < NJ; ++k) {
        if (k <= lnk) {
            const bool pr = is_prismatic(prism, k);
            const S v0 = w[0] - Os[k][0], v1 = w[1] - Os[k][1], v2 = w[2] - Os[k][2];
            const S c0 = pr ? Zs[k][0] : Zs[k][1] * v2 - Zs[k][2] * v1;
            const S c1 = pr ? Zs[k][1] : Zs[k][2] * v0 - Zs[k][0] * v2;
            const S c2 = pr ? Zs[k][2] : Zs[k][0] * v1 - Zs[k][1] * v0;
            g[k] += sgn * (u[0] * c0 + u[1] * c1 + u[2] * c2);
        }
    }
}

// Self and environment distances of configuration q (+inf where nothing is
// checked) and, with GRAD, their gradients.  With a finite `beyond`, pairs
// provably farther than it are skipped as well: a minimum above `beyond` is
// then reported as +inf (the residuals, which vanish beyond their margin,
// need no more).
template <typename S, bool GRAD, typename C, bool PRISM = true>
__device__ __forceinline__ void coll_distances(const RobotT<S> &rb, const C cap[NJ][7], int n_obs,
                                               const CPF_GLOBAL double *__restrict__ obs, const S *q, S dmin[2],
                                               S grad[2][NJ], S beyond = __builtin_inf()) {
    S Zs[NJ][3], Os[NJ][3], P0[NJ][3], P1[NJ][3];
    capsule_chain<S, C, PRISM>(rb, cap, q, Zs, Os, P0, P1);
    // bounding sphere of each capsule: centre and radius (half length + r)
    S cc[NJ][3], cr[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        S h2 = S(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            cc[i][k] = S(0.5) * (P0[i][k] + P1[i][k]);
            const S h = S(0.5) * (P1[i][k] - P0[i][k]);
            h2 += h * h;
        }
        cr[i] = sqrt(h2) + (S)cap[i][6];
    }
    auto gap = [&](const S a[3], const S b[3]) {
        const S x = a[0] - b[0], y = a[1] - b[1], z = a[2] - b[2];
        return sqrt(x * x + y * y + z * z);
    };
    dmin[0] = __builtin_inf();
    dmin[1] = __builtin_inf();
    int bi = -1, bj = 0;
    S bs = S(0), bt = S(0);
#pragma unroll
    for (int i = 0; i < NJ; ++i)
#pragma unroll
        for (int j = i + 3; j < NJ; ++j) {
            if (gap(cc[i], cc[j]) - cr[i] - cr[j] > fmin(dmin[0], beyond) + cull_slack<S>()) continue;
            S s, t;
            const S d = sqrt(seg_seg_d2(P0[i], P1[i], P0[j], P1[j], s, t)) - (S)cap[i][6] - (S)cap[j][6];
            if (d < dmin[0]) {
                dmin[0] = d;
                bi = i;
                bj = j;
                bs = s;
                bt = t;
            }
        }
    int li = -1, lo_idx = 0;
    S ls = S(0);
    for (int m = 0; m < n_obs; ++m) {
        const CPF_GLOBAL double *B = obs + (size_t)m * 18;
        S o[3], R[9], lo[3], hi[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            o[k] = (S)B[k];
            lo[k] = (S)B[12 + k];
            hi[k] = (S)B[15 + k];
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) R[k] = (S)B[3 + k];
        // the cuboid's bounding sphere: world centre and half diagonal
        S bc[3], bh2 = S(0);
        {
            S m[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                m[k] = S(0.5) * (lo[k] + hi[k]);
                const S h = S(0.5) * (hi[k] - lo[k]);
                bh2 += h * h;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) bc[k] = o[k] + R[3 * k] * m[0] + R[3 * k + 1] * m[1] + R[3 * k + 2] * m[2];
        }
        const S br = sqrt(bh2);
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            if (gap(cc[i], bc) - cr[i] - br > fmin(dmin[1], beyond) + cull_slack<S>()) continue;
            S A[3], D[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {   // R^T (P0 - o), R^T (P1 - P0)
                A[r] = R[r] * (P0[i][0] - o[0]) + R[3 + r] * (P0[i][1] - o[1]) + R[6 + r] * (P0[i][2] - o[2]);
                D[r] = R[r] * (P1[i][0] - P0[i][0]) + R[3 + r] * (P1[i][1] - P0[i][1]) +
                       R[6 + r] * (P1[i][2] - P0[i][2]);
            }
            S s;
            const S d = sqrt(seg_box_d2(A, D, lo, hi, s)) - (S)cap[i][6];
            if (d < dmin[1]) {
                dmin[1] = d;
                li = i;
                lo_idx = m;
                ls = s;
            }
        }
    }
    if (GRAD) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int k = 0; k < NJ; ++k) grad[h][k] = S(0);
        if (bi >= 0) {
            S pa[3], pb[3], u[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                pa[k] = P0[bi][k] + bs * (P1[bi][k] - P0[bi][k]);
                pb[k] = P0[bj][k] + bt * (P1[bj][k] - P0[bj][k]);
                u[k] = pa[k] - pb[k];
            }
            const S nrm = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            if (nrm > contact_eps<S>()) {
#pragma unroll
                for (int k = 0; k < 3; ++k) u[k] /= nrm;
                point_gradient<S, PRISM>(PRISM ? rb.prism : 0u, Zs, Os, bi, pa, u, S(1), grad[0]);
                point_gradient<S, PRISM>(PRISM ? rb.prism : 0u, Zs, Os, bj, pb, u, S(-1), grad[0]);
            }
        }
        if (li >= 0) {
            const CPF_GLOBAL double *B = obs + (size_t)lo_idx * 18;
            S pa[3], x[3], u[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) pa[k] = P0[li][k] + ls * (P1[li][k] - P0[li][k]);
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const S v = (S)B[3 + r] * (pa[0] - (S)B[0]) + (S)B[6 + r] * (pa[1] - (S)B[1]) +
                            (S)B[9 + r] * (pa[2] - (S)B[2]);
                x[r] = v < (S)B[12 + r] ? (S)B[12 + r] : (v > (S)B[15 + r] ? (S)B[15 + r] : v);
            }
#pragma unroll
            for (int k = 0; k < 3; ++k)
                u[k] = pa[k] - ((S)B[k] + (S)B[3 + 3 * k] * x[0] + (S)B[4 + 3 * k] * x[1] + (S)B[5 + 3 * k] * x[2]);
            const S nrm = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            if (nrm > contact_eps<S>()) {
#pragma unroll
                for (int k = 0; k < 3; ++k) u[k] /= nrm;
                point_gradient<S, PRISM>(PRISM ? rb.prism : 0u, Zs, Os, li, pa, u, S(1), grad[1]);
            }
        }
    }
}

}  // namespace CPF_JNS
}  // namespace cpf
