// dp.hip -- layered-graph search over candidate plans (Sec. III-B).
//
// Node (t, k) is candidate k at waypoint t.  The value of a node is the
// smallest achievable maximum joint change (mjac) of a path ending there,
// with the joint-limit penalty (and the caller's extra cost) added on the
// edge that enters a penalised node:
//   B_0(k) = pen_0(k)
//   B_t(k) = min_k' max(B_{t-1}(k'), e_t(k',k) + pen_t(k)),
//   e_t(k',k) = max_j |q_t^k[j] - q_{t-1}^k'[j]|.
// Ties are broken by the smallest (value, e, k'); every operation is an
// exact FP64 sub / abs / max / compare except the single rounding of
// e + pen, so the result does not depend on the order of evaluation.
//
// Two kernels:
//  1. dp_topm_kernel (whole GPU, no stage dependency): for every node (t, k),
//     the TOPM predecessors with the smallest (e_t(k',k), k'), in order.
//  2. dp_kernel (one workgroup per plan, stages in sequence): node (t, k)
//     first scans its TOPM list.  Every predecessor not in the list has
//     e >= e_M (the list's last edge) and B >= beta = min_k' B_{t-1}(k'), so
//     its value is at least max(beta, e_M + pen) (e + pen is monotone in e
//     under rounding).  If that bound exceeds the best value found, or equals
//     it with e_M >= the best edge (the list then also wins every tie), the
//     list result is the exact minimum; otherwise the lane falls back to the
//     full scan over all K predecessors.  Either way the answer equals the
//     exhaustive minimum, bit for bit.
#include <float.h>

#include "cpf_device.h"
#include "cpf_internal.h"

namespace cpf {

constexpr int DP_BS = 1024;        // serial kernel: one lane per destination (K <= 1024)
constexpr int TOPM_BS = 256;       // list kernel: one lane per node of a stage tile

__device__ __forceinline__ bool key_less(double v, double e, int k, double bv, double be, int bk) {
    return v < bv || (v == bv && (e < be || (e == be && k < bk)));
}

// Edge change between a destination (registers) and a predecessor (7 values).
template <typename Q>
__device__ __forceinline__ double edge(const double qk[NJ], const Q *pq, int stride) {
    double e = fabs(qk[0] - (double)pq[0]);
#pragma unroll
    for (int j = 1; j < NJ; ++j) e = fmax(e, fabs(qk[j] - (double)pq[j * stride]));
    return e;
}

// Grid: x = tile (stage t >= 1, block of TOPM_BS destinations), y = plan.
__global__ __launch_bounds__(TOPM_BS) void dp_topm_kernel(const DevPlan *__restrict__ plans) {
    const DevPlan &P = plans[blockIdx.y];
    const int T = P.T, K = P.K;
    if (T <= 1 || K <= 0) return;
    const int nkb = (K + TOPM_BS - 1) / TOPM_BS;
    const int t = 1 + blockIdx.x / nkb, kb = blockIdx.x % nkb;
    if (t >= T) return;
    extern __shared__ float qprev[];   // [7][K]: candidates of stage t-1
    const CPF_GLOBAL float *__restrict__ cand = P.cand;
    for (int x = threadIdx.x; x < NJ * K; x += TOPM_BS)
        qprev[x] = cand[(size_t)(t - 1) * NJ * K + x];
    __syncthreads();
    const int k = kb * TOPM_BS + threadIdx.x;
    if (k >= K) return;
    double qk[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) qk[j] = (double)cand[((size_t)t * NJ + j) * K + k];
    double le[TOPM];
    int li[TOPM];
#pragma unroll
    for (int m = 0; m < TOPM; ++m) {
        le[m] = __builtin_inf();
        li[m] = 0;
    }
    for (int kp = 0; kp < K; ++kp) {
        const double e = edge(qk, qprev + kp, K);
        if (e < le[TOPM - 1]) {   // ascending k': a tie on e never displaces an earlier k'
#pragma unroll
            for (int m = TOPM - 1; m > 0; --m) {
                const bool shift = e < le[m - 1];
                const bool here = !shift && e < le[m];
                le[m] = shift ? le[m - 1] : (here ? e : le[m]);
                li[m] = shift ? li[m - 1] : (here ? kp : li[m]);
            }
            if (e < le[0]) {
                le[0] = e;
                li[0] = kp;
            }
        }
    }
    const int meff = K < TOPM ? K : TOPM;
#pragma unroll
    for (int m = 0; m < TOPM; ++m)
        if (m < meff) P.topk[((size_t)t * TOPM + m) * K + k] = (uint16_t)li[m];
}

__global__ __launch_bounds__(DP_BS) void dp_kernel(const DevPlan *__restrict__ plans) {
    const DevPlan &P = plans[blockIdx.x];
    const int T = P.T, K = P.K;
    if (T <= 0 || K <= 0) return;
    extern __shared__ double prev[];   // [K][8]: q_{t-1}^k' (7) and B_{t-1}(k')
    __shared__ double wmin[DP_BS / 64];
    __shared__ double red[DP_BS];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int k = tid;
    const bool owner = k < K;
    const int meff = K < TOPM ? K : TOPM;

    double lom[NJ], him[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        lom[j] = P.lo[j] + P.margin;
        him[j] = P.hi[j] - P.margin;
    }
    const CPF_GLOBAL float *__restrict__ cand = P.cand;

    auto penalty = [&](const double *q, int t) -> double {
        bool near = false;
#pragma unroll
        for (int j = 0; j < NJ; ++j) near = near || (q[j] <= lom[j]) || (q[j] >= him[j]);
        const double ex = (P.has_extra && owner) ? P.extra[(size_t)t * K + k] : 0.0;
        return (near ? P.penalty : 0.0) + ex;
    };
    // beta = min over the values just written to prev (all waves call this)
    auto stage_min = [&](double b) -> double {
        double m = owner ? b : __builtin_inf();
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m = fmin(m, __shfl_xor(m, off));
        if (lane == 0) wmin[wave] = m;
        __syncthreads();
        double r = wmin[0];
#pragma unroll
        for (int w = 1; w < DP_BS / 64; ++w) r = fmin(r, wmin[w]);
        return r;
    };

    double qk[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) qk[j] = owner ? (double)cand[(size_t)j * K + k] : 0.0;
    double b0 = 0.0;
    if (owner) {
        b0 = penalty(qk, 0);
#pragma unroll
        for (int j = 0; j < NJ; ++j) prev[k * 8 + j] = qk[j];
        prev[k * 8 + 7] = b0;
    }
    double beta = stage_min(b0);   // includes the barrier that publishes prev

    // candidates and predecessor lists of the next stage, loaded one stage ahead
    float qn[NJ];
    int ln[TOPM];
#pragma unroll
    for (int j = 0; j < NJ; ++j) qn[j] = (owner && T > 1) ? cand[((size_t)1 * NJ + j) * K + k] : 0.f;
#pragma unroll
    for (int m = 0; m < TOPM; ++m)
        ln[m] = (owner && T > 1 && m < meff) ? P.topk[((size_t)1 * TOPM + m) * K + k] : 0;

    for (int t = 1; t < T; ++t) {
        double bv = __builtin_inf(), be = __builtin_inf();
        int bk = -1;
        if (owner) {
            int lc[TOPM];
#pragma unroll
            for (int j = 0; j < NJ; ++j) qk[j] = (double)qn[j];
#pragma unroll
            for (int m = 0; m < TOPM; ++m) lc[m] = ln[m];
            if (t + 1 < T) {
#pragma unroll
                for (int j = 0; j < NJ; ++j) qn[j] = cand[((size_t)(t + 1) * NJ + j) * K + k];
#pragma unroll
                for (int m = 0; m < TOPM; ++m)
                    if (m < meff) ln[m] = P.topk[((size_t)(t + 1) * TOPM + m) * K + k];
            }
            const double pen = penalty(qk, t);
            double eM = 0.0;
#pragma unroll
            for (int m = 0; m < TOPM; ++m) {
                if (m < meff) {
                    const int kp = lc[m];
                    const double *pq = prev + kp * 8;
                    const double e = edge(qk, pq, 1);
                    const double v = fmax(pq[7], e + pen);   // finite operands: exact max
                    if (key_less(v, e, kp, bv, be, bk)) {
                        bv = v;
                        be = e;
                        bk = kp;
                    }
                    eM = e;
                }
            }
            const double lb = fmax(beta, eM + pen);
            const bool exact = (meff == K) || (lb > bv) || (lb == bv && eM >= be);
            if (!exact) {   // full scan over every predecessor
                bv = __builtin_inf();
                be = __builtin_inf();
                bk = -1;
                for (int kp = 0; kp < K; ++kp) {
                    const double *pq = prev + kp * 8;
                    const double e = edge(qk, pq, 1);
                    const double v = fmax(pq[7], e + pen);
                    const bool upd = (v < bv) | ((v == bv) & (e < be));
                    bv = upd ? v : bv;
                    be = upd ? e : be;
                    bk = upd ? kp : bk;
                }
            }
            P.bp[(size_t)t * K + k] = (uint16_t)(bk >= 0 ? bk : 0);
        }
        __syncthreads();   // every lane has finished reading prev
        if (owner) {
#pragma unroll
            for (int j = 0; j < NJ; ++j) prev[k * 8 + j] = qk[j];
            prev[k * 8 + 7] = bv;
        }
        beta = stage_min(bv);
        __syncthreads();   // wmin is rewritten by the next stage
    }

    // End node: smallest (B_{T-1}(k), k); then follow the back-pointers.
    if (tid < 64) {
        double bb = __builtin_inf();
        int bkk = 0x7fffffff;
        for (int kk = tid; kk < K; kk += 64) {
            const double b = prev[kk * 8 + 7];
            if (b < bb) { bb = b; bkk = kk; }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_xor(bb, off);
            const int ok = __shfl_xor(bkk, off);
            if (ob < bb || (ob == bb && ok < bkk)) { bb = ob; bkk = ok; }
        }
        if (tid == 0) {
            P.dp_out[0] = bb;
            P.dp_out[2] = (double)bkk;
            // Validated inputs keep every value finite, so bkk and every
            // back-pointer are in [0, K); the clamps only keep memory safe.
            int cur = (bkk >= 0 && bkk < K) ? bkk : 0;
            P.path[T - 1] = cur;
            for (int t = T - 1; t > 0; --t) {
                cur = P.bp[(size_t)t * K + cur];
                cur = cur < K ? cur : 0;
                P.path[t - 1] = cur;
            }
        }
    }
    __syncthreads();

    // Seed gather xi[j][t] = q_t^{path[t]}[j] and its mjac.
    double m = 0.0;
    for (int t = tid; t < T; t += DP_BS) {
        const int kk = P.path[t];
#pragma unroll
        for (int j = 0; j < NJ; ++j) P.xi[(size_t)j * T + t] = (double)cand[((size_t)t * NJ + j) * K + kk];
        if (t + 1 < T) {
            const int k2 = P.path[t + 1];
#pragma unroll
            for (int j = 0; j < NJ; ++j)
                m = fmax(m, fabs((double)cand[((size_t)(t + 1) * NJ + j) * K + k2] -
                                 (double)cand[((size_t)t * NJ + j) * K + kk]));
        }
    }
    red[tid] = m;
    __syncthreads();
    for (int s = DP_BS / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
        __syncthreads();
    }
    if (tid == 0) {
        P.dp_out[1] = red[0];
        P.st->lambda = P.lam0;   // the LM starts afresh from this seed
        P.st->seeded = 0;
    }
}

hipError_t dp_launch(const DevPlan *d_plans, int nplans, int maxK, int maxT, hipStream_t s) {
    if (nplans <= 0) return hipSuccess;
    if (maxT > 1) {
        const int nkb = (maxK + TOPM_BS - 1) / TOPM_BS;
        const dim3 grid((unsigned)((maxT - 1) * nkb), (unsigned)nplans);
        hipLaunchKernelGGL(dp_topm_kernel, grid, dim3(TOPM_BS), (size_t)maxK * NJ * sizeof(float),
                           s, d_plans);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const size_t lds = (size_t)maxK * 8 * sizeof(double);
    hipLaunchKernelGGL(dp_kernel, dim3(nplans), dim3(DP_BS), lds, s, d_plans);
    return hipGetLastError();
}

}  // namespace cpf
