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
// e + pen, so the result does not depend on the reduction order.
//
// One workgroup of 1024 lanes per plan.  Lane (part, k) owns destination k
// and scans the predecessor range of its part; the previous stage's
// candidates and values sit in LDS as [K][8] doubles and are read by
// broadcast.  Partial minima are merged with the full key, so the split of
// the predecessor range does not change the answer.
#include <float.h>

#include "cpf_device.h"
#include "cpf_internal.h"

namespace cpf {

constexpr int DP_BS = 1024;

__device__ __forceinline__ bool key_less(double v, double e, int k, double bv, double be, int bk) {
    return v < bv || (v == bv && (e < be || (e == be && k < bk)));
}

__global__ __launch_bounds__(DP_BS) void dp_kernel(const DevPlan *__restrict__ plans) {
    const DevPlan &P = plans[blockIdx.x];
    const int T = P.T, K = P.K;
    if (T <= 0 || K <= 0) return;
    extern __shared__ double prev[];   // [K][8]: q_{t-1}^k' (7) and B_{t-1}(k')
    __shared__ double part_v[DP_BS], part_e[DP_BS];
    __shared__ int part_k[DP_BS];

    const int tid = threadIdx.x;
    const int Kp = (K + 63) & ~63;
    const int NP = Kp >= DP_BS ? 1 : DP_BS / Kp;
    const int k = tid % Kp, part = tid / Kp;
    const bool owner = part < NP && k < K;
    const int kp_lo = (part * K) / NP, kp_hi = ((part + 1) * K) / NP;

    double lom[NJ], him[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        lom[j] = P.lo[j] + P.margin;
        him[j] = P.hi[j] - P.margin;
    }
    const float *__restrict__ cand = P.cand;

    auto penalty = [&](const double *q, int t) -> double {
        bool near = false;
#pragma unroll
        for (int j = 0; j < NJ; ++j) near = near || (q[j] <= lom[j]) || (q[j] >= him[j]);
        const double ex = P.has_extra ? P.extra[(size_t)t * K + k] : 0.0;
        return (near ? P.penalty : 0.0) + ex;
    };

    double qk[NJ];
    if (owner) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) qk[j] = (double)cand[(size_t)j * K + k];
        if (part == 0) {
            const double pen = penalty(qk, 0);
#pragma unroll
            for (int j = 0; j < NJ; ++j) prev[k * 8 + j] = qk[j];
            prev[k * 8 + 7] = pen;
        }
    }
    __syncthreads();

    for (int t = 1; t < T; ++t) {
        double bv = __builtin_inf(), be = __builtin_inf();   // +inf
        int bk = -1;
        if (owner) {
#pragma unroll
            for (int j = 0; j < NJ; ++j) qk[j] = (double)cand[((size_t)t * NJ + j) * K + k];
            const double pen = penalty(qk, t);
            for (int kp = kp_lo; kp < kp_hi; ++kp) {
                const double *pq = prev + kp * 8;
                double e = fabs(qk[0] - pq[0]);
#pragma unroll
                for (int j = 1; j < NJ; ++j) e = fmax(e, fabs(qk[j] - pq[j]));
                double v = e + pen;
                const double b = pq[7];
                v = (b > v) ? b : v;
                if (v < bv || (v == bv && e < be)) { bv = v; be = e; bk = kp; }
            }
            part_v[tid] = bv; part_e[tid] = be; part_k[tid] = bk;
        }
        __syncthreads();
        if (owner && part == 0) {
            for (int p = 1; p < NP; ++p) {
                const int o = p * Kp + k;
                if (key_less(part_v[o], part_e[o], part_k[o], bv, be, bk)) {
                    bv = part_v[o]; be = part_e[o]; bk = part_k[o];
                }
            }
            P.bp[(size_t)t * K + k] = (uint16_t)(bk >= 0 ? bk : 0);
#pragma unroll
            for (int j = 0; j < NJ; ++j) prev[k * 8 + j] = qk[j];
            prev[k * 8 + 7] = bv;
        }
        __syncthreads();
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
    part_v[tid] = m;
    __syncthreads();
    for (int s = DP_BS / 2; s > 0; s >>= 1) {
        if (tid < s) part_v[tid] = fmax(part_v[tid], part_v[tid + s]);
        __syncthreads();
    }
    if (tid == 0) {
        P.dp_out[1] = part_v[0];
        P.st->lambda = P.lam0;   // the LM starts afresh from this seed
        P.st->seeded = 0;
    }
}

hipError_t dp_launch(const DevPlan *d_plans, int nplans, int maxK, hipStream_t s) {
    if (nplans <= 0) return hipSuccess;
    const size_t lds = (size_t)maxK * 8 * sizeof(double);
    hipLaunchKernelGGL(dp_kernel, dim3(nplans), dim3(DP_BS), lds, s, d_plans);
    return hipGetLastError();
}

}  // namespace cpf
