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
//  1. dp_topm_kernel (whole GPU, no stage dependency): the penalty of every
//     node, and for every node (t, k) with t >= 1 the TOPM predecessors with
//     the smallest (e_t(k',k), k'), in that order, with c = e + pen_t(k).
//     The rounding of e + pen is monotone in e, so c ascends along the list.
//  2. dp_kernel (one workgroup per plan, stages in sequence): node (t, k)
//     takes the best of its list under the key (value, e, k'), where
//     value = max(B_{t-1}(k'), c).  In list order (e, k') ascends, so the
//     first entry of smallest value is the key minimum.  Every predecessor
//     outside the list has e >= e_M (the list's last edge) and
//     B >= beta = min_k' B_{t-1}(k'), so its value is at least
//     lb = max(beta, c_M).  If lb > the list's best value, no outside
//     predecessor reaches it; if lb equals it, an outside predecessor can
//     only tie on value, and then loses on (e, k') because its e >= e_M >=
//     the best entry's edge (an equal e comes with a larger k', since the
//     list keeps the earliest k' of equal edges).  So lb >= best value proves
//     the list result exact; otherwise the node gets the full scan over all
//     K predecessors, done by a whole wavefront (the nodes needing one are
//     shared out among the wavefronts after the stage's barrier).  Either
//     way the answer equals the exhaustive minimum, bit for bit.  A stage
//     costs an LDS gather of TOPM / 2 values per lane (the list's second
//     half only where the first half cannot settle the node) and one
//     workgroup barrier (two more when a full scan is needed); the lists of
//     later stages are loaded ahead.
#include <float.h>

#include "coll_device.h"
#include "cpf_device.h"
#include "cpf_internal.h"

namespace cpf {
namespace CPF_JNS {

constexpr int TOPM_BS = 256;       // list kernel: one lane per node of a stage tile

// Edge change between a destination (registers) and a predecessor (NJ values).
template <typename Q>
__device__ __forceinline__ double edge(const double qk[NJ], const Q *pq, long stride) {
    double e = fabs(qk[0] - (double)pq[0]);
#pragma unroll
    for (int j = 1; j < NJ; ++j) e = fmax(e, fabs(qk[j] - (double)pq[j * stride]));
    return e;
}

// Node penalty: limit_penalty if any joint is within the margin of a limit,
// plus the caller's cost of the node, plus (collision geometry) the node's
// collision penalty from node_coll_kernel.
__device__ __forceinline__ double node_penalty(const DevPlan &P, const double q[NJ], int t, int k) {
    bool near = false;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const double m = is_prismatic((uint32_t)P.prism, j) ? P.margin_p : P.margin;
        near = near || (q[j] <= P.lo[j] + m) || (q[j] >= P.hi[j] - m);
    }
    const double ex = P.has_extra ? P.extra[(size_t)t * P.K + k] : 0.0;
    double pen = (near ? P.penalty : 0.0) + ex;
    if (P.has_coll) pen += P.cpen[(size_t)t * P.K + k];
    return pen;
}

// The collision checker of the search (Sec. III-B): coll_penalty for every
// node (t, k >= k_begin) whose configuration has a capsule distance below
// zero (FP64 kinematics on the float32 candidates), else 0.  One lane per
// node; its own kernel so that the list kernels keep their registers.
// Grid: x = tile (stage t, block of TOPM_BS nodes from k_begin), y = plan.
__global__ __launch_bounds__(TOPM_BS) void node_coll_kernel(const DevPlan *__restrict__ plans, int k_begin) {
    const DevPlan &P = plans[blockIdx.y];
    const int T = P.T, K = P.K;
    if (T <= 0 || K <= k_begin || !P.has_coll || P.dof != NJ) return;
    const int nkb = (K - k_begin + TOPM_BS - 1) / TOPM_BS;
    const int t = blockIdx.x / nkb, k = k_begin + (blockIdx.x % nkb) * TOPM_BS + threadIdx.x;
    if (t >= T || k >= K) return;
    double q[NJ], dm[2], g[2][NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) q[j] = (double)P.cand[((size_t)t * NJ + j) * K + k];
    coll_distances<double, false>(load_robot<double>(P), P.cap, P.n_obs, P.obs, q, dm, g);
    P.cpen[(size_t)t * K + k] = (dm[0] < 0.0 || dm[1] < 0.0) ? P.coll_penalty : 0.0;
}

static hipError_t node_coll_launch(const DevPlan *d_plans, int nplans, int maxK, int maxT, int k_begin,
                                   hipStream_t s) {
    const int nkb = (maxK - k_begin + TOPM_BS - 1) / TOPM_BS;
    if (nkb <= 0) return hipSuccess;
    hipLaunchKernelGGL(node_coll_kernel, dim3((unsigned)(maxT * nkb), (unsigned)nplans), dim3(TOPM_BS), 0, s,
                       d_plans, k_begin);
    return hipGetLastError();
}

// Sorted insertion into a TOPM list ordered by (e, k').  Callers offer k' in
// ascending order among equal e, so a tie on e never displaces an earlier k'.
__device__ __forceinline__ void list_insert(double le[TOPM], int li[TOPM], double e, int kp) {
    if (e < le[TOPM - 1]) {
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

// The lists of stage t are element-major, so that the lanes of a wavefront
// (consecutive k) read and write contiguous runs: the indices as pairs
// packed in 32-bit words, [T][TOPM / 2][K], the values as [T][TOPM][K].
__device__ __forceinline__ CPF_GLOBAL uint32_t *list_words(const DevPlan &P, int t, int k, int K) {
    return (CPF_GLOBAL uint32_t *)P.topk + (size_t)t * (TOPM / 2) * K + k;
}
__device__ __forceinline__ CPF_GLOBAL double *list_values(const DevPlan &P, int t, int k, int K) {
    return P.topc + (size_t)t * TOPM * K + k;
}

// Entry m of the stored list of node (t, k).
__device__ __forceinline__ int list_entry(const DevPlan &P, int t, int k, int K, int m) {
    const uint32_t w = list_words(P, t, k, K)[(size_t)(m >> 1) * K];
    return (int)((w >> ((m & 1) * 16)) & 0xffffu);
}

__device__ __forceinline__ void store_list(const DevPlan &P, int t, int k, int K, const double le[TOPM],
                                           const int li[TOPM], double pen) {
    CPF_GLOBAL uint32_t *ix = list_words(P, t, k, K);
#pragma unroll
    for (int m = 0; m < TOPM / 2; ++m) ix[(size_t)m * K] = (uint32_t)li[2 * m] | ((uint32_t)li[2 * m + 1] << 16);
    CPF_GLOBAL double *cv = list_values(P, t, k, K);
#pragma unroll
    for (int m = 0; m < TOPM; ++m) cv[(size_t)m * K] = le[m] + pen;
}

// Candidates buffered per lane between merges into its list (exact scan).
constexpr int LIST_BUF = 16;

// The previous stage's candidates in shared memory, in groups of four
// predecessors: group g holds joint j of predecessors 4g..4g+3 as one float4
// at (g * NJ + j) * 4, so a group is NJ consecutive float4s.  K is rounded up
// to whole groups (the padding holds +inf).
__host__ __device__ inline int topm_row(int K) { return (K + 3) & ~3; }
__device__ __forceinline__ int qidx(int j, int kp) { return ((kp >> 2) * NJ + j) * 4 + (kp & 3); }

// Shared memory of dp_topm_kernel for K candidates: the previous stage's
// candidates (float, NJ * topm_row(K)) and the merge buffers (uint16
// [LIST_BUF][TOPM_BS]).
__host__ __device__ inline size_t topm_shared_bytes(int K) {
    return (size_t)topm_row(K) * NJ * sizeof(float) + (size_t)LIST_BUF * TOPM_BS * sizeof(uint16_t);
}

// Selection keys.  The bit pattern of a non-negative float orders like its
// value.  Clamped to [2^-24, 2^8) and less the clamp's low end it fits in 28
// bits; shifted up by 4, with its low b bits replaced by the predecessor's
// index (b = max(4, ceil(log2 K)), so an index fits), it gives a 32-bit key
// that orders predecessors by FP32 edge, coarsened to buckets of 2^(b-4)
// consecutive floats, then by index.  Keys are distinct, and a bucket's
// edges are bounded by bucket_lower / bucket_upper.
constexpr uint32_t KEY_LO = 103u << 23;          // 2^-24
constexpr uint32_t KEY_HI = (135u << 23) - 1u;   // the largest float below 2^8

__device__ __forceinline__ uint32_t umed3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ __forceinline__ uint32_t edge_key(float e, uint32_t kmask, uint32_t kp) {
    const uint32_t x = min(max(__float_as_uint(e), KEY_LO), KEY_HI);
    return (((x - KEY_LO) << 4) & kmask) | kp;
}

// Bounds of the FP32 edges whose keys carry the bucket bits cb (a key with
// its index bits cleared): every such edge e has lower <= e < upper.  The
// lowest bucket takes every edge below the clamp, the highest every edge
// above it.
__device__ __forceinline__ double bucket_lower(uint32_t cb) {
    return cb == 0 ? 0.0 : (double)__uint_as_float((cb >> 4) + KEY_LO);
}
__device__ __forceinline__ double bucket_upper(uint32_t cb, uint32_t kmask, int b) {
    const uint32_t top = ((KEY_HI - KEY_LO) << 4) & kmask;
    return cb == top ? __builtin_inf() : (double)__uint_as_float((cb >> 4) + KEY_LO + (1u << (b - 4)));
}

// (e, k') order of two list entries.
__device__ __forceinline__ bool entry_before(double ea, int ia, double eb, int ib) {
    return ea < eb || (ea == eb && ia < ib);
}

// Grid: x = tile (stage t, block of TOPM_BS destinations), y = plan.
//
// One lane per destination k.  Its list is the TOPM predecessors with the
// smallest (e_t(k', k), k') under the exact FP64 edge e.  The FP32 edge ef
// of the float32 inputs is the FP32 rounding of the exact edge and the FP64
// edge its FP64 rounding, so ef orders predecessors like e up to a relative
// 2^-21 (twice FP32's rounding, with room to spare): e_a <= e_b implies
// ef_a <= ef_b (1 + 2^-21), and ef_a >= ef_b (1 + 2^-21) implies e_a > e_b.
//
//  1. Selection: every predecessor's 32-bit key (FP32 edge bucket, index)
//     goes through a sorted register list of the TOPM + 1 smallest keys,
//     branch-free: inserting x moves entry m to median(L[m-1], L[m], x).
//  2. When K <= TOPM the list holds every predecessor.  Otherwise, if the
//     (TOPM+1)-th key's bucket starts at or above the TOPM-th key's bucket
//     end times (1 + 2^-21), each of the first TOPM has a smaller exact edge
//     than every predecessor left out, so they are the list's members.
//     Their FP64 edges are computed and, should the key order differ from
//     the (e, k') order (equal buckets), they are sorted.
//  3. Otherwise (near-equal edges at the list's end) the lane rebuilds its
//     list exactly: each predecessor whose FP32 edge is below the TOPM-th
//     bucket's end times (1 + 2^-21) -- a set holding the whole list -- is
//     buffered, and the buffers are merged into a sorted FP64 list with
//     strict insertion in ascending k' (whenever some lane of the wavefront
//     has LIST_BUF of them), the screen tightening to the list's last edge
//     times (1 + 2^-21) as it fills.
// Each path yields the list the plain scan in ascending k' builds, bit for
// bit; with K < TOPM the entries past K keep index 0 and an infinite edge
// (the serial pass reads only the first min(K, TOPM)).
__global__ __launch_bounds__(TOPM_BS) void dp_topm_kernel(const DevPlan *__restrict__ plans) {
    const DevPlan &P = plans[blockIdx.y];
    const int T = P.T, K = P.K;
    if (T <= 0 || K <= 0 || P.dof != NJ) return;   // empty slot, or a chain of another length
    const int nkb = (K + TOPM_BS - 1) / TOPM_BS;
    const int t = blockIdx.x / nkb, kb = blockIdx.x % nkb;
    if (t >= T) return;
    const int Kr = topm_row(K);
    extern __shared__ float qprev[];   // candidates of stage t-1 (qidx), then the merge buffers
    uint16_t *buf = (uint16_t *)(qprev + (size_t)NJ * Kr) + threadIdx.x;   // [LIST_BUF][TOPM_BS]
    const CPF_GLOBAL float *__restrict__ cand = P.cand;
    if (t > 0) {
#pragma unroll
        for (int j = 0; j < NJ; ++j)
            for (int kp = threadIdx.x; kp < Kr; kp += TOPM_BS)
                qprev[qidx(j, kp)] = kp < K ? cand[((size_t)(t - 1) * NJ + j) * K + kp] : __builtin_inff();
    }
    __syncthreads();
    const int k = kb * TOPM_BS + threadIdx.x;
    if (k >= K) return;
    float qf[NJ];
    double qk[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        qf[j] = cand[((size_t)t * NJ + j) * K + k];
        qk[j] = (double)qf[j];
    }
    const double pen = node_penalty(P, qk, t, k);
    P.pen[(size_t)t * K + k] = pen;
    if (t == 0) return;

    // 1. the TOPM + 1 smallest keys
    const int b = K <= 16 ? 4 : 32 - __clz(K - 1);
    const uint32_t kmask = ~((1u << b) - 1u);
    uint32_t L[TOPM + 1];
#pragma unroll
    for (int m = 0; m <= TOPM; ++m) L[m] = 0xffffffffu;
    const float4 *rows = (const float4 *)qprev;
    for (int k4 = 0; k4 < Kr / 4; ++k4) {
        float4 p[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) p[j] = rows[k4 * NJ + j];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            auto pu = [&](int j) { return u == 0 ? p[j].x : (u == 1 ? p[j].y : (u == 2 ? p[j].z : p[j].w)); };
            float e = fabsf(qf[0] - pu(0));
#pragma unroll
            for (int j = 1; j < NJ; ++j) e = fmaxf(e, fabsf(qf[j] - pu(j)));
            const uint32_t key = edge_key(e, kmask, (uint32_t)(4 * k4 + u));
#pragma unroll
            for (int m = TOPM; m > 0; --m) L[m] = umed3(L[m - 1], L[m], key);
            L[0] = min(L[0], key);
        }
    }

#pragma unroll
    for (int j = 0; j < NJ; ++j) qk[j] = (double)qf[j];   // (not kept live through the selection)
    double le[TOPM];
    int li[TOPM];
    const int n = K < TOPM ? K : TOPM;
    bool exact_scan = false;
    if (K > TOPM) {
        const uint32_t c15 = L[TOPM - 1] & kmask, c16 = L[TOPM] & kmask;
        exact_scan = !(bucket_lower(c16) >= bucket_upper(c15, kmask, b) * (1.0 + 0x1p-21));
    }
    if (!exact_scan) {
        // 2. the first n keys are the list; FP64 edges, then the (e, k') order
        bool unsorted = false;
#pragma unroll
        for (int m = 0; m < TOPM; ++m) {
            li[m] = m < n ? (int)(L[m] & ~kmask) : 0;
            le[m] = m < n ? edge(qk, qprev + qidx(0, li[m]), 4) : __builtin_inf();
            if (m > 0) unsorted = unsorted || (m < n && entry_before(le[m], li[m], le[m - 1], li[m - 1]));
        }
        if (unsorted) {   // odd-even transposition sort of the first n entries
#pragma unroll
            for (int r = 0; r < TOPM; ++r) {
#pragma unroll
                for (int m = (r & 1) + 1; m < TOPM; m += 2) {
                    const bool sw = m < n && entry_before(le[m], li[m], le[m - 1], li[m - 1]);
                    const double ea = le[m - 1], eb = le[m];
                    const int ia = li[m - 1], ib = li[m];
                    le[m - 1] = sw ? eb : ea;
                    le[m] = sw ? ea : eb;
                    li[m - 1] = sw ? ib : ia;
                    li[m] = sw ? ia : ib;
                }
            }
        }
    } else {
        // 3. exact rebuild from the predecessors below the screen
        const double thr = bucket_upper(L[TOPM - 1] & kmask, kmask, b) * (1.0 + 0x1p-21);
#pragma unroll
        for (int m = 0; m < TOPM; ++m) {
            le[m] = __builtin_inf();
            li[m] = 0;
        }
        double tau = thr;
        int cnt = 0;
        for (int kp = 0; kp < K; ++kp) {
            const float *pq = qprev + qidx(0, kp);
            float e = fabsf(qf[0] - pq[0]);
#pragma unroll
            for (int j = 1; j < NJ; ++j) e = fmaxf(e, fabsf(qf[j] - pq[4 * j]));
            if ((double)e < tau) {
                buf[cnt * TOPM_BS] = (uint16_t)kp;
                ++cnt;
            }
            if (__any(cnt == LIST_BUF) || kp == K - 1) {   // uniform over the lanes in this branch
                for (int i = 0; i < cnt; ++i) {
                    const int kq = buf[i * TOPM_BS];
                    list_insert(le, li, edge(qk, qprev + qidx(0, kq), 4), kq);
                }
                cnt = 0;
                tau = fmin(thr, le[TOPM - 1] * (1.0 + 0x1p-21));
            }
        }
    }
    store_list(P, t, k, K, le, li, pen);
}

// After candidates K_old..K-1 were appended to a plan (Sec. III-B's
// re-search with more candidate plans), with the first K_old candidates'
// penalties and lists already copied into the plan's layout: penalties and
// full lists for the new nodes; for an old node, its list merged with the
// new predecessors only.  The TOPM smallest (e, k') over all K predecessors
// are among the old list and the new predecessors, and offering the old
// list in its order and then the new k' ascending keeps the (e, k') order of
// equal edges, so the merged list equals the list computed from scratch.
// The old entries' edges are recomputed (the stored c = e + pen is rounded).
__global__ __launch_bounds__(TOPM_BS) void dp_topm_append_kernel(const DevPlan *__restrict__ plans, int K_old) {
    const DevPlan &P = plans[blockIdx.y];
    const int T = P.T, K = P.K;
    if (T <= 0 || K <= 0 || P.dof != NJ) return;
    const int nkb = (K + TOPM_BS - 1) / TOPM_BS;
    const int t = blockIdx.x / nkb, kb = blockIdx.x % nkb;
    if (t >= T) return;
    extern __shared__ float qprev[];   // [NJ][K]: candidates of stage t-1
    const CPF_GLOBAL float *__restrict__ cand = P.cand;
    if (t > 0) {
        for (int x = threadIdx.x; x < NJ * K; x += TOPM_BS)
            qprev[x] = cand[(size_t)(t - 1) * NJ * K + x];
    }
    __syncthreads();
    const int k = kb * TOPM_BS + threadIdx.x;
    if (k >= K) return;
    double qk[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) qk[j] = (double)cand[((size_t)t * NJ + j) * K + k];
    const size_t node = (size_t)t * K + k;
    const bool old = k < K_old;
    double pen;
    if (old) {
        pen = P.pen[node];   // kept from the first search
    } else {
        pen = node_penalty(P, qk, t, k);
        P.pen[node] = pen;
    }
    if (t == 0) return;
    double le[TOPM];
    int li[TOPM];
#pragma unroll
    for (int m = 0; m < TOPM; ++m) {
        le[m] = __builtin_inf();
        li[m] = 0;
    }
    int kp0 = 0;
    if (old) {
        const int n_old = K_old < TOPM ? K_old : TOPM;
        for (int m = 0; m < n_old; ++m) {
            const int kp = list_entry(P, t, k, K, m);
            list_insert(le, li, edge(qk, qprev + kp, K), kp);
        }
        kp0 = K_old;
    }
    for (int kp = kp0; kp < K; ++kp) list_insert(le, li, edge(qk, qprev + kp, K), kp);
    store_list(P, t, k, K, le, li, pen);
}

// One stage's list of a destination, in registers.
struct StageList {
    uint4 ix0, ix1;       // TOPM packed 16-bit predecessor indices
    double c[TOPM];       // their edges plus the destination's penalty
};

__device__ __forceinline__ void load_list(const DevPlan &P, int t, int k, StageList &L) {
    const int K = P.K;
    const CPF_GLOBAL uint32_t *ix = list_words(P, t, k, K);
    L.ix0 = make_uint4(ix[0], ix[(size_t)K], ix[(size_t)2 * K], ix[(size_t)3 * K]);
    L.ix1 = make_uint4(ix[(size_t)4 * K], ix[(size_t)5 * K], ix[(size_t)6 * K], ix[(size_t)7 * K]);
    const CPF_GLOBAL double *cv = list_values(P, t, k, K);
#pragma unroll
    for (int m = 0; m < TOPM; ++m) L.c[m] = cv[(size_t)m * K];
}

// Lane-to-lane move of a double by a DPP control (ALU only, no LDS); rows
// outside row_mask keep their own value.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int plo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROW_MASK, 0xf, false);
    const int phi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROW_MASK, 0xf, false);
    return __hiloint2double(phi, plo);
}

// Minimum over the 64 lanes of a wavefront (every lane active): within
// quads, half rows and rows of 16 lanes, then row 0 into row 1 and row 2
// into row 3 (lane 15's broadcast), then rows 0-1 into row 3 (lane 31's);
// lane 63 ends up holding the minimum of all 64 lanes.
__device__ __forceinline__ double wave_min(double v) {
    auto mn = [](double a, double b) { return b < a ? b : a; };
    v = mn(v, dpp_f64<0xb1, 0xf>(v));    // quad_perm [1,0,3,2]
    v = mn(v, dpp_f64<0x4e, 0xf>(v));    // quad_perm [2,3,0,1]
    v = mn(v, dpp_f64<0x141, 0xf>(v));   // row_half_mirror
    v = mn(v, dpp_f64<0x140, 0xf>(v));   // row_mirror
    v = mn(v, dpp_f64<0x142, 0xa>(v));   // row_bcast:15 into rows 1 and 3
    v = mn(v, dpp_f64<0x143, 0xc>(v));   // row_bcast:31 into rows 2 and 3
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int list_index(const StageList &L, int m) {
    const uint4 &v = m < 8 ? L.ix0 : L.ix1;
    const int w = (m & 7) >> 1;
    const uint32_t word = w == 0 ? v.x : (w == 1 ? v.y : (w == 2 ? v.z : v.w));
    return (int)((word >> ((m & 1) * 16)) & 0xffffu);
}

// One lane per destination; BS >= K threads.  AHEAD stages of lists are in
// flight ahead of use (fewer with 1024 lanes, where registers are scarcer).
template <int BS, int AHEAD>
__global__ __launch_bounds__(BS) void dp_kernel(const DevPlan *__restrict__ plans) {
    const DevPlan &P = plans[blockIdx.x];
    const int T = P.T, K = P.K;
    if (T <= 0 || K <= 0 || P.dof != NJ) return;
    __shared__ double Bb[2][MAX_K];          // B_{t-1} and B_t (ping-pong)
    __shared__ double wmin[2][BS / 64];   // per-wave minima of each buffer
    __shared__ unsigned long long fmask[2][BS / 64];   // lanes whose list proved nothing
    __shared__ int ftag[2];   // = t when a lane of stage t needs a full scan (never cleared)
    __shared__ double red[BS];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nwave = (int)(blockDim.x >> 6);
    const int k = tid;
    const bool owner = k < K;
    const CPF_GLOBAL float *__restrict__ cand = P.cand;
    CPF_GLOBAL uint16_t *__restrict__ bp = P.bp;

    // publish a stage's values and its minimum (one barrier)
    auto publish = [&](int buf, double b) -> double {
        if (owner) Bb[buf][k] = b;
        const double m = wave_min(owner ? b : __builtin_inf());
        if (lane == 0) wmin[buf][wave] = m;
        __syncthreads();
        // all BS / 64 slots are read at once (in bounds; those past nwave
        // are not used), in the same order as a loop over the nwave waves
        double r = wmin[buf][0];
#pragma unroll
        for (int w = 1; w < BS / 64; ++w) {
            const double x = wmin[buf][w];
            r = (w < nwave && x < r) ? x : r;   // values are never NaN
        }
        return r;
    };

    if (tid < 2) ftag[tid] = -1;
    double beta = publish(0, owner ? P.pen[k] : 0.0);   // B_0 = pen_0 (the barrier orders ftag too)

    // Full scans of stage t for the nodes whose list could not prove their
    // minimum (fmask[cur]), one wavefront per node: lane l takes the
    // predecessors l, l + 64, ..., keeping the smallest (value, e, k') in
    // ascending k', then the wavefront reduces under the same key, which is
    // the serial scan's result.  Returns the new stage minimum.
    auto full_scans = [&](int t, int cur, int prv) -> double {
        const CPF_GLOBAL float *qp = cand + (size_t)(t - 1) * NJ * K;
        int i = 0;
        for (int w = 0; w < nwave; ++w) {
            unsigned long long m = fmask[cur][w];
            while (m) {
                const int node = w * 64 + __builtin_ctzll(m);
                m &= m - 1;
                if (i++ % nwave != wave) continue;
                double qk[NJ];
#pragma unroll
                for (int j = 0; j < NJ; ++j) qk[j] = (double)cand[((size_t)t * NJ + j) * K + node];
                const double pen = P.pen[(size_t)t * K + node];
                double bv = __builtin_inf(), be = __builtin_inf();
                int bk = 0x7fffffff;
                for (int kp = lane; kp < K; kp += 64) {
                    const double e = edge(qk, qp + kp, K);
                    const double vv = fmax(Bb[prv][kp], e + pen);
                    const bool upd = (vv < bv) | ((vv == bv) & (e < be));
                    bv = upd ? vv : bv;
                    be = upd ? e : be;
                    bk = upd ? kp : bk;
                }
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    const double ov = __shfl_xor(bv, off), oe = __shfl_xor(be, off);
                    const int ok = __shfl_xor(bk, off);
                    const bool take = (ov < bv) | ((ov == bv) & ((oe < be) | ((oe == be) & (ok < bk))));
                    bv = take ? ov : bv;
                    be = take ? oe : be;
                    bk = take ? ok : bk;
                }
                if (lane == 0) {
                    Bb[cur][node] = bv;
                    bp[(size_t)t * K + node] = (uint16_t)(bk < K ? bk : 0);
                }
            }
        }
        __syncthreads();
        return publish(cur, owner ? Bb[cur][k] : 0.0);
    };

    const int kc = owner ? k : K - 1;   // the node whose lists a lane loads
#ifdef CPF_PHASE_CYCLES
    // Diagnostic build only: shader-clock totals of the stage loop, thread 0
    // of plan 0: list evaluation, publication (its barrier), full scans.
    unsigned long long ph_gather = 0, ph_publish = 0, ph_scan = 0, n_scan = 0, ph_t = clock64();
    unsigned long long ph_read = 0, ph_eval = 0;
#define DP_MARK(acc)                                   \
    do {                                               \
        if (tid == 0 && blockIdx.x == 0) {             \
            const unsigned long long now_ = clock64(); \
            acc += now_ - ph_t;                        \
            ph_t = now_;                               \
        }                                              \
    } while (0)
#else
#define DP_MARK(acc) \
    do {             \
    } while (0)
#endif
    // The first entry of least value among list entries m0 .. m0 + TOPM/2 - 1,
    // by a pairwise tree: a right half replaces its left half only when
    // strictly smaller, so ties keep the earlier entry, as a scan in list
    // order would.  Entries past K (K < TOPM) carry c = +inf and never win.
    auto half_best = [&](const StageList &L, int prv, int m0, double &bv, int &bk) {
        constexpr int H = TOPM / 2;
        double tv[H];
        int tk[H];
#pragma unroll
        for (int m = 0; m < H; ++m) {
            tk[m] = list_index(L, m0 + m);
            tv[m] = Bb[prv][tk[m]];
        }
#ifdef CPF_PHASE_CYCLES
        {   // diagnostic build: wait for the gathered values here
            double sb = tv[0];
#pragma unroll
            for (int m = 1; m < H; ++m) sb += tv[m];
            if (sb == -1.0) bp[0] = 0;
        }
        DP_MARK(ph_read);
#endif
#pragma unroll
        for (int m = 0; m < H; ++m) tv[m] = fmax(tv[m], L.c[m0 + m]);
#pragma unroll
        for (int w = 1; w < H; w *= 2)
#pragma unroll
            for (int m = 0; m < H; m += 2 * w) {
                const bool right = tv[m + w] < tv[m];
                tv[m] = right ? tv[m + w] : tv[m];
                tk[m] = right ? tk[m + w] : tk[m];
            }
        bv = tv[0];
        bk = tk[0];
    };

    // One stage: the best of the list in `L`, the exactness check and, when
    // it fails anywhere, the cooperative full scans; `L` is refilled with the
    // list AHEAD stages on (clamped to a valid node, so every lane loads and
    // no branch separates the loads from their use).
    //
    // The list is evaluated in two halves.  Every entry m of the second half
    // has value max(B, c_m) >= c_m >= c_{TOPM/2}, and a later entry of equal
    // value loses the tie, so once the first half's best is at most
    // c_{TOPM/2} the second half cannot change the result; only when some
    // lane of the wavefront needs it does the wavefront gather the second
    // half (about one wavefront-stage in a hundred on the serving stream's
    // inputs).
    auto stage = [&](int t, StageList &L) {
        const int cur = t & 1, prv = cur ^ 1;
        double bv;
        int bk;
        half_best(L, prv, 0, bv, bk);
        if (__any(!(bv <= L.c[TOPM / 2]))) {   // uniform: the wavefront's lanes together
            double bv2;
            int bk2;
            half_best(L, prv, TOPM / 2, bv2, bk2);
            const bool right = bv2 < bv;
            bv = right ? bv2 : bv;
            bk = right ? bk2 : bk;
        }
        const bool exact = (K <= TOPM) || (fmax(beta, L.c[TOPM - 1]) >= bv);
#ifdef CPF_PHASE_CYCLES
        if (bv == -1.0) bp[0] = 0;   // diagnostic build: the evaluation is complete here
#endif
        DP_MARK(ph_eval);
        const unsigned long long need = __ballot(owner && !exact);
        if (lane == 0) {
            fmask[cur][wave] = need;
            if (need) ftag[cur] = t;
        }
        if (owner && exact) bp[(size_t)t * K + k] = (uint16_t)bk;
        load_list(P, min(t + AHEAD, T - 1), kc, L);
        DP_MARK(ph_gather);
        beta = publish(cur, bv);   // its barrier also publishes fmask[cur] and ftag[cur]
        DP_MARK(ph_publish);
        if (ftag[cur] == t) {
            beta = full_scans(t, cur, prv);
#ifdef CPF_PHASE_CYCLES
            ++n_scan;
#endif
            DP_MARK(ph_scan);
        }
    };

    // lists of the next AHEAD stages, in flight; buffer a serves the stages
    // t with (t - 1) % AHEAD == a, so no list is ever copied
    StageList buf[AHEAD];
#pragma unroll
    for (int a = 0; a < AHEAD; ++a) load_list(P, min(1 + a, T - 1), kc, buf[a]);
    // whole rounds of AHEAD stages keep the loop body free of branches
    // around the loads; the remaining stages follow
    int t0 = 1;
    for (; t0 + AHEAD <= T; t0 += AHEAD) {
#pragma unroll
        for (int a = 0; a < AHEAD; ++a) stage(t0 + a, buf[a]);
    }
#pragma unroll
    for (int a = 0; a < AHEAD; ++a)
        if (t0 + a < T) stage(t0 + a, buf[a]);

    // End node: smallest (B_{T-1}(k), k); then follow the back-pointers.
    const int last = (T - 1) & 1;
    if (tid < 64) {
        double bb = __builtin_inf();
        int bkk = 0x7fffffff;
        for (int kk = tid; kk < K; kk += 64) {
            const double b = Bb[last][kk];
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
                cur = bp[(size_t)t * K + cur];
                cur = cur < K ? cur : 0;
                P.path[t - 1] = cur;
            }
        }
    }
    __syncthreads();

    // Seed gather xi[j][t] = q_t^{path[t]}[j] and its largest steps of a
    // revolute and of a prismatic joint (the seed's mjac is the larger).
    double m[2] = {0.0, 0.0};
    for (int t = tid; t < T; t += (int)blockDim.x) {
        const int kk = P.path[t];
#pragma unroll
        for (int j = 0; j < NJ; ++j) P.xi[(size_t)j * T + t] = (double)cand[((size_t)t * NJ + j) * K + kk];
        if (t + 1 < T) {
            const int k2 = P.path[t + 1];
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const int h = is_prismatic((uint32_t)P.prism, j) ? 1 : 0;
                m[h] = fmax(m[h], fabs((double)cand[((size_t)(t + 1) * NJ + j) * K + k2] -
                                       (double)cand[((size_t)t * NJ + j) * K + kk]));
            }
        }
    }
    for (int h = 0; h < 2; ++h) {
        red[tid] = m[h];
        __syncthreads();
        for (int s = (int)blockDim.x / 2; s > 0; s >>= 1) {
            if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
            __syncthreads();
        }
        m[h] = red[0];
        __syncthreads();
    }
    if (tid == 0) {
        P.dp_out[1] = fmax(m[0], m[1]);
        P.dp_out[3] = m[0];
        P.dp_out[4] = m[1];
        P.st->lambda = P.lam0;   // the LM starts afresh from this seed
        P.st->seeded = 0;
    }
#ifdef CPF_PHASE_CYCLES
    if (tid == 0 && blockIdx.x == 0)
        printf("dp stage cycles T=%d K=%d: read %llu eval %llu lists %llu publish %llu scans %llu (stages with scans "
               "%llu)\n", T, K, ph_read, ph_eval, ph_gather, ph_publish, ph_scan, n_scan);
#endif
#undef DP_MARK
}

hipError_t dp_lists_launch(const DevPlan *d_plans, int nplans, int maxK, int maxT, bool coll, hipStream_t s) {
    if (nplans <= 0 || maxT <= 0 || maxK <= 0) return hipSuccess;
    if (maxK > MAX_K) return hipErrorInvalidValue;
    if (coll) {
        const hipError_t e = node_coll_launch(d_plans, nplans, maxK, maxT, 0, s);
        if (e != hipSuccess) return e;
    }
    const int nkb = (maxK + TOPM_BS - 1) / TOPM_BS;
    const dim3 grid((unsigned)(maxT * nkb), (unsigned)nplans);
    hipLaunchKernelGGL(dp_topm_kernel, grid, dim3(TOPM_BS), topm_shared_bytes(maxK), s, d_plans);
    return hipGetLastError();
}

hipError_t dp_stages_launch(const DevPlan *d_plans, int nplans, int maxK, hipStream_t s) {
    if (nplans <= 0 || maxK <= 0) return hipSuccess;
    if (maxK > MAX_K) return hipErrorInvalidValue;
    // one lane per destination, whole wavefronts (the seed reduction needs a power of two)
    int bs = 64;
    while (bs < maxK) bs <<= 1;
    if (bs <= 512)
        hipLaunchKernelGGL((dp_kernel<512, 2>), dim3(nplans), dim3(bs), 0, s, d_plans);
    else
        hipLaunchKernelGGL((dp_kernel<1024, 1>), dim3(nplans), dim3(bs), 0, s, d_plans);
    return hipGetLastError();
}

hipError_t dp_append_launch(const DevPlan *d_plan, int K_old, int K, int T, bool coll, hipStream_t s) {
    if (T <= 0 || K <= 0) return hipSuccess;
    if (K > MAX_K || K_old < 0 || K_old > K) return hipErrorInvalidValue;
    if (coll) {   // the new nodes' collision penalties (the old ones are kept)
        const hipError_t e = node_coll_launch(d_plan, 1, K, T, K_old, s);
        if (e != hipSuccess) return e;
    }
    const int nkb = (K + TOPM_BS - 1) / TOPM_BS;
    hipLaunchKernelGGL(dp_topm_append_kernel, dim3((unsigned)(T * nkb), 1), dim3(TOPM_BS),
                       (size_t)K * NJ * sizeof(float), s, d_plan, K_old);
    return hipGetLastError();
}

// One lane per candidate plan: its mjac, computed like the search computes
// edges (exact FP64 differences of the float32 values).
__global__ __launch_bounds__(256) void cand_mjac_kernel(const float *__restrict__ cand, int T, int K,
                                                        double *__restrict__ out) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= K) return;
    double m = 0.0;
    for (int t = 0; t + 1 < T; ++t)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
            m = fmax(m, fabs((double)cand[((size_t)(t + 1) * NJ + j) * K + k] -
                             (double)cand[((size_t)t * NJ + j) * K + k]));
    out[k] = m;
}

hipError_t cand_mjac_launch(const float *cand, int T, int K, double *out, hipStream_t s) {
    if (K <= 0) return hipSuccess;
    hipLaunchKernelGGL(cand_mjac_kernel, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, cand, T, K, out);
    return hipGetLastError();
}

}  // namespace CPF_JNS
}  // namespace cpf
