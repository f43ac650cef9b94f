// capi.cpp -- C ABI of the refinement path: context, device-memory budget,
// plans, synchronous search / LM calls and the batched solve.  The request
// server (cpf_submit / cpf_poll) lives in serve.cpp.
//
// A plan owns one device arena laid out as described in cpf_device.h.  The
// host converts the caller's AoS inputs to the device SoA layout once, at
// upload; kernels then run without further host traffic until results are
// read back.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <thread>

#include "runtime.h"

namespace cpf {

namespace {
thread_local std::string g_err;
}

// Working memory of cpf_solve_static: one plan arena in a static device
// array, so that the call needs no device allocation.  Host code reaches it
// only through the address hipGetSymbolAddress returns for the current
// device (set up by cpf_ctx_create; the array's name is a host stand-in).
constexpr uint64_t SCRATCH_BYTES = (uint64_t)64 << 20;
constexpr int MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
static void *g_scratch_ptr[MAX_DEVICES];
static std::mutex g_scratch_mu[MAX_DEVICES];   // one call at a time per device

// Address of this device's copy of the static scratch, looked up once per
// device with that device current.
static cpf_status scratch_setup(int device) {
    if (device < 0 || device >= MAX_DEVICES) return fail(CPF_E_UNSUPPORTED, "device %d beyond %d", device, MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_scratch_mu[device]);
    if (g_scratch_ptr[device]) return CPF_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(CPF_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
    return CPF_OK;
}

cpf_status fail(cpf_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// Bytes of the upload region: the caller's candidates ([K][T][dof], doubles
// or floats), then its targets ([T][12] doubles) from the next 256-byte
// boundary.
size_t raw_targets_offset(int T, int K, int dof, bool cand_f32) {
    return align256((size_t)T * K * dof * (cand_f32 ? sizeof(float) : sizeof(double)));
}
size_t raw_bytes(int T, int K, int dof, bool cand_f32) {
    return raw_targets_offset(T, K, dof, cand_f32) + (size_t)12 * T * sizeof(double);
}

Layout make_layout(int T, int K, int dof, bool extra, int n_obs, bool coll) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t t = (size_t)T, k = (size_t)K, nj = (size_t)dof, ntri = nj * (nj + 1) / 2;
    // what a read-back needs lies together at the start: one copy
    L.st = take(sizeof(LMState));
    L.report = take(8 * sizeof(double));
    L.dp_out = take(8 * sizeof(double));
    L.path = take(t * sizeof(int32_t));
    L.cand = take(t * nj * k * sizeof(float));
    L.extra = take(extra ? t * k * sizeof(double) : 0);
    L.pen = take(t * k * sizeof(double));
    L.bp = take(t * k * sizeof(uint16_t));
    L.topk = take(t * k * TOPM * sizeof(uint16_t));
    L.topc = take(std::max(t * k * TOPM * sizeof(double), raw_bytes(T, K, dof, false)));
    L.raw = L.topc;
    L.targets = take(12 * t * sizeof(double));
    L.xi = take(nj * t * sizeof(double));
    L.xt = take(nj * t * sizeof(double));
    L.A = take(ntri * t * sizeof(double));
    L.g = take(nj * t * sizeof(double));
    L.cr = take(cr_doubles(T, dof) * sizeof(double));
    L.dx = take(nj * t * sizeof(double));
    L.rb = take(nj * t * sizeof(double));
    L.xv = take(nj * t * sizeof(double));
    L.obs = take((size_t)n_obs * 18 * sizeof(double));
    L.cpen = take(coll ? t * k * sizeof(double) : 0);
    L.rr = take(RROWS * t * sizeof(double));
    L.rt = take(RROWS * t * sizeof(double));
    L.total = off;
    return L;
}

uint64_t plan_bytes(int T, int K, int dof, bool extra, int n_obs, bool coll) {
    return make_layout(T, K, dof, extra, n_obs, coll).total + align256(sizeof(DevPlan));
}

uint64_t plan_class_bytes(int T, int K, int dof, bool extra, int n_obs, bool coll) {
    const uint64_t b = plan_bytes(T, K, dof, extra, n_obs, coll);
    uint64_t c = (uint64_t)1 << 20;
    while (c < b) c <<= 1;
    return c;
}

cpf_status arena_get(cpf_ctx *ctx, uint64_t cls, void **out) {
    std::vector<void *> evict;
    {
        std::lock_guard<std::mutex> lk(ctx->pool_mu);
        if (ctx->used.load() + cls > ctx->budget)
            return fail(CPF_E_NOMEM, "plan needs %llu bytes; budget %llu, in use %llu",
                        (unsigned long long)cls, (unsigned long long)ctx->budget,
                        (unsigned long long)ctx->used.load());
        auto it = ctx->pool.find(cls);
        if (it != ctx->pool.end() && !it->second.empty()) {
            *out = it->second.back();
            it->second.pop_back();
            ctx->pooled -= cls;
            ctx->used += cls;
            return CPF_OK;
        }
        // make room among the cached arenas of other sizes
        for (auto &kv : ctx->pool) {
            while (!kv.second.empty() && ctx->used.load() + ctx->pooled + cls > ctx->budget) {
                evict.push_back(kv.second.back());
                kv.second.pop_back();
                ctx->pooled -= kv.first;
            }
        }
        ctx->used += cls;
    }
    for (void *p : evict) HIP_IGNORE(hipFree(p));
    hipError_t e = hipMalloc(out, cls);
    if (e != hipSuccess) {
        ctx->used -= cls;
        return fail(CPF_E_NOMEM, "hipMalloc(%llu): %s", (unsigned long long)cls, hipGetErrorString(e));
    }
    return CPF_OK;
}

void arena_put(cpf_ctx *ctx, void *p, uint64_t cls) {
    std::lock_guard<std::mutex> lk(ctx->pool_mu);
    ctx->used -= cls;
    ctx->pool[cls].push_back(p);
    ctx->pooled += cls;
}

void pool_clear(cpf_ctx *ctx) {
    std::lock_guard<std::mutex> lk(ctx->pool_mu);
    for (auto &kv : ctx->pool)
        for (void *p : kv.second) HIP_IGNORE(hipFree(p));
    ctx->pool.clear();
    ctx->pooled = 0;
    for (auto &kv : ctx->pinned)
        for (void *p : kv.second) HIP_IGNORE(hipHostFree(p));
    ctx->pinned.clear();
    ctx->pinned_total = 0;
}

void *pinned_get(cpf_ctx *ctx, uint64_t bytes, uint64_t *cls) {
    uint64_t c = (uint64_t)1 << 20;
    while (c < bytes) c <<= 1;
    *cls = c;
    {
        std::lock_guard<std::mutex> lk(ctx->pool_mu);
        auto it = ctx->pinned.find(c);
        if (it != ctx->pinned.end() && !it->second.empty()) {
            void *p = it->second.back();
            it->second.pop_back();
            return p;
        }
        if (ctx->pinned_total + c > ctx->pinned_cap) return nullptr;
        ctx->pinned_total += c;
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess) {
        std::lock_guard<std::mutex> lk(ctx->pool_mu);
        ctx->pinned_total -= c;
        return nullptr;
    }
    return p;
}

void pinned_put(cpf_ctx *ctx, void *p, uint64_t cls) {
    std::lock_guard<std::mutex> lk(ctx->pool_mu);
    ctx->pinned[cls].push_back(p);
}

void copy_parallel(void *dst, const void *src, size_t bytes) {
    const size_t chunk = (size_t)4 << 20;
    const int nt = (int)std::min<size_t>(4, (bytes + chunk - 1) / chunk);
    if (nt <= 1) {
        memcpy(dst, src, bytes);
        return;
    }
    const size_t per = (bytes + nt - 1) / nt;
    std::vector<std::thread> th;
    for (int i = 1; i < nt; ++i) {
        const size_t off = per * i, n = std::min(per, bytes - std::min(bytes, off));
        if (n) th.emplace_back([=] { memcpy((char *)dst + off, (const char *)src + off, n); });
    }
    memcpy(dst, src, std::min(per, bytes));
    for (auto &t : th) t.join();
}

static bool all_finite(const double *p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

cpf_status check_robot(const cpf_robot *r, HostRobot *out) {
    if (!r) return fail(CPF_E_ARG, "robot is NULL");
    if (!dof_supported(r->dof)) return fail(CPF_E_UNSUPPORTED, "dof=%d: chains of 7 or 8 joints are built", r->dof);
    if (!r->a || !r->d || !r->alpha || !r->q_lo || !r->q_hi)
        return fail(CPF_E_ARG, "robot array is NULL");
    *out = HostRobot{};
    out->dof = r->dof;
    const int nj = r->dof;
    for (int i = 0; i < nj; ++i) {
        const double off = r->theta_off ? r->theta_off[i] : 0.0;
        const double v[6] = {r->a[i], r->d[i], r->alpha[i], off, r->q_lo[i], r->q_hi[i]};
        if (!all_finite(v, 6)) return fail(CPF_E_ARG, "robot row %d is not finite", i);
        if (!(r->q_lo[i] <= r->q_hi[i])) return fail(CPF_E_ARG, "joint %d: q_lo > q_hi", i);
        out->a[i] = r->a[i];
        out->d[i] = r->d[i];
        out->alpha[i] = r->alpha[i];
        out->ca[i] = std::cos(r->alpha[i]);
        out->sa[i] = std::sin(r->alpha[i]);
        out->off[i] = off;
        out->lo[i] = r->q_lo[i];
        out->hi[i] = r->q_hi[i];
    }
    out->prism = 0;
    if (r->joint_type)
        for (int i = 0; i < nj; ++i) {
            if (r->joint_type[i] != 0 && r->joint_type[i] != 1)
                return fail(CPF_E_ARG, "joint %d: joint_type %d (0 revolute, 1 prismatic)", i, r->joint_type[i]);
            if (r->joint_type[i] == 1) out->prism |= 1u << i;
        }
    out->has_caps = r->capsules != nullptr;
    if (r->capsules) {
        if (!all_finite(r->capsules, (size_t)nj * 7)) return fail(CPF_E_ARG, "capsules not finite");
        for (int i = 0; i < nj; ++i) {
            if (!(r->capsules[7 * i + 6] >= 0.0)) return fail(CPF_E_ARG, "capsule %d: negative radius", i);
            for (int c = 0; c < 7; ++c) out->cap[i][c] = r->capsules[7 * i + c];
        }
    }
    return CPF_OK;
}

cpf_status check_plan_robot(const HostRobot &hr) {
    if (hr.has_caps && hr.prism)
        return fail(CPF_E_UNSUPPORTED, "plans with collision capsules and a prismatic joint are switched off");
    return CPF_OK;
}

hipError_t search_launch(cpf_ctx *ctx, const DevPlan *d_plans, int nplans, int maxK, int maxT, bool lists_ready,
                         bool coll, int dofs, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int dof = 7; dof <= 8 && e == hipSuccess; ++dof) {
        if (!(dofs & dof_bit(dof))) continue;
        if (!lists_ready)
            e = timed(ctx, KIND_DPL, s,
                      [&] { return CPF_BY_DOF(dof, dp_lists_launch(d_plans, nplans, maxK, maxT, coll, s)); });
        if (e == hipSuccess)
            e = timed(ctx, KIND_DP, s, [&] { return CPF_BY_DOF(dof, dp_stages_launch(d_plans, nplans, maxK, s)); });
    }
    return e;
}

hipError_t event_pair(cpf_ctx *ctx, hipEvent_t *a, hipEvent_t *b) {
    {
        std::lock_guard<std::mutex> lk(ctx->prof_mu);
        if (ctx->ev_free.size() >= 2) {
            *a = ctx->ev_free.back();
            ctx->ev_free.pop_back();
            *b = ctx->ev_free.back();
            ctx->ev_free.pop_back();
            return hipSuccess;
        }
    }
    hipError_t e = hipEventCreate(a);
    if (e == hipSuccess) e = hipEventCreate(b);
    return e;
}

cpf_status check_obstacles(int32_t n, const double *obs) {
    if (n < 0 || n > MAX_OBS) return fail(CPF_E_ARG, "n_obstacles=%d must be in [0, %d]", n, MAX_OBS);
    if (n > 0 && !obs) return fail(CPF_E_ARG, "obstacles is NULL");
    if (n > 0 && !all_finite(obs, (size_t)n * 18)) return fail(CPF_E_ARG, "obstacles not finite");
    for (int m = 0; m < n; ++m)
        for (int k = 0; k < 3; ++k)
            if (!(obs[18 * m + 12 + k] <= obs[18 * m + 15 + k]))
                return fail(CPF_E_ARG, "obstacle %d: p_min > p_max", m);
    return CPF_OK;
}

cpf_status check_problem(const cpf_problem *p, int dof) {
    if (!p) return fail(CPF_E_ARG, "problem is NULL");
    if (p->T < 1 || p->K < 1) return fail(CPF_E_ARG, "T=%d K=%d must be >= 1", p->T, p->K);
    if (p->K > MAX_K) return fail(CPF_E_UNSUPPORTED, "K=%d exceeds %d", p->K, MAX_K);
    if (p->T > (1 << 24)) return fail(CPF_E_UNSUPPORTED, "T=%d too large", p->T);
    if (p->mem != CPF_MEM_HOST && p->mem != CPF_MEM_DEVICE) return fail(CPF_E_ARG, "mem %d", p->mem);
    if (p->mem == CPF_MEM_DEVICE) {   // device values are checked on the device (stage_kernel)
        if (!p->targets || !p->cand_f32) return fail(CPF_E_ARG, "device inputs need targets and cand_f32");
    } else {
        if (!p->targets || (!p->cand && !p->cand_f32)) return fail(CPF_E_ARG, "targets / cand is NULL");
        if (!all_finite(p->targets, (size_t)p->T * 12)) return fail(CPF_E_ARG, "targets not finite");
        const size_t n = (size_t)p->K * p->T * dof;
        if (p->cand_f32) {
            for (size_t i = 0; i < n; ++i)
                if (!std::isfinite(p->cand_f32[i])) return fail(CPF_E_ARG, "cand_f32 not finite");
        } else if (!all_finite(p->cand, n)) {
            return fail(CPF_E_ARG, "cand not finite");
        }
    }
    if (p->node_pen) {
        for (size_t i = 0; i < (size_t)p->T * p->K; ++i)
            if (!(std::fabs(p->node_pen[i]) <= 1e30))
                return fail(CPF_E_ARG, "node_pen must be finite with |value| <= 1e30");
    }
    return check_obstacles(p->n_obstacles, p->obstacles);
}

cpf_status check_opts(const cpf_opts *o) {
    if (!o) return fail(CPF_E_ARG, "opts is NULL");
    const double v[7] = {o->w_pose, o->w_smooth, o->lambda0, o->lambda_min, o->lambda_max,
                         o->limit_margin, o->limit_penalty};
    if (!all_finite(v, 7)) return fail(CPF_E_ARG, "options not finite");
    if (!(std::fabs(o->limit_penalty) <= 1e30) || !(o->limit_margin >= 0))
        return fail(CPF_E_ARG, "limit_penalty / limit_margin out of range");
    if (o->w_pose < 0 || o->w_smooth < 0) return fail(CPF_E_ARG, "negative weight");
    if (!(o->lambda_min > 0) || !(o->lambda_min <= o->lambda0) || !(o->lambda0 <= o->lambda_max))
        return fail(CPF_E_ARG, "need 0 < lambda_min <= lambda0 <= lambda_max");
    if (o->prec != CPF_MIXED && o->prec != CPF_FP64) return fail(CPF_E_ARG, "prec %d", o->prec);
    if (o->iters < 0 || o->refine_steps < 0 || o->refine_steps > 8)
        return fail(CPF_E_ARG, "iters / refine_steps out of range");
    if (o->schedule != 0 && o->schedule != 1) return fail(CPF_E_ARG, "schedule %d", o->schedule);
    const double tv[3] = {o->valid_pos_m, o->valid_rot_rad, o->valid_step_rad};
    if (!all_finite(tv, 3) || tv[0] < 0 || tv[1] < 0 || tv[2] < 0)
        return fail(CPF_E_ARG, "validity thresholds must be finite and >= 0");
    const double cv[3] = {o->coll_margin, o->w_coll, o->coll_penalty};
    if (!all_finite(cv, 3) || cv[0] < 0 || cv[1] < 0 || !(std::fabs(cv[2]) <= 1e30))
        return fail(CPF_E_ARG, "collision options out of range");
    const double pv[2] = {o->limit_margin_m, o->valid_step_m};
    if (!all_finite(pv, 2) || pv[0] < 0 || pv[1] < 0)
        return fail(CPF_E_ARG, "prismatic margin / step threshold must be finite and >= 0");
    return CPF_OK;
}

// Host image of the device descriptor of an arena.
static void fill_desc(cpf_plan *p, bool has_extra) {
    DevPlan &D = p->desc;
    memset(&D, 0, sizeof(D));
    D.T = p->T;
    D.K = p->K;
    D.has_extra = has_extra ? 1 : 0;
    D.prec = p->opts.prec;
    D.refine_steps = p->opts.refine_steps;
    D.w_p = p->opts.w_pose;
    D.w_s = p->opts.w_smooth;
    D.lam0 = p->opts.lambda0;
    D.lam_min = p->opts.lambda_min;
    D.lam_max = p->opts.lambda_max;
    D.margin = p->opts.limit_margin;
    D.margin_p = p->opts.limit_margin_m;
    D.penalty = p->opts.limit_penalty;
    D.schedule = p->opts.schedule;
    D.prism = (int32_t)p->robot.prism;
    D.dof = p->robot.dof;
    D.vtol[0] = p->opts.valid_pos_m;
    D.vtol[1] = p->opts.valid_rot_rad;
    D.vtol[2] = p->opts.valid_step_rad;
    D.vtol[3] = p->opts.valid_step_m;
    D.has_coll = p->robot.has_caps ? 1 : 0;
    D.n_obs = p->n_obs;
    D.coll_margin = p->opts.coll_margin;
    D.w_coll = p->opts.w_coll;
    D.coll_penalty = p->opts.coll_penalty;
    const HostRobot &r = p->robot;
    for (int i = 0; i < r.dof; ++i)
        for (int c = 0; c < 7; ++c) {
            D.cap[i][c] = r.cap[i][c];
            D.capf[i][c] = (float)r.cap[i][c];
        }
    for (int i = 0; i < r.dof; ++i) {
        D.a[i] = r.a[i]; D.d[i] = r.d[i]; D.ca[i] = r.ca[i]; D.sa[i] = r.sa[i]; D.off[i] = r.off[i];
        D.lo[i] = r.lo[i]; D.hi[i] = r.hi[i];
        D.af[i] = (float)r.a[i]; D.df[i] = (float)r.d[i]; D.caf[i] = (float)r.ca[i];
        D.saf[i] = (float)r.sa[i]; D.offf[i] = (float)r.off[i];
    }
    char *b = p->arena;
    const Layout &L = p->L;
    set_dev_ptr(D.cand, b + L.cand);
    set_dev_ptr(D.extra, has_extra ? b + L.extra : nullptr);
    set_dev_ptr(D.bp, b + L.bp);
    set_dev_ptr(D.pen, b + L.pen);
    set_dev_ptr(D.topk, b + L.topk);
    set_dev_ptr(D.topc, b + L.topc);
    set_dev_ptr(D.path, b + L.path);
    set_dev_ptr(D.dp_out, b + L.dp_out);
    set_dev_ptr(D.targets, b + L.targets);
    set_dev_ptr(D.xi, b + L.xi);
    set_dev_ptr(D.xt, b + L.xt);
    set_dev_ptr(D.A, b + L.A);
    set_dev_ptr(D.g, b + L.g);
    set_dev_ptr(D.cr, b + L.cr);
    set_dev_ptr(D.dx, b + L.dx);
    set_dev_ptr(D.rb, b + L.rb);
    set_dev_ptr(D.st, b + L.st);
    set_dev_ptr(D.report, b + L.report);
    set_dev_ptr(D.xv, b + L.xv);
    set_dev_ptr(D.obs, b + L.obs);
    set_dev_ptr(D.cpen, b + L.cpen);
    set_dev_ptr(D.rr, b + L.rr);
    set_dev_ptr(D.rt, b + L.rt);
}

// A plan of T waypoints and K candidates with an arena from the pool, its
// descriptor and initial LM state uploaded on s; no problem data yet.
// Every array the descriptor points at lies inside the plan's arena, at its
// layout offset, with the extent its shape needs (recomputed here from T, K,
// the obstacle count and the flags, independently of make_layout's
// arithmetic), and the descriptor itself sits after the last array.
static bool desc_in_arena(const cpf_plan *p, bool has_extra) {
    const char *a = p->arena;
    const size_t end = p->L.total;
    const size_t t = (size_t)p->T, k = (size_t)p->K, d = sizeof(double);
    const size_t nj = (size_t)p->robot.dof, ntri = nj * (nj + 1) / 2;
    const DevPlan &D = p->desc;
    struct Span { const void *ptr; size_t bytes; };
    const Span spans[] = {
        {(const void *)D.cand, t * k * nj * sizeof(float)}, {(const void *)D.pen, t * k * d},
        {(const void *)D.bp, t * k * sizeof(uint16_t)}, {(const void *)D.topk, t * k * TOPM * sizeof(uint16_t)},
        {(const void *)D.topc, t * k * TOPM * d}, {(const void *)D.path, t * sizeof(int32_t)},
        {(const void *)D.dp_out, 8 * d}, {(const void *)D.targets, 12 * t * d}, {(const void *)D.xi, nj * t * d},
        {(const void *)D.xt, nj * t * d}, {(const void *)D.A, ntri * t * d}, {(const void *)D.g, nj * t * d},
        {(const void *)D.cr, cr_doubles(p->T, (int)nj) * d}, {(const void *)D.dx, nj * t * d},
        {(const void *)D.rb, nj * t * d}, {(const void *)D.st, sizeof(LMState)}, {(const void *)D.report, 8 * d},
        {(const void *)D.xv, nj * t * d}, {(const void *)D.rr, RROWS * t * d}, {(const void *)D.rt, RROWS * t * d},
        {(const void *)D.obs, (size_t)p->n_obs * 18 * d},
        {(const void *)D.cpen, p->robot.has_caps ? t * k * d : 0},
        {(const void *)D.extra, has_extra ? t * k * d : 0}};
    for (const Span &sp : spans) {
        if (sp.bytes == 0) continue;
        const char *q = (const char *)sp.ptr;
        if (q < a || q + sp.bytes > a + end) return false;
    }
    return (const char *)p->d_desc >= a + end;
}

// Fill a plan's host fields and descriptor for an arena already in p->arena
// and queue the descriptor, the initial LM state and the cleared input flag
// on s.
static hipError_t plan_setup(cpf_plan *p, cpf_ctx *ctx, const HostRobot &hr, int T, int K, bool has_extra, int n_obs,
                             const cpf_opts *opts, int32_t iters_target, hipStream_t s) {
    p->ctx = ctx;
    p->T = T;
    p->K = K;
    p->n_obs = n_obs;
    p->robot = hr;
    p->opts = *opts;
    p->L = make_layout(T, K, hr.dof, has_extra, n_obs, hr.has_caps);
    p->d_desc = (DevPlan *)(p->arena + p->L.total);
    fill_desc(p, has_extra);
    if (!desc_in_arena(p, has_extra)) return hipErrorInvalidValue;   // a layout mistake, caught on the host
    p->init = LMState{};
    p->init.lambda = opts->lambda0;
    p->init.nu = 2.0;
    p->init.iters_target = iters_target;
    hipError_t e = hipMemcpyAsync(p->arena + p->L.st, &p->init, sizeof(LMState), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(p->d_desc, &p->desc, sizeof(DevPlan), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(input_flag(p), 0, sizeof(int), s);
    return e;
}

cpf_status plan_alloc(cpf_ctx *ctx, const HostRobot &hr, int T, int K, bool has_extra, int n_obs,
                      const cpf_opts *opts, int32_t iters_target, hipStream_t s, cpf_plan **out) {
    const uint64_t cls = plan_class_bytes(T, K, hr.dof, has_extra, n_obs, hr.has_caps);
    void *mem = nullptr;
    cpf_status st = arena_get(ctx, cls, &mem);
    if (st != CPF_OK) return st;
    std::unique_ptr<cpf_plan> p(new cpf_plan());
    p->bytes = cls;
    p->arena = (char *)mem;
    const hipError_t e = plan_setup(p.get(), ctx, hr, T, K, has_extra, n_obs, opts, iters_target, s);
    if (e != hipSuccess) {
        HIP_IGNORE(hipStreamSynchronize(s));
        arena_put(ctx, mem, cls);
        return fail(CPF_E_DEVICE, "upload failed: %s", hipGetErrorString(e));
    }
    *out = p.release();
    return CPF_OK;
}

// Queue the problem's inputs into a set-up plan on s: host arrays go up as
// they are into the upload region and a kernel converts them (or
// device-resident ones in place) into the device layout (candidates to
// float, joint-major; targets component-major); node costs and obstacles
// are copied.
static hipError_t plan_upload(cpf_plan *p, const cpf_problem *prob, hipStream_t s) {
    const int T = p->T, K = p->K, dof = p->robot.dof;
    const size_t n_cand = (size_t)T * K * dof;
    const bool f32 = prob->mem == CPF_MEM_DEVICE || prob->cand_f32 != nullptr;
    const void *cin = nullptr;
    const double *tin = nullptr;
    int *bad = nullptr;
    hipError_t e = hipSuccess;
    if (prob->mem == CPF_MEM_DEVICE) {   // checked on the device (the flag was cleared by plan_setup)
        cin = prob->cand_f32;
        tin = prob->targets;
        bad = input_flag(p);
    } else {
        char *raw = p->arena + p->L.raw;
        const size_t toff = raw_targets_offset(T, K, dof, f32);
        e = hipMemcpyAsync(raw, f32 ? (const void *)prob->cand_f32 : (const void *)prob->cand,
                           n_cand * (f32 ? sizeof(float) : sizeof(double)), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(raw + toff, prob->targets, (size_t)12 * T * sizeof(double), hipMemcpyHostToDevice, s);
        cin = raw;
        tin = (const double *)(raw + toff);
    }
    if (e == hipSuccess)
        e = CPF_BY_DOF(dof, stage_launch(cin, f32, tin, T, K, (float *)(p->arena + p->L.cand),
                                         (double *)(p->arena + p->L.targets), bad, s));
    if (e == hipSuccess && prob->node_pen)
        e = hipMemcpyAsync(p->arena + p->L.extra, prob->node_pen, (size_t)T * K * sizeof(double),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess && prob->n_obstacles > 0)
        e = hipMemcpyAsync(p->arena + p->L.obs, prob->obstacles, (size_t)prob->n_obstacles * 18 * sizeof(double),
                           hipMemcpyHostToDevice, s);
    return e;
}

cpf_status plan_create(cpf_ctx *ctx, const HostRobot &hr, const cpf_problem *prob,
                       const cpf_opts *opts, int32_t iters_target, hipStream_t s, cpf_plan **out) {
    cpf_plan *p = nullptr;
    cpf_status st = plan_alloc(ctx, hr, prob->T, prob->K, prob->node_pen != nullptr, prob->n_obstacles, opts,
                               iters_target, s, &p);
    if (st != CPF_OK) return st;
    const hipError_t e = plan_upload(p, prob, s);
    if (e != hipSuccess) {
        HIP_IGNORE(hipStreamSynchronize(s));
        plan_destroy(p);
        return fail(CPF_E_DEVICE, "upload failed: %s", hipGetErrorString(e));
    }
    *out = p;
    return CPF_OK;
}

int *input_flag(cpf_plan *p) { return (int *)(p->arena + p->L.report + 7 * sizeof(double)); }

bool input_flag_set(const double *report) {
    int v;
    memcpy(&v, &report[7], sizeof(int));
    return v != 0;
}

void plan_destroy(cpf_plan *p) {
    if (!p) return;
    if (p->arena) arena_put(p->ctx, p->arena, p->bytes);
    delete p;
}

cpf_status read_plan(cpf_plan *p, hipStream_t s, const LMState *state_dev, PlanReadback *rb,
                     double *xi_out, int32_t *path_out, double *xv_out) {
    std::vector<double> xs, vs;
    // the LM state, report, search output and path lead the arena (make_layout)
    const Layout &L = p->L;
    const size_t head = L.path + (path_out ? (size_t)p->T * sizeof(int32_t) : 0);
    std::vector<char> hb(head);
    HIP_TRY(hipMemcpyAsync(hb.data(), p->arena, head, hipMemcpyDeviceToHost, s));
    if (state_dev) HIP_TRY(hipMemcpyAsync(&rb->st, state_dev, sizeof(LMState), hipMemcpyDeviceToHost, s));
    if (xi_out) {
        xs.resize((size_t)p->robot.dof * p->T);
        HIP_TRY(hipMemcpyAsync(xs.data(), p->arena + p->L.xi, xs.size() * sizeof(double),
                               hipMemcpyDeviceToHost, s));
    }
    if (xv_out) {
        vs.resize((size_t)p->robot.dof * p->T);
        HIP_TRY(hipMemcpyAsync(vs.data(), p->arena + p->L.xv, vs.size() * sizeof(double),
                               hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    if (!state_dev) memcpy(&rb->st, hb.data() + L.st, sizeof(LMState));
    memcpy(rb->report, hb.data() + L.report, sizeof(rb->report));
    memcpy(rb->dp_out, hb.data() + L.dp_out, sizeof(rb->dp_out));
    if (path_out) memcpy(path_out, hb.data() + L.path, (size_t)p->T * sizeof(int32_t));
    if (xi_out) soa_to_rows(xs.data(), p->T, p->robot.dof, xi_out);
    if (xv_out && rb->st.n_valid > 0) soa_to_rows(vs.data(), p->T, p->robot.dof, xv_out);
    return CPF_OK;
}

void soa_to_rows(const double *soa, int T, int dof, double *rows) {
    for (int t = 0; t < T; ++t)
        for (int j = 0; j < dof; ++j) rows[(size_t)t * dof + j] = soa[(size_t)j * T + t];
}

void report_from(const LMState &ls, const double *report, cpf_lm_report *rep) {
    rep->cost0 = ls.cost0;
    rep->cost = ls.cost;
    rep->lambda = ls.lambda;
    rep->grad_inf = ls.grad_inf;
    rep->n_accepted = ls.n_acc;
    rep->iters_done = ls.iters_done;
    rep->max_pos_err_m = report[0];
    rep->max_rot_err_rad = report[1];
    rep->mjac = report[2];
    rep->n_valid = ls.n_valid;
    rep->first_valid = ls.first_valid;
    rep->pose_steps = ls.pose_steps;
    rep->diff_steps = ls.diff_steps;
    rep->valid_length = ls.valid_length;
    rep->min_self_dist_m = report[3];
    rep->min_env_dist_m = report[4];
}

void fill_report(const PlanReadback &rb, cpf_lm_report *rep) { report_from(rb.st, rb.report, rep); }

}  // namespace cpf

using namespace cpf;

// ---------------------------------------------------------------------------
// Public API (synchronous part)
// ---------------------------------------------------------------------------

extern "C" {

void cpf_opts_default(cpf_opts *o) {
    if (!o) return;
    o->w_pose = 1.0;
    o->w_smooth = 0.1;
    o->lambda0 = 1e-3;
    o->lambda_min = 1e-10;
    o->lambda_max = 1e10;
    o->limit_margin = 1.5 * 3.14159265358979323846 / 180.0;
    o->limit_penalty = 10.0;
    o->iters = 50;
    o->prec = CPF_MIXED;
    o->refine_steps = 1;
    o->schedule = 0;
    o->valid_pos_m = 1e-4;
    o->valid_rot_rad = 0.1 * 3.14159265358979323846 / 180.0;
    o->valid_step_rad = 7.0 * 3.14159265358979323846 / 180.0;
    o->coll_margin = 0.02;
    o->w_coll = 1.0;
    o->coll_penalty = 100.0;
    o->limit_margin_m = 0.03;
    o->valid_step_m = 0.02;
}

const char *cpf_last_error(void) { return cpf::g_err.c_str(); }

cpf_status cpf_ctx_create(int device, uint64_t mem_budget_bytes, cpf_ctx **out) {
    if (!out) return fail(CPF_E_ARG, "out is NULL");
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(CPF_E_ARG, "device %d of %d", device, n);
    HIP_TRY(hipSetDevice(device));
    cpf_status st = scratch_setup(device);
    if (st != CPF_OK) return st;
    std::unique_ptr<cpf_ctx> c(new cpf_ctx());
    c->device = device;
    c->budget = mem_budget_bytes ? mem_budget_bytes : (uint64_t)64 << 30;
    HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    *out = c.release();
    return CPF_OK;
}

void cpf_ctx_destroy(cpf_ctx *ctx) {
    if (!ctx) return;
    server_stop_and_join(ctx);
    HIP_IGNORE(hipSetDevice(ctx->device));
    cpf_ctx_profile(ctx, 0);
    for (hipEvent_t ev : ctx->ev_free) HIP_IGNORE(hipEventDestroy(ev));
    ctx->ev_free.clear();
    if (ctx->stream) HIP_IGNORE(hipStreamSynchronize(ctx->stream));
    pool_clear(ctx);
    if (ctx->stream) HIP_IGNORE(hipStreamDestroy(ctx->stream));
    delete ctx;
}

uint64_t cpf_ctx_bytes_in_use(const cpf_ctx *ctx) { return ctx ? ctx->used.load() : 0; }

cpf_status cpf_plan_init(cpf_ctx *ctx, const cpf_robot *robot, const cpf_problem *prob,
                         const cpf_opts *opts, cpf_plan **out) {
    if (!ctx || !out) return fail(CPF_E_ARG, "ctx / out is NULL");
    HostRobot hr;
    cpf_status st;
    if ((st = check_robot(robot, &hr)) != CPF_OK) return st;
    if ((st = check_plan_robot(hr)) != CPF_OK) return st;
    if ((st = check_problem(prob, hr.dof)) != CPF_OK) return st;
    cpf_opts o;
    cpf_opts_default(&o);
    if (opts) o = *opts;
    if ((st = check_opts(&o)) != CPF_OK) return st;
    HIP_TRY(hipSetDevice(ctx->device));
    cpf_plan *p = nullptr;
    if ((st = plan_create(ctx, hr, prob, &o, 0, ctx->stream, &p)) != CPF_OK) return st;
    int bad = 0;
    hipError_t e = hipSuccess;
    if (prob->mem == CPF_MEM_DEVICE)
        e = hipMemcpyAsync(&bad, input_flag(p), sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        plan_destroy(p);
        return fail(CPF_E_DEVICE, "plan upload: %s", hipGetErrorString(e));
    }
    if (bad) {
        plan_destroy(p);
        return fail(CPF_E_ARG, "a device-resident target or candidate value is not finite");
    }
    *out = p;
    return CPF_OK;
}

void cpf_plan_free(cpf_plan *plan) {
    if (!plan) return;
    HIP_IGNORE(hipSetDevice(plan->ctx->device));
    HIP_IGNORE(hipStreamSynchronize(plan->ctx->stream));
    plan_destroy(plan);
}

cpf_status cpf_fk_batch(cpf_ctx *ctx, const cpf_robot *robot, int64_t M, int32_t prec,
                        const void *q_dev, void *pose_dev, void *jac_dev, void *hip_stream) {
    if (!ctx) return fail(CPF_E_ARG, "ctx is NULL");
    HostRobot hr;
    cpf_status st;
    if ((st = check_robot(robot, &hr)) != CPF_OK) return st;
    if (M < 0) return fail(CPF_E_ARG, "M=%lld", (long long)M);
    if (prec != CPF_F32 && prec != CPF_F64) return fail(CPF_E_ARG, "prec %d", prec);
    if (M > 0 && (!q_dev || !pose_dev)) return fail(CPF_E_ARG, "q / pose pointer is NULL");
    if ((uint64_t)M > ((uint64_t)1 << 38)) return fail(CPF_E_ARG, "M too large");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_TRY(timed(ctx, KIND_FK, s,
                  [&] { return CPF_BY_DOF(hr.dof, fk_batch_launch(hr, M, prec, q_dev, pose_dev, jac_dev, s)); }));
    return CPF_OK;
}

cpf_status cpf_coll_batch(cpf_ctx *ctx, const cpf_robot *robot, int32_t n_obstacles, const double *obstacles_dev,
                          int64_t M, int32_t prec, const void *q_dev, void *dist_dev, void *grad_dev,
                          void *hip_stream) {
    if (!ctx) return fail(CPF_E_ARG, "ctx is NULL");
    HostRobot hr;
    cpf_status st;
    if ((st = check_robot(robot, &hr)) != CPF_OK) return st;
    if (!hr.has_caps) return fail(CPF_E_ARG, "robot has no capsules");
    if (n_obstacles < 0 || n_obstacles > MAX_OBS)
        return fail(CPF_E_ARG, "n_obstacles=%d must be in [0, %d]", n_obstacles, MAX_OBS);
    if (n_obstacles > 0 && !obstacles_dev) return fail(CPF_E_ARG, "obstacles_dev is NULL");
    if (M < 0) return fail(CPF_E_ARG, "M=%lld", (long long)M);
    if (prec != CPF_F32 && prec != CPF_F64) return fail(CPF_E_ARG, "prec %d", prec);
    if (M > 0 && (!q_dev || !dist_dev)) return fail(CPF_E_ARG, "q / dist pointer is NULL");
    if ((uint64_t)M > ((uint64_t)1 << 38)) return fail(CPF_E_ARG, "M too large");
    HIP_TRY(hipSetDevice(ctx->device));
    HostCaps caps;
    memcpy(caps.v, hr.cap, sizeof(caps.v));
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_TRY(timed(ctx, KIND_FK, s, [&] {
        return CPF_BY_DOF(hr.dof,
                          coll_batch_launch(hr, caps, n_obstacles, obstacles_dev, M, prec, q_dev, dist_dev, grad_dev, s));
    }));
    return CPF_OK;
}

cpf_status cpf_dp_search(cpf_plan *plan, int32_t *path_out, double *best_out, double *mjac_out) {
    if (!plan) return fail(CPF_E_ARG, "plan is NULL");
    cpf_ctx *ctx = plan->ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(search_launch(ctx, plan->d_desc, 1, plan->K, plan->T, plan->lists_valid, plan->robot.has_caps,
                          dof_bit(plan->robot.dof), ctx->stream));
    PlanReadback rb;
    cpf_status st = read_plan(plan, ctx->stream, nullptr, &rb, nullptr, path_out, nullptr);
    if (st != CPF_OK) return st;
    plan->searched = true;
    plan->lists_valid = true;
    plan->seed_steps[0] = rb.dp_out[3];
    plan->seed_steps[1] = rb.dp_out[4];
    if (best_out) *best_out = rb.dp_out[0];
    if (mjac_out) *mjac_out = rb.dp_out[1];
    return CPF_OK;
}

cpf_status cpf_dp_needs_research(const cpf_plan *plan, int32_t *out) {
    if (!plan || !out) return fail(CPF_E_ARG, "plan / out is NULL");
    if (!plan->searched) return fail(CPF_E_STATE, "the plan has not been searched");
    *out = (plan->seed_steps[0] > CPF_RESEARCH_MJAC_RAD || plan->seed_steps[1] > CPF_RESEARCH_MJAC_M) ? 1 : 0;
    return CPF_OK;
}

cpf_status cpf_dp_seed_steps(const cpf_plan *plan, double *rev_rad_out, double *pri_m_out) {
    if (!plan) return fail(CPF_E_ARG, "plan is NULL");
    if (!plan->searched) return fail(CPF_E_STATE, "the plan has not been searched");
    if (rev_rad_out) *rev_rad_out = plan->seed_steps[0];
    if (pri_m_out) *pri_m_out = plan->seed_steps[1];
    return CPF_OK;
}

static_assert(TOPM == CPF_TOPM, "list length of the ABI and the kernels");

cpf_status cpf_dp_lists(const cpf_plan *plan, int32_t t0, int32_t nt, uint16_t *idx_out, double *c_out) {
    if (!plan || (!idx_out && !c_out)) return fail(CPF_E_ARG, "plan / both outputs NULL");
    if (!plan->lists_valid) return fail(CPF_E_STATE, "the plan has no current search lists");
    const int T = plan->T, K = plan->K;
    if (t0 < 1 || nt < 0 || (int64_t)t0 + nt > T) return fail(CPF_E_ARG, "waypoints %d + %d outside [1, %d)", t0, nt, T);
    if (nt == 0) return CPF_OK;
    cpf_ctx *ctx = plan->ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    // device layout: indices as pairs in 32-bit words [T][TOPM / 2][K], values [T][TOPM][K]
    std::vector<uint32_t> w((size_t)nt * (TOPM / 2) * K);
    std::vector<double> c((size_t)nt * TOPM * K);
    hipStream_t s = ctx->stream;
    HIP_TRY(hipMemcpyAsync(w.data(), plan->arena + plan->L.topk + (size_t)t0 * (TOPM / 2) * K * sizeof(uint32_t),
                           w.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(c.data(), plan->arena + plan->L.topc + (size_t)t0 * TOPM * K * sizeof(double),
                           c.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int t = 0; t < nt; ++t)
        for (int k = 0; k < K; ++k)
            for (int m = 0; m < TOPM; ++m) {
                const size_t o = ((size_t)t * K + k) * TOPM + m;
                if (idx_out) idx_out[o] = (uint16_t)(w[((size_t)t * (TOPM / 2) + m / 2) * K + k] >> (16 * (m & 1)));
                if (c_out) c_out[o] = c[((size_t)t * TOPM + m) * K + k];
            }
    return CPF_OK;
}

cpf_status cpf_plan_append(cpf_plan *plan, int32_t K_add, const double *cand_add, const double *node_pen_add) {
    if (!plan || !cand_add) return fail(CPF_E_ARG, "plan / cand_add is NULL");
    if (K_add < 1) return fail(CPF_E_ARG, "K_add=%d must be >= 1", K_add);
    const int T = plan->T, K0 = plan->K, K2 = K0 + K_add, dof = plan->robot.dof;
    if (K2 > MAX_K) return fail(CPF_E_UNSUPPORTED, "K=%d + %d exceeds %d", K0, K_add, MAX_K);
    if (!all_finite(cand_add, (size_t)K_add * T * dof)) return fail(CPF_E_ARG, "cand_add not finite");
    if (node_pen_add)
        for (size_t i = 0; i < (size_t)T * K_add; ++i)
            if (!(std::fabs(node_pen_add[i]) <= 1e30))
                return fail(CPF_E_ARG, "node_pen_add must be finite with |value| <= 1e30");
    cpf_ctx *ctx = plan->ctx;
    hipStream_t s = ctx->stream;
    HIP_TRY(hipSetDevice(ctx->device));
    const bool old_extra = plan->desc.has_extra != 0;
    const bool has_extra = old_extra || node_pen_add != nullptr;
    // A plan searched before has current penalties and lists to merge into;
    // otherwise the next search computes them for all candidates.
    const bool merge = plan->lists_valid;
    cpf_plan *np = nullptr;
    cpf_status st = plan_alloc(ctx, plan->robot, T, K2, has_extra, plan->n_obs, &plan->opts, plan->init.iters_target,
                               s, &np);
    if (st != CPF_OK) return st;
    char *a2 = np->arena;
    const char *a1 = plan->arena;
    const Layout &L1 = plan->L, &L2 = np->L;
    // 1. the new candidates go up through the raw region and are converted
    //    into columns K0.. of the new candidate array
    hipError_t e = hipMemcpyAsync(a2 + L2.raw, cand_add, (size_t)K_add * T * dof * sizeof(double),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = CPF_BY_DOF(dof, stage_append_launch((const double *)(a2 + L2.raw), T, K_add, K2, K0,
                                                (float *)(a2 + L2.cand), s));
    // 2. kept on the device: candidates, node costs, penalties, predecessor
    //    lists and targets (the lists overwrite the raw region, in stream order)
    auto cols = [&](size_t off2, size_t off1, size_t elem, int rows) {
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(a2 + off2, (size_t)K2 * elem, a1 + off1, (size_t)K0 * elem, (size_t)K0 * elem,
                                 (size_t)rows, hipMemcpyDeviceToDevice, s);
    };
    cols(L2.cand, L1.cand, sizeof(float), T * dof);
    if (merge) {
        cols(L2.pen, L1.pen, sizeof(double), T);
        cols(L2.topk, L1.topk, sizeof(uint32_t), T * TOPM / 2);   // [T][TOPM / 2][K] index pairs
        cols(L2.topc, L1.topc, sizeof(double), T * TOPM);         // [T][TOPM][K] values
        if (plan->robot.has_caps) cols(L2.cpen, L1.cpen, sizeof(double), T);
    }
    if (has_extra) {
        if (old_extra) cols(L2.extra, L1.extra, sizeof(double), T);
        else if (e == hipSuccess)
            e = hipMemset2DAsync(a2 + L2.extra, (size_t)K2 * sizeof(double), 0, (size_t)K0 * sizeof(double), T, s);
        if (e == hipSuccess && node_pen_add)
            e = hipMemcpy2DAsync(a2 + L2.extra + (size_t)K0 * sizeof(double), (size_t)K2 * sizeof(double),
                                 node_pen_add, (size_t)K_add * sizeof(double), (size_t)K_add * sizeof(double),
                                 (size_t)T, hipMemcpyHostToDevice, s);
        else if (e == hipSuccess)
            e = hipMemset2DAsync(a2 + L2.extra + (size_t)K0 * sizeof(double), (size_t)K2 * sizeof(double), 0,
                                 (size_t)K_add * sizeof(double), T, s);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(a2 + L2.targets, a1 + L1.targets, (size_t)12 * T * sizeof(double),
                           hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && plan->n_obs > 0)
        e = hipMemcpyAsync(a2 + L2.obs, a1 + L1.obs, (size_t)plan->n_obs * 18 * sizeof(double),
                           hipMemcpyDeviceToDevice, s);
    // 3. penalties and lists of the new nodes; the old nodes' lists merged
    if (e == hipSuccess && merge)
        e = timed(ctx, KIND_DPL, s, [&] {
            return CPF_BY_DOF(dof, dp_append_launch(np->d_desc, K0, K2, T, plan->robot.has_caps, s));
        });
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        HIP_IGNORE(hipStreamSynchronize(s));
        plan_destroy(np);
        return fail(CPF_E_DEVICE, "append: %s", hipGetErrorString(e));
    }
    // The caller's handle takes the new arena; the old one returns to the pool.
    std::swap(plan->arena, np->arena);
    std::swap(plan->L, np->L);
    std::swap(plan->bytes, np->bytes);
    std::swap(plan->desc, np->desc);
    std::swap(plan->d_desc, np->d_desc);
    std::swap(plan->K, np->K);
    plan_destroy(np);
    plan->searched = false;
    plan->lists_valid = merge;
    return CPF_OK;
}

cpf_status cpf_lm_refine(cpf_plan *plan, int32_t iters, double *xi_out, cpf_lm_report *rep) {
    if (!plan) return fail(CPF_E_ARG, "plan is NULL");
    if (iters < 0) return fail(CPF_E_ARG, "iters=%d", iters);
    if (!plan->searched) return fail(CPF_E_STATE, "lm_refine before dp_search");
    cpf_ctx *ctx = plan->ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(timed(ctx, KIND_LM, ctx->stream,
                  [&] {
                      return CPF_BY_DOF(plan->robot.dof, lm_launch(plan->d_desc, 1, plan->opts.prec, plan->opts.schedule,
                                                                   plan_geo(plan->robot), iters, ctx->stream));
                  }));
    HIP_TRY(timed(ctx, KIND_EVAL, ctx->stream, [&] {
        return CPF_BY_DOF(plan->robot.dof, eval_launch(plan->d_desc, 1, 0, plan_geo(plan->robot), ctx->stream));
    }));
    PlanReadback rb;
    cpf_status st = read_plan(plan, ctx->stream, nullptr, &rb, xi_out, nullptr, nullptr);
    if (st != CPF_OK) return st;
    if (rep) fill_report(rb, rep);
    if (rb.st.status != 0) return fail(CPF_E_NUMERIC, "non-positive pivot in the block solve");
    return CPF_OK;
}

cpf_status cpf_plan_solve(cpf_plan *plan, int32_t *path_out, double *best_out, double *xi_out,
                          cpf_lm_report *rep) {
    if (!plan) return fail(CPF_E_ARG, "plan is NULL");
    cpf_ctx *ctx = plan->ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const bool coll = plan->robot.has_caps;
    const int dof = plan->robot.dof;
    HIP_TRY(search_launch(ctx, plan->d_desc, 1, plan->K, plan->T, false, coll, dof_bit(dof), s));
    plan->lists_valid = true;
    HIP_TRY(timed(ctx, KIND_LM, s, [&] {
        return CPF_BY_DOF(dof, lm_launch(plan->d_desc, 1, plan->opts.prec, plan->opts.schedule, plan_geo(plan->robot),
                                         plan->opts.iters, s));
    }));
    HIP_TRY(timed(ctx, KIND_EVAL, s,
                  [&] { return CPF_BY_DOF(dof, eval_launch(plan->d_desc, 1, 0, plan_geo(plan->robot), s)); }));
    PlanReadback rb;
    cpf_status st = read_plan(plan, s, nullptr, &rb, xi_out, path_out, nullptr);
    if (st != CPF_OK) return st;
    plan->searched = true;
    plan->seed_steps[0] = rb.dp_out[3];
    plan->seed_steps[1] = rb.dp_out[4];
    if (best_out) *best_out = rb.dp_out[0];
    if (rep) fill_report(rb, rep);
    if (rb.st.status != 0) return fail(CPF_E_NUMERIC, "non-positive pivot in the block solve");
    return CPF_OK;
}

cpf_status cpf_solve_static(cpf_ctx *ctx, const cpf_robot *robot, const cpf_problem *prob, const cpf_opts *opts,
                            int32_t *path_out, double *best_out, double *xi_out, cpf_lm_report *rep) {
    if (!ctx) return fail(CPF_E_ARG, "ctx is NULL");
    HostRobot hr;
    cpf_status st;
    if ((st = check_robot(robot, &hr)) != CPF_OK) return st;
    if ((st = check_plan_robot(hr)) != CPF_OK) return st;
    if ((st = check_problem(prob, hr.dof)) != CPF_OK) return st;
    cpf_opts o;
    cpf_opts_default(&o);
    if (opts) o = *opts;
    if ((st = check_opts(&o)) != CPF_OK) return st;
    const int T = prob->T, K = prob->K;
    const bool has_extra = prob->node_pen != nullptr;
    const int dof = hr.dof;
    const Layout L = make_layout(T, K, dof, has_extra, prob->n_obstacles, hr.has_caps);
    const uint64_t need = L.total + align256(sizeof(DevPlan));
    if (need > SCRATCH_BYTES)
        return fail(CPF_E_NOMEM, "T=%d K=%d needs %llu bytes of working memory; the static scratch holds %llu", T, K,
                    (unsigned long long)need, (unsigned long long)SCRATCH_BYTES);
    char head[1024];   // LM state, report, search output: the arena's first bytes
    if (L.path > sizeof(head)) return fail(CPF_E_STATE, "arena head of %zu bytes", L.path);
    HIP_TRY(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> lk(g_scratch_mu[ctx->device]);
    char *base = (char *)g_scratch_ptr[ctx->device];
    if (!base) return fail(CPF_E_STATE, "no static scratch on device %d", ctx->device);
    cpf_plan p;   // on the stack, its arena the device's scratch
    p.arena = base;
    hipStream_t s = ctx->stream;
    const bool coll = hr.has_caps;
    const int geo = plan_geo(hr);
    hipError_t e = plan_setup(&p, ctx, hr, T, K, has_extra, prob->n_obstacles, &o, 0, s);
    if (e == hipSuccess) e = plan_upload(&p, prob, s);
    if (e == hipSuccess) e = CPF_BY_DOF(dof, dp_lists_launch(p.d_desc, 1, K, T, coll, s));
    if (e == hipSuccess) e = CPF_BY_DOF(dof, dp_stages_launch(p.d_desc, 1, K, s));
    if (e == hipSuccess) e = CPF_BY_DOF(dof, lm_launch(p.d_desc, 1, o.prec, o.schedule, geo, o.iters, s));
    if (e == hipSuccess) e = CPF_BY_DOF(dof, eval_launch(p.d_desc, 1, 0, geo, s));
    if (e == hipSuccess) e = hipMemcpyAsync(head, base, L.path, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && path_out)
        e = hipMemcpyAsync(path_out, base + L.path, (size_t)T * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && xi_out) {   // rows [T][dof] into the trial-point area, then straight to the caller
        e = CPF_BY_DOF(dof, soa_rows_launch((const double *)(base + L.xi), T, (double *)(base + L.xt), s));
        if (e == hipSuccess)
            e = hipMemcpyAsync(xi_out, base + L.xt, (size_t)T * dof * sizeof(double), hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        HIP_IGNORE(hipStreamSynchronize(s));
        return fail(CPF_E_DEVICE, "static solve: %s", hipGetErrorString(e));
    }
    LMState ls;
    double report[8], dp_out[8];
    memcpy(&ls, head + L.st, sizeof(ls));
    memcpy(report, head + L.report, sizeof(report));
    memcpy(dp_out, head + L.dp_out, sizeof(dp_out));
    if (input_flag_set(report)) return fail(CPF_E_ARG, "a device-resident target or candidate value is not finite");
    if (best_out) *best_out = dp_out[0];
    if (rep) report_from(ls, report, rep);
    if (ls.status != 0) return fail(CPF_E_NUMERIC, "non-positive pivot in the block solve");
    return CPF_OK;
}

cpf_status cpf_lm_latest_valid(cpf_plan *plan, double *xi_out) {
    if (!plan || !xi_out) return fail(CPF_E_ARG, "plan / xi_out is NULL");
    if (!plan->opts.schedule) return fail(CPF_E_STATE, "plan was not created with opts.schedule = 1");
    cpf_ctx *ctx = plan->ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    PlanReadback rb;
    cpf_status st = read_plan(plan, ctx->stream, nullptr, &rb, nullptr, nullptr, xi_out);
    if (st != CPF_OK) return st;
    if (!plan->searched || rb.st.seeded == 0 || rb.st.n_valid == 0)
        return fail(CPF_E_STATE, "no valid trajectory yet");
    return CPF_OK;
}

cpf_status cpf_solve_batch(cpf_ctx *ctx, int32_t nplans, const cpf_robot *robots,
                           const cpf_problem *probs, const cpf_opts *opts, cpf_result *results) {
    if (!ctx || nplans < 0 || (nplans > 0 && (!robots || !probs || !results)))
        return fail(CPF_E_ARG, "bad batch arguments");
    cpf_opts o;
    cpf_opts_default(&o);
    if (opts) o = *opts;
    cpf_status st;
    if ((st = check_opts(&o)) != CPF_OK) return st;
    std::vector<HostRobot> hrs(nplans);
    for (int i = 0; i < nplans; ++i) {
        if ((st = check_robot(&robots[i], &hrs[i])) != CPF_OK) return st;
        if ((st = check_plan_robot(hrs[i])) != CPF_OK) return st;
        if ((st = check_problem(&probs[i], hrs[i].dof)) != CPF_OK) return st;
    }
    if (nplans == 0) return CPF_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    std::vector<cpf_plan *> plans;
    DevPlan *d_descs = nullptr;
    auto cleanup = [&]() {
        HIP_IGNORE(hipStreamSynchronize(ctx->stream));
        if (d_descs) HIP_IGNORE(hipFree(d_descs));
        for (auto *p : plans) plan_destroy(p);
    };
    int maxK = 0, maxT = 0, dofs = 0;
    bool kinds[GEO_KINDS] = {false, false, false};   // geometry kinds present
    for (int i = 0; i < nplans; ++i) {
        kinds[plan_geo(hrs[i])] = true;
        dofs |= dof_bit(hrs[i].dof);
        cpf_plan *p = nullptr;
        if ((st = plan_create(ctx, hrs[i], &probs[i], &o, 0, ctx->stream, &p)) != CPF_OK) {
            cleanup();
            return st;
        }
        plans.push_back(p);
        maxK = std::max(maxK, probs[i].K);
        maxT = std::max(maxT, probs[i].T);
    }
    std::vector<DevPlan> host(nplans);
    for (int i = 0; i < nplans; ++i) host[i] = plans[i]->desc;
    hipError_t e = hipMalloc((void **)&d_descs, host.size() * sizeof(DevPlan));
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_descs, host.data(), host.size() * sizeof(DevPlan),
                           hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    const int64_t t0 = now_ns();
    if (e == hipSuccess)
        e = search_launch(ctx, d_descs, nplans, maxK, maxT, false, kinds[GEO_COLL], dofs, ctx->stream);
    if (e == hipSuccess)
        e = timed(ctx, KIND_LM, ctx->stream,
                  [&] {
                      hipError_t r = hipSuccess;
                      for (int dof = 7; dof <= 8; ++dof)
                          for (int c = 0; c < GEO_KINDS && r == hipSuccess; ++c)
                              if (kinds[c] && (dofs & dof_bit(dof)))
                                  r = CPF_BY_DOF(dof, lm_launch(d_descs, nplans, o.prec, o.schedule, c, o.iters,
                                                                ctx->stream));
                      return r;
                  });
    if (e == hipSuccess)
        e = timed(ctx, KIND_EVAL, ctx->stream,
                  [&] {
                      hipError_t r = hipSuccess;
                      for (int dof = 7; dof <= 8; ++dof)
                          for (int c = 0; c < GEO_KINDS && r == hipSuccess; ++c)
                              if (kinds[c] && (dofs & dof_bit(dof)))
                                  r = CPF_BY_DOF(dof, eval_launch(d_descs, nplans, 0, c, ctx->stream));
                      return r;
                  });
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    const int64_t t1 = now_ns();
    if (e != hipSuccess) {
        cleanup();
        return fail(CPF_E_DEVICE, "batch launch: %s", hipGetErrorString(e));
    }
    for (int i = 0; i < nplans; ++i) {
        PlanReadback rb;
        if ((st = read_plan(plans[i], ctx->stream, nullptr, &rb, results[i].xi, results[i].path,
                            results[i].xi_valid)) !=
            CPF_OK) {
            cleanup();
            return st;
        }
        fill_report(rb, &results[i].report);
        results[i].search_best = rb.dp_out[0];
        results[i].search_mjac = rb.dp_out[1];
        results[i].status = input_flag_set(rb.report) ? CPF_E_ARG : (rb.st.status != 0 ? CPF_E_NUMERIC : CPF_OK);
        results[i].t_submit_ns = t0;
        results[i].t_admit_ns = t0;
        results[i].t_search_done_ns = t1;
        results[i].t_done_ns = t1;
    }
    cleanup();
    return CPF_OK;
}

cpf_status cpf_batchopt(cpf_ctx *ctx, const cpf_robot *robot, const cpf_problem *prob,
                        const cpf_opts *opts, int32_t M, int32_t *idx_out, cpf_result *results) {
    if (!ctx || !idx_out || !results) return fail(CPF_E_ARG, "ctx / idx_out / results is NULL");
    HostRobot hr;
    cpf_status st;
    if ((st = check_robot(robot, &hr)) != CPF_OK) return st;
    if ((st = check_plan_robot(hr)) != CPF_OK) return st;
    if ((st = check_problem(prob, hr.dof)) != CPF_OK) return st;
    if (M < 1 || M > prob->K) return fail(CPF_E_ARG, "M=%d with K=%d", M, prob->K);
    cpf_opts o;
    cpf_opts_default(&o);
    if (opts) o = *opts;
    if ((st = check_opts(&o)) != CPF_OK) return st;
    HIP_TRY(hipSetDevice(ctx->device));
    // 1. the candidates' mjac on the device (the uploaded plan's penalty
    //    array is free until a search runs)
    const int T = prob->T, K = prob->K;
    cpf_plan *p = nullptr;
    if ((st = plan_create(ctx, hr, prob, &o, 0, ctx->stream, &p)) != CPF_OK) return st;
    std::vector<double> m(K);
    hipError_t e = CPF_BY_DOF(hr.dof, cand_mjac_launch((const float *)(p->arena + p->L.cand), T, K,
                                                       (double *)(p->arena + p->L.pen), ctx->stream));
    if (e == hipSuccess)
        e = hipMemcpyAsync(m.data(), p->arena + p->L.pen, (size_t)K * sizeof(double), hipMemcpyDeviceToHost,
                           ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    plan_destroy(p);
    if (e != hipSuccess) return fail(CPF_E_DEVICE, "candidate mjac: %s", hipGetErrorString(e));
    // 2. the M smallest (mjac, index)
    std::vector<int> order(K);
    for (int k = 0; k < K; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return m[a] < m[b]; });
    // 3. one single-candidate problem each (views into the caller's arrays;
    //    a caller node cost is gathered per candidate)
    std::vector<cpf_robot> robots(M, *robot);
    std::vector<cpf_problem> probs(M);
    std::vector<std::vector<double>> pens(M);
    for (int i = 0; i < M; ++i) {
        const int k = order[i];
        idx_out[i] = k;
        const size_t off = (size_t)k * T * hr.dof;
        probs[i] = cpf_problem{T, 1, prob->targets, prob->cand ? prob->cand + off : nullptr, nullptr,
                               prob->n_obstacles, prob->obstacles,
                               prob->cand_f32 ? prob->cand_f32 + off : nullptr, prob->mem};
        if (prob->node_pen) {
            pens[i].resize(T);
            for (int t = 0; t < T; ++t) pens[i][t] = prob->node_pen[(size_t)t * K + k];
            probs[i].node_pen = pens[i].data();
        }
    }
    return cpf_solve_batch(ctx, M, robots.data(), probs.data(), &o, results);
}

cpf_status cpf_ctx_profile(cpf_ctx *ctx, int32_t enable) {
    if (!ctx) return fail(CPF_E_ARG, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    for (auto &ev : ctx->events) {
        HIP_IGNORE(hipEventSynchronize(ev.b));
        ctx->ev_free.push_back(ev.a);
        ctx->ev_free.push_back(ev.b);
    }
    ctx->events.clear();
    for (int i = 0; i < KIND_COUNT; ++i) {
        ctx->prof_ms[i] = 0;
        ctx->prof_n[i] = 0;
    }
    ctx->prof.store(enable != 0);
    return CPF_OK;
}

cpf_status cpf_ctx_kernel_stats(cpf_ctx *ctx, const char *kernel, double *total_ms,
                                int64_t *launches) {
    if (!ctx || !kernel) return fail(CPF_E_ARG, "ctx / kernel is NULL");
    static const char *names[KIND_COUNT] = {"fk", "dp", "lm", "eval", "dp_lists"};
    int kind = -1;
    for (int i = 0; i < KIND_COUNT; ++i)
        if (strcmp(kernel, names[i]) == 0) kind = i;
    if (kind < 0) return fail(CPF_E_ARG, "unknown kernel '%s'", kernel);
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    for (auto &ev : ctx->events) {
        float ms = 0.f;
        HIP_TRY(hipEventSynchronize(ev.b));
        HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
        ctx->prof_ms[ev.kind] += ms;
        ctx->prof_n[ev.kind] += 1;
        ctx->ev_free.push_back(ev.a);
        ctx->ev_free.push_back(ev.b);
    }
    ctx->events.clear();
    if (total_ms) *total_ms = ctx->prof_ms[kind];
    if (launches) *launches = ctx->prof_n[kind];
    return CPF_OK;
}

}  // extern "C"
