// capi.cpp -- C ABI of the refinement path: context, device-memory budget,
// plans, batched solve and the continuously batched request server.
//
// A plan owns one device arena laid out as described in cpf_device.h.  The
// host converts the caller's AoS inputs to the device SoA layout once, in
// plan_init; kernels then run without further host traffic until the result
// is read back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/cpf.h"
#include "cpf_device.h"
#include "cpf_internal.h"

using namespace cpf;

// Best-effort cleanup calls whose status cannot be reported.
#define HIP_IGNORE(expr) ((void)(expr))

namespace {

thread_local std::string g_err;

cpf_status fail(cpf_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(CPF_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Byte offsets of one plan's buffers inside its arena.
struct Layout {
    size_t cand, extra, bp, path, dp_out, targets, xi, xt, A, g, P, y, dx, rb, st, report, total;
};

Layout make_layout(int T, int K, bool extra) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t t = (size_t)T, k = (size_t)K;
    L.cand = take(t * NJ * k * sizeof(float));
    L.extra = take(extra ? t * k * sizeof(double) : 0);
    L.bp = take(t * k * sizeof(uint16_t));
    L.path = take(t * sizeof(int32_t));
    L.dp_out = take(8 * sizeof(double));
    L.targets = take(12 * t * sizeof(double));
    L.xi = take(NJ * t * sizeof(double));
    L.xt = take(NJ * t * sizeof(double));
    L.A = take(NTRI * t * sizeof(double));
    L.g = take(NJ * t * sizeof(double));
    L.P = take(NBLK * t * sizeof(double));
    L.y = take(NJ * t * sizeof(double));
    L.dx = take(NJ * t * sizeof(double));
    L.rb = take(NJ * t * sizeof(double));
    L.st = take(sizeof(LMState));
    L.report = take(8 * sizeof(double));
    L.total = off;
    return L;
}

bool all_finite(const double *p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

cpf_status check_robot(const cpf_robot *r, HostRobot *out) {
    if (!r) return fail(CPF_E_ARG, "robot is NULL");
    if (r->dof != NJ) return fail(CPF_E_UNSUPPORTED, "dof=%d: only 7-joint chains are built", r->dof);
    if (!r->a || !r->d || !r->alpha || !r->q_lo || !r->q_hi)
        return fail(CPF_E_ARG, "robot array is NULL");
    for (int i = 0; i < NJ; ++i) {
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
    return CPF_OK;
}

cpf_status check_problem(const cpf_problem *p) {
    if (!p) return fail(CPF_E_ARG, "problem is NULL");
    if (p->T < 1 || p->K < 1) return fail(CPF_E_ARG, "T=%d K=%d must be >= 1", p->T, p->K);
    if (p->K > MAX_K) return fail(CPF_E_UNSUPPORTED, "K=%d exceeds %d", p->K, MAX_K);
    if (p->K > 65535) return fail(CPF_E_UNSUPPORTED, "K too large for 16-bit back-pointers");
    if (!p->targets || !p->cand) return fail(CPF_E_ARG, "targets / cand is NULL");
    if (!all_finite(p->targets, (size_t)p->T * 12)) return fail(CPF_E_ARG, "targets not finite");
    if (!all_finite(p->cand, (size_t)p->K * p->T * NJ)) return fail(CPF_E_ARG, "cand not finite");
    if (p->node_pen) {
        for (size_t i = 0; i < (size_t)p->T * p->K; ++i)
            if (!(std::fabs(p->node_pen[i]) <= 1e30))
                return fail(CPF_E_ARG, "node_pen must be finite with |value| <= 1e30");
    }
    return CPF_OK;
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
    return CPF_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Context and plan objects
// ---------------------------------------------------------------------------

struct Request;
static void request_delete(Request *r);

struct cpf_ctx {
    int device = 0;
    uint64_t budget = 0;
    std::atomic<uint64_t> used{0};
    hipStream_t stream = nullptr;     // synchronous plan calls
    hipStream_t serve_stream = nullptr;
    // serving
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> pending;
    std::map<uint64_t, Request *> tickets;
    uint64_t next_ticket = 1;
    bool stop = false;
    bool server_started = false;
    std::thread server;
    int iters_per_tick = 5;
    // kernel timing (cpf_ctx_profile)
    std::mutex prof_mu;
    std::atomic<bool> prof{false};
    struct Ev {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Ev> events;
    double prof_ms[4] = {0, 0, 0, 0};
    int64_t prof_n[4] = {0, 0, 0, 0};

    bool reserve(uint64_t b) {
        uint64_t cur = used.load();
        while (true) {
            if (cur + b > budget) return false;
            if (used.compare_exchange_weak(cur, cur + b)) return true;
        }
    }
    void release(uint64_t b) { used.fetch_sub(b); }
};

struct cpf_plan {
    cpf_ctx *ctx = nullptr;
    int T = 0, K = 0;
    HostRobot robot{};
    cpf_opts opts{};
    Layout L{};
    char *arena = nullptr;
    DevPlan desc{};
    DevPlan *d_desc = nullptr;
    bool searched = false;
    int iters_done = 0;
};

namespace {

enum { KIND_FK = 0, KIND_DP = 1, KIND_LM = 2, KIND_EVAL = 3 };

// Launch through `launch`; with profiling on, bracket it with events on s.
template <class F>
hipError_t timed(cpf_ctx *ctx, int kind, hipStream_t s, F &&launch) {
    if (!ctx->prof.load()) return launch();
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventRecord(a, s);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    ctx->events.push_back({kind, a, b});
    return e;
}

// Build the host image of the device descriptor for an arena.
void fill_desc(cpf_plan *p, bool has_extra) {
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
    D.penalty = p->opts.limit_penalty;
    for (int i = 0; i < NJ; ++i) {
        const HostRobot &r = p->robot;
        D.a[i] = r.a[i]; D.d[i] = r.d[i]; D.ca[i] = r.ca[i]; D.sa[i] = r.sa[i]; D.off[i] = r.off[i];
        D.lo[i] = r.lo[i]; D.hi[i] = r.hi[i];
        D.af[i] = (float)r.a[i]; D.df[i] = (float)r.d[i]; D.caf[i] = (float)r.ca[i];
        D.saf[i] = (float)r.sa[i]; D.offf[i] = (float)r.off[i];
    }
    char *b = p->arena;
    const Layout &L = p->L;
    D.cand = (const float *)(b + L.cand);
    D.extra = has_extra ? (const double *)(b + L.extra) : nullptr;
    D.bp = (uint16_t *)(b + L.bp);
    D.path = (int32_t *)(b + L.path);
    D.dp_out = (double *)(b + L.dp_out);
    D.targets = (double *)(b + L.targets);
    D.xi = (double *)(b + L.xi);
    D.xt = (double *)(b + L.xt);
    D.A = (double *)(b + L.A);
    D.g = (double *)(b + L.g);
    D.P = (double *)(b + L.P);
    D.y = (double *)(b + L.y);
    D.dx = (double *)(b + L.dx);
    D.rb = (double *)(b + L.rb);
    D.st = (LMState *)(b + L.st);
    D.report = (double *)(b + L.report);
}

uint64_t plan_bytes(int T, int K, bool extra) {
    return make_layout(T, K, extra).total + align256(sizeof(DevPlan));
}

// Allocate and upload one plan on stream s (asynchronous; host staging is
// kept alive by the caller until the stream is synchronised).
cpf_status plan_create(cpf_ctx *ctx, const HostRobot &hr, const cpf_problem *prob,
                       const cpf_opts *opts, hipStream_t s, std::vector<char> &staging,
                       cpf_plan **out) {
    const bool has_extra = prob->node_pen != nullptr;
    const uint64_t bytes = plan_bytes(prob->T, prob->K, has_extra);
    if (!ctx->reserve(bytes))
        return fail(CPF_E_NOMEM, "plan needs %llu bytes; budget %llu, in use %llu",
                    (unsigned long long)bytes, (unsigned long long)ctx->budget,
                    (unsigned long long)ctx->used.load());
    std::unique_ptr<cpf_plan> p(new cpf_plan());
    p->ctx = ctx;
    p->T = prob->T;
    p->K = prob->K;
    p->robot = hr;
    p->opts = *opts;
    p->L = make_layout(p->T, p->K, has_extra);
    void *mem = nullptr;
    hipError_t e = hipMalloc(&mem, p->L.total + align256(sizeof(DevPlan)));
    if (e != hipSuccess) {
        ctx->release(bytes);
        return fail(CPF_E_NOMEM, "hipMalloc(%llu): %s", (unsigned long long)bytes,
                    hipGetErrorString(e));
    }
    p->arena = (char *)mem;
    p->d_desc = (DevPlan *)(p->arena + p->L.total);
    fill_desc(p.get(), has_extra);

    // Host staging: SoA candidates (float), SoA targets, LM state, descriptor.
    const int T = p->T, K = p->K;
    const size_t n_cand = (size_t)T * NJ * K;
    const size_t stage_bytes = n_cand * sizeof(float) + (size_t)12 * T * sizeof(double) +
                               sizeof(LMState) + sizeof(DevPlan);
    staging.resize(stage_bytes);
    float *cs = (float *)staging.data();
    double *ts = (double *)(staging.data() + n_cand * sizeof(float));
    LMState *ss = (LMState *)(ts + (size_t)12 * T);
    DevPlan *ds = (DevPlan *)(ss + 1);
    for (int k = 0; k < K; ++k)
        for (int t = 0; t < T; ++t) {
            const double *src = prob->cand + ((size_t)k * T + t) * NJ;
            for (int j = 0; j < NJ; ++j) cs[((size_t)t * NJ + j) * K + k] = (float)src[j];
        }
    for (int t = 0; t < T; ++t)
        for (int c = 0; c < 12; ++c) ts[(size_t)c * T + t] = prob->targets[(size_t)t * 12 + c];
    memset(ss, 0, sizeof(LMState));
    ss->lambda = opts->lambda0;
    ss->nu = 2.0;
    ss->iters_target = 0;
    *ds = p->desc;

    e = hipMemcpyAsync(p->arena + p->L.cand, cs, n_cand * sizeof(float), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->arena + p->L.targets, ts, (size_t)12 * T * sizeof(double),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess && has_extra)
        e = hipMemcpyAsync(p->arena + p->L.extra, prob->node_pen, (size_t)T * K * sizeof(double),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->arena + p->L.st, ss, sizeof(LMState), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->d_desc, ds, sizeof(DevPlan), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
        HIP_IGNORE(hipFree(mem));
        ctx->release(bytes);
        return fail(CPF_E_DEVICE, "upload failed: %s", hipGetErrorString(e));
    }
    *out = p.release();
    return CPF_OK;
}

void plan_destroy(cpf_plan *p) {
    if (!p) return;
    if (p->arena) {
        HIP_IGNORE(hipFree(p->arena));
        p->ctx->release(plan_bytes(p->T, p->K, p->desc.has_extra != 0));
    }
    delete p;
}

// Read the LM state, report and (optionally) xi of a plan; stream-synchronous.
struct PlanReadback {
    LMState st;
    double report[8];
    double dp_out[8];
};

cpf_status read_state(cpf_plan *p, hipStream_t s, PlanReadback *rb, double *xi_out,
                      int32_t *path_out) {
    std::vector<double> xs;
    HIP_TRY(hipMemcpyAsync(&rb->st, p->arena + p->L.st, sizeof(LMState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(rb->report, p->arena + p->L.report, 8 * sizeof(double),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(rb->dp_out, p->arena + p->L.dp_out, 8 * sizeof(double),
                           hipMemcpyDeviceToHost, s));
    if (xi_out) {
        xs.resize((size_t)NJ * p->T);
        HIP_TRY(hipMemcpyAsync(xs.data(), p->arena + p->L.xi, xs.size() * sizeof(double),
                               hipMemcpyDeviceToHost, s));
    }
    if (path_out)
        HIP_TRY(hipMemcpyAsync(path_out, p->arena + p->L.path, (size_t)p->T * sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (xi_out)
        for (int t = 0; t < p->T; ++t)
            for (int j = 0; j < NJ; ++j) xi_out[(size_t)t * NJ + j] = xs[(size_t)j * p->T + t];
    return CPF_OK;
}

void fill_report(const PlanReadback &rb, cpf_lm_report *rep) {
    rep->cost0 = rb.st.cost0;
    rep->cost = rb.st.cost;
    rep->lambda = rb.st.lambda;
    rep->grad_inf = rb.st.grad_inf;
    rep->n_accepted = rb.st.n_acc;
    rep->iters_done = rb.st.iters_done;
    rep->max_pos_err_m = rb.report[0];
    rep->max_rot_err_rad = rb.report[1];
    rep->mjac = rb.report[2];
}

// Upload descriptors of several plans into one device array (caller frees).
cpf_status upload_descs(const std::vector<cpf_plan *> &plans, hipStream_t s, DevPlan **d_out,
                        std::vector<DevPlan> &host) {
    host.resize(plans.size());
    for (size_t i = 0; i < plans.size(); ++i) host[i] = plans[i]->desc;
    void *d = nullptr;
    HIP_TRY(hipMalloc(&d, host.size() * sizeof(DevPlan)));
    hipError_t e = hipMemcpyAsync(d, host.data(), host.size() * sizeof(DevPlan),
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
        HIP_IGNORE(hipFree(d));
        return fail(CPF_E_DEVICE, "descriptor upload: %s", hipGetErrorString(e));
    }
    *d_out = (DevPlan *)d;
    return CPF_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Public API
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
}

const char *cpf_last_error(void) { return g_err.c_str(); }

static void server_main(cpf_ctx *ctx);

cpf_status cpf_ctx_create(int device, uint64_t mem_budget_bytes, cpf_ctx **out) {
    if (!out) return fail(CPF_E_ARG, "out is NULL");
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(CPF_E_ARG, "device %d of %d", device, n);
    HIP_TRY(hipSetDevice(device));
    std::unique_ptr<cpf_ctx> c(new cpf_ctx());
    c->device = device;
    c->budget = mem_budget_bytes ? mem_budget_bytes : (uint64_t)64 << 30;
    HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&c->serve_stream, hipStreamNonBlocking));
    *out = c.release();
    return CPF_OK;
}

void cpf_ctx_destroy(cpf_ctx *ctx) {
    if (!ctx) return;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->stop = true;
    }
    ctx->cv_work.notify_all();
    if (ctx->server.joinable()) ctx->server.join();
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (auto &kv : ctx->tickets) request_delete(kv.second);
        ctx->tickets.clear();
    }
    HIP_IGNORE(hipSetDevice(ctx->device));
    if (ctx->stream) HIP_IGNORE(hipStreamDestroy(ctx->stream));
    if (ctx->serve_stream) HIP_IGNORE(hipStreamDestroy(ctx->serve_stream));
    delete ctx;
}

uint64_t cpf_ctx_bytes_in_use(const cpf_ctx *ctx) { return ctx ? ctx->used.load() : 0; }

cpf_status cpf_plan_init(cpf_ctx *ctx, const cpf_robot *robot, const cpf_problem *prob,
                         const cpf_opts *opts, cpf_plan **out) {
    if (!ctx || !out) return fail(CPF_E_ARG, "ctx / out is NULL");
    HostRobot hr;
    cpf_status st;
    if ((st = check_robot(robot, &hr)) != CPF_OK) return st;
    if ((st = check_problem(prob)) != CPF_OK) return st;
    cpf_opts o;
    cpf_opts_default(&o);
    if (opts) o = *opts;
    if ((st = check_opts(&o)) != CPF_OK) return st;
    HIP_TRY(hipSetDevice(ctx->device));
    std::vector<char> staging;
    cpf_plan *p = nullptr;
    if ((st = plan_create(ctx, hr, prob, &o, ctx->stream, staging, &p)) != CPF_OK) return st;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        plan_destroy(p);
        return fail(CPF_E_DEVICE, "plan upload: %s", hipGetErrorString(e));
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
    HIP_TRY(timed(ctx, KIND_FK, (hipStream_t)hip_stream, [&] { return fk_batch_launch(hr, M, prec, q_dev, pose_dev, jac_dev, (hipStream_t)hip_stream); }));
    return CPF_OK;
}

cpf_status cpf_dp_search(cpf_plan *plan, int32_t *path_out, double *best_out, double *mjac_out) {
    if (!plan) return fail(CPF_E_ARG, "plan is NULL");
    cpf_ctx *ctx = plan->ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(timed(ctx, KIND_DP, ctx->stream, [&] { return dp_launch(plan->d_desc, 1, plan->K, ctx->stream); }));
    PlanReadback rb;
    cpf_status st = read_state(plan, ctx->stream, &rb, nullptr, path_out);
    if (st != CPF_OK) return st;
    plan->searched = true;
    plan->iters_done = 0;
    if (best_out) *best_out = rb.dp_out[0];
    if (mjac_out) *mjac_out = rb.dp_out[1];
    return CPF_OK;
}

cpf_status cpf_lm_refine(cpf_plan *plan, int32_t iters, double *xi_out, cpf_lm_report *rep) {
    if (!plan) return fail(CPF_E_ARG, "plan is NULL");
    if (iters < 0) return fail(CPF_E_ARG, "iters=%d", iters);
    if (!plan->searched) return fail(CPF_E_STATE, "lm_refine before dp_search");
    cpf_ctx *ctx = plan->ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(timed(ctx, KIND_LM, ctx->stream, [&] { return lm_launch(plan->d_desc, 1, plan->opts.prec, iters, ctx->stream); }));
    HIP_TRY(timed(ctx, KIND_EVAL, ctx->stream, [&] { return eval_launch(plan->d_desc, 1, ctx->stream); }));
    PlanReadback rb;
    cpf_status st = read_state(plan, ctx->stream, &rb, xi_out, nullptr);
    if (st != CPF_OK) return st;
    plan->iters_done = rb.st.iters_done;
    if (rep) fill_report(rb, rep);
    if (rb.st.status != 0)
        return fail(CPF_E_NUMERIC, "non-positive pivot in the block solve");
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
        if ((st = check_problem(&probs[i])) != CPF_OK) return st;
    }
    if (nplans == 0) return CPF_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    std::vector<cpf_plan *> plans;
    std::vector<std::vector<char>> staging(nplans);
    auto cleanup = [&]() {
        HIP_IGNORE(hipStreamSynchronize(ctx->stream));
        for (auto *p : plans) plan_destroy(p);
    };
    int maxK = 0;
    for (int i = 0; i < nplans; ++i) {
        cpf_plan *p = nullptr;
        if ((st = plan_create(ctx, hrs[i], &probs[i], &o, ctx->stream, staging[i], &p)) != CPF_OK) {
            cleanup();
            return st;
        }
        plans.push_back(p);
        maxK = std::max(maxK, probs[i].K);
    }
    std::vector<DevPlan> host_descs;
    DevPlan *d_descs = nullptr;
    if ((st = upload_descs(plans, ctx->stream, &d_descs, host_descs)) != CPF_OK) {
        cleanup();
        return st;
    }
    const int64_t t0 = now_ns();
    hipError_t e = timed(ctx, KIND_DP, ctx->stream, [&] { return dp_launch(d_descs, nplans, maxK, ctx->stream); });
    if (e == hipSuccess) e = timed(ctx, KIND_LM, ctx->stream, [&] { return lm_launch(d_descs, nplans, o.prec, o.iters, ctx->stream); });
    if (e == hipSuccess) e = timed(ctx, KIND_EVAL, ctx->stream, [&] { return eval_launch(d_descs, nplans, ctx->stream); });
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    const int64_t t1 = now_ns();
    if (e != hipSuccess) {
        HIP_IGNORE(hipFree(d_descs));
        cleanup();
        return fail(CPF_E_DEVICE, "batch launch: %s", hipGetErrorString(e));
    }
    for (int i = 0; i < nplans; ++i) {
        PlanReadback rb;
        if ((st = read_state(plans[i], ctx->stream, &rb, results[i].xi, results[i].path)) != CPF_OK) {
            HIP_IGNORE(hipFree(d_descs));
            cleanup();
            return st;
        }
        fill_report(rb, &results[i].report);
        results[i].search_best = rb.dp_out[0];
        results[i].search_mjac = rb.dp_out[1];
        results[i].status = rb.st.status != 0 ? CPF_E_NUMERIC : CPF_OK;
        results[i].t_submit_ns = t0;
        results[i].t_admit_ns = t0;
        results[i].t_search_done_ns = t1;
        results[i].t_done_ns = t1;
    }
    HIP_IGNORE(hipFree(d_descs));
    cleanup();
    return CPF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Serving: submit / poll with continuous batching
// ---------------------------------------------------------------------------

struct Request {
    uint64_t ticket = 0;
    HostRobot robot{};
    cpf_opts opts{};
    int T = 0, K = 0;
    std::vector<double> targets, cand, node_pen;
    uint64_t bytes = 0;
    cpf_plan *plan = nullptr;
    std::vector<char> staging;
    bool done = false;
    cpf_status status = CPF_OK;
    std::vector<double> xi;
    std::vector<int32_t> path;
    cpf_lm_report report{};
    double best = 0, smjac = 0;
    int64_t t_submit = 0, t_admit = 0, t_search = 0, t_done = 0;
};

static void request_delete(Request *r) { delete r; }

extern "C" cpf_status cpf_submit(cpf_ctx *ctx, const cpf_robot *robot, const cpf_problem *prob,
                                 const cpf_opts *opts, uint64_t *ticket) {
    if (!ctx || !ticket) return fail(CPF_E_ARG, "ctx / ticket is NULL");
    HostRobot hr;
    cpf_status st;
    if ((st = check_robot(robot, &hr)) != CPF_OK) return st;
    if ((st = check_problem(prob)) != CPF_OK) return st;
    cpf_opts o;
    cpf_opts_default(&o);
    if (opts) o = *opts;
    if ((st = check_opts(&o)) != CPF_OK) return st;
    const uint64_t bytes = plan_bytes(prob->T, prob->K, prob->node_pen != nullptr);
    if (bytes > ctx->budget)
        return fail(CPF_E_NOMEM, "request needs %llu bytes, budget is %llu",
                    (unsigned long long)bytes, (unsigned long long)ctx->budget);
    std::unique_ptr<Request> r(new Request());
    r->robot = hr;
    r->opts = o;
    r->T = prob->T;
    r->K = prob->K;
    r->targets.assign(prob->targets, prob->targets + (size_t)prob->T * 12);
    r->cand.assign(prob->cand, prob->cand + (size_t)prob->K * prob->T * NJ);
    if (prob->node_pen) r->node_pen.assign(prob->node_pen, prob->node_pen + (size_t)prob->T * prob->K);
    r->bytes = bytes;
    r->t_submit = now_ns();
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (ctx->stop) return fail(CPF_E_STATE, "context is shutting down");
        if (!ctx->server_started) {
            ctx->server = std::thread(server_main, ctx);
            ctx->server_started = true;
        }
        r->ticket = ctx->next_ticket++;
        *ticket = r->ticket;
        ctx->tickets[r->ticket] = r.get();
        ctx->pending.push_back(r.release());
    }
    ctx->cv_work.notify_one();
    return CPF_OK;
}

extern "C" cpf_status cpf_poll(cpf_ctx *ctx, uint64_t ticket, int32_t timeout_ms, cpf_result *out) {
    if (!ctx) return fail(CPF_E_ARG, "ctx is NULL");
    std::unique_lock<std::mutex> lk(ctx->mu);
    auto it = ctx->tickets.find(ticket);
    if (it == ctx->tickets.end()) return fail(CPF_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second;
    if (!r->done) {
        if (timeout_ms == 0) return CPF_PENDING;
        auto pred = [&] { return r->done; };
        if (timeout_ms < 0) ctx->cv_done.wait(lk, pred);
        else if (!ctx->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred))
            return CPF_PENDING;
    }
    if (out) {
        if (out->xi && !r->xi.empty()) memcpy(out->xi, r->xi.data(), r->xi.size() * sizeof(double));
        if (out->path && !r->path.empty()) memcpy(out->path, r->path.data(), r->path.size() * sizeof(int32_t));
        out->report = r->report;
        out->search_best = r->best;
        out->search_mjac = r->smjac;
        out->status = r->status;
        out->t_submit_ns = r->t_submit;
        out->t_admit_ns = r->t_admit;
        out->t_search_done_ns = r->t_search;
        out->t_done_ns = r->t_done;
    }
    ctx->tickets.erase(it);
    delete r;
    return CPF_OK;
}

namespace {

// Finish a request: read results back, free its plan (caller holds no lock).
void retire(cpf_ctx *ctx, Request *r, hipStream_t s, cpf_status dev_status) {
    if (r->plan && dev_status == CPF_OK) {
        PlanReadback rb;
        r->xi.resize((size_t)r->T * NJ);
        r->path.resize(r->T);
        cpf_status st = read_state(r->plan, s, &rb, r->xi.data(), r->path.data());
        if (st == CPF_OK) {
            fill_report(rb, &r->report);
            r->best = rb.dp_out[0];
            r->smjac = rb.dp_out[1];
            r->status = rb.st.status != 0 ? CPF_E_NUMERIC : CPF_OK;
        } else {
            r->status = st;
        }
    } else if (dev_status != CPF_OK) {
        r->status = dev_status;
    }
    if (r->plan) {
        plan_destroy(r->plan);
        r->plan = nullptr;
    }
    r->cand.clear();
    r->cand.shrink_to_fit();
    r->t_done = now_ns();
    std::lock_guard<std::mutex> lk(ctx->mu);
    r->done = true;
    ctx->cv_done.notify_all();
}

}  // namespace

// Server loop.  Each tick: admit queued requests whose bytes fit the free
// budget (upload + search in one launch over the newly admitted), then run
// up to iters_per_tick LM iterations for every admitted request in one
// launch, then retire the finished ones.  Requests submitted during a tick
// join at the next tick, so their work overlaps with the ones in flight.
static void server_main(cpf_ctx *ctx) {
    HIP_IGNORE(hipSetDevice(ctx->device));
    hipStream_t s = ctx->serve_stream;
    std::vector<Request *> active;
    while (true) {
        std::vector<Request *> admitted;
        {
            std::unique_lock<std::mutex> lk(ctx->mu);
            ctx->cv_work.wait(lk, [&] { return ctx->stop || !ctx->pending.empty() || !active.empty(); });
            if (ctx->stop && ctx->pending.empty() && active.empty()) break;
            while (!ctx->pending.empty()) {
                Request *r = ctx->pending.front();
                if (!ctx->reserve(r->bytes)) break;   // wait for budget
                ctx->release(r->bytes);               // plan_create reserves it again
                ctx->pending.pop_front();
                admitted.push_back(r);
            }
        }
        std::vector<cpf_plan *> new_plans;
        for (Request *r : admitted) {
            cpf_problem pb{r->T, r->K, r->targets.data(), r->cand.data(),
                           r->node_pen.empty() ? nullptr : r->node_pen.data()};
            r->t_admit = now_ns();
            cpf_status st = plan_create(ctx, r->robot, &pb, &r->opts, s, r->staging, &r->plan);
            if (st != CPF_OK) {
                r->plan = nullptr;
                retire(ctx, r, s, st);
                continue;
            }
            new_plans.push_back(r->plan);
            active.push_back(r);
        }
        cpf_status dev = CPF_OK;
        if (!new_plans.empty()) {
            int maxK = 0;
            for (auto *p : new_plans) maxK = std::max(maxK, p->K);
            std::vector<DevPlan> hd;
            DevPlan *dd = nullptr;
            dev = upload_descs(new_plans, s, &dd, hd);
            if (dev == CPF_OK) {
                // per-plan iteration targets
                for (Request *r : admitted)
                    if (r->plan) {
                        LMState tmp{};
                        (void)tmp;
                    }
                hipError_t e = timed(ctx, KIND_DP, s, [&] { return dp_launch(dd, (int)new_plans.size(), maxK, s); });
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                HIP_IGNORE(hipFree(dd));
                if (e != hipSuccess) dev = fail(CPF_E_DEVICE, "search launch: %s", hipGetErrorString(e));
            }
            const int64_t ts = now_ns();
            for (Request *r : admitted)
                if (r->plan) r->t_search = ts;
        }
        if (!active.empty() && dev == CPF_OK) {
            std::vector<cpf_plan *> ap;
            int prec = active[0]->opts.prec;
            for (Request *r : active) ap.push_back(r->plan);
            std::vector<DevPlan> hd;
            DevPlan *dd = nullptr;
            dev = upload_descs(ap, s, &dd, hd);
            if (dev == CPF_OK) {
                // set iteration targets (host-side counters mirror the device)
                hipError_t e = hipSuccess;
                for (Request *r : active) {
                    const int32_t tgt = r->opts.iters;
                    e = hipMemcpyAsync((char *)r->plan->arena + r->plan->L.st + offsetof(LMState, iters_target),
                                       &r->opts.iters, sizeof(int32_t), hipMemcpyHostToDevice, s);
                    (void)tgt;
                    if (e != hipSuccess) break;
                }
                // Plans of both precisions are advanced by their own launch.
                std::vector<cpf_plan *> by_prec[2];
                for (Request *r : active) by_prec[r->opts.prec == CPF_FP64 ? 1 : 0].push_back(r->plan);
                (void)prec;
                for (int pr = 0; pr < 2 && e == hipSuccess; ++pr) {
                    if (by_prec[pr].empty()) continue;
                    std::vector<DevPlan> hd2;
                    DevPlan *dd2 = nullptr;
                    if (upload_descs(by_prec[pr], s, &dd2, hd2) != CPF_OK) { e = hipErrorUnknown; break; }
                    e = timed(ctx, KIND_LM, s, [&] { return lm_launch(dd2, (int)by_prec[pr].size(), pr, ctx->iters_per_tick, s); });
                    if (e == hipSuccess) e = timed(ctx, KIND_EVAL, s, [&] { return eval_launch(dd2, (int)by_prec[pr].size(), s); });
                    if (e == hipSuccess) e = hipStreamSynchronize(s);
                    HIP_IGNORE(hipFree(dd2));
                }
                HIP_IGNORE(hipFree(dd));
                if (e != hipSuccess) dev = fail(CPF_E_DEVICE, "LM tick: %s", hipGetErrorString(e));
            }
        }
        // Retire finished (or failed) requests.
        std::vector<Request *> still;
        for (Request *r : active) {
            bool finished = dev != CPF_OK;
            if (!finished) {
                LMState stt;
                if (hipMemcpy(&stt, (char *)r->plan->arena + r->plan->L.st, sizeof(LMState),
                              hipMemcpyDeviceToHost) != hipSuccess) {
                    finished = true;
                } else {
                    finished = stt.iters_done >= r->opts.iters || stt.status != 0;
                }
            }
            if (finished) retire(ctx, r, s, dev);
            else still.push_back(r);
        }
        active.swap(still);
    }
}

extern "C" cpf_status cpf_ctx_profile(cpf_ctx *ctx, int32_t enable) {
    if (!ctx) return fail(CPF_E_ARG, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    for (auto &ev : ctx->events) {
        HIP_IGNORE(hipEventSynchronize(ev.b));
        HIP_IGNORE(hipEventDestroy(ev.a));
        HIP_IGNORE(hipEventDestroy(ev.b));
    }
    ctx->events.clear();
    for (int i = 0; i < 4; ++i) {
        ctx->prof_ms[i] = 0;
        ctx->prof_n[i] = 0;
    }
    ctx->prof.store(enable != 0);
    return CPF_OK;
}

extern "C" cpf_status cpf_ctx_kernel_stats(cpf_ctx *ctx, const char *kernel, double *total_ms,
                                           int64_t *launches) {
    if (!ctx || !kernel) return fail(CPF_E_ARG, "ctx / kernel is NULL");
    static const char *names[4] = {"fk", "dp", "lm", "eval"};
    int kind = -1;
    for (int i = 0; i < 4; ++i)
        if (strcmp(kernel, names[i]) == 0) kind = i;
    if (kind < 0) return fail(CPF_E_ARG, "unknown kernel '%s'", kernel);
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    for (auto &ev : ctx->events) {
        float ms = 0.f;
        HIP_TRY(hipEventSynchronize(ev.b));
        HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
        ctx->prof_ms[ev.kind] += ms;
        ctx->prof_n[ev.kind] += 1;
        HIP_IGNORE(hipEventDestroy(ev.a));
        HIP_IGNORE(hipEventDestroy(ev.b));
    }
    ctx->events.clear();
    if (total_ms) *total_ms = ctx->prof_ms[kind];
    if (launches) *launches = ctx->prof_n[kind];
    return CPF_OK;
}
