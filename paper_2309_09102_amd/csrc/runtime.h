// runtime.h -- host-side runtime objects shared by capi.cpp and serve.cpp:
// the context (device, budget, streams, server state), plans and their
// device arenas, error reporting and kernel timing.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/cpf.h"
#include "cpf_plan.h"
#include "cpf_internal.h"

// Best-effort cleanup calls whose status cannot be reported.
#define HIP_IGNORE(expr) ((void)(expr))

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return cpf::fail(CPF_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

namespace cpf {

cpf_status fail(cpf_status st, const char *fmt, ...);
int64_t now_ns();
inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Byte offsets of one plan's buffers inside its arena.  `raw` receives the
// caller's candidates ([K][T][dof] doubles or floats) and targets ([T][12])
// as uploaded;
// a kernel converts them into the device layout before the search, so the
// region is shared with the search lists (topc), which are written later.
struct Layout {
    size_t cand, extra, pen, bp, topk, topc, raw, path, dp_out, targets, xi, xt, A, g, cr, dx, rb, st,
        report, xv, obs, cpen, rr, rt, total;
};
Layout make_layout(int T, int K, int dof, bool extra, int n_obs, bool coll);
uint64_t plan_bytes(int T, int K, int dof, bool extra, int n_obs, bool coll);
// Device bytes a plan takes from the budget: its arena rounded up to a
// power of two (at least 1 MiB), the unit the arena pool recycles.
uint64_t plan_class_bytes(int T, int K, int dof, bool extra, int n_obs, bool coll);

cpf_status check_robot(const cpf_robot *r, HostRobot *out);
// Robots a plan may use (CPF_E_UNSUPPORTED for collision capsules together
// with a prismatic joint: that combination is switched off in plans).
cpf_status check_plan_robot(const HostRobot &hr);
cpf_status check_problem(const cpf_problem *p, int dof);
cpf_status check_opts(const cpf_opts *o);

enum { KIND_FK = 0, KIND_DP = 1, KIND_LM = 2, KIND_EVAL = 3, KIND_DPL = 4, KIND_COUNT = 5 };

struct Request;
struct Server;

}  // namespace cpf

struct cpf_ctx {
    int device = 0;
    uint64_t budget = 0;
    std::atomic<uint64_t> used{0};   // arenas held by live plans
    hipStream_t stream = nullptr;    // synchronous plan calls
    // Arena pool: freed arenas are kept by size class and handed out again,
    // so steady serving makes no device allocation or free; cached bytes
    // count against the budget together with `used`.
    std::mutex pool_mu;
    std::map<uint64_t, std::vector<void *>> pool;
    uint64_t pooled = 0;
    // Pinned host staging for submitted requests (same scheme, capped), so
    // their uploads are asynchronous DMA.
    std::map<uint64_t, std::vector<void *>> pinned;
    uint64_t pinned_total = 0;
    uint64_t pinned_cap = (uint64_t)4 << 30;
    // serving
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<cpf::Request *> pending;
    std::map<uint64_t, cpf::Request *> tickets;
    uint64_t next_ticket = 1;
    bool stop = false;
    cpf::Server *server = nullptr;
    std::thread server_thread;
    int32_t slots = 256;           // concurrent requests on the device
    int32_t iters_per_tick = 30;   // LM iterations per graph replay, at most
    int32_t tick_budget = 6000;    // and about tick_budget / (T + 330) of them for a plan of T waypoints
    // kernel timing
    std::mutex prof_mu;
    std::atomic<bool> prof{false};
    struct Ev {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Ev> events;
    std::vector<hipEvent_t> ev_free;   // created events ready for reuse (no create in a timed launch)
    double prof_ms[cpf::KIND_COUNT] = {};
    int64_t prof_n[cpf::KIND_COUNT] = {};

};

struct cpf_plan {
    cpf_ctx *ctx = nullptr;
    int T = 0, K = 0, n_obs = 0;
    cpf::HostRobot robot{};
    cpf_opts opts{};
    cpf::Layout L{};
    char *arena = nullptr;
    uint64_t bytes = 0;   // size class taken from the pool
    cpf::DevPlan desc{};
    cpf::DevPlan *d_desc = nullptr;
    cpf::LMState init{};  // host source of the initial LM state upload
    bool searched = false;
    bool lists_valid = false;   // the search's predecessor lists are current
    double seed_steps[2] = {0.0, 0.0};   // last search: largest revolute / prismatic step
};

namespace cpf {

// A pair of events from the context's pool (created when it is empty).
hipError_t event_pair(cpf_ctx *ctx, hipEvent_t *a, hipEvent_t *b);

// Launch through `launch`; with profiling on, bracket it with events on s.
template <class F>
hipError_t timed(cpf_ctx *ctx, int kind, hipStream_t s, F &&launch) {
    if (!ctx->prof.load()) return launch();
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = event_pair(ctx, &a, &b);
    if (e == hipSuccess) e = hipEventRecord(a, s);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    ctx->events.push_back({kind, a, b});
    return e;
}

// The search of nplans plans on s, each launch timed: the lists (unless
// lists_ready: the plans' lists are current) as "dp_lists", the stages as
// "dp"; dofs: the chain lengths among the plans (dof_bit), one set of
// launches each.
hipError_t search_launch(cpf_ctx *ctx, const DevPlan *d_plans, int nplans, int maxK, int maxT, bool lists_ready,
                         bool coll, int dofs, hipStream_t s);

// Arena of `cls` bytes from the pool (or a new allocation within the
// budget); E_NOMEM when the budget does not allow it.
cpf_status arena_get(cpf_ctx *ctx, uint64_t cls, void **out);
void arena_put(cpf_ctx *ctx, void *p, uint64_t cls);
void pool_clear(cpf_ctx *ctx);
// Pinned host buffer of at least `bytes` (class written to *cls), or
// nullptr when the pinned cap is reached (the caller then uses pageable
// memory).
void *pinned_get(cpf_ctx *ctx, uint64_t bytes, uint64_t *cls);
void pinned_put(cpf_ctx *ctx, void *p, uint64_t cls);
// memcpy split over a few threads for large copies.
void copy_parallel(void *dst, const void *src, size_t bytes);

// Take an arena and upload one plan on stream s (asynchronous: the caller's
// arrays in `prob` must stay alive until s is synchronised).  iters_target =
// 0 lets each lm_refine call run the iterations it asks for.
cpf_status plan_alloc(cpf_ctx *ctx, const HostRobot &hr, int T, int K, bool has_extra, int n_obs,
                      const cpf_opts *opts, int32_t iters_target, hipStream_t s, cpf_plan **out);
cpf_status plan_create(cpf_ctx *ctx, const HostRobot &hr, const cpf_problem *prob,
                       const cpf_opts *opts, int32_t iters_target, hipStream_t s, cpf_plan **out);
void plan_destroy(cpf_plan *p);
// Flag of a plan's device-resident inputs (an int in the report's last
// slot): cleared when the arena is taken, set by the staging kernel when a
// device input value is not finite.
int *input_flag(cpf_plan *p);
bool input_flag_set(const double *report);

struct PlanReadback {
    LMState st;
    double report[8];
    double dp_out[8];
};
// Read state / report / search output and optionally xi ([T][dof]), path and
// the latest valid trajectory ([T][dof], written only when one exists).
cpf_status read_plan(cpf_plan *p, hipStream_t s, const LMState *state_dev, PlanReadback *rb,
                     double *xi_out, int32_t *path_out, double *xv_out);
// Device [dof][T] to caller [T][dof].
void soa_to_rows(const double *soa, int T, int dof, double *rows);
void report_from(const LMState &ls, const double *report, cpf_lm_report *rep);
void fill_report(const PlanReadback &rb, cpf_lm_report *rep);

// Server lifetime (serve.cpp).
void server_stop_and_join(cpf_ctx *ctx);

}  // namespace cpf
