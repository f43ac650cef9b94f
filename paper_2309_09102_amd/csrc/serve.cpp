// serve.cpp -- continuously batched request server behind cpf_submit /
// cpf_poll.
//
// The device holds a fixed table of `slots` plan descriptors (the work list)
// and their LM states in one contiguous array.  One server thread loops:
//   1. admission: while a slot is free and the request's arena fits the
//      memory budget, take an arena from the pool and upload the request on
//      a search lane's stream; the admitted requests are searched in one
//      launch there (one workgroup per request).  SEARCH_LANES batches can
//      be in flight at once on their own streams, so a batch admitted while
//      another is searched does not wait for it (a batch's stage recursion
//      lasts as long as its longest request, however few requests it has),
//      while
//   2. the LM stream replays a tick graph over the work list: the LM kernel
//      instances of both precisions, for the kinds of plan in the table
//      (weighted objective or schedule, with or without collision
//      geometry), over every slot (each instance skips empty slots and the
//      other instances' plans), every plan advancing up to `iters_per_tick`
//      iterations, then the report kernel for plans that just finished;
//   3. a searched batch joins the work list at the next tick (its
//      descriptors are written into their slots on the LM stream);
//   4. after each tick all slot states come back in one copy, and the
//      finished requests are read back together and retired (their arenas
//      go back to the pool).
// Requests submitted while the GPU is busy join at the next tick, so their
// search and iterations overlap on the device with the requests in flight.
// A graph is captured once per context and combination of plan kinds (at
// its first use): its kernels read the work list from device memory, so
// admissions and retirements only rewrite descriptor slots between replays,
// and a table of plain plans never launches the other kinds' instances
// (whose larger scratch needs slow every dispatch).
#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <thread>

#include "runtime.h"

namespace cpf {

struct Request {
    uint64_t ticket = 0;
    HostRobot robot{};
    cpf_opts opts{};
    int T = 0, K = 0;
    // copies of the caller's host arrays (candidates as given, double or
    // float, targets, node costs, obstacles) in one buffer, pinned when the
    // pinned pool allows, else pageable; device-resident candidates and
    // targets are not copied (prob points at them)
    cpf_problem prob{};
    int n_obs = 0;
    void *stage = nullptr;
    uint64_t stage_cls = 0;
    std::vector<double> stage_vec;
    uint64_t bytes = 0;
    cpf_plan *plan = nullptr;
    int slot = -1;
    bool done = false;
    cpf_status status = CPF_OK;
    std::vector<double> xi, xi_soa, xv, xv_soa;
    std::vector<int32_t> path;
    double report[8] = {0}, dp_out[8] = {0};
    cpf_lm_report rep{};
    double best = 0, smjac = 0;
    int64_t t_submit = 0, t_admit = 0, t_search = 0, t_done = 0;
};

// A search lane: one admitted batch at a time, uploaded and searched on the
// lane's stream.
struct SearchLane {
    hipStream_t s = nullptr;
    hipEvent_t searched = nullptr;
    DevPlan *d_new = nullptr;           // [cap] descriptors of the batch
    std::vector<DevPlan> h_new;
    std::vector<Request *> searching;   // the batch in flight (empty: lane free)
};
constexpr int SEARCH_LANES = 2;

struct Server {
    int cap = 0;
    int ipt = 0;
    int budget = 0;   // waypoint-iterations per plan and tick (0: iters_per_tick for every plan)
    hipStream_t s_lm = nullptr;    // tick graph, work-list updates, read-back
    SearchLane lane[SEARCH_LANES];
    DevPlan *d_work = nullptr;     // [cap]
    LMState *d_states = nullptr;   // [cap]
    std::vector<DevPlan> h_work;
    std::vector<LMState> h_states, h_init;
    std::vector<Request *> slot_req;
    // tick graphs by kinds present: bit 0 schedule, bit 1 collision geometry,
    // bit 2 a prismatic joint, bit 3 an 8-joint chain
    hipGraph_t graph[16] = {};
    hipGraphExec_t exec[16] = {};
};

namespace {

cpf_status server_init(cpf_ctx *ctx, Server *sv) {
    sv->cap = ctx->slots;
    sv->ipt = ctx->iters_per_tick;
    sv->budget = ctx->tick_budget;
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipStreamCreateWithFlags(&sv->s_lm, hipStreamNonBlocking));
    for (SearchLane &ln : sv->lane) {
        HIP_TRY(hipStreamCreateWithFlags(&ln.s, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&ln.searched, hipEventDisableTiming));
        HIP_TRY(hipMalloc((void **)&ln.d_new, sizeof(DevPlan) * sv->cap));
        ln.h_new.assign(sv->cap, DevPlan{});
    }
    HIP_TRY(hipMalloc((void **)&sv->d_work, sizeof(DevPlan) * sv->cap));
    HIP_TRY(hipMalloc((void **)&sv->d_states, sizeof(LMState) * sv->cap));
    sv->h_work.assign(sv->cap, DevPlan{});     // T = 0: empty slot
    sv->h_states.assign(sv->cap, LMState{});
    sv->h_init.assign(sv->cap, LMState{});
    sv->slot_req.assign(sv->cap, nullptr);
    HIP_TRY(hipMemcpyAsync(sv->d_work, sv->h_work.data(), sizeof(DevPlan) * sv->cap,
                           hipMemcpyHostToDevice, sv->s_lm));
    HIP_TRY(hipMemcpyAsync(sv->d_states, sv->h_states.data(), sizeof(LMState) * sv->cap,
                           hipMemcpyHostToDevice, sv->s_lm));
    HIP_TRY(hipStreamSynchronize(sv->s_lm));
    return CPF_OK;
}

// The tick graph for the plan kinds in `kinds` (bit 0 schedule, bit 1
// collision geometry, bit 2 a prismatic joint, bit 3 an 8-joint chain),
// captured at its first use: the LM instances of both precisions for those
// kinds and the plain ones, then the report kernels; those of 7-joint chains
// always, those of 8-joint chains with bit 3.
cpf_status tick_graph(Server *sv, int kinds, hipGraphExec_t *out) {
    if (!sv->exec[kinds]) {
        HIP_TRY(hipStreamBeginCapture(sv->s_lm, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        const bool geos[GEO_KINDS] = {true, ((kinds >> 1) & 1) != 0, ((kinds >> 2) & 1) != 0};
        const int top_dof = (kinds >> 3) & 1 ? 8 : 7;
        for (int dof = 7; dof <= top_dof; ++dof) {
            for (int geo = 0; geo < GEO_KINDS; ++geo)
                for (int sched = 0; sched <= (kinds & 1) && geos[geo]; ++sched)
                    for (int prec = 0; prec < 2 && e == hipSuccess; ++prec)
                        e = CPF_BY_DOF(dof, lm_launch(sv->d_work, sv->cap, prec, sched, geo, sv->ipt, sv->s_lm,
                                                      sv->budget));
            for (int geo = 0; geo < GEO_KINDS && e == hipSuccess; ++geo)
                if (geos[geo]) e = CPF_BY_DOF(dof, eval_launch(sv->d_work, sv->cap, 1, geo, sv->s_lm));
        }
        hipError_t e2 = hipStreamEndCapture(sv->s_lm, &sv->graph[kinds]);
        if (e != hipSuccess) return fail(CPF_E_DEVICE, "tick capture: %s", hipGetErrorString(e));
        if (e2 != hipSuccess) return fail(CPF_E_DEVICE, "tick capture end: %s", hipGetErrorString(e2));
        HIP_TRY(hipGraphInstantiate(&sv->exec[kinds], sv->graph[kinds], nullptr, nullptr, 0));
    }
    *out = sv->exec[kinds];
    return CPF_OK;
}

void server_free(Server *sv) {
    for (SearchLane &ln : sv->lane)
        if (ln.s) HIP_IGNORE(hipStreamSynchronize(ln.s));
    if (sv->s_lm) HIP_IGNORE(hipStreamSynchronize(sv->s_lm));
    for (int g = 0; g < 16; ++g) {
        if (sv->exec[g]) HIP_IGNORE(hipGraphExecDestroy(sv->exec[g]));
        if (sv->graph[g]) HIP_IGNORE(hipGraphDestroy(sv->graph[g]));
    }
    if (sv->d_work) HIP_IGNORE(hipFree(sv->d_work));
    if (sv->d_states) HIP_IGNORE(hipFree(sv->d_states));
    for (SearchLane &ln : sv->lane) {
        if (ln.searched) HIP_IGNORE(hipEventDestroy(ln.searched));
        if (ln.d_new) HIP_IGNORE(hipFree(ln.d_new));
        if (ln.s) HIP_IGNORE(hipStreamDestroy(ln.s));
    }
    if (sv->s_lm) HIP_IGNORE(hipStreamDestroy(sv->s_lm));
}

void release_stage(cpf_ctx *ctx, Request *r) {
    if (r->stage) pinned_put(ctx, r->stage, r->stage_cls);
    r->stage = nullptr;
    std::vector<double>().swap(r->stage_vec);
    r->prob = cpf_problem{};
}

// Release a request's slot, plan and inputs and wake its pollers.  The slot's
// descriptor is cleared on the LM stream, ahead of the next tick.
void finish(cpf_ctx *ctx, Server *sv, Request *r) {
    if (r->slot >= 0) {
        sv->h_work[r->slot] = DevPlan{};
        HIP_IGNORE(hipMemcpyAsync(sv->d_work + r->slot, &sv->h_work[r->slot], sizeof(DevPlan),
                                  hipMemcpyHostToDevice, sv->s_lm));
        sv->slot_req[r->slot] = nullptr;
        r->slot = -1;
    }
    if (r->plan) {
        plan_destroy(r->plan);
        r->plan = nullptr;
    }
    release_stage(ctx, r);
    std::vector<double>().swap(r->xi_soa);
    std::vector<double>().swap(r->xv_soa);
    r->t_done = now_ns();
    std::lock_guard<std::mutex> lk(ctx->mu);
    r->done = true;
    ctx->cv_done.notify_all();
}

// Read back the finished requests together (one synchronisation), then
// release them.
void retire(cpf_ctx *ctx, Server *sv, const std::vector<Request *> &fin, cpf_status dev) {
    if (fin.empty()) return;
    hipError_t e = hipSuccess;
    if (dev == CPF_OK) {
        for (Request *r : fin) {
            if (!r->plan) continue;
            const Layout &L = r->plan->L;
            const char *a = r->plan->arena;
            r->xi_soa.resize((size_t)r->robot.dof * r->T);
            r->path.resize(r->T);
            if (e == hipSuccess)
                e = hipMemcpyAsync(r->xi_soa.data(), a + L.xi, r->xi_soa.size() * sizeof(double),
                                   hipMemcpyDeviceToHost, sv->s_lm);
            if (e == hipSuccess)
                e = hipMemcpyAsync(r->path.data(), a + L.path, (size_t)r->T * sizeof(int32_t),
                                   hipMemcpyDeviceToHost, sv->s_lm);
            if (e == hipSuccess)
                e = hipMemcpyAsync(r->report, a + L.report, sizeof(r->report), hipMemcpyDeviceToHost, sv->s_lm);
            if (e == hipSuccess)
                e = hipMemcpyAsync(r->dp_out, a + L.dp_out, sizeof(r->dp_out), hipMemcpyDeviceToHost, sv->s_lm);
            if (r->opts.schedule && sv->h_states[r->slot].n_valid > 0) {
                r->xv_soa.resize((size_t)r->robot.dof * r->T);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(r->xv_soa.data(), a + L.xv, r->xv_soa.size() * sizeof(double),
                                       hipMemcpyDeviceToHost, sv->s_lm);
            }
        }
        if (e == hipSuccess) e = hipStreamSynchronize(sv->s_lm);
        if (e != hipSuccess) dev = fail(CPF_E_DEVICE, "read-back: %s", hipGetErrorString(e));
    }
    for (Request *r : fin) {
        if (dev != CPF_OK || !r->plan) {
            if (r->status == CPF_OK) r->status = dev;
        } else {
            const LMState &ls = sv->h_states[r->slot];
            const int dof = r->robot.dof;
            r->xi.resize((size_t)r->T * dof);
            soa_to_rows(r->xi_soa.data(), r->T, dof, r->xi.data());
            if (!r->xv_soa.empty()) {
                r->xv.resize((size_t)r->T * dof);
                soa_to_rows(r->xv_soa.data(), r->T, dof, r->xv.data());
            }
            report_from(ls, r->report, &r->rep);
            r->best = r->dp_out[0];
            r->smjac = r->dp_out[1];
            r->status = input_flag_set(r->report) ? CPF_E_ARG : (ls.status != 0 ? CPF_E_NUMERIC : CPF_OK);
        }
        finish(ctx, sv, r);
    }
}

// Admit queued requests into free slots while their arenas fit the budget,
// upload them on a free search lane's stream and launch their search there.
// Returns the number admitted; requests that fail to upload are retired with
// their status.
int admit(cpf_ctx *ctx, Server *sv, SearchLane &ln, int free_slots) {
    std::vector<Request *> batch;
    int maxK = 0, maxT = 0, dofs = 0;
    bool any_coll = false;
    while (free_slots > 0) {
        Request *r = nullptr;
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            if (ctx->pending.empty()) break;
            r = ctx->pending.front();
            ctx->pending.pop_front();
        }
        r->t_admit = now_ns();
        cpf_status st = plan_create(ctx, r->robot, &r->prob, &r->opts, r->opts.iters, ln.s, &r->plan);
        if (st == CPF_E_NOMEM) {   // wait for arenas to come back
            std::lock_guard<std::mutex> lk(ctx->mu);
            ctx->pending.push_front(r);
            break;
        }
        if (st != CPF_OK) {
            r->plan = nullptr;
            r->status = st;
            finish(ctx, sv, r);
            continue;
        }
        int slot = 0;
        while (sv->slot_req[slot]) ++slot;
        r->slot = slot;
        sv->slot_req[slot] = r;
        LMState &ls = sv->h_init[slot];
        memset(&ls, 0, sizeof(ls));
        ls.lambda = r->opts.lambda0;
        ls.nu = 2.0;
        ls.iters_target = r->opts.iters;
        HIP_IGNORE(hipMemcpyAsync(sv->d_states + slot, &ls, sizeof(LMState), hipMemcpyHostToDevice, ln.s));
        DevPlan d = r->plan->desc;
        set_dev_ptr(d.st, sv->d_states + slot);
        ln.h_new[batch.size()] = d;
        batch.push_back(r);
        maxK = std::max(maxK, r->K);
        maxT = std::max(maxT, r->T);
        any_coll = any_coll || r->robot.has_caps;
        dofs |= dof_bit(r->robot.dof);
        --free_slots;
    }
    if (batch.empty()) return 0;
    hipError_t e = hipMemcpyAsync(ln.d_new, ln.h_new.data(), sizeof(DevPlan) * batch.size(),
                                  hipMemcpyHostToDevice, ln.s);
    if (e == hipSuccess)
        e = search_launch(ctx, ln.d_new, (int)batch.size(), maxK, maxT, false, any_coll, dofs, ln.s);
    if (e == hipSuccess) e = hipEventRecord(ln.searched, ln.s);
    if (e != hipSuccess) {
        HIP_IGNORE(hipStreamSynchronize(ln.s));
        const cpf_status dev = fail(CPF_E_DEVICE, "search launch: %s", hipGetErrorString(e));
        for (Request *r : batch) r->status = dev;
        retire(ctx, sv, batch, dev);
        return 0;
    }
    ln.searching = batch;
    return (int)batch.size();
}

// A searched batch joins the work list (descriptors written on s_lm, so the
// next tick sees them).
void activate(cpf_ctx *ctx, Server *sv, SearchLane &ln) {
    const int64_t ts = now_ns();
    for (Request *r : ln.searching) {
        DevPlan d = r->plan->desc;
        set_dev_ptr(d.st, sv->d_states + r->slot);
        sv->h_work[r->slot] = d;
        HIP_IGNORE(hipMemcpyAsync(sv->d_work + r->slot, &sv->h_work[r->slot], sizeof(DevPlan),
                                  hipMemcpyHostToDevice, sv->s_lm));
        r->t_search = ts;
        release_stage(ctx, r);   // the inputs are on the device now
    }
    ln.searching.clear();
}

void server_main(cpf_ctx *ctx) {
    std::unique_ptr<Server> sv(new Server());
    const cpf_status init = server_init(ctx, sv.get());
    std::vector<Request *> active;   // in the work list
    while (true) {
        bool searching = false;
        for (const SearchLane &ln : sv->lane) searching = searching || !ln.searching.empty();
        const bool busy = !active.empty() || searching;
        {
            std::unique_lock<std::mutex> lk(ctx->mu);
            if (!busy)
                ctx->cv_work.wait(lk, [&] { return ctx->stop || !ctx->pending.empty(); });
            if (ctx->stop && ctx->pending.empty() && !busy) break;
        }
        if (init != CPF_OK) {   // no device server: fail everything queued
            std::vector<Request *> q;
            {
                std::lock_guard<std::mutex> lk(ctx->mu);
                q.assign(ctx->pending.begin(), ctx->pending.end());
                ctx->pending.clear();
            }
            for (Request *r : q) {
                r->status = init;
                finish(ctx, sv.get(), r);
            }
            continue;
        }
        // 1. admit and search a new batch on a free lane
        for (SearchLane &ln : sv->lane) {
            if (!ln.searching.empty()) continue;
            int used = 0;
            for (Request *r : sv->slot_req) used += r != nullptr;
            admit(ctx, sv.get(), ln, sv->cap - used);
            break;
        }
        // 2. finished searches join the work list before the next tick
        bool pending_search = false;
        for (SearchLane &ln : sv->lane) {
            if (ln.searching.empty()) continue;
            const hipError_t q = hipEventQuery(ln.searched);
            if (q == hipSuccess) {
                for (Request *r : ln.searching) active.push_back(r);
                activate(ctx, sv.get(), ln);
            } else if (q == hipErrorNotReady) {
                pending_search = true;
            } else {
                const cpf_status dev = fail(CPF_E_DEVICE, "search: %s", hipGetErrorString(q));
                std::vector<Request *> b = ln.searching;
                ln.searching.clear();
                retire(ctx, sv.get(), b, dev);
            }
        }
        if (active.empty()) {
            // nothing to tick yet: poll the searches (and admit new requests
            // to a free lane meanwhile)
            if (pending_search) std::this_thread::sleep_for(std::chrono::microseconds(50));
            continue;
        }
        // 3. one LM tick over every slot, then all slot states in one copy
        int kinds = 0;
        for (Request *r : active)
            kinds |= (r->opts.schedule ? 1 : 0) | (r->robot.has_caps ? 2 : 0) | (r->robot.prism ? 4 : 0) |
                     (r->robot.dof == 8 ? 8 : 0);
        hipGraphExec_t exec = nullptr;
        cpf_status dev = tick_graph(sv.get(), kinds, &exec);
        hipError_t e = dev == CPF_OK ? hipSuccess : hipErrorUnknown;
        if (e == hipSuccess) e = timed(ctx, KIND_LM, sv->s_lm, [&] { return hipGraphLaunch(exec, sv->s_lm); });
        if (e == hipSuccess)
            e = hipMemcpyAsync(sv->h_states.data(), sv->d_states, sizeof(LMState) * sv->cap,
                               hipMemcpyDeviceToHost, sv->s_lm);
        if (e == hipSuccess) e = hipStreamSynchronize(sv->s_lm);
        if (dev == CPF_OK && e != hipSuccess) dev = fail(CPF_E_DEVICE, "LM tick: %s", hipGetErrorString(e));
        // 4. retire finished (or failed) requests together
        std::vector<Request *> still, fin;
        for (Request *r : active) {
            bool finished = dev != CPF_OK;
            if (!finished) {
                const LMState &ls = sv->h_states[r->slot];
                finished = ls.status != 0 || (ls.iters_done >= r->opts.iters && ls.reported);
            }
            (finished ? fin : still).push_back(r);
        }
        retire(ctx, sv.get(), fin, dev);
        active.swap(still);
    }
    server_free(sv.get());
}

}  // namespace

void server_stop_and_join(cpf_ctx *ctx) {
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->stop = true;
    }
    ctx->cv_work.notify_all();
    if (ctx->server_thread.joinable()) ctx->server_thread.join();
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (auto &kv : ctx->tickets) delete kv.second;
    ctx->tickets.clear();
}

}  // namespace cpf

using namespace cpf;

extern "C" cpf_status cpf_ctx_config(cpf_ctx *ctx, int32_t slots, int32_t iters_per_tick, int32_t tick_budget) {
    if (!ctx) return fail(CPF_E_ARG, "ctx is NULL");
    if (slots < 1 || slots > 65536 || iters_per_tick < 1 || iters_per_tick > 100000)
        return fail(CPF_E_ARG, "slots %d / iters_per_tick %d out of range", slots, iters_per_tick);
    if (tick_budget < 0) return fail(CPF_E_ARG, "tick_budget %d < 0", tick_budget);
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->server_thread.joinable()) return fail(CPF_E_STATE, "server already running");
    ctx->slots = slots;
    ctx->iters_per_tick = iters_per_tick;
    ctx->tick_budget = tick_budget;
    return CPF_OK;
}

extern "C" cpf_status cpf_submit(cpf_ctx *ctx, const cpf_robot *robot, const cpf_problem *prob,
                                 const cpf_opts *opts, uint64_t *ticket) {
    if (!ctx || !ticket) return fail(CPF_E_ARG, "ctx / ticket is NULL");
    HostRobot hr;
    cpf_status st;
    if ((st = check_robot(robot, &hr)) != CPF_OK) return st;
    if ((st = check_plan_robot(hr)) != CPF_OK) return st;
    if ((st = check_problem(prob, hr.dof)) != CPF_OK) return st;
    cpf_opts o;
    cpf_opts_default(&o);
    if (opts) o = *opts;
    if ((st = check_opts(&o)) != CPF_OK) return st;
    if (o.iters < 1) return fail(CPF_E_ARG, "iters=%d: a served request runs at least one LM iteration", o.iters);
    const uint64_t bytes =
        plan_class_bytes(prob->T, prob->K, hr.dof, prob->node_pen != nullptr, prob->n_obstacles, hr.has_caps);
    if (bytes > ctx->budget)
        return fail(CPF_E_NOMEM, "request needs %llu bytes, budget is %llu",
                    (unsigned long long)bytes, (unsigned long long)ctx->budget);
    std::unique_ptr<Request> r(new Request());
    r->robot = hr;
    r->opts = o;
    r->T = prob->T;
    r->K = prob->K;
    // staging bytes: [candidates][targets][node costs][obstacles], each part
    // starting on an 8-byte boundary; device-resident candidates and targets
    // stay where they are
    const bool dev = prob->mem == CPF_MEM_DEVICE;
    const bool f32 = prob->cand_f32 != nullptr;
    const size_t n_cand = (size_t)prob->K * prob->T * hr.dof, n_tg = (size_t)prob->T * 12;
    const size_t b_cand = dev ? 0 : ((n_cand * (f32 ? sizeof(float) : sizeof(double)) + 7) & ~size_t(7));
    const size_t b_tg = dev ? 0 : n_tg * sizeof(double);
    const size_t n_pen = prob->node_pen ? (size_t)prob->T * prob->K : 0;
    const size_t n_ob = (size_t)prob->n_obstacles * 18;
    const size_t b_all = b_cand + b_tg + (n_pen + n_ob) * sizeof(double);
    char *buf = nullptr;
    if (b_all > 0) {
        r->stage = pinned_get(ctx, b_all, &r->stage_cls);
        buf = (char *)r->stage;
        if (!buf) {
            r->stage_vec.resize((b_all + 7) / 8);
            buf = (char *)r->stage_vec.data();
        }
    }
    cpf_problem &pb = r->prob;
    pb.T = prob->T;
    pb.K = prob->K;
    pb.mem = prob->mem;
    if (dev) {
        pb.cand_f32 = prob->cand_f32;
        pb.targets = prob->targets;
    } else {
        if (f32) {
            pb.cand_f32 = (const float *)buf;
            copy_parallel(buf, prob->cand_f32, n_cand * sizeof(float));
        } else {
            pb.cand = (const double *)buf;
            copy_parallel(buf, prob->cand, n_cand * sizeof(double));
        }
        pb.targets = (const double *)(buf + b_cand);
        memcpy(buf + b_cand, prob->targets, b_tg);
    }
    double *tail = buf ? (double *)(buf + b_cand + b_tg) : nullptr;
    if (n_pen) {
        pb.node_pen = tail;
        copy_parallel(tail, prob->node_pen, n_pen * sizeof(double));
    }
    r->n_obs = prob->n_obstacles;
    pb.n_obstacles = prob->n_obstacles;
    if (n_ob) {
        pb.obstacles = tail + n_pen;
        memcpy(tail + n_pen, prob->obstacles, n_ob * sizeof(double));
    }
    r->bytes = bytes;
    r->t_submit = now_ns();
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (ctx->stop) {
            release_stage(ctx, r.get());
            return fail(CPF_E_STATE, "context is shutting down");
        }
        if (!ctx->server_thread.joinable()) ctx->server_thread = std::thread(server_main, ctx);
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
    if (it == ctx->tickets.end())
        return fail(CPF_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
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
        if (out->path && !r->path.empty())
            memcpy(out->path, r->path.data(), r->path.size() * sizeof(int32_t));
        if (out->xi_valid && !r->xv.empty())
            memcpy(out->xi_valid, r->xv.data(), r->xv.size() * sizeof(double));
        out->report = r->rep;
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
