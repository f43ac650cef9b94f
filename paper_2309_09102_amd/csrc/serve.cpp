// serve.cpp -- continuously batched request server behind cpf_submit /
// cpf_poll.
//
// The device holds a fixed table of `slots` plan descriptors (the work list)
// and their LM states in one contiguous array.  One server thread runs ticks:
//   1. admit queued requests while a slot is free and their arena fits the
//      memory budget (upload on the server stream);
//   2. search the newly admitted requests in one launch (one workgroup each);
//   3. replay the LM tick graph: lm_kernel<float> and lm_kernel<double> over
//      every slot (each skips empty slots and the other precision), each
//      plan advancing up to `iters_per_tick` iterations, then the report
//      kernel for plans that just finished;
//   4. read all slot states back in one copy and retire finished requests.
// Requests submitted while a tick runs join at the next tick, so their work
// overlaps on the device with the requests already in flight.  The graph is
// captured once per context: its kernels read the work list from device
// memory, so admissions and retirements only rewrite descriptor slots
// between replays.
#include <algorithm>
#include <cstring>
#include <memory>

#include "runtime.h"

namespace cpf {

struct Request {
    uint64_t ticket = 0;
    HostRobot robot{};
    cpf_opts opts{};
    int T = 0, K = 0;
    std::vector<double> targets, cand, node_pen;
    uint64_t bytes = 0;
    cpf_plan *plan = nullptr;
    std::vector<char> staging;
    int slot = -1;
    bool done = false;
    cpf_status status = CPF_OK;
    std::vector<double> xi;
    std::vector<int32_t> path;
    cpf_lm_report report{};
    double best = 0, smjac = 0;
    int64_t t_submit = 0, t_admit = 0, t_search = 0, t_done = 0;
};

struct Server {
    int cap = 0;
    int ipt = 0;
    hipStream_t s = nullptr;
    DevPlan *d_work = nullptr;     // [cap]
    LMState *d_states = nullptr;   // [cap]
    DevPlan *d_new = nullptr;      // [cap] descriptors of the tick's admissions
    std::vector<DevPlan> h_work;
    std::vector<LMState> h_states;
    std::vector<Request *> slot_req;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

cpf_status server_init(cpf_ctx *ctx, Server *sv) {
    sv->cap = ctx->slots;
    sv->ipt = ctx->iters_per_tick;
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipStreamCreateWithFlags(&sv->s, hipStreamNonBlocking));
    HIP_TRY(hipMalloc((void **)&sv->d_work, sizeof(DevPlan) * sv->cap));
    HIP_TRY(hipMalloc((void **)&sv->d_states, sizeof(LMState) * sv->cap));
    HIP_TRY(hipMalloc((void **)&sv->d_new, sizeof(DevPlan) * sv->cap));
    sv->h_work.assign(sv->cap, DevPlan{});     // T = 0: empty slot
    sv->h_states.assign(sv->cap, LMState{});
    sv->slot_req.assign(sv->cap, nullptr);
    HIP_TRY(hipMemcpyAsync(sv->d_work, sv->h_work.data(), sizeof(DevPlan) * sv->cap,
                           hipMemcpyHostToDevice, sv->s));
    HIP_TRY(hipMemcpyAsync(sv->d_states, sv->h_states.data(), sizeof(LMState) * sv->cap,
                           hipMemcpyHostToDevice, sv->s));
    HIP_TRY(hipStreamSynchronize(sv->s));
    // Capture the LM tick: both precisions over every slot, then the report
    // for plans that finished in this tick.
    HIP_TRY(hipStreamBeginCapture(sv->s, hipStreamCaptureModeThreadLocal));
    hipError_t e = lm_launch(sv->d_work, sv->cap, 0, sv->ipt, sv->s);
    if (e == hipSuccess) e = lm_launch(sv->d_work, sv->cap, 1, sv->ipt, sv->s);
    if (e == hipSuccess) e = eval_launch(sv->d_work, sv->cap, 1, sv->s);
    hipError_t e2 = hipStreamEndCapture(sv->s, &sv->graph);
    if (e != hipSuccess) return fail(CPF_E_DEVICE, "tick capture: %s", hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(CPF_E_DEVICE, "tick capture end: %s", hipGetErrorString(e2));
    HIP_TRY(hipGraphInstantiate(&sv->exec, sv->graph, nullptr, nullptr, 0));
    return CPF_OK;
}

void server_free(Server *sv) {
    if (sv->s) HIP_IGNORE(hipStreamSynchronize(sv->s));
    if (sv->exec) HIP_IGNORE(hipGraphExecDestroy(sv->exec));
    if (sv->graph) HIP_IGNORE(hipGraphDestroy(sv->graph));
    if (sv->d_work) HIP_IGNORE(hipFree(sv->d_work));
    if (sv->d_states) HIP_IGNORE(hipFree(sv->d_states));
    if (sv->d_new) HIP_IGNORE(hipFree(sv->d_new));
    if (sv->s) HIP_IGNORE(hipStreamDestroy(sv->s));
}

// Finish a request: read its results, free its plan and slot, wake pollers.
void retire(cpf_ctx *ctx, Server *sv, Request *r, cpf_status dev_status) {
    if (r->plan && dev_status == CPF_OK) {
        PlanReadback rb;
        r->xi.resize((size_t)r->T * NJ);
        r->path.resize(r->T);
        cpf_status st = read_plan(r->plan, sv->s, sv->d_states + r->slot, &rb, r->xi.data(),
                                  r->path.data());
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
    if (r->slot >= 0) {
        sv->h_work[r->slot] = DevPlan{};
        HIP_IGNORE(hipMemcpyAsync(sv->d_work + r->slot, &sv->h_work[r->slot], sizeof(DevPlan),
                                  hipMemcpyHostToDevice, sv->s));
        HIP_IGNORE(hipStreamSynchronize(sv->s));
        sv->slot_req[r->slot] = nullptr;
        r->slot = -1;
    }
    if (r->plan) {
        plan_destroy(r->plan);
        r->plan = nullptr;
    }
    r->cand.clear();
    r->cand.shrink_to_fit();
    r->staging.clear();
    r->staging.shrink_to_fit();
    r->t_done = now_ns();
    std::lock_guard<std::mutex> lk(ctx->mu);
    r->done = true;
    ctx->cv_done.notify_all();
}

void server_main(cpf_ctx *ctx) {
    std::unique_ptr<Server> sv(new Server());
    cpf_status init = server_init(ctx, sv.get());
    std::vector<Request *> active;
    while (true) {
        std::vector<Request *> admitted;
        {
            std::unique_lock<std::mutex> lk(ctx->mu);
            ctx->cv_work.wait(lk, [&] { return ctx->stop || !ctx->pending.empty() || !active.empty(); });
            if (ctx->stop && ctx->pending.empty() && active.empty()) break;
            int free_slots = sv->cap - (int)active.size();
            uint64_t planned = 0;
            while (!ctx->pending.empty() && free_slots > 0 && init == CPF_OK) {
                Request *r = ctx->pending.front();
                if (ctx->used.load() + planned + r->bytes > ctx->budget) break;   // wait for budget
                ctx->pending.pop_front();
                admitted.push_back(r);
                planned += r->bytes;
                --free_slots;
            }
            if (init != CPF_OK) {   // no device server: fail everything queued
                while (!ctx->pending.empty()) {
                    admitted.push_back(ctx->pending.front());
                    ctx->pending.pop_front();
                }
            }
        }
        if (init != CPF_OK) {
            for (Request *r : admitted) retire(ctx, sv.get(), r, init);
            continue;
        }
        // 1. upload and place the admitted requests
        std::vector<DevPlan> fresh;
        int maxK = 0, maxT = 0;
        for (Request *r : admitted) {
            cpf_problem pb{r->T, r->K, r->targets.data(), r->cand.data(),
                           r->node_pen.empty() ? nullptr : r->node_pen.data()};
            r->t_admit = now_ns();
            cpf_status st = plan_create(ctx, r->robot, &pb, &r->opts, r->opts.iters, sv->s,
                                        r->staging, &r->plan);
            if (st != CPF_OK) {
                r->plan = nullptr;
                retire(ctx, sv.get(), r, st);
                continue;
            }
            int slot = 0;
            while (sv->slot_req[slot]) ++slot;
            r->slot = slot;
            sv->slot_req[slot] = r;
            DevPlan d = r->plan->desc;
            set_dev_ptr(d.st, sv->d_states + slot);
            sv->h_work[slot] = d;
            LMState &ls = sv->h_states[slot];
            memset(&ls, 0, sizeof(ls));
            ls.lambda = r->opts.lambda0;
            ls.nu = 2.0;
            ls.iters_target = r->opts.iters;
            HIP_IGNORE(hipMemcpyAsync(sv->d_states + slot, &ls, sizeof(LMState),
                                      hipMemcpyHostToDevice, sv->s));
            HIP_IGNORE(hipMemcpyAsync(sv->d_work + slot, &sv->h_work[slot], sizeof(DevPlan),
                                      hipMemcpyHostToDevice, sv->s));
            fresh.push_back(d);
            maxK = std::max(maxK, r->K);
            maxT = std::max(maxT, r->T);
            active.push_back(r);
        }
        cpf_status dev = CPF_OK;
        // 2. search the admitted requests
        if (!fresh.empty()) {
            hipError_t e = hipMemcpyAsync(sv->d_new, fresh.data(), sizeof(DevPlan) * fresh.size(),
                                          hipMemcpyHostToDevice, sv->s);
            if (e == hipSuccess)
                e = timed(ctx, KIND_DP, sv->s,
                          [&] { return dp_launch(sv->d_new, (int)fresh.size(), maxK, maxT, sv->s); });
            if (e == hipSuccess) e = hipStreamSynchronize(sv->s);
            if (e != hipSuccess) dev = fail(CPF_E_DEVICE, "search launch: %s", hipGetErrorString(e));
            const int64_t ts = now_ns();
            for (Request *r : admitted)
                if (r->plan) r->t_search = ts;
        }
        // 3. one LM tick over every slot
        if (dev == CPF_OK && !active.empty()) {
            hipError_t e = timed(ctx, KIND_LM, sv->s, [&] { return hipGraphLaunch(sv->exec, sv->s); });
            if (e == hipSuccess)
                e = hipMemcpyAsync(sv->h_states.data(), sv->d_states, sizeof(LMState) * sv->cap,
                                   hipMemcpyDeviceToHost, sv->s);
            if (e == hipSuccess) e = hipStreamSynchronize(sv->s);
            if (e != hipSuccess) dev = fail(CPF_E_DEVICE, "LM tick: %s", hipGetErrorString(e));
        }
        // 4. retire finished (or failed) requests
        std::vector<Request *> still;
        for (Request *r : active) {
            bool finished = dev != CPF_OK;
            if (!finished) {
                const LMState &ls = sv->h_states[r->slot];
                finished = ls.status != 0 || (ls.iters_done >= r->opts.iters && ls.reported);
            }
            if (finished) retire(ctx, sv.get(), r, dev);
            else still.push_back(r);
        }
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

extern "C" cpf_status cpf_ctx_config(cpf_ctx *ctx, int32_t slots, int32_t iters_per_tick) {
    if (!ctx) return fail(CPF_E_ARG, "ctx is NULL");
    if (slots < 1 || slots > 65536 || iters_per_tick < 1 || iters_per_tick > 100000)
        return fail(CPF_E_ARG, "slots %d / iters_per_tick %d out of range", slots, iters_per_tick);
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->server_thread.joinable()) return fail(CPF_E_STATE, "server already running");
    ctx->slots = slots;
    ctx->iters_per_tick = iters_per_tick;
    return CPF_OK;
}

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
