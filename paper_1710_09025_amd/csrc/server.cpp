// server.cpp -- serving loop with continuous batching.
//
// Requests (instances) are queued by pamc_server_submit.  A host thread
// admits queued requests, first come first served, whenever their device
// footprint fits the remaining HBM budget and a slot is free; admitted
// instances join the batched step loop at their own step 0 and leave when
// their last step has run.  Because every random number is keyed by the
// instance's own seed and row, a request's result does not depend on what
// else is running.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "runner.h"

namespace pamc {
int make_inst(int L, const int8_t *J, const int32_t *Jq, int64_t R, const double *beta, int nT, int NS,
              uint64_t seed, const pamc_options &opt, HostInst &h);
void tune_cache_load();
}

using pamc::HostInst;
using pamc::Runner;

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

enum ReqState { kQueued = 0, kActive = 1, kDone = 2, kCancelled = 3 };

struct Request {
    uint64_t id = 0;
    HostInst h;
    size_t bytes = 0;
    int state = kQueued;
    int slot = -1;
    int status = PAMC_OK;
    int n_temps = 0;
    std::vector<pamc_step_obs> obs;
    double t_submit = 0, t_admit = 0, t_finish = 0;
    bool cancel = false;
};

}  // namespace

struct pamc_server {
    Runner run;
    size_t budget = 0;
    size_t used = 0;
    int max_active = 256;
    int device = -1;
    bool autotune = false;  // sweep shapes chosen by measurement at submission
    int spin_format = PAMC_SPINS_INT8;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> queue;
    std::map<uint64_t, Request> reqs;
    std::vector<uint64_t> active;  // request ids on the device
    std::thread loop;
    bool stop = false;
    uint64_t next_id = 1;
    int64_t completed = 0;
    int loop_status = PAMC_OK;
    double t_start = 0.0;   // host clock at creation
    double busy_ms = 0.0;   // device time of the steps run so far
    hipEvent_t ev_busy[2] = {nullptr, nullptr};

    void run_loop();
};

void pamc_server::run_loop()
{
    bool work_changed = false;
    for (;;) {
        std::vector<uint64_t> admit;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                if (stop) return;
                // drop cancelled requests still in the queue
                while (!queue.empty() && reqs[queue.front()].cancel) {
                    reqs[queue.front()].state = kCancelled;
                    queue.pop_front();
                }
                size_t inflight = used;
                int nact = (int)active.size();
                while (!queue.empty() && nact + (int)admit.size() < max_active) {
                    Request &r = reqs[queue.front()];
                    if (r.cancel) {
                        r.state = kCancelled;
                        queue.pop_front();
                        continue;
                    }
                    if (inflight + r.bytes > budget) break;  // first come first served
                    inflight += r.bytes;
                    admit.push_back(r.id);
                    queue.pop_front();
                }
                used = inflight;
                if (!active.empty() || !admit.empty()) break;
                cv.wait(lk);
            }
        }
        // admissions: device memory, tables, initial population
        for (uint64_t id : admit) {
            Request *r;
            {
                std::lock_guard<std::mutex> lk(mu);
                r = &reqs[id];
            }
            const int slot = run.add_instance(std::move(r->h));
            int st = slot < 0 ? slot : run.init_instances({slot});
            std::lock_guard<std::mutex> lk(mu);
            if (slot < 0 || st != PAMC_OK) {
                r->status = slot < 0 ? slot : st;
                r->state = kDone;
                r->t_finish = now_s();
                used -= r->bytes;
                if (slot >= 0) run.remove_instance(slot);
                ++completed;
                continue;
            }
            r->slot = slot;
            r->state = kActive;
            r->t_admit = now_s();
            active.push_back(id);
            work_changed = true;
        }
        // cancellations of running requests
        {
            std::lock_guard<std::mutex> lk(mu);
            for (size_t j = 0; j < active.size();) {
                Request &r = reqs[active[j]];
                if (r.cancel) {
                    run.remove_instance(r.slot);
                    used -= r.bytes;
                    r.state = kCancelled;
                    r.t_finish = now_s();
                    active.erase(active.begin() + (long)j);
                    work_changed = true;
                } else {
                    ++j;
                }
            }
        }
        if (active.empty()) continue;
        if (work_changed) {
            std::vector<int> slots;
            for (uint64_t id : active) slots.push_back(reqs[id].slot);
            if (run.build_work(slots) != PAMC_OK) {
                std::lock_guard<std::mutex> lk(mu);
                loop_status = PAMC_ERR_DEVICE;
                stop = true;
                return;
            }
            work_changed = false;
        }
        // run steps: as many as possible before the next instance finishes,
        // but return to admission after a few steps when requests wait
        int until_finish = 1 << 30;
        for (uint64_t id : active) {
            const HostInst &h = run.inst(reqs[id].slot);
            until_finish = std::min(until_finish, h.nT - h.k_enq);
        }
        bool waiting;
        {
            std::lock_guard<std::mutex> lk(mu);
            waiting = !queue.empty();
        }
        const int nsteps = std::max(1, std::min(until_finish, waiting ? 1 : 16));
        (void)hipEventRecord(ev_busy[0], run.stream());
        int st = run.enqueue_steps(nsteps);
        (void)hipEventRecord(ev_busy[1], run.stream());
        if (st == PAMC_OK) st = run.sync();
        if (st == PAMC_OK) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev_busy[0], ev_busy[1]) == hipSuccess) {
                std::lock_guard<std::mutex> lk(mu);
                busy_ms += ms;
            }
        }
        if (st != PAMC_OK) {
            std::lock_guard<std::mutex> lk(mu);
            loop_status = st;
            for (uint64_t id : active) {
                reqs[id].status = st;
                reqs[id].state = kDone;
                reqs[id].t_finish = now_s();
            }
            active.clear();
            stop = true;
            return;
        }
        // retire finished instances
        std::lock_guard<std::mutex> lk(mu);
        for (size_t j = 0; j < active.size();) {
            Request &r = reqs[active[j]];
            const HostInst &h = run.inst(r.slot);
            if (h.k_enq >= h.nT) {
                r.status = run.inst_status(r.slot, nullptr, nullptr);
                r.obs.resize((size_t)h.nT);
                const int so = run.observables(r.slot, r.obs.data(), h.nT);
                if (r.status == PAMC_OK && so != PAMC_OK) r.status = so;
                run.remove_instance(r.slot);
                used -= r.bytes;
                r.state = kDone;
                r.t_finish = now_s();
                ++completed;
                active.erase(active.begin() + (long)j);
                work_changed = true;
            } else {
                ++j;
            }
        }
    }
}

extern "C" {

int pamc_server_create(size_t hbm_budget_bytes, const pamc_server_options *opt, pamc_server **out)
{
    if (!out || hbm_budget_bytes == 0) {
        pamc::set_error("server: invalid arguments");
        return PAMC_ERR_INVALID;
    }
    *out = nullptr;
    pamc_server *s = new (std::nothrow) pamc_server();
    if (!s) return PAMC_ERR_NOMEM;
    s->budget = hbm_budget_bytes;
    s->max_active = (opt && opt->max_active > 0) ? opt->max_active : 256;
    s->device = opt ? opt->device : -1;
    s->autotune = opt && opt->autotune;
    s->spin_format = opt ? opt->spin_format : PAMC_SPINS_INT8;
    if (s->autotune) pamc::tune_cache_load();
    pamc_options o;
    pamc_default_options(&o);
    o.device = s->device;
    int st = s->run.setup(o, s->max_active);
    if (st != PAMC_OK) {
        delete s;
        return st;
    }
    if (hipEventCreate(&s->ev_busy[0]) != hipSuccess || hipEventCreate(&s->ev_busy[1]) != hipSuccess) {
        delete s;
        pamc::set_error("server: hipEventCreate failed");
        return PAMC_ERR_DEVICE;
    }
    s->t_start = now_s();
    s->loop = std::thread([s] { s->run_loop(); });
    *out = s;
    return PAMC_OK;
}

int pamc_server_submit(pamc_server *s, const pamc_instance *inst, uint64_t *req_id)
{
    if (!s || !inst || !req_id) {
        pamc::set_error("server submit: NULL argument");
        return PAMC_ERR_INVALID;
    }
    pamc_options o;
    pamc_default_options(&o);
    o.device = s->device;
    o.autotune = s->autotune ? 1 : 0;
    o.spin_format = s->spin_format;
    o.pop_schedule = inst->pop_schedule;
    Request r;
    int st = pamc::make_inst(inst->L, inst->real_couplings ? nullptr : inst->couplings, inst->real_couplings,
                             inst->R, inst->beta, inst->n_temps, inst->sweeps, inst->seed, o, r.h);
    if (st != PAMC_OK) return st;
    r.bytes = pamc::inst_device_bytes(inst->L, r.h.Rcap, inst->n_temps, r.h.ovl_n, r.h.packed != 0,
                                      r.h.real != 0) +
              4096;
    r.n_temps = inst->n_temps;
    if (r.bytes > s->budget) {
        pamc::set_error("request needs " + std::to_string(r.bytes) + " bytes, more than the budget");
        return PAMC_ERR_REJECTED;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
        pamc::set_error("server stopped");
        return s->loop_status != PAMC_OK ? s->loop_status : PAMC_ERR_STATE;
    }
    r.id = s->next_id++;
    r.t_submit = now_s();
    *req_id = r.id;
    s->queue.push_back(r.id);
    s->reqs.emplace(r.id, std::move(r));
    s->cv.notify_one();
    return PAMC_OK;
}

int pamc_server_poll(pamc_server *s, uint64_t req_id, pamc_result *out)
{
    if (!s || !out) {
        pamc::set_error("server poll: NULL argument");
        return PAMC_ERR_INVALID;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) {
        pamc::set_error("unknown request id");
        return PAMC_ERR_INVALID;
    }
    Request &r = it->second;
    if (r.state == kQueued || r.state == kActive) return PAMC_ERR_BUSY;
    out->status = r.state == kCancelled ? PAMC_ERR_STATE : r.status;
    out->n_temps = r.n_temps;
    out->submit_time_s = r.t_submit;
    out->admit_time_s = r.t_admit;
    out->finish_time_s = r.t_finish;
    if (out->obs && !r.obs.empty()) std::memcpy(out->obs, r.obs.data(), sizeof(pamc_step_obs) * r.obs.size());
    return PAMC_OK;
}

int pamc_server_cancel(pamc_server *s, uint64_t req_id)
{
    if (!s) return PAMC_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) {
        pamc::set_error("unknown request id");
        return PAMC_ERR_INVALID;
    }
    if (it->second.state == kDone || it->second.state == kCancelled) return PAMC_ERR_STATE;
    it->second.cancel = true;
    s->cv.notify_one();
    return PAMC_OK;
}

int pamc_server_stats(pamc_server *s, int64_t *completed, int64_t *queued, int64_t *active)
{
    if (!s) return PAMC_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    if (completed) *completed = s->completed;
    if (queued) *queued = (int64_t)s->queue.size();
    if (active) *active = (int64_t)s->active.size();
    return s->loop_status;
}

int pamc_server_usage(pamc_server *s, size_t *used_bytes, size_t *budget_bytes, double *busy_s, double *wall_s)
{
    if (!s) return PAMC_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    if (used_bytes) *used_bytes = s->used;
    if (budget_bytes) *budget_bytes = s->budget;
    if (busy_s) *busy_s = s->busy_ms * 1e-3;
    if (wall_s) *wall_s = now_s() - s->t_start;
    return s->loop_status;
}

void pamc_server_destroy(pamc_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->loop.joinable()) s->loop.join();
    for (hipEvent_t e : s->ev_busy)
        if (e) (void)hipEventDestroy(e);
    delete s;
}

}  // extern "C"
