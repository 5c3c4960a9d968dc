// server.cpp -- serving loop with continuous batching.
//
// Requests (instances) are queued by pamc_server_submit.  A host thread
// admits queued requests, first come first served, whenever their device
// footprint fits the remaining HBM budget and a slot is free; admitted
// instances join the batched step loop at their own step 0 and leave when
// their last step has run.  Because every random number is keyed by the
// instance's own seed and row, a request's result does not depend on what
// else is running.
//
// The loop never drains the device to change its work: steps are queued on
// the main stream in chunks, at most two chunks ahead; admissions (tables,
// initial population) and result reads go through a second stream; device
// memory comes from one arena reserved at creation (no hipMalloc or hipFree
// while serving); an instance that leaves, and work lists that are
// replaced, are released only after an event behind the steps that may
// still read them (Runner serving mode).
#include <algorithm>
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
bool shape_valid(const HostInst &h, int tile_rows, int rp, const char **why);
int tune_shape(HostInst &h, const pamc_options &opt, double *ns_per_attempt);
}

using pamc::HostInst;
using pamc::Runner;

namespace {
constexpr int64_t kServeShapeRows = 100000;  // population the serving shapes are tuned for
}

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
    bool no_room_idle = false;  // the arena had no room with nothing running
    hipEvent_t done = nullptr;  // behind the request's last step, once queued
};

// First-fit allocator over one device allocation; 256-byte granules.  Used
// by the loop thread only (and by creation and destruction).
class Arena {
public:
    ~Arena()
    {
        if (base_) (void)hipFree(base_);
    }
    bool init(size_t bytes)
    {
        bytes = (bytes + 255) & ~size_t(255);
        if (hipMalloc(&base_, bytes) != hipSuccess) {
            base_ = nullptr;
            return false;
        }
        free_[0] = bytes;
        return true;
    }
    void *get(size_t bytes)
    {
        bytes = std::max<size_t>(256, (bytes + 255) & ~size_t(255));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            used_[off] = bytes;
            return static_cast<uint8_t *>(base_) + off;
        }
        return nullptr;
    }
    void put(void *p)
    {
        if (!p) return;
        const size_t off = (size_t)(static_cast<uint8_t *>(p) - static_cast<uint8_t *>(base_));
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t start = off, len = u->second;
        used_.erase(u);
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && nx->first == off + len) {
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == start) {
                start = pv->first;
                len += pv->second;
                free_.erase(pv);
            }
        }
        free_[start] = len;
    }
    // Whether a block of this size could be carved now.
    bool fits(size_t bytes) const
    {
        bytes = (bytes + 255) & ~size_t(255);
        for (const auto &f : free_)
            if (f.second >= bytes) return true;
        return false;
    }

private:
    void *base_ = nullptr;
    std::map<size_t, size_t> free_;  // offset -> length
    std::map<size_t, size_t> used_;  // offset -> length
};

void *arena_alloc(size_t bytes, void *user) { return static_cast<Arena *>(user)->get(bytes); }
void arena_free(void *p, void *user) { static_cast<Arena *>(user)->put(p); }

// Steps queued per chunk: up to kChunk when nobody waits, kChunkWaiting
// when requests are queued (so that memory freed by a leaving instance is
// offered to them soon), and never past the next instance's last step.
constexpr int kChunk = 16;
constexpr int kChunkWaiting = 4;

}  // namespace

struct pamc_server {
    Arena arena;
    Runner run;  // destroyed before the arena
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
    double t_start = 0.0;  // host clock at creation
    double busy_ms = 0.0;  // device time of the steps run so far
    struct Chunk {
        hipEvent_t begin, end;
    };
    std::deque<Chunk> inflight;  // queued chunks, oldest first
    std::vector<hipEvent_t> ev_pool;

    void run_loop();
    hipEvent_t event();
    void recycle(hipEvent_t e) { ev_pool.push_back(e); }
    int retire_chunk(bool wait);
    void fail_all(int st);
};

hipEvent_t pamc_server::event()
{
    if (!ev_pool.empty()) {
        hipEvent_t e = ev_pool.back();
        ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Accounts the oldest queued chunk once it has run (wait: wait for it);
// returns PAMC_OK, PAMC_ERR_BUSY (not yet run) or PAMC_ERR_DEVICE.
int pamc_server::retire_chunk(bool wait)
{
    if (inflight.empty()) return PAMC_OK;
    Chunk c = inflight.front();
    const hipError_t q = wait ? hipEventSynchronize(c.end) : hipEventQuery(c.end);
    if (q == hipErrorNotReady) return PAMC_ERR_BUSY;
    if (q != hipSuccess) {
        pamc::set_error(std::string("server: ") + hipGetErrorString(q));
        return PAMC_ERR_DEVICE;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c.begin, c.end) == hipSuccess) {
        std::lock_guard<std::mutex> lk(mu);
        busy_ms += ms;
    }
    inflight.pop_front();
    recycle(c.begin);
    recycle(c.end);
    return PAMC_OK;
}

void pamc_server::fail_all(int st)
{
    std::lock_guard<std::mutex> lk(mu);
    loop_status = st;
    for (uint64_t id : active) {
        reqs[id].status = st;
        reqs[id].state = kDone;
        reqs[id].t_finish = now_s();
    }
    active.clear();
    stop = true;
}

void pamc_server::run_loop()
{
    bool work_changed = false;
    for (;;) {
        // -- what to admit and what to cancel, under the lock
        std::vector<uint64_t> admit, cancelled;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                if (stop) return;
                // keep the queue's order: stop at the first request that does
                // not fit yet (first come first served)
                size_t inflight_bytes = used;
                const int slots = run.free_slots();
                while (!queue.empty() && slots > (int)admit.size() &&
                       (int)active.size() + (int)admit.size() < max_active) {
                    Request &r = reqs[queue.front()];
                    if (r.cancel) {
                        r.state = kCancelled;
                        r.t_finish = now_s();
                        queue.pop_front();
                        continue;
                    }
                    if (inflight_bytes + r.bytes > budget || !arena.fits(r.bytes)) break;
                    inflight_bytes += r.bytes;
                    admit.push_back(r.id);
                    queue.pop_front();
                }
                used = inflight_bytes;
                for (uint64_t id : active)
                    if (reqs[id].cancel) cancelled.push_back(id);
                if (!active.empty() || !admit.empty() || !inflight.empty()) break;
                cv.wait(lk);
            }
        }
        // -- admissions: tables and initial population through the second
        // stream; the steps already queued keep running
        for (size_t a = 0; a < admit.size(); ++a) {
            const uint64_t id = admit[a];
            Request *r;
            {
                std::lock_guard<std::mutex> lk(mu);
                r = &reqs[id];
            }
            HostInst h = r->h;  // kept for a retry if the arena has no room yet
            const int slot = run.add_instance(std::move(h));
            if (slot == PAMC_ERR_NOMEM) {
                // the budget admits it but the arena is fragmented or still
                // held by fences: back to the head of the queue, with the
                // rest of this pass, until memory is released
                std::lock_guard<std::mutex> lk(mu);
                for (size_t b = admit.size(); b-- > a + 1;) {
                    queue.push_front(admit[b]);
                    used -= reqs[admit[b]].bytes;
                }
                used -= r->bytes;
                admit.resize(a);
                if (active.empty() && r->no_room_idle) {
                    // nothing runs and nothing is held: it will never fit
                    r->status = PAMC_ERR_NOMEM;
                    r->state = kDone;
                    r->t_finish = now_s();
                    ++completed;
                    break;
                }
                queue.push_front(id);
                if (active.empty()) {
                    r->no_room_idle = true;
                    if (run.release_fenced(true) != PAMC_OK) {
                        loop_status = PAMC_ERR_DEVICE;
                        stop = true;
                        return;
                    }
                }
                break;
            }
            const int st = slot < 0 ? slot : run.init_instances({slot});
            if (st == PAMC_ERR_DEVICE || run.poisoned()) {
                fail_all(PAMC_ERR_DEVICE);
                return;
            }
            std::lock_guard<std::mutex> lk(mu);
            if (slot < 0 || st != PAMC_OK) {
                r->status = st;
                r->state = kDone;
                r->t_finish = now_s();
                used -= r->bytes;
                if (slot >= 0) run.remove_instance(slot);
                ++completed;
                continue;
            }
            r->slot = slot;
            r->state = kActive;
            r->no_room_idle = false;
            r->t_admit = now_s();
            active.push_back(id);
            work_changed = true;
        }
        // -- cancellations of running requests (released behind the queue)
        for (uint64_t id : cancelled) {
            std::lock_guard<std::mutex> lk(mu);
            Request &r = reqs[id];
            run.remove_instance(r.slot);
            if (r.done) recycle(r.done);
            r.done = nullptr;
            used -= r.bytes;
            r.state = kCancelled;
            r.t_finish = now_s();
            active.erase(std::find(active.begin(), active.end(), id));
            work_changed = true;
        }
        // -- retire requests whose last step has run
        for (size_t j = 0; j < active.size();) {
            Request *r;
            {
                std::lock_guard<std::mutex> lk(mu);
                r = &reqs[active[j]];
            }
            if (!r->done || hipEventQuery(r->done) != hipSuccess) {
                ++j;
                continue;
            }
            const int nT = run.inst(r->slot).nT;
            int status = run.inst_status(r->slot, nullptr, nullptr);
            std::vector<pamc_step_obs> obs((size_t)nT);
            const int so = run.observables(r->slot, obs.data(), nT);
            if (status == PAMC_OK && so != PAMC_OK) status = so;
            if (status == PAMC_ERR_DEVICE || run.poisoned()) {
                fail_all(PAMC_ERR_DEVICE);
                return;
            }
            run.remove_instance(r->slot);
            recycle(r->done);
            std::lock_guard<std::mutex> lk(mu);
            r->done = nullptr;
            r->obs = std::move(obs);
            r->status = status;
            used -= r->bytes;
            r->state = kDone;
            r->t_finish = now_s();
            ++completed;
            active.erase(active.begin() + (long)j);
            work_changed = true;
        }
        if (run.release_fenced(false) != PAMC_OK) {
            fail_all(PAMC_ERR_DEVICE);
            return;
        }
        if (work_changed) {
            std::vector<int> slots;
            {
                std::lock_guard<std::mutex> lk(mu);
                for (uint64_t id : active) slots.push_back(reqs[id].slot);
            }
            if (run.build_work(slots) != PAMC_OK) {
                fail_all(PAMC_ERR_DEVICE);
                return;
            }
            work_changed = false;
        }
        // -- queue the next chunk of steps, up to the next instance's end
        int until_finish = 1 << 30;
        bool waiting;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (uint64_t id : active) {
                const HostInst &h = run.inst(reqs[id].slot);
                if (h.k_enq < h.nT) until_finish = std::min(until_finish, h.nT - h.k_enq);
            }
            waiting = !queue.empty();
        }
        if (until_finish < (1 << 30)) {
            const int n = std::max(1, std::min(until_finish, waiting ? kChunkWaiting : kChunk));
            const Chunk c{event(), event()};
            if (!c.begin || !c.end) {
                fail_all(PAMC_ERR_DEVICE);
                return;
            }
            int st = hipEventRecord(c.begin, run.stream()) == hipSuccess ? PAMC_OK : PAMC_ERR_DEVICE;
            if (st == PAMC_OK) st = run.enqueue_steps(n);
            // requests whose last step is now queued: an event behind it,
            // recorded before the chunk's end so that it has completed when
            // the chunk has
            if (st == PAMC_OK) {
                std::lock_guard<std::mutex> lk(mu);
                for (uint64_t id : active) {
                    Request &r = reqs[id];
                    if (r.done || run.inst(r.slot).k_enq < run.inst(r.slot).nT) continue;
                    r.done = event();
                    if (!r.done || hipEventRecord(r.done, run.stream()) != hipSuccess) st = PAMC_ERR_DEVICE;
                }
            }
            if (st == PAMC_OK && hipEventRecord(c.end, run.stream()) != hipSuccess) st = PAMC_ERR_DEVICE;
            if (st != PAMC_OK) {
                fail_all(st);
                return;
            }
            inflight.push_back(c);
        }
        // -- at most two chunks ahead of the device; with nothing left to
        // queue, wait for the oldest chunk (the next retirement)
        const bool all_queued = until_finish == (1 << 30);
        while (!inflight.empty()) {
            const bool must_wait = inflight.size() > 2 || all_queued;
            const int st = retire_chunk(must_wait);
            if (st == PAMC_ERR_BUSY) break;
            if (st != PAMC_OK) {
                fail_all(st);
                return;
            }
            if (must_wait) break;
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
    if (s->device >= 0 && hipSetDevice(s->device) != hipSuccess) {
        delete s;
        pamc::set_error("server: hipSetDevice failed");
        return PAMC_ERR_DEVICE;
    }
    // the requests' blocks plus room for the work lists, the instance
    // table and the n ln n table, all carved from one allocation
    const size_t reserve = (size_t(64) << 20) + hbm_budget_bytes / 16;
    if (!s->arena.init(hbm_budget_bytes + reserve)) {
        delete s;
        pamc::set_error("server: device allocation of the arena failed");
        return PAMC_ERR_NOMEM;
    }
    pamc_options o;
    pamc_default_options(&o);
    o.device = s->device;
    o.graphs = 0;  // the work changes with every admission
    o.alloc = arena_alloc;
    o.free = arena_free;
    o.alloc_user = &s->arena;
    int st = s->run.setup(o, s->max_active);
    if (st == PAMC_OK) st = s->run.enable_async(size_t(8) << 20);
    // the n ln n table at the arena's start, sized for populations up to
    // 2^17 rows, so that it rarely grows (and moves) while serving
    if (st == PAMC_OK) st = s->run.reserve_nlnn(int64_t(1) << 17);
    if (st != PAMC_OK) {
        delete s;
        return st;
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
    o.spin_format = s->spin_format;
    o.pop_schedule = inst->pop_schedule;
    Request r;
    int st = pamc::make_inst(inst->L, inst->real_couplings ? nullptr : inst->couplings, inst->real_couplings,
                             inst->R, inst->beta, inst->n_temps, inst->sweeps, inst->seed, o, r.h);
    if (st != PAMC_OK) return st;
    if (s->autotune) {
        // The requests of one lattice size in flight together sweep as one
        // launch of about kServeShapeRows rows: the shape is the one tuned
        // for that population, not for the request alone (whose own tuning
        // favours small tiles to fill the chip by itself), and requests of
        // one size share it, hence one launch per size and step.
        HostInst t = r.h;
        t.R = kServeShapeRows;
        t.Rcap = pamc::default_capacity(kServeShapeRows);
        o.autotune = 1;
        st = pamc::tune_shape(t, o, nullptr);
        if (st != PAMC_OK) return st;
        if (pamc::shape_valid(r.h, t.tile_rows, t.rp, nullptr)) {
            r.h.tile_rows = t.tile_rows;
            r.h.rp = t.rp;
        }
    }
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
    if (s->run.stream()) (void)hipStreamSynchronize(s->run.stream());
    for (auto &c : s->inflight) {
        (void)hipEventDestroy(c.begin);
        (void)hipEventDestroy(c.end);
    }
    for (auto &kv : s->reqs)
        if (kv.second.done) (void)hipEventDestroy(kv.second.done);
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    delete s;
}

}  // extern "C"
