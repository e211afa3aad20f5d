// mxfft_serve.cpp -- request serving: a scheduler thread admits queued
// transform requests in arrival order onto stream slots while the pooled
// plans fit a device-memory budget, and reports per-request times and status.
// A planner thread creates and releases plans, so the scheduler never waits
// on an allocation or a free: it keeps polling completions meanwhile.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mxfft.h"
#include "mxfft_internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;
constexpr int kMaxSlots = 16;
constexpr int kMaxCoils = 65535;

static_assert((int)MXFFT_E4M3 == (int)mxk::MODE_E4M3 && (int)MXFFT_E5M2 == (int)mxk::MODE_E5M2 &&
                  (int)MXFFT_E2M3 == (int)mxk::MODE_E2M3 && (int)MXFFT_E3M2 == (int)mxk::MODE_E3M2,
              "public formats and kernel modes share their values");

struct PooledPlan {
    int n = 0, cap = 0;
    mxfft_params p{};
    mxfft_plan_t plan = nullptr;
    uint64_t bytes = 0;       // device bytes counted against the budget
    bool ready = false;       // created (false while the planner builds it)
    mxfft_status error = MXFFT_OK;   // creation failed
    bool busy = false;        // reserved for, or running, a request
    uint64_t last_use = 0;
};

struct Request {
    mxfft_request r{};
    int state = 0;        // 0 queued, 1 running, 2 done
    int cap = 0;          // plan batch capacity
    uint64_t need = 0;    // device bytes of a new plan for it
    PooledPlan* building = nullptr;   // plan the planner is creating for it
    mxfft_result res{};
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    int32_t* h_status = nullptr;   // pinned copy of the request's status words
    uint64_t ticket = 0;           // 0: free
    PooledPlan* plan = nullptr;
    bool has_status = false;
};

// Plans are shared only between requests of identical parameters; the block
// size matters for every MX element format (MXFP8 and MXFP6).
bool same_params(const mxfft_params& a, const mxfft_params& b)
{
    const bool mx = mxk::is_mx_mode(a.format);
    return a.format == b.format && (!mx || a.block == b.block) && a.k_min == b.k_min && a.k_max == b.k_max &&
           a.flags == b.flags && a.target == b.target && a.tau_pct == b.tau_pct && a.tau_min == b.tau_min;
}

int capacity_of(int coils)
{
    int c = 1;
    while (c < coils) c <<= 1;
    return c > kMaxCoils ? kMaxCoils : c;
}

struct PlanJob {
    bool create;          // create pp's plan, else release it
    PooledPlan* pp;
};

}  // namespace

struct mxfft_server_s {
    uint64_t budget = 0;
    int device = 0;
    Clock::time_point t0;
    hipStream_t setup = nullptr;   // plan uploads (planner thread)
    std::vector<Slot> slots;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Request> reqs;
    std::vector<PooledPlan*> pool;
    std::deque<PlanJob> jobs;      // planner work, in order
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_plan;
    std::thread th, planner;
    bool stop = false, planner_stop = false;
    uint64_t next_ticket = 1, use_clock = 0;
    uint64_t events = 0;           // submissions and finished plan jobs (wakes the idle scheduler)
    uint64_t freeing = 0;          // bytes of evicted plans the planner has yet to free
    mxfft_serve_counters c{};

    double now_ms() const { return std::chrono::duration<double, std::milli>(Clock::now() - t0).count(); }

    void finish(Request& q, int32_t status)
    {
        q.res.status = status;
        q.res.t_done_ms = now_ms();
        q.state = 2;
        c.completed++;
        cv_done.notify_all();
    }

    void remove_from_pool(PooledPlan* pp)
    {
        for (size_t i = 0; i < pool.size(); i++)
            if (pool[i] == pp) {
                pool.erase(pool.begin() + i);
                return;
            }
    }

    // Planner thread: creates plans on its own stream and releases evicted
    // ones, without the server lock; the bytes of an evicted plan stay
    // counted until it is freed.
    void plan_loop()
    {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            cv_plan.wait(lk, [&] { return planner_stop || !jobs.empty(); });
            if (jobs.empty()) break;
            const PlanJob j = jobs.front();
            jobs.pop_front();
            PooledPlan* pp = j.pp;
            lk.unlock();
            mxfft_status st = MXFFT_OK;
            mxfft_plan_t h = nullptr;
            if (j.create) st = mxfft_plan(&h, pp->n, pp->cap, &pp->p, setup);
            else mxk::plan_release_idle(pp->plan);   // idle: its last event has completed
            lk.lock();
            if (j.create) {
                const uint64_t reserved = pp->bytes;
                if (st == MXFFT_OK) {
                    pp->plan = h;
                    pp->bytes = mxfft_plan_device_bytes(h);
                    c.plans_created++;
                } else {
                    pp->error = st;
                    pp->bytes = 0;
                }
                c.plan_bytes = c.plan_bytes - reserved + pp->bytes;
                if (c.plan_bytes > c.peak_plan_bytes) c.peak_plan_bytes = c.plan_bytes;
                pp->ready = true;
            } else {
                c.plan_bytes -= pp->bytes;
                freeing -= pp->bytes;
                c.plans_evicted++;
                delete pp;
            }
            events++;
            cv_work.notify_all();
        }
    }

    // The plan for the head-of-queue request q.  Returns a ready plan, or
    // nullptr to wait (a plan being created, or running requests holding the
    // budget); *err is set when creation failed.
    PooledPlan* acquire(Request& q, mxfft_status* err)
    {
        *err = MXFFT_OK;
        if (PooledPlan* pp = q.building) {
            if (!pp->ready) return nullptr;
            q.building = nullptr;
            if (pp->error != MXFFT_OK) {
                *err = pp->error;
                remove_from_pool(pp);
                delete pp;
                return nullptr;
            }
            return pp;
        }
        for (PooledPlan* pp : pool)
            if (pp->ready && !pp->busy && pp->n == q.r.n && pp->cap == q.cap && same_params(pp->p, q.r.params)) {
                pp->busy = true;
                return pp;
            }
        // evict idle plans, least recently used first, until the plans that
        // stay fit with the new one; then wait until they are freed
        bool queued = false;
        while (c.plan_bytes - freeing + q.need > budget) {
            PooledPlan* victim = nullptr;
            for (PooledPlan* pp : pool)
                if (pp->ready && !pp->busy && (!victim || pp->last_use < victim->last_use)) victim = pp;
            if (!victim) break;   // running requests hold the rest of the budget
            remove_from_pool(victim);
            freeing += victim->bytes;
            jobs.push_back({false, victim});
            queued = true;
        }
        if (queued) cv_plan.notify_one();
        if (c.plan_bytes + q.need > budget) return nullptr;
        PooledPlan* pp = new PooledPlan();
        pp->n = q.r.n;
        pp->cap = q.cap;
        pp->p = q.r.params;
        pp->bytes = q.need;          // reserved until the planner reports the plan's own size
        pp->busy = true;
        c.plan_bytes += q.need;
        if (c.plan_bytes > c.peak_plan_bytes) c.peak_plan_bytes = c.plan_bytes;
        pool.push_back(pp);
        jobs.push_back({true, pp});
        q.building = pp;
        cv_plan.notify_one();
        return nullptr;
    }

    // Enqueue q on slot si with plan pp (reserved: busy).  When an enqueue
    // fails the request is finished at once with that status and the slot
    // stays free.
    void launch(uint64_t ticket, Request& q, PooledPlan* pp, int si)
    {
        Slot& s = slots[si];
        pp->last_use = ++use_clock;
        q.state = 1;
        q.res.slot = si;
        q.res.t_start_ms = now_ms();
        const mxfft_request& r = q.r;
        mxfft_status st = MXFFT_OK;
        if (r.ready && hipStreamWaitEvent(s.stream, (hipEvent_t)r.ready, 0) != hipSuccess) st = MXFFT_EHIP;
        if (st == MXFFT_OK) {
            switch (r.op) {
            case 0: st = mxfft_forward(pp->plan, r.in, r.out, r.coils, r.k_out, s.stream); break;
            case 1: st = mxfft_inverse(pp->plan, r.in, r.out, r.coils, nullptr, s.stream); break;
            default: st = mxfft_roundtrip(pp->plan, r.in, r.out, r.coils, r.k_out, s.stream); break;
            }
        }
        s.has_status = mxk::plan_has_status(pp->plan);
        if (st == MXFFT_OK && s.has_status &&
            hipMemcpyAsync(s.h_status, mxk::plan_status_words(pp->plan), sizeof(int32_t) * (size_t)r.coils,
                           hipMemcpyDeviceToHost, s.stream) != hipSuccess)
            st = MXFFT_EHIP;
        if (st == MXFFT_OK && hipEventRecord(s.done, s.stream) != hipSuccess) st = MXFFT_EHIP;
        c.admitted++;
        if (st != MXFFT_OK) {
            pp->busy = false;
            finish(q, st);
            return;
        }
        s.ticket = ticket;
        s.plan = pp;
        c.in_flight++;
    }

    void loop()
    {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        uint64_t seen = 0;
        for (;;) {
            bool busy = false;
            seen = events;
            // completions
            for (Slot& s : slots) {
                if (!s.ticket) continue;
                const hipError_t e = hipEventQuery(s.done);
                if (e == hipErrorNotReady) {
                    busy = true;
                    continue;
                }
                Request& q = reqs[s.ticket];
                int32_t status = (e == hipSuccess) ? MXFFT_OK : MXFFT_EHIP;
                if (e == hipSuccess && s.has_status)
                    for (int i = 0; i < q.r.coils; i++)
                        if (s.h_status[i] != 0) {
                            status = s.h_status[i];
                            break;
                        }
                s.plan->busy = false;
                s.plan->last_use = ++use_clock;
                s.ticket = 0;
                s.plan = nullptr;
                c.in_flight--;
                finish(q, status);
            }
            // admissions, in arrival order
            while (!queue.empty()) {
                int si = -1;
                for (int i = 0; i < (int)slots.size(); i++)
                    if (!slots[i].ticket) {
                        si = i;
                        break;
                    }
                if (si < 0) break;
                const uint64_t t = queue.front();
                Request& q = reqs[t];
                mxfft_status err;
                PooledPlan* pp = acquire(q, &err);
                if (!pp && err == MXFFT_OK) break;   // wait for a plan or for budget
                queue.pop_front();
                c.queued--;
                if (!pp) {
                    c.admitted++;
                    finish(q, err);
                    continue;
                }
                launch(t, q, pp, si);
                if (slots[si].ticket) busy = true;
            }
            if (stop && queue.empty() && !busy) break;
            if (busy) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            } else {
                // idle: until a submission, a finished plan job or stop
                cv_work.wait(lk, [&] { return stop || events != seen; });
            }
        }
    }
};

extern "C" {

mxfft_status mxfft_serve_create(mxfft_server_t* out, uint64_t hbm_budget_bytes, int32_t slots)
{
    if (!out || slots < 1 || slots > kMaxSlots || hbm_budget_bytes == 0) return MXFFT_EINVAL;
    *out = nullptr;
    mxfft_server_s* s = new mxfft_server_s();
    s->budget = hbm_budget_bytes;
    s->c.budget = hbm_budget_bytes;
    s->t0 = Clock::now();
    bool ok = hipGetDevice(&s->device) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&s->setup, hipStreamNonBlocking) == hipSuccess;
    s->slots.resize(slots);
    for (Slot& sl : s->slots) {
        ok = ok && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess;
        ok = ok && hipHostMalloc((void**)&sl.h_status, sizeof(int32_t) * kMaxCoils, hipHostMallocDefault) == hipSuccess;
    }
    if (!ok) {
        for (Slot& sl : s->slots) {
            if (sl.h_status) (void)hipHostFree(sl.h_status);
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
        }
        if (s->setup) (void)hipStreamDestroy(s->setup);
        delete s;
        return MXFFT_EHIP;
    }
    s->planner = std::thread([s] { s->plan_loop(); });
    s->th = std::thread([s] { s->loop(); });
    *out = s;
    return MXFFT_OK;
}

mxfft_status mxfft_serve_submit(mxfft_server_t srv, const mxfft_request* req, uint64_t* ticket)
{
    if (!srv || !req || !ticket || !req->in || !req->out) return MXFFT_EINVAL;
    if (req->coils < 1 || req->coils > kMaxCoils || req->op < 0 || req->op > 2) return MXFFT_EINVAL;
    Request q;
    q.r = *req;
    q.cap = capacity_of(req->coils);
    const mxfft_status st = mxfft_plan_bytes(req->n, q.cap, &req->params, &q.need);
    if (st != MXFFT_OK) return st;
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->c.submitted++;
    if (q.need > srv->budget) {
        srv->c.rejected++;
        return MXFFT_EBUDGET;
    }
    q.res.t_submit_ms = srv->now_ms();
    const uint64_t t = srv->next_ticket++;
    srv->reqs.emplace(t, q);
    srv->queue.push_back(t);
    srv->c.queued++;
    srv->events++;
    *ticket = t;
    srv->cv_work.notify_one();
    return MXFFT_OK;
}

mxfft_status mxfft_serve_wait(mxfft_server_t srv, uint64_t ticket, mxfft_result* res)
{
    if (!srv || !res) return MXFFT_EINVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->reqs.find(ticket) == srv->reqs.end()) return MXFFT_EINVAL;
    srv->cv_done.wait(lk, [&] {
        auto it = srv->reqs.find(ticket);
        return it == srv->reqs.end() || it->second.state == 2;
    });
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return MXFFT_EINVAL;   // answered to another waiter
    *res = it->second.res;
    srv->reqs.erase(it);
    return MXFFT_OK;
}

mxfft_status mxfft_serve_poll(mxfft_server_t srv, uint64_t ticket, mxfft_result* res)
{
    if (!srv || !res) return MXFFT_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return MXFFT_EINVAL;
    if (it->second.state != 2) return MXFFT_EBUSY;
    *res = it->second.res;
    srv->reqs.erase(it);
    return MXFFT_OK;
}

mxfft_status mxfft_serve_stats(mxfft_server_t srv, mxfft_serve_counters* out)
{
    if (!srv || !out) return MXFFT_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->c;
    return MXFFT_OK;
}

mxfft_status mxfft_serve_destroy(mxfft_server_t srv)
{
    if (!srv) return MXFFT_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv_work.notify_all();
    }
    srv->th.join();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->planner_stop = true;
        srv->cv_plan.notify_all();
    }
    srv->planner.join();   // finishes its queued jobs first
    for (PooledPlan* pp : srv->pool) {
        if (pp->plan) mxfft_plan_destroy(pp->plan);
        delete pp;
    }
    for (Slot& sl : srv->slots) {
        (void)hipHostFree(sl.h_status);
        (void)hipEventDestroy(sl.done);
        (void)hipStreamDestroy(sl.stream);
    }
    (void)hipStreamDestroy(srv->setup);
    delete srv;
    return MXFFT_OK;
}

}  // extern "C"
