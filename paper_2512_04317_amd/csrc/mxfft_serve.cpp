// mxfft_serve.cpp -- request serving: a scheduler thread admits queued
// transform requests in arrival order onto stream slots while the pooled
// plans fit a device-memory budget, and reports per-request times and status.
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

struct PooledPlan {
    int n = 0, cap = 0;
    mxfft_params p{};
    mxfft_plan_t plan = nullptr;
    uint64_t bytes = 0;
    bool busy = false;
    uint64_t last_use = 0;
};

struct Request {
    mxfft_request r{};
    int state = 0;        // 0 queued, 1 running, 2 done
    int cap = 0;          // plan batch capacity
    uint64_t need = 0;    // device bytes of a new plan for it
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

bool same_params(const mxfft_params& a, const mxfft_params& b)
{
    const bool mx = a.format == MXFFT_E4M3 || a.format == MXFFT_E5M2;
    return a.format == b.format && (!mx || a.block == b.block) && a.k_min == b.k_min && a.k_max == b.k_max &&
           a.flags == b.flags && a.target == b.target && a.tau_pct == b.tau_pct && a.tau_min == b.tau_min;
}

int capacity_of(int coils)
{
    int c = 1;
    while (c < coils) c <<= 1;
    return c > kMaxCoils ? kMaxCoils : c;
}

}  // namespace

struct mxfft_server_s {
    uint64_t budget = 0;
    int device = 0;
    Clock::time_point t0;
    hipStream_t setup = nullptr;   // plan uploads
    std::vector<Slot> slots;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Request> reqs;
    std::vector<PooledPlan*> pool;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread th;
    bool stop = false;
    uint64_t next_ticket = 1, use_clock = 0;
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

    void drop_plan(PooledPlan* pp)
    {
        mxfft_plan_destroy(pp->plan);
        c.plan_bytes -= pp->bytes;
        c.plans_evicted++;
        for (size_t i = 0; i < pool.size(); i++)
            if (pool[i] == pp) {
                pool.erase(pool.begin() + i);
                break;
            }
        delete pp;
    }

    // An idle pooled plan for q, or a new one within the budget (evicting
    // idle plans, least recently used first).  nullptr: wait for running
    // requests to free budget; *err set when creation failed.
    PooledPlan* acquire(const Request& q, mxfft_status* err)
    {
        *err = MXFFT_OK;
        for (PooledPlan* pp : pool)
            if (!pp->busy && pp->n == q.r.n && pp->cap == q.cap && same_params(pp->p, q.r.params)) return pp;
        while (c.plan_bytes + q.need > budget) {
            PooledPlan* victim = nullptr;
            for (PooledPlan* pp : pool)
                if (!pp->busy && (!victim || pp->last_use < victim->last_use)) victim = pp;
            if (!victim) return nullptr;
            drop_plan(victim);
        }
        PooledPlan* pp = new PooledPlan();
        pp->n = q.r.n;
        pp->cap = q.cap;
        pp->p = q.r.params;
        *err = mxfft_plan(&pp->plan, q.r.n, q.cap, &q.r.params, setup);
        if (*err != MXFFT_OK) {
            delete pp;
            return nullptr;
        }
        pp->bytes = mxfft_plan_device_bytes(pp->plan);
        pool.push_back(pp);
        c.plans_created++;
        c.plan_bytes += pp->bytes;
        if (c.plan_bytes > c.peak_plan_bytes) c.peak_plan_bytes = c.plan_bytes;
        return pp;
    }

    // Enqueue q on slot si with plan pp.  When an enqueue fails the request is
    // finished at once with that status and the slot stays free.
    void launch(uint64_t ticket, Request& q, PooledPlan* pp, int si)
    {
        Slot& s = slots[si];
        pp->busy = true;
        pp->last_use = ++use_clock;
        q.state = 1;
        q.res.slot = si;
        q.res.t_start_ms = now_ms();
        const mxfft_request& r = q.r;
        mxfft_status st;
        switch (r.op) {
        case 0: st = mxfft_forward(pp->plan, r.in, r.out, r.coils, r.k_out, s.stream); break;
        case 1: st = mxfft_inverse(pp->plan, r.in, r.out, r.coils, nullptr, s.stream); break;
        default: st = mxfft_roundtrip(pp->plan, r.in, r.out, r.coils, r.k_out, s.stream); break;
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
        for (;;) {
            bool busy = false;
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
                if (!pp && err == MXFFT_OK) break;   // wait for running requests
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
                cv_work.wait(lk, [&] { return stop || !queue.empty(); });
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
    for (PooledPlan* pp : srv->pool) {
        mxfft_plan_destroy(pp->plan);
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
