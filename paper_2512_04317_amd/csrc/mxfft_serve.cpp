// mxfft_serve.cpp -- request serving: a scheduler thread admits queued
// transform requests in arrival order onto stream slots while the pooled
// plans fit a device-memory budget, and reports per-request times and status.
// A planner thread creates and releases plans, so the scheduler never waits
// on an allocation or a free: it keeps polling completions meanwhile.
#include <hip/hip_runtime.h>

#include <algorithm>
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
// Pooled plans hold at least this many slices, so that small requests queued
// together can share one launch sequence; a shared launch takes at most
// kMaxGroup slices and looks at most kGroupScan queued requests ahead.
constexpr int kMinCap = 32;
constexpr int kMaxGroup = 1024;
constexpr int kGroupScan = 64;

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

// A request of a launch and its first slice in it.
struct Member {
    uint64_t ticket;
    int first;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    int32_t* h_status = nullptr;   // pinned copy of the launch's status words
    unsigned long long* h_off = nullptr;   // pinned: input then output slice offsets of a shared launch
    unsigned long long* d_off = nullptr;   // their device copy
    int32_t* d_k = nullptr;        // k of a shared launch, before its copy to each request
    uint64_t ticket = 0;           // 0: free; else the (first) request
    std::vector<Member> members;   // every request of the launch
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
    int c = kMinCap;
    while (c < coils) c <<= 1;
    return c > kMaxCoils ? kMaxCoils : c;
}

// Requests that one launch sequence can serve together: the same size,
// parameters and operation, and complex64 buffers (8-byte aligned, so that
// their slices are element offsets from the lowest address).
bool can_share(const mxfft_request& a, const mxfft_request& b)
{
    auto aligned = [](const mxfft_request& r) {
        return ((uintptr_t)r.in % 8) == 0 && ((uintptr_t)r.out % 8) == 0;
    };
    return a.n == b.n && a.op == b.op && same_params(a.params, b.params) && aligned(a) && aligned(b);
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
    bool held = false;             // admissions paused (mxfft_serve_hold)
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
        s.members.assign(1, Member{ticket, 0});
        s.plan = pp;
        c.in_flight++;
    }

    // Enqueue the requests `group` (the first one q, whose plan pp has room
    // for all of them) on slot si as one launch sequence over their slices:
    // per-slice offset tables address each request's input and output
    // buffers from the lowest of them; k goes to the slot's array and then to
    // each request's k_out.  Each request's result is the one it would have
    // alone: every slice is transformed independently.  When an enqueue
    // fails every request of the group is finished with that status.
    void launch_group(const std::vector<uint64_t>& group, PooledPlan* pp, int si)
    {
        if (group.size() == 1) {
            launch(group[0], reqs[group[0]], pp, si);
            return;
        }
        Slot& s = slots[si];
        pp->last_use = ++use_clock;
        const double t = now_ms();
        const size_t nn = (size_t)pp->n * pp->n;
        uintptr_t in0 = UINTPTR_MAX, out0 = UINTPTR_MAX;
        int total = 0;
        bool want_k = false;
        for (uint64_t tk : group) {
            const mxfft_request& r = reqs[tk].r;
            in0 = std::min(in0, (uintptr_t)r.in);
            out0 = std::min(out0, (uintptr_t)r.out);
            total += r.coils;
            want_k |= r.k_out != nullptr;
        }
        s.members.clear();
        int first = 0;
        for (uint64_t tk : group) {
            Request& q = reqs[tk];
            q.state = 1;
            q.res.slot = si;
            q.res.t_start_ms = t;
            const unsigned long long bi = ((uintptr_t)q.r.in - in0) / 8, bo = ((uintptr_t)q.r.out - out0) / 8;
            for (int j = 0; j < q.r.coils; j++) {
                s.h_off[first + j] = bi + (unsigned long long)j * nn;
                s.h_off[total + first + j] = bo + (unsigned long long)j * nn;
            }
            s.members.push_back(Member{tk, first});
            first += q.r.coils;
        }
        mxfft_status st = MXFFT_OK;
        for (uint64_t tk : group) {
            const mxfft_request& r = reqs[tk].r;
            if (st == MXFFT_OK && r.ready && hipStreamWaitEvent(s.stream, (hipEvent_t)r.ready, 0) != hipSuccess)
                st = MXFFT_EHIP;
        }
        if (st == MXFFT_OK && hipMemcpyAsync(s.d_off, s.h_off, sizeof(unsigned long long) * 2 * (size_t)total,
                                             hipMemcpyHostToDevice, s.stream) != hipSuccess)
            st = MXFFT_EHIP;
        if (st == MXFFT_OK) {
            mxk::Workspace w = mxk::plan_workspace(pp->plan);
            w.slice_off = s.d_off;
            w.slice_off_out = s.d_off + total;
            int32_t* kb = want_k ? s.d_k : nullptr;
            const mxfft_request& r0 = reqs[group[0]].r;
            switch (r0.op) {
            case 0: st = mxk::plan_forward_ws(pp->plan, w, (const void*)in0, (void*)out0, total, kb, s.stream); break;
            case 1: st = mxk::plan_inverse_ws(pp->plan, w, (const void*)in0, (void*)out0, total, nullptr, s.stream); break;
            default: st = mxk::plan_roundtrip_ws(pp->plan, w, (const void*)in0, (void*)out0, total, kb, s.stream); break;
            }
            for (const Member& m : s.members) {
                const mxfft_request& r = reqs[m.ticket].r;
                if (st == MXFFT_OK && kb && r.k_out && r.op != 1 &&
                    hipMemcpyAsync(r.k_out, kb + m.first, sizeof(int32_t) * (size_t)r.coils, hipMemcpyDeviceToDevice,
                                   s.stream) != hipSuccess)
                    st = MXFFT_EHIP;
            }
        }
        s.has_status = mxk::plan_has_status(pp->plan);
        if (st == MXFFT_OK && s.has_status &&
            hipMemcpyAsync(s.h_status, mxk::plan_status_words(pp->plan), sizeof(int32_t) * (size_t)total,
                           hipMemcpyDeviceToHost, s.stream) != hipSuccess)
            st = MXFFT_EHIP;
        if (st == MXFFT_OK && hipEventRecord(s.done, s.stream) != hipSuccess) st = MXFFT_EHIP;
        c.admitted += group.size();
        if (st != MXFFT_OK) {
            pp->busy = false;
            for (uint64_t tk : group) finish(reqs[tk], st);
            s.members.clear();
            return;
        }
        c.coalesced_launches++;
        c.coalesced_requests += group.size();
        s.ticket = group[0];
        s.plan = pp;
        c.in_flight += group.size();
    }

    // The head-of-queue request and the queued requests after it that can
    // share its launch (its plan has room; they wait on no plan of their own),
    // taken out of the queue in arrival order.
    std::vector<uint64_t> take_group(PooledPlan* pp)
    {
        std::vector<uint64_t> g{queue.front()};
        const Request& q = reqs[queue.front()];
        int total = q.r.coils;
        const int room = std::min(pp->cap, kMaxGroup);
        auto it = queue.begin() + 1;
        for (int looked = 0; it != queue.end() && looked < kGroupScan && total < room; looked++) {
            const Request& o = reqs[*it];
            if (!o.building && total + o.r.coils <= room && can_share(q.r, o.r)) {
                total += o.r.coils;
                g.push_back(*it);
                it = queue.erase(it);
            } else {
                ++it;
            }
        }
        queue.pop_front();
        c.queued -= g.size();
        return g;
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
                for (const Member& m : s.members) {
                    Request& q = reqs[m.ticket];
                    int32_t status = (e == hipSuccess) ? MXFFT_OK : MXFFT_EHIP;
                    if (e == hipSuccess && s.has_status)
                        for (int i = 0; i < q.r.coils; i++)
                            if (s.h_status[m.first + i] != 0) {
                                status = s.h_status[m.first + i];
                                break;
                            }
                    c.in_flight--;
                    finish(q, status);
                }
                s.plan->busy = false;
                s.plan->last_use = ++use_clock;
                s.ticket = 0;
                s.members.clear();
                s.plan = nullptr;
            }
            // admissions, in arrival order
            while (!queue.empty() && !held) {
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
                if (!pp) {
                    queue.pop_front();
                    c.queued--;
                    c.admitted++;
                    finish(q, err);
                    continue;
                }
                launch_group(take_group(pp), pp, si);
                if (slots[si].ticket) busy = true;
            }
            if (stop && (queue.empty() || held) && !busy) {
                if (!held) break;
                held = false;      // stopping: the queued requests still run
                continue;
            }
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
        ok = ok && hipHostMalloc((void**)&sl.h_off, sizeof(unsigned long long) * 2 * kMaxGroup, hipHostMallocDefault) ==
                       hipSuccess;
        ok = ok && hipMalloc((void**)&sl.d_off, sizeof(unsigned long long) * 2 * kMaxGroup) == hipSuccess;
        ok = ok && hipMalloc((void**)&sl.d_k, sizeof(int32_t) * kMaxGroup) == hipSuccess;
    }
    if (!ok) {
        for (Slot& sl : s->slots) {
            if (sl.h_status) (void)hipHostFree(sl.h_status);
            if (sl.h_off) (void)hipHostFree(sl.h_off);
            (void)hipFree(sl.d_off);
            (void)hipFree(sl.d_k);
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

mxfft_status mxfft_serve_hold(mxfft_server_t srv, int32_t hold)
{
    if (!srv || (hold != 0 && hold != 1)) return MXFFT_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->held = hold != 0;
    srv->events++;
    srv->cv_work.notify_one();
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
        (void)hipHostFree(sl.h_off);
        (void)hipFree(sl.d_off);
        (void)hipFree(sl.d_k);
        (void)hipEventDestroy(sl.done);
        (void)hipStreamDestroy(sl.stream);
    }
    (void)hipStreamDestroy(srv->setup);
    delete srv;
    return MXFFT_OK;
}

}  // extern "C"
