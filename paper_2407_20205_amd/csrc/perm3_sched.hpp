// The scheduler behind perm_server_*: continuous batching of permanent
// requests, free of HIP.  Everything the device does goes through an executor
// (SchedExecutor); perm3_server.hip gives the HIP one, and a CPU test drives
// the same scheduler with a mock that computes the tallies on the host.
//
// A worker thread repeatedly
//   1. admits queued requests into free slots while the admitted work (Gray
//      indices still to visit) stays within the work budget (a request larger
//      than the budget is admitted alone);
//   2. plans a tick: up to `quantum` indices of 64-chunk tasks taken from the
//      active slots in policy order (least remaining work first, or admission
//      order); a slot whose last chunk is taken finishes in this tick;
//   3. launches the tick, and while it runs serves the fast lane: requests of
//      order <= fast_n in batches of up to 64 (and 2^28 Gray indices), each
//      one executor call;
//   4. completes the tick and hands the finished requests to poll().
// The chunk length of a slot is the block decomposition of Section 3.1:
// aligned runs of 2^m consecutive Gray states, each started at its own state.
// A tick that has not finished within tick_timeout_ms (when set) fails the
// server: every request still held or queued completes with PERM_EDEVICE.
#pragma once

#include <stdint.h>
#include <string.h>
#include <time.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "perm3.h"
#include "perm3_plan.hpp"

namespace perm3 {

inline uint64_t sched_now_ns()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

struct Request {
    uint64_t tag = 0;
    int32_t n = 0;
    uint64_t t_submit = 0;
    std::vector<uint8_t> A;
};

constexpr int SLOT_ROWS = 64;        // rows a slot holds (n <= 63)
constexpr int FAST_DEFAULT_N = 28;   // fast_max_n = 0
constexpr int FAST_MAX_N = 28;       // one request of this order is 2^28 Gray indices: one launch

// What the device does for the scheduler.  Only the worker thread calls it,
// one call at a time; a non-zero return is a status code (PERM_E*) that fails
// the server.
struct SchedExecutor {
    virtual ~SchedExecutor() = default;
    // Put request r's matrix into slot s (its rows packed by phi, Section 2)
    // and start the slot's tally at 0.
    virtual int32_t admit(int s, const Request &r) = 0;
    // Start a tick over tasks[0..nt); the slots fin[0..nfin) take their last
    // chunks in it.
    virtual int32_t launch(const TickTask *tasks, size_t nt, const int32_t *fin, uint32_t nfin) = 0;
    // Whether the tick in flight has finished, without waiting.
    virtual int32_t query(bool *finished) = 0;
    // Wait for the tick in flight: fin_out[i] = perm mod 3 of slot fin[i]
    // ((-1)^n times its tally, reduced mod 3, eq. (2)).
    virtual int32_t complete(uint8_t *fin_out) = 0;
    // perm mod 3 of `count` small matrices in one call.
    virtual int32_t run_fast(const uint8_t *const *As, const int32_t *ns, int32_t count, uint8_t *out) = 0;
};

// How a slot's Gray range is cut, from the tuning of the batch class.
struct SchedParams {
    perm_server_cfg cfg;   // validated; quantum != 0
    int fast_n = -1;       // requests with n <= fast_n take the fast lane (-1: none)
    int body_log = 5, body_log_mid = 4, mid_max_n = 31, direct_max_n = 11, chunk_log_max = 20;
    size_t max_tasks = 0;  // tasks one tick may hold
};

// Tasks a tick may hold for a configuration: every slot contributes at most
// quantum / 2^m + 1 tasks with m >= 0.
inline size_t sched_max_tasks(const perm_server_cfg &cfg)
{
    return std::min<size_t>((size_t)(cfg.quantum >> 6) + 2 * (size_t)cfg.max_slots + 64, (size_t)1 << 22);
}

class Scheduler {
public:
    Scheduler(const SchedParams &p, SchedExecutor *ex) : P(p), X(ex)
    {
        slots.assign((size_t)P.cfg.max_slots, Slot());
        for (int s = P.cfg.max_slots - 1; s >= 0; --s) free_slots.push_back(s);
        tasks.resize(P.max_tasks);
    }
    Scheduler(const Scheduler &) = delete;
    Scheduler &operator=(const Scheduler &) = delete;
    ~Scheduler() { (void)shutdown(); }

    void start() { worker = std::thread([this] { run(); }); }

    // Queue one request (A: n*n bytes, checked by the caller; copied).
    int32_t submit(const uint8_t *A, int32_t n, uint64_t tag)
    {
        Request r;
        r.tag = tag;
        r.n = n;
        r.t_submit = sched_now_ns();
        r.A.assign(A, A + (size_t)n * n);
        {
            std::lock_guard<std::mutex> g(mu);
            if (stop) return PERM_ESTATE;
            if ((int64_t)(queue.size() + fast_queue.size()) >= (int64_t)P.cfg.queue_cap) return PERM_EAGAIN;
            stats_.submitted += 1;
            if (n == 0) {
                // the empty product needs no device work
                perm_done d;
                memset(&d, 0, sizeof d);
                d.tag = tag;
                d.result = 1;
                d.t_submit_ns = d.t_admit_ns = d.t_done_ns = r.t_submit;
                done.push_back(d);
                stats_.completed += 1;
                cv_done.notify_all();
                return PERM_OK;
            }
            if (n <= P.fast_n)
                fast_queue.push_back(std::move(r));
            else
                queue.push_back(std::move(r));
        }
        cv_work.notify_one();
        return PERM_OK;
    }

    int32_t poll(perm_done *out, int32_t max, int32_t *got, int64_t timeout_us)
    {
        *got = 0;
        std::unique_lock<std::mutex> g(mu);
        if (done.empty() && timeout_us > 0)
            cv_done.wait_for(g, std::chrono::microseconds(timeout_us),
                             [&] { return !done.empty() || fatal != PERM_OK; });
        int32_t k = 0;
        while (k < max && !done.empty()) {
            out[k++] = done.front();
            done.pop_front();
        }
        *got = k;
        return PERM_OK;
    }

    perm_server_stats stats()
    {
        std::lock_guard<std::mutex> g(mu);
        return stats_;
    }

    // Finish all admitted and queued work and stop the worker; returns the
    // status that failed the server, or PERM_OK.
    int32_t shutdown()
    {
        {
            std::lock_guard<std::mutex> g(mu);
            stop = true;
        }
        cv_work.notify_all();
        if (worker.joinable()) worker.join();
        std::lock_guard<std::mutex> g(mu);
        return fatal;
    }

private:
    struct Slot {
        bool used = false;
        Request req;
        uint64_t t_admit = 0;
        int32_t m = 0, mode = MODE_DIRECT, ul = 5;
        uint64_t next_chunk = 0, nchunks = 0;
        uint64_t seq = 0;
        uint64_t remaining() const { return (nchunks - next_chunk) << m; }
    };

    SchedParams P;
    SchedExecutor *X;

    // worker-only state
    std::vector<Slot> slots;
    std::vector<int> free_slots;
    std::deque<Request> fast;          // fast-lane requests taken by the worker
    std::vector<TickTask> tasks;       // the tick being planned or in flight
    std::vector<int32_t> tick_fin;     // slots finishing in the tick in flight
    size_t tick_nt = 0;
    uint64_t admitted_work = 0;
    uint64_t seq = 0;

    // shared state, under mu
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> queue;
    std::deque<Request> fast_queue;
    std::deque<perm_done> done;
    bool stop = false;
    int32_t fatal = PERM_OK;
    perm_server_stats stats_{};
    std::thread worker;

    // Move requests into free slots while the work budget allows (caller holds mu).
    void admit(std::vector<int> &to_pack)
    {
        while (!queue.empty() && !free_slots.empty()) {
            const uint64_t work = 1ull << queue.front().n;
            const bool any_active = free_slots.size() < slots.size();
            if (P.cfg.work_budget && any_active && admitted_work + work > P.cfg.work_budget) break;
            const int s = free_slots.back();
            free_slots.pop_back();
            Slot &sl = slots[s];
            sl.used = true;
            sl.req = std::move(queue.front());
            queue.pop_front();
            sl.t_admit = sched_now_ns();
            sl.seq = seq++;
            const int n = sl.req.n;
            sl.ul = n <= P.mid_max_n ? P.body_log_mid : P.body_log;
            if (n > P.direct_max_n && n >= sl.ul + 7) {
                sl.mode = MODE_FAST;
                // chunks small enough that one quantum spreads over many waves
                int m = 14;
                const int mmax = std::min(P.chunk_log_max, n - 6);
                if (m > mmax) m = mmax;
                if (m < sl.ul + 1) m = sl.ul + 1;
                sl.m = m;
            } else {
                sl.mode = MODE_DIRECT;
                int m = n - 6;
                if (m > 10) m = 10;
                if (m < 0) m = 0;
                sl.m = m;
            }
            sl.next_chunk = 0;
            sl.nchunks = (1ull << n) >> sl.m;
            if (sl.nchunks == 0) sl.nchunks = 1;
            admitted_work += work;
            to_pack.push_back(s);
        }
    }

    // Take the submitted fast-lane requests (caller holds mu).
    void take_fast()
    {
        while (!fast_queue.empty()) {
            fast.push_back(std::move(fast_queue.front()));
            fast_queue.pop_front();
        }
    }

    void publish(std::vector<perm_done> &finished)
    {
        if (finished.empty()) return;
        std::lock_guard<std::mutex> g(mu);
        for (auto &d : finished) done.push_back(d);
        stats_.completed += finished.size();
        finished.clear();
        cv_done.notify_all();
    }

    // One batch of the fast lane: up to 64 requests and 2^28 Gray indices.
    int32_t serve_fast()
    {
        int32_t count = 0;
        uint64_t work = 0;
        while (count < (int32_t)fast.size() && count < SMALL_PLAN_MAX &&
               (count == 0 || work + (1ull << fast[count].n) <= SMALL_FUSED_WORK))
            work += 1ull << fast[count++].n;
        if (count == 0) return PERM_OK;
        const uint64_t t_admit = sched_now_ns();
        std::vector<const uint8_t *> As(count);
        std::vector<int32_t> ns(count);
        std::vector<uint8_t> out(count);
        for (int32_t k = 0; k < count; ++k) {
            As[k] = fast[k].A.data();
            ns[k] = fast[k].n;
        }
        const int32_t rc = X->run_fast(As.data(), ns.data(), count, out.data());
        if (rc) return rc;
        const uint64_t t = sched_now_ns();
        std::vector<perm_done> finished(count);
        for (int32_t k = 0; k < count; ++k) {
            perm_done &d = finished[k];
            memset(&d, 0, sizeof d);
            d.tag = fast[k].tag;
            d.status = PERM_OK;
            d.n = fast[k].n;
            d.result = out[k];
            d.t_submit_ns = fast[k].t_submit;
            d.t_admit_ns = t_admit;
            d.t_done_ns = t;
        }
        fast.erase(fast.begin(), fast.begin() + count);
        publish(finished);
        return PERM_OK;
    }

    // Plan the next tick over the active slots and launch it.
    int32_t tick_launch(bool &launched)
    {
        launched = false;
        std::vector<int> order;
        for (int s = 0; s < (int)slots.size(); ++s)
            if (slots[s].used && slots[s].next_chunk < slots[s].nchunks) order.push_back(s);
        if (order.empty()) return PERM_OK;
        if (P.cfg.policy == PERM_POLICY_FIFO) {
            std::sort(order.begin(), order.end(), [&](int a, int b) { return slots[a].seq < slots[b].seq; });
        } else {
            std::sort(order.begin(), order.end(), [&](int a, int b) {
                const uint64_t ra = slots[a].remaining(), rb = slots[b].remaining();
                return ra != rb ? ra < rb : slots[a].seq < slots[b].seq;
            });
        }
        uint64_t budget = P.cfg.quantum;
        size_t nt = 0;
        tick_fin.clear();
        for (int s : order) {
            if (budget == 0 || nt >= P.max_tasks) break;
            Slot &sl = slots[s];
            const uint64_t per_chunk = 1ull << sl.m;
            uint64_t take = sl.nchunks - sl.next_chunk;
            const uint64_t afford = std::max<uint64_t>(budget / per_chunk, 1);
            if (take > afford) take = (afford + 63) & ~63ull;   // whole tasks
            if (take > sl.nchunks - sl.next_chunk) take = sl.nchunks - sl.next_chunk;
            const uint64_t room = (uint64_t)(P.max_tasks - nt) * 64;
            if (take > room) take = room;
            uint64_t c = sl.next_chunk;
            const uint64_t end = sl.next_chunk + take;
            while (c < end) {
                const uint64_t k = std::min<uint64_t>(64, end - c);
                TickTask &t = tasks[nt++];
                t.slot = s;
                t.m = sl.m;
                t.mode = sl.mode;
                t.nchunks = (int32_t)k;
                t.c_first = c;
                t.ul = sl.ul;
                t.pad = 0;
                c += k;
            }
            sl.next_chunk = end;
            const uint64_t used = take * per_chunk;
            budget = used >= budget ? 0 : budget - used;
            if (sl.next_chunk >= sl.nchunks) tick_fin.push_back(s);
        }
        const int32_t rc = X->launch(tasks.data(), nt, tick_fin.data(), (uint32_t)tick_fin.size());
        if (rc) return rc;
        tick_nt = nt;
        launched = true;
        return PERM_OK;
    }

    // Wait for the tick in flight; requests finishing in it are appended.
    int32_t tick_complete(std::vector<perm_done> &finished)
    {
        std::vector<uint8_t> fin_out(tick_fin.size());
        const int32_t rc = X->complete(fin_out.data());
        if (rc) return rc;
        const uint64_t t = sched_now_ns();
        uint64_t visited = 0;
        for (size_t i = 0; i < tick_nt; ++i) visited += (uint64_t)tasks[i].nchunks << tasks[i].m;
        {
            std::lock_guard<std::mutex> g(mu);
            stats_.ticks += 1;
            stats_.tick_indices += visited;
        }
        for (size_t i = 0; i < tick_fin.size(); ++i) {
            const int s = tick_fin[i];
            Slot &sl = slots[s];
            perm_done d;
            memset(&d, 0, sizeof d);
            d.tag = sl.req.tag;
            d.status = PERM_OK;
            d.n = sl.req.n;
            d.result = fin_out[i];
            d.t_submit_ns = sl.req.t_submit;
            d.t_admit_ns = sl.t_admit;
            d.t_done_ns = t;
            finished.push_back(d);
            admitted_work -= 1ull << sl.req.n;
            sl.used = false;
            sl.req.A.clear();
            free_slots.push_back(s);
        }
        tick_fin.clear();
        tick_nt = 0;
        return PERM_OK;
    }

    // Fail every request still held or queued with status rc (caller holds mu).
    void fail_all(int32_t rc)
    {
        auto fail = [&](uint64_t tag, int32_t n, uint64_t t_submit) {
            perm_done d;
            memset(&d, 0, sizeof d);
            d.tag = tag;
            d.status = rc;
            d.n = n;
            d.t_submit_ns = t_submit;
            d.t_done_ns = sched_now_ns();
            done.push_back(d);
        };
        for (auto &sl : slots)
            if (sl.used) {
                fail(sl.req.tag, sl.req.n, sl.req.t_submit);
                sl.used = false;
            }
        for (auto &r : fast) fail(r.tag, r.n, r.t_submit);
        fast.clear();
        for (auto &r : fast_queue) fail(r.tag, r.n, r.t_submit);
        fast_queue.clear();
        for (auto &r : queue) fail(r.tag, r.n, r.t_submit);
        queue.clear();
    }

    void run()
    {
        std::vector<perm_done> finished;
        uint64_t busy_start = 0;
        const uint64_t timeout_ns = (uint64_t)(P.cfg.tick_timeout_ms > 0 ? P.cfg.tick_timeout_ms : 0) * 1000000ull;
        for (;;) {
            bool stopping;
            std::vector<int> to_pack;
            {
                // admit straight from the submission queue, so queue_cap bounds the waiting requests
                std::unique_lock<std::mutex> g(mu);
                const bool idle = free_slots.size() == slots.size() && fast.empty();
                if (idle && queue.empty() && fast_queue.empty() && !stop)
                    cv_work.wait(g, [&] { return stop || !queue.empty() || !fast_queue.empty(); });
                take_fast();
                admit(to_pack);
                stopping = stop;
            }
            int32_t rc = PERM_OK;
            for (size_t i = 0; i < to_pack.size() && rc == PERM_OK; ++i)
                rc = X->admit(to_pack[i], slots[to_pack[i]].req);
            const bool active = free_slots.size() < slots.size();
            bool launched = false;
            uint64_t t_launch = 0;
            if (rc == PERM_OK && active) {
                if (!busy_start) busy_start = sched_now_ns();
                rc = tick_launch(launched);
                t_launch = sched_now_ns();
            }
            // the fast lane: small requests in batches, beside the tick in flight
            while (rc == PERM_OK) {
                if (!fast.empty()) {
                    rc = serve_fast();
                    continue;
                }
                if (!launched) break;
                bool fin = false;
                rc = X->query(&fin);
                if (rc || fin) break;
                if (timeout_ns && sched_now_ns() - t_launch > timeout_ns) {
                    rc = PERM_EDEVICE;   // the tick did not finish in time
                    break;
                }
                std::unique_lock<std::mutex> g(mu);
                cv_work.wait_for(g, std::chrono::microseconds(20), [&] { return !fast_queue.empty(); });
                take_fast();
            }
            if (rc == PERM_OK && launched) rc = tick_complete(finished);
            std::lock_guard<std::mutex> g(mu);
            if (busy_start && (rc != PERM_OK || free_slots.size() == slots.size())) {
                stats_.busy_ns += sched_now_ns() - busy_start;
                busy_start = 0;
            }
            if (rc != PERM_OK) {
                fatal = rc;
                fail_all(rc);
                stop = true;
            }
            for (auto &d : finished) done.push_back(d);
            stats_.completed += finished.size();
            int act = 0;
            for (auto &sl : slots) act += sl.used ? 1 : 0;
            stats_.active_slots = act;
            stats_.queued = (int32_t)(queue.size() + fast_queue.size() + fast.size());
            if (!finished.empty() || rc != PERM_OK) cv_done.notify_all();
            finished.clear();
            const bool drained = act == 0 && queue.empty() && fast_queue.empty() && fast.empty();
            if ((stopping && drained) || rc != PERM_OK) {
                cv_done.notify_all();
                return;
            }
        }
    }
};

}  // namespace perm3
