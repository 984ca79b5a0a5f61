// perm_server_*: a request loop with continuous batching.
//
// A worker thread owns a stream and device-resident slots.  Each admitted
// request occupies one slot: its rows (packed on the device by k_slot_pack)
// and its int64 partial tally stay in device memory until it finishes.  The
// worker repeatedly
//   1. admits queued requests while a slot is free and the admitted work
//      (Gray indices still to visit) stays within the work budget;
//   2. builds a tick: up to `quantum` indices of 64-chunk tasks taken from
//      the active slots in policy order (least remaining work first, or
//      admission order); a slot whose last chunk is taken finishes in this tick;
//   3. launches k_tick (persistent waves over the task list; tallies added
//      atomically per slot) and k_finish (finished slots' tallies reduced mod 3),
//      copies the finished results back and hands them to perm_server_poll.
// Requests arriving while a tick runs join the next one, so large and small
// jobs share the device instead of queueing behind each other.
//
// Small requests (n <= fast_max_n) skip the slots: they wait in a queue of
// their own, and while a tick is in flight (or when none is) the worker takes
// them in batches of up to 64 requests and 2^28 Gray indices and runs each
// batch as one small host call of the library: planned, packed and walked by
// one launch on the library's stream, whose waves raise their issue priority.
// The tick's grid leaves a block slot free on a quarter of the CUs, so such a
// batch runs beside the tick and finishes in tens of microseconds instead of
// waiting for the next tick.
#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "perm3.h"
#include "perm3_internal.h"
#include "perm3_runtime.h"
#include "perm3_walk.hpp"

using namespace perm3;

namespace {

uint64_t now_ns()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

struct Request {
    uint64_t tag;
    int32_t n;
    uint64_t t_submit;
    std::vector<uint8_t> A;
};

struct Slot {
    bool used = false;
    Request req;
    uint64_t t_admit = 0;
    int32_t m = 0, mode = MODE_DIRECT, ul = 5;
    uint64_t next_chunk = 0, nchunks = 0;
    uint64_t seq = 0;
    uint64_t remaining() const { return (nchunks - next_chunk) << m; }
};

constexpr int SLOT_ROWS = 64;

}  // namespace

constexpr int FAST_DEFAULT_N = 28;   // fast_max_n = 0
constexpr int FAST_MAX_N = 28;       // one request of this order is 2^28 Gray indices: one launch

struct perm_server {
    perm_server_cfg cfg{};
    perm_tuning tuning{};
    int device = 0, cus = 0;
    int fast_n = -1;                  // requests with n <= fast_n take the fast lane
    Context *ctx = nullptr;           // the library context the fast lane calls into
    hipStream_t stream = nullptr;
    hipEvent_t ev_tick = nullptr;

    // device buffers
    RowW *d_rows = nullptr;
    SlotInfo *d_slots = nullptr;
    int64_t *d_tally = nullptr;
    TickTask *d_tasks = nullptr;
    uint32_t *d_counts = nullptr;     // [0] ntasks, [1] nfin, [2] queue
    int32_t *d_fin = nullptr;
    uint8_t *d_fin_out = nullptr;
    uint8_t *d_upload = nullptr;      // matrices being admitted
    // pinned host staging
    TickTask *h_tasks = nullptr;
    uint32_t *h_counts = nullptr;
    int32_t *h_fin = nullptr;
    uint8_t *h_fin_out = nullptr;
    uint8_t *h_upload = nullptr;
    SlotInfo *h_slots = nullptr;
    size_t max_tasks = 0;

    std::vector<Slot> slots;
    std::vector<int> free_slots;
    std::deque<Request> fast;          // fast-lane requests taken by the worker (worker only)
    // the tick in flight
    size_t tick_nt = 0;
    uint32_t tick_nfin = 0;
    std::vector<int> tick_fin;
    uint64_t admitted_work = 0;
    uint64_t seq = 0;

    std::mutex mu;                    // guards queue, done, stats, stop
    std::condition_variable cv_work, cv_done;
    std::deque<Request> queue;
    std::deque<Request> fast_queue;   // submitted requests for the fast lane
    std::deque<perm_done> done;
    bool stop = false;
    int32_t fatal = PERM_OK;
    perm_server_stats stats{};
    std::thread worker;

    int32_t init();
    void release();
    void run();
    int32_t tick_launch(bool &launched);
    int32_t tick_complete(std::vector<perm_done> &finished);
    void admit(std::deque<Request> &incoming, std::vector<int> &to_pack);
    void take_fast();
    int32_t serve_fast();
    void publish(std::vector<perm_done> &finished);
};

#define SRV_TRY(expr)                                        \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return hip_fail(_e, #expr);    \
    } while (0)

int32_t perm_server::init()
{
    SRV_TRY(hipGetDevice(&device));
    hipDeviceProp_t prop;
    SRV_TRY(hipGetDeviceProperties(&prop, device));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_error(PERM_EDEVICE, "device is %s; this library is built for gfx950 only", prop.gcnArchName);
    cus = prop.multiProcessorCount;
    SRV_TRY(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
    SRV_TRY(hipEventCreateWithFlags(&ev_tick, hipEventDisableTiming));
    const size_t S = (size_t)cfg.max_slots;
    // every slot can contribute at most quantum / 2^m + 1 tasks, and m >= 0
    max_tasks = std::min<size_t>((size_t)(cfg.quantum >> 6) + 2 * S + 64, (size_t)1 << 22);
    SRV_TRY(hipMalloc(&d_rows, S * SLOT_ROWS * sizeof(RowW)));
    SRV_TRY(hipMalloc(&d_slots, S * sizeof(SlotInfo)));
    SRV_TRY(hipMalloc(&d_tally, S * sizeof(int64_t)));
    SRV_TRY(hipMemsetAsync(d_tally, 0, S * sizeof(int64_t), stream));
    SRV_TRY(hipMalloc(&d_tasks, max_tasks * sizeof(TickTask)));
    SRV_TRY(hipMalloc(&d_counts, 4 * sizeof(uint32_t)));
    SRV_TRY(hipMemsetAsync(d_counts, 0, 4 * sizeof(uint32_t), stream));
    SRV_TRY(hipMalloc(&d_fin, S * sizeof(int32_t)));
    SRV_TRY(hipMalloc(&d_fin_out, S));
    SRV_TRY(hipMalloc(&d_upload, S * SLOT_ROWS * SLOT_ROWS));
    SRV_TRY(hipHostMalloc((void **)&h_tasks, max_tasks * sizeof(TickTask), hipHostMallocDefault));
    SRV_TRY(hipHostMalloc((void **)&h_counts, 4 * sizeof(uint32_t), hipHostMallocDefault));
    SRV_TRY(hipHostMalloc((void **)&h_fin, S * sizeof(int32_t), hipHostMallocDefault));
    SRV_TRY(hipHostMalloc((void **)&h_fin_out, S, hipHostMallocDefault));
    SRV_TRY(hipHostMalloc((void **)&h_upload, S * SLOT_ROWS * SLOT_ROWS, hipHostMallocDefault));
    SRV_TRY(hipHostMalloc((void **)&h_slots, S * sizeof(SlotInfo), hipHostMallocDefault));
    SRV_TRY(hipStreamSynchronize(stream));
    slots.assign(S, Slot());
    free_slots.clear();
    for (int s = (int)S - 1; s >= 0; --s) free_slots.push_back(s);
    return PERM_OK;
}

void perm_server::release()
{
    if (stream) (void)hipStreamSynchronize(stream);
    (void)hipFree(d_rows);
    (void)hipFree(d_slots);
    (void)hipFree(d_tally);
    (void)hipFree(d_tasks);
    (void)hipFree(d_counts);
    (void)hipFree(d_fin);
    (void)hipFree(d_fin_out);
    (void)hipFree(d_upload);
    (void)hipHostFree(h_tasks);
    (void)hipHostFree(h_counts);
    (void)hipHostFree(h_fin);
    (void)hipHostFree(h_fin_out);
    (void)hipHostFree(h_upload);
    (void)hipHostFree(h_slots);
    if (ev_tick) (void)hipEventDestroy(ev_tick);
    if (stream) (void)hipStreamDestroy(stream);
}

// Move requests into free slots while the work budget allows.
void perm_server::admit(std::deque<Request> &incoming, std::vector<int> &to_pack)
{
    while (!incoming.empty() && !free_slots.empty()) {
        const Request &r = incoming.front();
        const uint64_t work = 1ull << r.n;
        const bool any_active = free_slots.size() < slots.size();
        if (cfg.work_budget && any_active && admitted_work + work > cfg.work_budget) break;
        const int s = free_slots.back();
        free_slots.pop_back();
        Slot &sl = slots[s];
        sl.used = true;
        sl.req = std::move(incoming.front());
        incoming.pop_front();
        sl.t_admit = now_ns();
        sl.seq = seq++;
        const int n = sl.req.n;
        sl.ul = n <= tuning.mid_max_n ? tuning.body_log_mid : tuning.body_log;
        if (n > tuning.direct_max_n && n >= sl.ul + 7) {
            sl.mode = MODE_FAST;
            // chunks small enough that one quantum spreads over many waves
            int m = 14;
            const int mmax = std::min(tuning.chunk_log_max, n - 6);
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
void perm_server::take_fast()
{
    while (!fast_queue.empty()) {
        fast.push_back(std::move(fast_queue.front()));
        fast_queue.pop_front();
    }
}

// Run fast-lane requests, up to 64 of them and 2^28 Gray indices in all (one
// launch walks them), as one host call into the library context and publish
// their results at once.
int32_t perm_server::serve_fast()
{
    int32_t count = 0;
    uint64_t work = 0;
    while (count < (int32_t)fast.size() && count < SMALL_PLAN_MAX &&
           (count == 0 || work + (1ull << fast[count].n) <= SMALL_FUSED_WORK))
        work += 1ull << fast[count++].n;
    if (count == 0) return PERM_OK;
    const uint64_t t_admit = now_ns();
    std::vector<const uint8_t *> As(count);
    std::vector<int32_t> ns(count);
    std::vector<uint8_t> out(count);
    for (int32_t k = 0; k < count; ++k) {
        As[k] = fast[k].A.data();
        ns[k] = fast[k].n;
    }
    int32_t rc;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        rc = ctx->run_host(As.data(), ns.data(), count, false, 0, 0, out.data(), nullptr);
    }
    if (rc) return rc;
    const uint64_t t = now_ns();
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

// Hand finished requests to perm_server_poll.
void perm_server::publish(std::vector<perm_done> &finished)
{
    if (finished.empty()) return;
    std::lock_guard<std::mutex> g(mu);
    for (auto &d : finished) done.push_back(d);
    stats.completed += finished.size();
    finished.clear();
    cv_done.notify_all();
}

// Plan and launch one tick (asynchronous; tick_complete waits for it).
int32_t perm_server::tick_launch(bool &launched)
{
    launched = false;
    std::vector<int> order;
    for (int s = 0; s < (int)slots.size(); ++s)
        if (slots[s].used && slots[s].next_chunk < slots[s].nchunks) order.push_back(s);
    if (order.empty()) return PERM_OK;
    if (cfg.policy == PERM_POLICY_FIFO) {
        std::sort(order.begin(), order.end(), [&](int a, int b) { return slots[a].seq < slots[b].seq; });
    } else {
        std::sort(order.begin(), order.end(), [&](int a, int b) {
            const uint64_t ra = slots[a].remaining(), rb = slots[b].remaining();
            return ra != rb ? ra < rb : slots[a].seq < slots[b].seq;
        });
    }
    uint64_t budget = cfg.quantum;
    size_t nt = 0;
    uint32_t nfin = 0;
    std::vector<int> fin_slots;
    for (int s : order) {
        if (budget == 0 || nt >= max_tasks) break;
        Slot &sl = slots[s];
        const uint64_t per_chunk = 1ull << sl.m;
        uint64_t take = sl.nchunks - sl.next_chunk;
        const uint64_t afford = std::max<uint64_t>(budget / per_chunk, 1);
        if (take > afford) take = (afford + 63) & ~63ull;   // whole tasks
        if (take > sl.nchunks - sl.next_chunk) take = sl.nchunks - sl.next_chunk;
        const uint64_t room = (uint64_t)(max_tasks - nt) * 64;
        if (take > room) take = room;
        uint64_t c = sl.next_chunk;
        const uint64_t end = sl.next_chunk + take;
        while (c < end) {
            const uint64_t k = std::min<uint64_t>(64, end - c);
            TickTask &t = h_tasks[nt++];
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
        if (sl.next_chunk >= sl.nchunks) {
            h_fin[nfin++] = s;
            fin_slots.push_back(s);
        }
    }
    h_counts[0] = (uint32_t)nt;
    h_counts[1] = nfin;
    SRV_TRY(hipMemcpyAsync(d_tasks, h_tasks, nt * sizeof(TickTask), hipMemcpyHostToDevice, stream));
    SRV_TRY(hipMemcpyAsync(d_counts, h_counts, 2 * sizeof(uint32_t), hipMemcpyHostToDevice, stream));
    if (nfin) SRV_TRY(hipMemcpyAsync(d_fin, h_fin, nfin * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    TickArgs ta;
    ta.rows = d_rows;
    ta.slots = d_slots;
    ta.tasks = d_tasks;
    ta.ntasks = d_counts;
    ta.tally = d_tally;
    ta.queue = d_counts + 2;
    // with a fast lane, one block slot on a quarter of the CUs stays free for
    // its launches (about 3% of the tick's waves at 8 waves per SIMD)
    const int per_cu = std::min(tuning.waves_per_simd, walk_resident_per_cu(0));
    int blocks = cus * per_cu;
    if (fast_n >= 1 && blocks > cus / 4) blocks -= std::max(1, cus / 4);
    const int need = (int)((nt + 3) / 4);
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    SRV_TRY(launch_tick(ta, blocks, stream));
    FinishArgs fa;
    fa.fin_slots = d_fin;
    fa.nfin = d_counts + 1;
    fa.slots = d_slots;
    fa.tally = d_tally;
    fa.fin_out = d_fin_out;
    fa.queue = d_counts + 2;
    SRV_TRY(launch_finish(fa, (int)nfin, stream));
    if (nfin) SRV_TRY(hipMemcpyAsync(h_fin_out, d_fin_out, nfin, hipMemcpyDeviceToHost, stream));
    SRV_TRY(hipEventRecord(ev_tick, stream));
    tick_nt = nt;
    tick_nfin = nfin;
    tick_fin.swap(fin_slots);
    launched = true;
    return PERM_OK;
}

// Wait for the tick in flight; requests finishing in it are appended.
int32_t perm_server::tick_complete(std::vector<perm_done> &finished)
{
    SRV_TRY(hipEventSynchronize(ev_tick));
    const uint64_t t = now_ns();
    {
        std::lock_guard<std::mutex> g(mu);
        stats.ticks += 1;
        for (size_t i = 0; i < tick_nt; ++i) stats.tick_indices += (uint64_t)h_tasks[i].nchunks << h_tasks[i].m;
    }
    for (uint32_t i = 0; i < tick_nfin; ++i) {
        const int s = tick_fin[i];
        Slot &sl = slots[s];
        perm_done d;
        memset(&d, 0, sizeof d);
        d.tag = sl.req.tag;
        d.status = PERM_OK;
        d.n = sl.req.n;
        d.result = h_fin_out[i];
        d.t_submit_ns = sl.req.t_submit;
        d.t_admit_ns = sl.t_admit;
        d.t_done_ns = t;
        finished.push_back(d);
        admitted_work -= 1ull << sl.req.n;
        sl.used = false;
        sl.req.A.clear();
        free_slots.push_back(s);
    }
    return PERM_OK;
}

void perm_server::run()
{
    (void)hipSetDevice(device);
    std::vector<perm_done> finished;
    uint64_t busy_start = 0;
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
            admit(queue, to_pack);
            stopping = stop;
        }
        int32_t rc = PERM_OK;
        // upload and pack the newly admitted matrices
        for (size_t i = 0; i < to_pack.size() && rc == PERM_OK; ++i) {
            const int s = to_pack[i];
            const Slot &sl = slots[s];
            const int n = sl.req.n;
            uint8_t *h = h_upload + (size_t)s * SLOT_ROWS * SLOT_ROWS;
            if (n) memcpy(h, sl.req.A.data(), (size_t)n * n);
            h_slots[s].n = n;
            h_slots[s].pad = 0;
            h_slots[s].row_base = (int64_t)s * SLOT_ROWS;
            uint8_t *d = d_upload + (size_t)s * SLOT_ROWS * SLOT_ROWS;
            hipError_t e = hipMemcpyAsync(d, h, (size_t)n * n, hipMemcpyHostToDevice, stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(d_slots + s, h_slots + s, sizeof(SlotInfo), hipMemcpyHostToDevice, stream);
            if (e == hipSuccess) e = launch_slot_pack(d, n, d_rows + (size_t)s * SLOT_ROWS, stream);
            if (e != hipSuccess) rc = hip_fail(e, "admit");
        }
        const bool active = free_slots.size() < slots.size();
        bool launched = false;
        if (rc == PERM_OK && active) {
            if (!busy_start) busy_start = now_ns();
            rc = tick_launch(launched);
        }
        // the fast lane: small requests in batches, beside the tick in flight
        while (rc == PERM_OK) {
            if (!fast.empty()) {
                rc = serve_fast();
                continue;
            }
            if (!launched) break;
            const hipError_t q = hipEventQuery(ev_tick);
            if (q == hipSuccess) break;
            if (q != hipErrorNotReady) {
                rc = hip_fail(q, "hipEventQuery");
                break;
            }
            std::unique_lock<std::mutex> g(mu);
            cv_work.wait_for(g, std::chrono::microseconds(20), [&] { return !fast_queue.empty(); });
            take_fast();
        }
        if (rc == PERM_OK && launched) rc = tick_complete(finished);
        {
            std::lock_guard<std::mutex> g(mu);
            if (busy_start && (rc != PERM_OK || free_slots.size() == slots.size())) {
                stats.busy_ns += now_ns() - busy_start;
                busy_start = 0;
            }
            if (rc != PERM_OK) {
                fatal = rc;
                // fail everything still held or queued
                auto fail = [&](uint64_t tag, int32_t n, uint64_t t_submit) {
                    perm_done d;
                    memset(&d, 0, sizeof d);
                    d.tag = tag;
                    d.status = rc;
                    d.n = n;
                    d.t_submit_ns = t_submit;
                    d.t_done_ns = now_ns();
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
                stop = true;
            }
            for (auto &d : finished) done.push_back(d);
            stats.completed += finished.size();
            int act = 0;
            for (auto &sl : slots) act += sl.used ? 1 : 0;
            stats.active_slots = act;
            stats.queued = (int32_t)(queue.size() + fast_queue.size() + fast.size());
            if (!finished.empty() || rc != PERM_OK) cv_done.notify_all();
            finished.clear();
            const bool drained = act == 0 && queue.empty() && fast_queue.empty() && fast.empty();
            if ((stopping && drained) || rc != PERM_OK) {
                cv_done.notify_all();
                return;
            }
        }
    }
}

extern "C" {

int32_t perm_server_create(const perm_server_cfg *cfg, perm_server **out)
{
    if (!cfg || !out) return set_error(PERM_EINVAL, "null pointer");
    if (cfg->max_slots < 1 || cfg->max_slots > 65536 || cfg->queue_cap < 1 || cfg->queue_cap > (1 << 24) ||
        (cfg->policy != PERM_POLICY_SRPT && cfg->policy != PERM_POLICY_FIFO) || cfg->fast_max_n < -1 ||
        cfg->fast_max_n > FAST_MAX_N)
        return set_error(PERM_EINVAL, "server configuration out of range");
    Context *c = nullptr;
    int32_t rc = get_context(&c);
    if (rc) return rc;
    perm_server *s = new perm_server();
    s->cfg = *cfg;
    s->ctx = c;
    s->fast_n = cfg->fast_max_n == 0 ? FAST_DEFAULT_N : cfg->fast_max_n;
    if (s->cfg.quantum == 0) s->cfg.quantum = 1ull << 33;
    {
        std::lock_guard<std::mutex> g(c->mu);
        s->tuning = c->tunings[PERM_TUNE_BATCH];
    }
    rc = s->init();
    if (rc) {
        s->release();
        delete s;
        return rc;
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return PERM_OK;
}

int32_t perm_server_submit(perm_server *s, const uint8_t *A, int32_t n, uint64_t tag)
{
    if (!s) return set_error(PERM_EINVAL, "null server");
    if (n < 0 || n > PERM_MAX_N) return set_error(PERM_EINVAL, "n = %d is outside [0, %d]", n, PERM_MAX_N);
    if (n > 0 && !A) return set_error(PERM_EINVAL, "null matrix pointer");
    for (int64_t i = 0; i < (int64_t)n * n; ++i)
        if (A[i] > 2) {
            set_error_index(i);
            return set_error(PERM_EDOMAIN, "entry %lld is %u; entries must be 0, 1 or 2", (long long)i,
                             (unsigned)A[i]);
        }
    Request r;
    r.tag = tag;
    r.n = n;
    r.t_submit = now_ns();
    r.A.assign(A, A + (size_t)n * n);
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) return set_error(PERM_ESTATE, "server is shutting down");
        if ((int32_t)(s->queue.size() + s->fast_queue.size()) >= s->cfg.queue_cap) return PERM_EAGAIN;
        if (n == 0) {
            // the empty product needs no device work
            perm_done d;
            memset(&d, 0, sizeof d);
            d.tag = tag;
            d.result = 1;
            d.t_submit_ns = d.t_admit_ns = d.t_done_ns = r.t_submit;
            s->done.push_back(d);
            s->stats.submitted += 1;
            s->stats.completed += 1;
            s->cv_done.notify_all();
            return PERM_OK;
        }
        if (n <= s->fast_n)
            s->fast_queue.push_back(std::move(r));
        else
            s->queue.push_back(std::move(r));
        s->stats.submitted += 1;
    }
    s->cv_work.notify_one();
    return PERM_OK;
}

int32_t perm_server_poll(perm_server *s, perm_done *out, int32_t max, int32_t *got, int64_t timeout_us)
{
    if (!s || !got || (max > 0 && !out) || max < 0) return set_error(PERM_EINVAL, "bad argument");
    *got = 0;
    std::unique_lock<std::mutex> g(s->mu);
    if (s->done.empty() && timeout_us > 0)
        s->cv_done.wait_for(g, std::chrono::microseconds(timeout_us), [&] { return !s->done.empty() || s->fatal; });
    int32_t k = 0;
    while (k < max && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *got = k;
    return PERM_OK;
}

int32_t perm_server_stats_get(perm_server *s, perm_server_stats *st)
{
    if (!s || !st) return set_error(PERM_EINVAL, "null pointer");
    std::lock_guard<std::mutex> g(s->mu);
    *st = s->stats;
    return PERM_OK;
}

int32_t perm_server_destroy(perm_server *s)
{
    if (!s) return set_error(PERM_EINVAL, "null server");
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    const int32_t fatal = s->fatal;
    s->release();
    delete s;
    return fatal;
}

}  // extern "C"
