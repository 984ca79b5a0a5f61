// perm_server_*: a request loop with continuous batching.
//
// The scheduling (admission, tick planning, the fast lane, the watchdog) is
// the HIP-free Scheduler of perm3_sched.hpp; this file is its device side.
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

#include <algorithm>
#include <cstring>
#include <memory>
#include <vector>

#include "perm3.h"
#include "perm3_internal.h"
#include "perm3_runtime.h"
#include "perm3_sched.hpp"
#include "perm3_walk.hpp"

using namespace perm3;

namespace {

#define SRV_TRY(expr)                                        \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return hip_fail(_e, #expr);    \
    } while (0)

// The device side of the server: a stream, device-resident slots (rows and
// int64 partial tallies), the tick's task list, and pinned staging.  The fast
// lane calls into the library context as a small host call.
struct HipExecutor final : SchedExecutor {
    perm_server_cfg cfg{};
    int waves_per_simd = 8;
    int device = 0, cus = 0;
    bool fast_lane = false;           // leave room on the CUs for fast-lane launches
    Context *ctx = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev_tick = nullptr;
    size_t max_tasks = 0;
    uint32_t tick_nfin = 0;

    RowW *d_rows = nullptr;
    SlotInfo *d_slots = nullptr;
    int64_t *d_tally = nullptr;
    TickTask *d_tasks = nullptr;
    uint32_t *d_counts = nullptr;     // [0] ntasks, [1] nfin, [2] queue
    int32_t *d_fin = nullptr;
    uint8_t *d_fin_out = nullptr;
    uint8_t *d_upload = nullptr;      // matrices being admitted
    TickTask *h_tasks = nullptr;
    uint32_t *h_counts = nullptr;
    int32_t *h_fin = nullptr;
    uint8_t *h_fin_out = nullptr;
    uint8_t *h_upload = nullptr;
    SlotInfo *h_slots = nullptr;

    int32_t init();
    void release();
    int32_t admit(int s, const Request &r) override;
    int32_t launch(const TickTask *tasks, size_t nt, const int32_t *fin, uint32_t nfin) override;
    int32_t query(bool *finished) override;
    int32_t complete(uint8_t *fin_out) override;
    int32_t run_fast(const uint8_t *const *As, const int32_t *ns, int32_t count, uint8_t *out) override;
};

int32_t HipExecutor::init()
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
    max_tasks = sched_max_tasks(cfg);
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
    return PERM_OK;
}

void HipExecutor::release()
{
    // work still queued (a tick the watchdog gave up on included) ends before its buffers go
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

// Upload the matrix of an admitted request into its slot and pack its rows.
int32_t HipExecutor::admit(int s, const Request &r)
{
    const int n = r.n;
    uint8_t *h = h_upload + (size_t)s * SLOT_ROWS * SLOT_ROWS;
    if (n) memcpy(h, r.A.data(), (size_t)n * n);
    h_slots[s].n = n;
    h_slots[s].pad = 0;
    h_slots[s].row_base = (int64_t)s * SLOT_ROWS;
    uint8_t *d = d_upload + (size_t)s * SLOT_ROWS * SLOT_ROWS;
    SRV_TRY(hipMemcpyAsync(d, h, (size_t)n * n, hipMemcpyHostToDevice, stream));
    SRV_TRY(hipMemcpyAsync(d_slots + s, h_slots + s, sizeof(SlotInfo), hipMemcpyHostToDevice, stream));
    SRV_TRY(launch_slot_pack(d, n, d_rows + (size_t)s * SLOT_ROWS, stream));
    return PERM_OK;
}

// Copy the tick's task list in, launch k_tick and k_finish, queue the
// finished results' copy out, and record the tick's event.
int32_t HipExecutor::launch(const TickTask *tasks, size_t nt, const int32_t *fin, uint32_t nfin)
{
    if (nt > max_tasks || nfin > (uint32_t)cfg.max_slots)
        return set_error(PERM_EINVAL, "tick of %zu tasks and %u finishing slots exceeds its buffers", nt, nfin);
    memcpy(h_tasks, tasks, nt * sizeof(TickTask));
    if (nfin) memcpy(h_fin, fin, nfin * sizeof(int32_t));
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
    const int per_cu = std::min(waves_per_simd, walk_resident_per_cu(0));
    int blocks = cus * per_cu;
    if (fast_lane && blocks > cus / 4) blocks -= std::max(1, cus / 4);
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
    tick_nfin = nfin;
    return PERM_OK;
}

int32_t HipExecutor::query(bool *finished)
{
    const hipError_t q = hipEventQuery(ev_tick);
    if (q == hipErrorNotReady) {
        *finished = false;
        return PERM_OK;
    }
    if (q != hipSuccess) return hip_fail(q, "hipEventQuery");
    *finished = true;
    return PERM_OK;
}

int32_t HipExecutor::complete(uint8_t *fin_out)
{
    SRV_TRY(hipEventSynchronize(ev_tick));
    if (tick_nfin) memcpy(fin_out, h_fin_out, tick_nfin);
    return PERM_OK;
}

// A fast-lane batch: one small host call of the library (planned, packed and
// walked by one launch on the library's stream).
int32_t HipExecutor::run_fast(const uint8_t *const *As, const int32_t *ns, int32_t count, uint8_t *out)
{
    std::lock_guard<std::mutex> g(ctx->mu);
    return ctx->run_host(As, ns, count, false, 0, 0, out, nullptr);
}

}  // namespace

struct perm_server {
    HipExecutor exec;
    std::unique_ptr<Scheduler> sched;
};

extern "C" {

int32_t perm_server_create(const perm_server_cfg *cfg, perm_server **out)
{
    if (!cfg || !out) return set_error(PERM_EINVAL, "null pointer");
    if (cfg->max_slots < 1 || cfg->max_slots > 65536 || cfg->queue_cap < 1 || cfg->queue_cap > (1 << 24) ||
        (cfg->policy != PERM_POLICY_SRPT && cfg->policy != PERM_POLICY_FIFO) || cfg->fast_max_n < -1 ||
        cfg->fast_max_n > FAST_MAX_N || cfg->tick_timeout_ms < 0 || cfg->reserved != 0)
        return set_error(PERM_EINVAL, "server configuration out of range");
    Context *c = nullptr;
    int32_t rc = get_context(&c);
    if (rc) return rc;
    std::unique_ptr<perm_server> s(new perm_server());
    SchedParams p;
    p.cfg = *cfg;
    if (p.cfg.quantum == 0) p.cfg.quantum = 1ull << 33;
    p.fast_n = cfg->fast_max_n == 0 ? FAST_DEFAULT_N : cfg->fast_max_n;
    p.max_tasks = sched_max_tasks(p.cfg);
    {
        std::lock_guard<std::mutex> g(c->mu);
        const perm_tuning &t = c->tunings[PERM_TUNE_BATCH];
        p.body_log = t.body_log;
        p.body_log_mid = t.body_log_mid;
        p.mid_max_n = t.mid_max_n;
        p.direct_max_n = t.direct_max_n;
        p.chunk_log_max = t.chunk_log_max;
        s->exec.waves_per_simd = t.waves_per_simd;
    }
    s->exec.cfg = p.cfg;
    s->exec.ctx = c;
    s->exec.fast_lane = p.fast_n >= 1;
    rc = s->exec.init();
    if (rc) {
        s->exec.release();
        return rc;
    }
    s->sched.reset(new Scheduler(p, &s->exec));
    s->sched->start();
    *out = s.release();
    return PERM_OK;
}

int32_t perm_server_submit(perm_server *s, const uint8_t *A, int32_t n, uint64_t tag)
{
    set_error_index(-1);
    if (!s) return set_error(PERM_EINVAL, "null server");
    if (n < 0 || n > PERM_MAX_N) return set_error(PERM_EINVAL, "n = %d is outside [0, %d]", n, PERM_MAX_N);
    if (n > 0 && !A) return set_error(PERM_EINVAL, "null matrix pointer");
    for (int64_t i = 0; i < (int64_t)n * n; ++i)
        if (A[i] > 2) {
            set_error_index(i);
            return set_error(PERM_EDOMAIN, "entry %lld is %u; entries must be 0, 1 or 2", (long long)i,
                             (unsigned)A[i]);
        }
    const int32_t rc = s->sched->submit(A, n, tag);
    if (rc == PERM_ESTATE) return set_error(PERM_ESTATE, "server is shutting down");
    return rc;
}

int32_t perm_server_poll(perm_server *s, perm_done *out, int32_t max, int32_t *got, int64_t timeout_us)
{
    if (!s || !got || (max > 0 && !out) || max < 0) return set_error(PERM_EINVAL, "bad argument");
    return s->sched->poll(out, max, got, timeout_us);
}

int32_t perm_server_stats_get(perm_server *s, perm_server_stats *st)
{
    if (!s || !st) return set_error(PERM_EINVAL, "null pointer");
    *st = s->sched->stats();
    return PERM_OK;
}

int32_t perm_server_destroy(perm_server *s)
{
    if (!s) return set_error(PERM_EINVAL, "null server");
    const int32_t fatal = s->sched->shutdown();
    s->sched.reset();
    s->exec.release();
    delete s;
    if (fatal == PERM_EDEVICE) return set_error(PERM_EDEVICE, "the server failed on the device (or its tick watchdog fired)");
    return fatal;
}

}  // extern "C"
