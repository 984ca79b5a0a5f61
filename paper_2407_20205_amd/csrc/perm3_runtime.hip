// Host runtime of libperm3: the C ABI of include/perm3.h.
//
// One context per device holds a stream, growable work buffers, a cache of
// captured HIP graphs, the tuning table and timing events.  Every compute
// entry point runs the same three launches on the device:
//   plan (one workgroup) -> pack (phi, validation) -> persistent walk,
// so validation, packing, the Gray walk, the reductions and the final mod 3
// all happen in kernels; host code only checks arguments, moves bytes and
// launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "perm3.h"
#include "perm3_internal.h"
#include "perm3_runtime.h"
#include "perm3_walk.hpp"

namespace perm3 {

// ------------------------------------------------------------------ errors

static thread_local std::string tl_error;
static thread_local int64_t tl_error_index = -1;

int32_t set_error(int32_t code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    tl_error = buf;
    return code;
}

void set_error_index(int64_t idx) { tl_error_index = idx; }

int32_t hip_fail(hipError_t e, const char *what)
{
    return set_error(PERM_EDEVICE, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

#define HIP_TRY(expr)                                         \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return hip_fail(_e, #expr);     \
    } while (0)

// ------------------------------------------------------------------ tuning

perm_tuning default_tuning()
{
    perm_tuning t;
    memset(&t, 0, sizeof t);
    t.waves_per_simd = 8;
    t.body_log = 5;
    t.chunk_log_max = 20;
    t.tasks_per_wave = 16;
    t.direct_max_n = 11;
    t.use_graphs = 1;
    t.states_per_lane = 1;
    t.body_log_mid = 4;
    t.mid_max_n = 31;
    t.max_tasks_log = 10;
    t.min_task_log = 19;
    t.queue_task_log = 18;
    return t;
}

bool tuning_valid(const perm_tuning &t)
{
    return t.waves_per_simd >= 1 && t.waves_per_simd <= 16 && t.body_log >= 4 && t.body_log <= 6 &&
           t.chunk_log_max >= 8 && t.chunk_log_max <= 24 && t.tasks_per_wave >= 1 &&
           t.tasks_per_wave <= 1024 && t.direct_max_n >= t.body_log + 6 && t.direct_max_n <= 63 &&
           (t.use_graphs == 0 || t.use_graphs == 1) &&
           (t.states_per_lane == 1 || t.states_per_lane == 2 || t.states_per_lane == 4) &&
           t.body_log_mid >= 4 && t.body_log_mid <= 6 && t.mid_max_n >= 0 && t.mid_max_n <= 63 &&
           t.direct_max_n >= t.body_log_mid + 6 && t.min_task_log >= 0 && t.min_task_log <= 30 &&
           t.max_tasks_log >= 0 && t.max_tasks_log <= 40 && t.queue_task_log >= 0 && t.queue_task_log <= 30;
}

int tune_class_host(int32_t count, int32_t n0)
{
    if (count != 1) return PERM_TUNE_BATCH;
    if (n0 <= 24) return PERM_TUNE_SMALL;
    if (n0 <= 31) return PERM_TUNE_MID;
    return PERM_TUNE_LARGE;
}

// ------------------------------------------------------------------ context

DevBuf::~DevBuf()
{
    if (p) (void)hipFree(p);
}

hipError_t DevBuf::reserve(size_t n)
{
    if (n <= cap) return hipSuccess;
    if (p) {
        // earlier asynchronous calls may still read the old buffer
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return e;
        e = hipFree(p);
        p = nullptr;
        cap = 0;
        if (e != hipSuccess) return e;
    }
    size_t want = std::max<size_t>(n, 256);
    hipError_t e = hipMalloc(&p, want);
    if (e == hipSuccess) cap = want;
    return e;
}

HostBuf::~HostBuf()
{
    if (p) (void)hipHostFree(p);
}

hipError_t HostBuf::reserve(size_t n)
{
    if (n <= cap) return hipSuccess;
    if (p) {
        // a copy from the old buffer may still be queued after a failed call
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return e;
        (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
    }
    size_t want = std::max<size_t>(n, 4096);
    hipError_t e = hipHostMalloc(&p, want, flags);
    if (e == hipSuccess) cap = want;
    return e;
}

size_t workset_bytes(int32_t count, int64_t rows, bool acc) { return workset_layout(count, rows, acc).off[9]; }

WorkSet workset_carve(void *base, int32_t count, int64_t rows, bool acc)
{
    const WorkSetLayout L = workset_layout(count, rows, acc);
    const size_t *off = L.off;
    uint8_t *b = (uint8_t *)base;
    WorkSet w;
    w.meta = (MatMeta *)(b + off[0]);
    w.order = (int32_t *)(b + off[1]);
    w.task_start = (uint64_t *)(b + off[2]);
    w.tally = (int64_t *)(b + off[3]);
    w.done = (uint64_t *)(b + off[4]);
    w.status = b + off[5];
    w.counters = (uint64_t *)(b + off[6]);
    w.rows = (RowW *)(b + off[7]);
    w.acc = acc ? (uint64_t *)(b + off[8]) : nullptr;
    return w;
}

Context::~Context()
{
    for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
    if (ev_walk0) (void)hipEventDestroy(ev_walk0);
    if (ev_walk1) (void)hipEventDestroy(ev_walk1);
    if (ev_all0) (void)hipEventDestroy(ev_all0);
    if (ev_all1) (void)hipEventDestroy(ev_all1);
    if (ev_done) (void)hipEventDestroy(ev_done);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (stream) (void)hipStreamDestroy(stream);
}

static std::mutex g_ctx_mu;
static std::map<int, std::unique_ptr<Context>> g_ctx;
static thread_local bool tl_timing = false;

// The context of the current device, made on first use.  Making one creates
// a stream and events and allocates no device memory: work buffers come with
// the first call that needs them.
int32_t get_context(Context **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> g(g_ctx_mu);
    auto it = g_ctx.find(dev);
    if (it != g_ctx.end()) {
        *out = it->second.get();
        return PERM_OK;
    }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_error(PERM_EDEVICE, "device %d is %s; this library is built for gfx950 only", dev,
                         prop.gcnArchName);
    std::unique_ptr<Context> c(new Context());
    c->device = dev;
    c->cus = prop.multiProcessorCount;
    c->clock_khz = prop.clockRate;
    snprintf(c->arch, sizeof c->arch, "%s", prop.gcnArchName);
    for (int k = 0; k < PERM_TUNE_CLASSES; ++k) {
        c->tunings[k] = default_tuning();
        c->tune_src[k] = PERM_TUNE_SRC_DEFAULT;
    }
    // a tuning cache beside the library (or named by the environment), if any
    load_default_cache(*c);
    int32_t rc = noalloc_init(*c);
    if (rc) return rc;
    HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreate(&c->ev_walk0));
    HIP_TRY(hipEventCreate(&c->ev_walk1));
    HIP_TRY(hipEventCreate(&c->ev_all0));
    HIP_TRY(hipEventCreate(&c->ev_all1));
    HIP_TRY(hipEventCreateWithFlags(&c->ev_done, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
    *out = c.get();
    g_ctx[dev] = std::move(c);
    return PERM_OK;
}

bool timing_enabled() { return tl_timing; }

// The persistent walk's workgroups (4 waves each, one per SIMD): waves_per_simd
// per CU, but no more than fit on a CU at once.
int Context::grid_blocks(const perm_tuning &tn) const
{
    return cus * std::min(tn.waves_per_simd, walk_resident_per_cu(tn.states_per_lane));
}

void Context::set_tuning(int cls, const perm_tuning &t, int32_t src)
{
    tunings[cls] = t;
    tune_src[cls] = src;
    drop_graphs();
}

void Context::drop_graphs()
{
    for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
}

// Make sure the shared work set holds `count` matrices with `rows` rows in total.
int32_t Context::reserve_work(int32_t count, int64_t rows)
{
    if (!small_acc.p) {
        HIP_TRY(small_acc.reserve(SMALL_PLAN_MAX * sizeof(uint64_t)));
        HIP_TRY(hipMemset(small_acc.p, 0, SMALL_PLAN_MAX * sizeof(uint64_t)));
    }
    count = std::max(count, 1);
    rows = std::max<int64_t>(rows, 1);
    if (work.p && count <= ws_count && rows <= ws_rows) return PERM_OK;
    const int32_t c = std::max(count, ws_count);
    const int64_t r = std::max(rows, ws_rows);
    void *before = work.p;
    HIP_TRY(work.reserve(workset_bytes(c, r, false)));
    ws = workset_carve(work.p, c, r, false);
    ws.acc = (uint64_t *)small_acc.p;
    ws_count = c;
    ws_rows = r;
    if (work.p != before) drop_graphs();
    return PERM_OK;
}

// Order this call after every earlier call of the context (they share buffers).
int32_t Context::join(hipStream_t st)
{
    if (have_last && last_stream != st) HIP_TRY(hipStreamWaitEvent(st, ev_done, 0));
    return PERM_OK;
}

int32_t Context::mark(hipStream_t st)
{
    HIP_TRY(hipEventRecord(ev_done, st));
    last_stream = st;
    have_last = true;
    return PERM_OK;
}

PlanArgs Context::plan_args(const WorkSet &w, const perm_tuning &tn, const int32_t *ns_dev, int32_t count,
                            uint8_t *out_dev, uint64_t *hist_dev) const
{
    PlanArgs a;
    memset(&a, 0, sizeof a);
    a.ns = ns_dev;
    a.count = count;
    a.body_log = tn.body_log;
    a.chunk_log_max = tn.chunk_log_max;
    a.direct_max_n = tn.direct_max_n;
    a.direct_chunk_log_max = 10;
    a.body_log_mid = tn.body_log_mid;
    a.mid_max_n = tn.mid_max_n;
    a.states_log = tn.states_per_lane == 4 ? 2 : (tn.states_per_lane == 2 ? 1 : 0);
    a.max_tasks_log = tn.max_tasks_log;
    a.min_task_log = tn.min_task_log;
    a.queue_task_log = tn.queue_task_log;
    a.waves_total = 4 * grid_blocks(tn);
    a.tasks_per_wave = tn.tasks_per_wave;
    a.meta = w.meta;
    a.order = w.order;
    a.task_start = w.task_start;
    a.tally = w.tally;
    a.done = w.done;
    a.status = w.status;
    a.counters = w.counters;
    a.out = out_dev;
    a.hist = hist_dev;
    return a;
}

WalkArgs Context::walk_args(const WorkSet &w, int32_t count, uint8_t *out_dev, uint64_t *hist_dev) const
{
    WalkArgs a;
    a.rows = w.rows;
    a.meta = w.meta;
    a.order = w.order;
    a.task_start = w.task_start;
    a.count = count;
    a.tally = w.tally;
    a.done = w.done;
    a.status = w.status;
    a.counters = w.counters;
    a.out = out_dev;
    a.hist = hist_dev;
    return a;
}

// Enqueue plan -> pack -> walk on the work set w.  pack_kind: 0 bytes, 1 planes.
int32_t Context::enqueue(const Launch &L, const WorkSet &w, const perm_tuning &tn, hipStream_t st, bool timed)
{
    PlanArgs pa = plan_args(w, tn, L.ns_dev, L.count, L.out_dev, L.hist_dev);
    pa.use_range = L.use_range;
    pa.range_lo = L.range_lo;
    pa.range_hi = L.range_hi;
    if (timed) HIP_TRY(hipEventRecord(ev_all0, st));
    PackU8Args pk;
    pk.mats = L.mats_dev;
    pk.offs = L.offs_dev;
    pk.meta = w.meta;
    pk.count = L.count;
    pk.rows = w.rows;
    pk.status = w.status;
    PackPlanesArgs pp;
    pp.planes = L.planes_dev;
    pp.row_off = L.row_off_dev;
    pp.meta = w.meta;
    pp.count = L.count;
    pp.rows = w.rows;
    pp.status = w.status;
    const bool small = L.count <= SMALL_PLAN_MAX;
    const bool bytes = L.pack_kind == 0;
    const int grid = grid_blocks(tn);
    if (small) {
        // one launch plans and packs and, for little work, walks too
        SmallAcc sa;
        sa.word = w.acc;
        if (L.zero_acc) HIP_TRY(launch_fill_u64(w.acc, SMALL_PLAN_MAX, 0, st));
        if (timed && L.fused_only) HIP_TRY(hipEventRecord(ev_walk0, st));
        const int blocks = L.small_blocks > 0 ? std::min(L.small_blocks, grid) : grid;
        HIP_TRY(launch_small(pa, pk, pp, sa, bytes ? 0 : 1, !L.use_range, std::max(blocks, L.count + 1), st));
        if (L.fused_only) {
            if (timed) {
                HIP_TRY(hipEventRecord(ev_walk1, st));
                HIP_TRY(hipEventRecord(ev_all1, st));
            }
            last_timing_valid = timed;
            last_launches = L.zero_acc ? 2 : 1;
            return PERM_OK;
        }
    } else {
        HIP_TRY(launch_plan(pa, st));
        HIP_TRY(bytes ? launch_pack_u8(pk, st) : launch_pack_planes(pp, st));
    }
    if (timed) HIP_TRY(hipEventRecord(ev_walk0, st));
    HIP_TRY(launch_walk(walk_args(w, L.count, L.out_dev, L.hist_dev), tn.states_per_lane, L.defer != 0, grid, st));
    if (timed) {
        HIP_TRY(hipEventRecord(ev_walk1, st));
        HIP_TRY(hipEventRecord(ev_all1, st));
    }
    last_timing_valid = timed;
    last_launches = (small ? 2 : 3) + (L.zero_acc ? 1 : 0);
    return PERM_OK;
}

// Run a launch: eagerly when timed, else through a cached HIP graph.
int32_t Context::run(const Launch &L, hipStream_t st, bool use_graph)
{
    const bool timed = tl_timing;
    int32_t rc = join(st);
    if (rc) return rc;
    last_graph = 0;
    // Calls of up to SMALL_PLAN_MAX matrices are two launches, issued directly:
    // replaying them as a graph costs more than it saves.
    const perm_tuning &tune = tn(L.cls);
    if (timed || !use_graph || !tune.use_graphs || L.count <= SMALL_PLAN_MAX) {
        rc = enqueue(L, ws, tune, st, timed);
        if (rc) return rc;
        return mark(st);
    }
    GraphKey key{L.pack_kind,
                 (uintptr_t)(L.pack_kind == 0 ? (const void *)L.mats_dev : (const void *)L.planes_dev),
                 (uintptr_t)(L.pack_kind == 0 ? (const void *)L.offs_dev : (const void *)L.row_off_dev),
                 (uintptr_t)L.ns_dev,
                 (uintptr_t)L.out_dev,
                 (uintptr_t)L.hist_dev,
                 (uintptr_t)st,
                 L.count,
                 0};   // tuning changes drop every cached graph
    auto it = graphs.find(key);
    if (it == graphs.end()) {
        if (graphs.size() >= 32) drop_graphs();
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        rc = enqueue(L, ws, tune, st, false);
        hipError_t e = hipStreamEndCapture(st, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        it = graphs.emplace(key, ex).first;
    } else {
        last_graph = 1;
    }
    HIP_TRY(hipGraphLaunch(it->second, st));
    last_timing_valid = false;
    last_launches = 3;   // graphs are used for calls of more than SMALL_PLAN_MAX matrices only
    return mark(st);
}

// A device-input call issued while the caller captures `st` into a graph of
// its own.  The launches go straight into that capture: no graph of the
// library's, no event waits or records, no timing.  The call gets a work set
// of its own, allocated now and kept until the context ends, so that replays
// of the caller's graph neither race with other calls into the library nor
// lose their buffers when the shared set grows.  Its accumulator words are
// cleared by a kernel at the start of every replay.
int32_t Context::run_captured(const Launch &L, hipStream_t st)
{
    const int64_t rows = (int64_t)L.count * PERM_MAX_N;
    std::unique_ptr<DevBuf> buf(new DevBuf());
    // allocation is not a stream operation; let it pass a capture in global mode
    hipStreamCaptureMode mode = hipStreamCaptureModeRelaxed;
    HIP_TRY(hipThreadExchangeStreamCaptureMode(&mode));
    const hipError_t e = buf->reserve(workset_bytes(L.count, rows, true));
    (void)hipThreadExchangeStreamCaptureMode(&mode);
    if (e != hipSuccess) return hip_fail(e, "work buffers for a captured call");
    const WorkSet w = workset_carve(buf->p, L.count, rows, true);
    captured.push_back(std::move(buf));
    Launch C = L;
    C.zero_acc = L.count <= SMALL_PLAN_MAX ? 1 : 0;
    const int32_t rc = enqueue(C, w, tn(L.cls), st, false);
    last_timing_valid = false;
    last_graph = 0;
    return rc;
}

// A device-input call on the caller's stream.  For a NULL stream (where torch
// runs unless told otherwise): a call launched directly goes on the NULL
// stream itself; a graph, which cannot be captured there, is replayed on the
// library's stream, ordered after earlier and before later work on the NULL
// stream.
int32_t Context::run_dev(const Launch &L, hipStream_t user)
{
    if (user) return run(L, user, true);
    // a call launched directly (no graph capture) goes on the NULL stream itself
    if (L.count <= SMALL_PLAN_MAX || !tn(L.cls).use_graphs) return run(L, nullptr, false);
    HIP_TRY(hipEventRecord(ev_in, nullptr));
    HIP_TRY(hipStreamWaitEvent(stream, ev_in, 0));
    int32_t rc = run(L, stream, true);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(ev_out, stream));
    HIP_TRY(hipStreamWaitEvent(nullptr, ev_out, 0));
    return PERM_OK;
}

// Stage host matrices into device memory (pinned copy) and run them; results
// to host.  All matrices have been validated by the caller.
int32_t Context::run_host(const uint8_t *const *As, const int32_t *ns, int32_t count, bool use_range,
                          uint64_t lo, uint64_t hi, uint8_t *out_host, int64_t *tally_host)
{
    int64_t bytes = 0, rows = 0;
    int32_t nmax = 0;
    for (int32_t k = 0; k < count; ++k) {
        bytes += (int64_t)ns[k] * ns[k];
        rows += ns[k];
        nmax = std::max(nmax, ns[k]);
    }
    const size_t offs_bytes = (size_t)count * sizeof(int64_t);
    const size_t ns_bytes = (size_t)count * sizeof(int32_t);
    const size_t offs_at = (((size_t)bytes + 15) / 16) * 16;
    const size_t ns_at = offs_at + offs_bytes;
    const size_t stage_bytes = ns_at + ns_bytes;
    // the orders are known here: a small call whose walk k_small takes alone
    // needs no k_walk after it (the kernel makes the same decision)
    const int cls = tune_class_host(count, ns[0]);
    const bool fused_only = small_call_fused(ns, count, use_range);
    uint64_t tasks = 0;
    if (fused_only) tasks = small_call_tasks(plan_args(ws, tn(cls), nullptr, count, nullptr, nullptr), ns, count);
    // Such a call reads its inputs straight from coherent pinned memory when
    // that moves little over the host link (each of its waves reads the
    // orders, the offsets and its matrix once): no staging copy before it.
    const bool zero_copy =
        fused_only && tasks * (uint64_t)(12 * count + nmax * nmax) <= (1ull << 20);
    HostBuf &hst = zero_copy ? h_zc : h_stage;
    HIP_TRY(hst.reserve(stage_bytes));
    if (!zero_copy) HIP_TRY(d_stage.reserve(stage_bytes));
    // results go straight to pinned host memory: no copy after the walk
    HIP_TRY(h_out.reserve((size_t)std::max(count, 1)));
    uint8_t *out_dev = nullptr;
    HIP_TRY(hipHostGetDevicePointer((void **)&out_dev, h_out.p, 0));
    int32_t rc = reserve_work(count, rows);
    if (rc) return rc;
    uint8_t *h = (uint8_t *)hst.p;
    int64_t *hoffs = (int64_t *)(h + offs_at);
    int32_t *hns = (int32_t *)(h + ns_at);
    int64_t o = 0;
    for (int32_t k = 0; k < count; ++k) {
        const int64_t sz = (int64_t)ns[k] * ns[k];
        if (sz) memcpy(h + o, As[k], (size_t)sz);
        hoffs[k] = o;
        hns[k] = ns[k];
        o += sz;
    }
    hipStream_t st = stream;
    rc = join(st);
    if (rc) return rc;
    uint8_t *d = nullptr;
    if (zero_copy) {
        HIP_TRY(hipHostGetDevicePointer((void **)&d, hst.p, 0));
    } else {
        HIP_TRY(hipMemcpyAsync(d_stage.p, h_stage.p, stage_bytes, hipMemcpyHostToDevice, st));
        d = (uint8_t *)d_stage.p;
    }
    Launch L;
    memset(&L, 0, sizeof L);
    L.pack_kind = 0;
    L.mats_dev = d;
    L.offs_dev = (const int64_t *)(d + offs_at);
    L.ns_dev = (const int32_t *)(d + ns_at);
    L.count = count;
    L.out_dev = out_dev;
    L.hist_dev = nullptr;
    L.use_range = use_range ? 1 : 0;
    L.range_lo = lo;
    L.range_hi = hi;
    L.fused_only = fused_only ? 1 : 0;
    L.cls = cls;
    L.defer = count > 1 || ns[0] <= 32 ? 1 : 0;
    // one wave per task (4 per block): blocks beyond the tasks would only start and leave
    if (fused_only) L.small_blocks = (int32_t)std::min<uint64_t>((tasks + 3) / 4, (uint64_t)grid_blocks(tn(cls)));
    rc = run(L, st, false);
    if (rc) return rc;
    if (tally_host) HIP_TRY(hipMemcpyAsync(tally_host, ws.tally, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (out_host) memcpy(out_host, h_out.p, (size_t)count);
    return PERM_OK;
}

int32_t Context::timing(perm_timing *t)
{
    memset(t, 0, sizeof *t);
    t->launches = last_launches;
    t->graph_replayed = last_graph;
    if (!last_timing_valid) return PERM_OK;
    HIP_TRY(hipEventSynchronize(ev_all1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev_walk0, ev_walk1));
    t->hot_kernel_ms = ms;
    HIP_TRY(hipEventElapsedTime(&ms, ev_all0, ev_all1));
    t->total_ms = ms;
    return PERM_OK;
}

// ------------------------------------------------------------------ host checks

static int32_t check_matrix(const uint8_t *A, int32_t n, int64_t *bad_at)
{
    if (n < 0 || n > PERM_MAX_N) return set_error(PERM_EINVAL, "n = %d is outside [0, %d]", n, PERM_MAX_N);
    if (n > 0 && !A) return set_error(PERM_EINVAL, "null matrix pointer");
    const int64_t cells = (int64_t)n * n;
    for (int64_t i = 0; i < cells; ++i) {
        if (A[i] > 2) {
            if (bad_at) *bad_at = i;
            return set_error(PERM_EDOMAIN, "entry %lld is %u; entries must be 0, 1 or 2", (long long)i,
                             (unsigned)A[i]);
        }
    }
    return PERM_OK;
}

}  // namespace perm3

using namespace perm3;

// ------------------------------------------------------------------ C ABI

extern "C" {

int32_t perm_mod3(const uint8_t *A, int32_t n, uint8_t *out)
{
    set_error_index(-1);
    if (!out) return set_error(PERM_EINVAL, "null output pointer");
    int64_t bad = -1;
    int32_t rc = check_matrix(A, n, &bad);
    if (rc) {
        set_error_index(bad);
        return rc;
    }
    Context *c = nullptr;
    if ((rc = get_context(&c))) return rc;
    std::lock_guard<std::mutex> g(c->mu);
    const uint8_t *As[1] = {A};
    int32_t ns[1] = {n};
    return c->run_host(As, ns, 1, false, 0, 0, out, nullptr);
}

int32_t perm_mod3_range_tally(const uint8_t *A, int32_t n, uint64_t begin, uint64_t end, int64_t *tally)
{
    set_error_index(-1);
    if (!tally) return set_error(PERM_EINVAL, "null tally pointer");
    int64_t bad = -1;
    int32_t rc = check_matrix(A, n, &bad);
    if (rc) {
        set_error_index(bad);
        return rc;
    }
    const uint64_t total = 1ull << n;
    if (begin > end || end > total)
        return set_error(PERM_EINVAL, "range [%llu, %llu) is not inside [0, 2^%d]", (unsigned long long)begin,
                         (unsigned long long)end, n);
    Context *c = nullptr;
    if ((rc = get_context(&c))) return rc;
    std::lock_guard<std::mutex> g(c->mu);
    const uint8_t *As[1] = {A};
    int32_t ns[1] = {n};
    return c->run_host(As, ns, 1, true, begin, end, nullptr, tally);
}

int32_t perm_mod3_batch(const uint8_t *const *As, const int32_t *ns, int32_t count, uint8_t *out)
{
    set_error_index(-1);
    if (count < 0 || count > PERM_MAX_BATCH) return set_error(PERM_EINVAL, "count = %d out of range", count);
    if (count == 0) return PERM_OK;
    if (!As || !ns || !out) return set_error(PERM_EINVAL, "null pointer argument");
    for (int32_t k = 0; k < count; ++k) {
        int32_t rc = check_matrix(As[k], ns[k], nullptr);
        if (rc) {
            set_error_index(k);
            return rc;
        }
    }
    Context *c = nullptr;
    int32_t rc = get_context(&c);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(c->mu);
    return c->run_host(As, ns, count, false, 0, 0, out, nullptr);
}

// The device-input calls: into the caller's capture when `stream` is being
// captured, else eagerly or through the library's cached graphs.
static int32_t run_device_call(Launch &L, void *stream)
{
    const hipStream_t st = (hipStream_t)stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (st) HIP_TRY(hipStreamIsCapturing(st, &cs));
    if (cs == hipStreamCaptureStatusInvalidated)
        return set_error(PERM_EDEVICE, "the stream's capture has been invalidated");
    const bool capturing = cs == hipStreamCaptureStatusActive;
    Context *c = nullptr;
    int32_t rc;
    if (capturing) {
        // making the context (first call on a device) is no stream operation either
        hipStreamCaptureMode mode = hipStreamCaptureModeRelaxed;
        HIP_TRY(hipThreadExchangeStreamCaptureMode(&mode));
        rc = get_context(&c);
        (void)hipThreadExchangeStreamCaptureMode(&mode);
    } else {
        rc = get_context(&c);
    }
    if (rc) return rc;
    std::lock_guard<std::mutex> g(c->mu);
    if (capturing) return c->run_captured(L, st);
    if ((rc = c->reserve_work(L.count, (int64_t)L.count * PERM_MAX_N))) return rc;
    return c->run_dev(L, st);
}

int32_t perm_mod3_batch_dev(const uint8_t *mats_dev, const int64_t *offs_dev, const int32_t *ns_dev,
                            int32_t count, uint8_t *out_dev, uint64_t *hist_dev, void *stream)
{
    set_error_index(-1);
    if (count < 0 || count > PERM_MAX_BATCH) return set_error(PERM_EINVAL, "count = %d out of range", count);
    if (count == 0) return PERM_OK;
    if (!mats_dev || !offs_dev || !ns_dev || !out_dev) return set_error(PERM_EINVAL, "null pointer argument");
    Launch L;
    memset(&L, 0, sizeof L);
    L.pack_kind = 0;
    L.mats_dev = mats_dev;
    L.offs_dev = offs_dev;
    L.ns_dev = ns_dev;
    L.count = count;
    L.out_dev = out_dev;
    L.hist_dev = hist_dev;
    L.cls = count == 1 ? PERM_TUNE_LARGE : PERM_TUNE_BATCH;
    L.defer = count > 1 ? 1 : 0;
    return run_device_call(L, stream);
}

int32_t perm_mod3_batch_packed(const uint64_t *planes_dev, const int64_t *row_off_dev, const int32_t *ns_dev,
                               int32_t count, uint8_t *out_dev, uint64_t *hist_dev, void *stream)
{
    set_error_index(-1);
    if (count < 0 || count > PERM_MAX_BATCH) return set_error(PERM_EINVAL, "count = %d out of range", count);
    if (count == 0) return PERM_OK;
    if (!planes_dev || !row_off_dev || !ns_dev || !out_dev)
        return set_error(PERM_EINVAL, "null pointer argument");
    Launch L;
    memset(&L, 0, sizeof L);
    L.pack_kind = 1;
    L.planes_dev = planes_dev;
    L.row_off_dev = row_off_dev;
    L.ns_dev = ns_dev;
    L.count = count;
    L.out_dev = out_dev;
    L.hist_dev = hist_dev;
    L.cls = count == 1 ? PERM_TUNE_LARGE : PERM_TUNE_BATCH;
    L.defer = count > 1 ? 1 : 0;
    return run_device_call(L, stream);
}

int32_t perm_mod3_from_tallies(int32_t n, const int64_t *tallies, int32_t count, uint8_t *out)
{
    set_error_index(-1);
    if (n < 0 || n > PERM_MAX_N) return set_error(PERM_EINVAL, "n = %d is outside [0, %d]", n, PERM_MAX_N);
    if (count < 1 || count > PERM_MAX_TALLIES)
        return set_error(PERM_EINVAL, "count = %d is outside [1, %d]", count, PERM_MAX_TALLIES);
    if (!tallies || !out) return set_error(PERM_EINVAL, "null pointer argument");
    Context *c = nullptr;
    int32_t rc = get_context(&c);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(c->mu);
    const size_t bytes = (size_t)count * sizeof(int64_t);
    HIP_TRY(c->h_zc.reserve(bytes));
    HIP_TRY(c->h_out.reserve(1));
    memcpy(c->h_zc.p, tallies, bytes);
    int64_t *t_dev = nullptr;
    uint8_t *out_dev = nullptr;
    HIP_TRY(hipHostGetDevicePointer((void **)&t_dev, c->h_zc.p, 0));
    HIP_TRY(hipHostGetDevicePointer((void **)&out_dev, c->h_out.p, 0));
    const hipStream_t st = c->stream;
    if ((rc = c->join(st))) return rc;
    HIP_TRY(launch_finish_tallies(t_dev, count, n, out_dev, st));
    HIP_TRY(hipStreamSynchronize(st));
    *out = *(volatile uint8_t *)c->h_out.p;
    c->last_timing_valid = false;
    c->last_launches = 1;
    c->last_graph = 0;
    return c->mark(st);
}

int32_t perm_mod3_pack(const uint8_t *A, int32_t n, uint64_t *planes)
{
    set_error_index(-1);
    if (!planes && n > 0) return set_error(PERM_EINVAL, "null planes pointer");
    int64_t bad = -1;
    int32_t rc = check_matrix(A, n, &bad);
    if (rc) {
        set_error_index(bad);
        return rc;
    }
    for (int32_t r = 0; r < n; ++r) {
        uint64_t mag = 0, sgn = 0;
        for (int32_t j = 0; j < n; ++j) {
            const uint8_t v = A[(int64_t)r * n + j];
            const uint64_t bit = 1ull << (n - 1 - j);
            if (v != 0) mag |= bit;
            if (v == 2) sgn |= bit;
        }
        planes[2 * r] = mag;
        planes[2 * r + 1] = sgn;
    }
    return PERM_OK;
}

int32_t perm_mod3_census(int32_t n, int32_t generator, uint64_t key, uint64_t first, uint64_t count,
                         uint64_t *counts)
{
    set_error_index(-1);
    if (!counts) return set_error(PERM_EINVAL, "null counts pointer");
    if (n < 1 || n > PERM_MAX_N) return set_error(PERM_EINVAL, "n = %d is outside [1, %d]", n, PERM_MAX_N);
    if (generator != PERM_GEN_ENUMERATE && generator != PERM_GEN_SPLITMIX)
        return set_error(PERM_EINVAL, "unknown generator %d", generator);
    if (generator == PERM_GEN_ENUMERATE) {
        if (n > 6) return set_error(PERM_EINVAL, "enumeration needs n <= 6");
        uint64_t total = 1;
        for (int k = 0; k < n * n; ++k) total *= 3u;
        if (first > total || count > total - first)
            return set_error(PERM_EINVAL, "matrices [%llu, +%llu) exceed 3^%d", (unsigned long long)first,
                             (unsigned long long)count, n * n);
    }
    counts[0] = counts[1] = counts[2] = 0;
    if (count == 0) return PERM_OK;
    Context *c = nullptr;
    int32_t rc = get_context(&c);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(c->mu);
    hipStream_t st = c->stream;
    if ((rc = c->join(st))) return rc;
    HIP_TRY(c->d_census.reserve(64 * 3 * sizeof(uint64_t)));
    unsigned long long *dcounts = (unsigned long long *)c->d_census.p;
    HIP_TRY(hipMemsetAsync(dcounts, 0, 64 * 3 * sizeof(uint64_t), st));
    if (n <= CENSUS_LANE_MAX_N) {
        CensusArgs a;
        a.n = n;
        a.gen = generator;
        a.key = key;
        a.first = first;
        a.count = count;
        a.counts = dcounts;
        HIP_TRY(launch_census_lanes(a, c->cus, st));
    } else {
        // generate chunks into device memory and walk them as a batch; the
        // histogram row 3n..3n+2 accumulates the results
        const uint32_t chunk = 1u << 16;
        const uint64_t nn = (uint64_t)n * n;
        HIP_TRY(c->d_gen.reserve((size_t)chunk * (nn + sizeof(int64_t) + sizeof(int32_t) + 1) + 64));
        uint8_t *mats = (uint8_t *)c->d_gen.p;
        int64_t *offs = (int64_t *)(mats + (((size_t)chunk * nn + 15) / 16) * 16);
        int32_t *ns = (int32_t *)(offs + chunk);
        uint8_t *out = (uint8_t *)(ns + chunk);
        if ((rc = c->reserve_work((int32_t)chunk, (int64_t)chunk * n))) return rc;
        for (uint64_t done = 0; done < count; done += chunk) {
            const uint32_t cnt = (uint32_t)std::min<uint64_t>(chunk, count - done);
            GenArgs ga;
            ga.n = n;
            ga.gen = generator;
            ga.key = key;
            ga.first = first + done;
            ga.count = cnt;
            ga.mats = mats;
            ga.offs = offs;
            ga.ns = ns;
            HIP_TRY(launch_generate(ga, st));
            Launch L;
            memset(&L, 0, sizeof L);
            L.pack_kind = 0;
            L.mats_dev = mats;
            L.offs_dev = offs;
            L.ns_dev = ns;
            L.count = (int32_t)cnt;
            L.out_dev = out;
            L.hist_dev = (uint64_t *)dcounts;
            L.cls = PERM_TUNE_BATCH;
            L.defer = 1;
            if ((rc = c->enqueue(L, c->ws, c->tn(PERM_TUNE_BATCH), st, false))) return rc;
        }
    }
    uint64_t h[64 * 3];
    HIP_TRY(hipMemcpyAsync(h, dcounts, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const int row = n <= CENSUS_LANE_MAX_N ? 0 : 3 * n;
    counts[0] = h[row];
    counts[1] = h[row + 1];
    counts[2] = h[row + 2];
    return c->mark(st);
}

int32_t perm_tuning_get(perm_tuning *t)
{
    if (!t) return set_error(PERM_EINVAL, "null pointer");
    Context *c = nullptr;
    int32_t rc = get_context(&c);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(c->mu);
    *t = c->tunings[PERM_TUNE_LARGE];
    return PERM_OK;
}

int32_t perm_tuning_set(const perm_tuning *t)
{
    if (!t) return set_error(PERM_EINVAL, "null pointer");
    if (!tuning_valid(*t)) return set_error(PERM_EINVAL, "tuning out of range");
    Context *c = nullptr;
    int32_t rc = get_context(&c);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(c->mu);
    for (int k = 0; k < PERM_TUNE_CLASSES; ++k) c->set_tuning(k, *t, PERM_TUNE_SRC_SET);
    return PERM_OK;
}

int32_t perm_tuning_get_class(int32_t cls, perm_tuning *t, int32_t *source)
{
    if (!t) return set_error(PERM_EINVAL, "null pointer");
    if (cls < 0 || cls >= PERM_TUNE_CLASSES) return set_error(PERM_EINVAL, "unknown tuning class %d", cls);
    Context *c = nullptr;
    int32_t rc = get_context(&c);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(c->mu);
    *t = c->tunings[cls];
    if (source) *source = c->tune_src[cls];
    return PERM_OK;
}

int32_t perm_tuning_set_class(int32_t cls, const perm_tuning *t)
{
    if (!t) return set_error(PERM_EINVAL, "null pointer");
    if (cls < 0 || cls >= PERM_TUNE_CLASSES) return set_error(PERM_EINVAL, "unknown tuning class %d", cls);
    if (!tuning_valid(*t)) return set_error(PERM_EINVAL, "tuning out of range");
    Context *c = nullptr;
    int32_t rc = get_context(&c);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(c->mu);
    c->set_tuning(cls, *t, PERM_TUNE_SRC_SET);
    return PERM_OK;
}

int32_t perm_tuning_reset(int32_t with_cache)
{
    Context *c = nullptr;
    int32_t rc = get_context(&c);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(c->mu);
    for (int k = 0; k < PERM_TUNE_CLASSES; ++k) c->set_tuning(k, default_tuning(), PERM_TUNE_SRC_DEFAULT);
    if (with_cache) load_default_cache(*c);
    return PERM_OK;
}

int32_t perm_timing_enable(int32_t on)
{
    tl_timing = on != 0;
    return PERM_OK;
}

int32_t perm_timing_last(perm_timing *t)
{
    if (!t) return set_error(PERM_EINVAL, "null pointer");
    Context *c = nullptr;
    int32_t rc = get_context(&c);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(c->mu);
    return c->timing(t);
}

int32_t perm_device_info_get(perm_device_info *info)
{
    if (!info) return set_error(PERM_EINVAL, "null pointer");
    Context *c = nullptr;
    int32_t rc = get_context(&c);
    if (rc) return rc;
    memset(info, 0, sizeof *info);
    info->compute_units = c->cus;
    info->simds_per_cu = 4;
    info->wave_size = 64;
    info->max_clock_khz = c->clock_khz;
    snprintf(info->arch, sizeof info->arch, "%s", c->arch);
    return PERM_OK;
}

int32_t perm_bipedal_ops(const uint32_t *in, int32_t count, uint32_t *out)
{
    if (count < 0 || count > (1 << 24)) return set_error(PERM_EINVAL, "count out of range");
    if (count == 0) return PERM_OK;
    if (!in || !out) return set_error(PERM_EINVAL, "null pointer");
    Context *c = nullptr;
    int32_t rc = get_context(&c);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(c->mu);
    DevBuf din, dout;
    HIP_TRY(din.reserve((size_t)count * 16));
    HIP_TRY(dout.reserve((size_t)count * 32));
    HIP_TRY(hipMemcpyAsync(din.p, in, (size_t)count * 16, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(launch_bipedal_ops((const uint32_t *)din.p, count, (uint32_t *)dout.p, c->stream));
    HIP_TRY(hipMemcpyAsync(out, dout.p, (size_t)count * 32, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return PERM_OK;
}

const char *perm_strerror(int32_t code)
{
    switch (code) {
    case PERM_OK: return "ok";
    case PERM_EINVAL: return "invalid argument";
    case PERM_EDOMAIN: return "matrix entry outside {0,1,2} or packed bit beyond n";
    case PERM_ENOMEM: return "out of memory";
    case PERM_EDEVICE: return "HIP device error";
    case PERM_EAGAIN: return "queue full, try again";
    case PERM_ESTATE: return "object shut down or busy";
    default: return "unknown status";
    }
}

const char *perm_last_error(void) { return tl_error.c_str(); }
int64_t perm_last_error_index(void) { return tl_error_index; }
const char *perm_version(void) { return "perm3 1.0 gfx950"; }

}  // extern "C"
