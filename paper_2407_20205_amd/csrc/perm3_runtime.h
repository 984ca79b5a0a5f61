// Host-side context of libperm3 (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "perm3.h"
#include "perm3_internal.h"
#include "perm3_walk.hpp"

namespace perm3 {

int32_t set_error(int32_t code, const char *fmt, ...);
void set_error_index(int64_t idx);
int32_t hip_fail(hipError_t e, const char *what);
perm_tuning default_tuning();
bool tuning_valid(const perm_tuning &t);
// The tuning class of a host call of `count` matrices whose first order is n0.
int tune_class_host(int32_t count, int32_t n0);

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf();
    hipError_t reserve(size_t n);
};

struct HostBuf {   // pinned host memory
    void *p = nullptr;
    size_t cap = 0;
    unsigned flags = hipHostMallocDefault;
    HostBuf() = default;
    explicit HostBuf(unsigned f) : flags(f) {}
    HostBuf(const HostBuf &) = delete;
    HostBuf &operator=(const HostBuf &) = delete;
    ~HostBuf();
    hipError_t reserve(size_t n);
};

// Device work buffers of one call: plan records, packed rows, tallies,
// completion counts, status, the queue counters, and the accumulator words of
// one-launch small calls (SMALL_PLAN_MAX of them, zero between calls).
struct WorkSet {
    MatMeta *meta = nullptr;
    int32_t *order = nullptr;
    uint64_t *task_start = nullptr;   // count + 1
    int64_t *tally = nullptr;
    uint64_t *done = nullptr;
    uint8_t *status = nullptr;
    uint64_t *counters = nullptr;     // CNT_COUNT
    RowW *rows = nullptr;
    uint64_t *acc = nullptr;          // SMALL_PLAN_MAX
};

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// The pieces of a work set, in order, each 256-byte aligned; off[9] is the total.
struct WorkSetLayout {
    size_t off[10];
};

constexpr WorkSetLayout workset_layout(int32_t count, int64_t rows, bool acc)
{
    const size_t c = (size_t)(count > 1 ? count : 1);
    const size_t r = (size_t)(rows > 1 ? rows : 1);
    const size_t sz[9] = {c * sizeof(MatMeta), c * sizeof(int32_t), (c + 1) * sizeof(uint64_t),
                          c * sizeof(int64_t), c * sizeof(uint64_t), c, CNT_COUNT * sizeof(uint64_t),
                          r * sizeof(RowW), acc ? SMALL_PLAN_MAX * sizeof(uint64_t) : 0};
    WorkSetLayout L{};
    L.off[0] = 0;
    for (int i = 0; i < 9; ++i) L.off[i + 1] = L.off[i] + align256(sz[i]);
    return L;
}

// Bytes of a work set for `count` matrices and `rows` rows in all (with the
// accumulator words when `acc`), and its buffers carved from one block of at
// least that many bytes (256-byte aligned pieces).
size_t workset_bytes(int32_t count, int64_t rows, bool acc);
WorkSet workset_carve(void *base, int32_t count, int64_t rows, bool acc);

// One device launch sequence: plan -> pack -> walk.
struct Launch {
    int32_t pack_kind;            // 0: byte matrices, 1: uint64 planes
    const uint8_t *mats_dev;
    const int64_t *offs_dev;
    const uint64_t *planes_dev;
    const int64_t *row_off_dev;
    const int32_t *ns_dev;
    int32_t count;
    uint8_t *out_dev;
    uint64_t *hist_dev;
    int32_t use_range;
    uint64_t range_lo, range_hi;
    int32_t fused_only;           // the caller knows the call is walked by k_small alone
    int32_t small_blocks;         // k_small's grid when the caller knows the work (0: the full grid)
    int32_t zero_acc;             // clear the accumulator words first (a set not known to hold zeros)
    int32_t cls;                  // tuning class (PERM_TUNE_*)
    int32_t defer;                // the walk re-walks candidate blocks one lane each (batches)
};

using GraphKey = std::tuple<int, uintptr_t, uintptr_t, uintptr_t, uintptr_t, uintptr_t, uintptr_t, int, int>;

struct Context {
    int device = 0;
    int cus = 0;
    int clock_khz = 0;
    char arch[64] = {0};
    perm_tuning tunings[PERM_TUNE_CLASSES]{};
    int32_t tune_src[PERM_TUNE_CLASSES]{};
    hipStream_t stream = nullptr;
    std::mutex mu;

    DevBuf work;                     // the shared work set (grown on demand)
    DevBuf d_stage, d_census, d_gen, d_wide;
    DevBuf small_acc;                // its accumulator words: SMALL_PLAN_MAX, zero between calls
    WorkSet ws{};
    int32_t ws_count = 0;
    int64_t ws_rows = 0;
    std::vector<std::unique_ptr<DevBuf>> captured;   // work sets of calls captured into callers' graphs
    void *noalloc_scratch = nullptr;   // this device's address of the allocation-free calls' work set
    HostBuf h_stage, h_wide;
    HostBuf h_out;                   // host-call results, written by the kernels directly
    HostBuf h_zc{hipHostMallocCoherent};   // small host calls' inputs, read by the kernel directly

    std::map<GraphKey, hipGraphExec_t> graphs;
    hipEvent_t ev_walk0 = nullptr, ev_walk1 = nullptr, ev_all0 = nullptr, ev_all1 = nullptr;
    hipEvent_t ev_done = nullptr, ev_in = nullptr, ev_out = nullptr;
    hipStream_t last_stream = nullptr;   // stream of the last call (valid when have_last)
    bool have_last = false;
    bool last_timing_valid = false;
    int last_launches = 0;
    int last_graph = 0;

    ~Context();
    const perm_tuning &tn(int cls) const { return tunings[cls]; }
    void set_tuning(int cls, const perm_tuning &t, int32_t src);
    void drop_graphs();
    int32_t reserve_work(int32_t count, int64_t rows);
    int32_t join(hipStream_t st);
    int32_t mark(hipStream_t st);
    PlanArgs plan_args(const WorkSet &w, const perm_tuning &tn, const int32_t *ns_dev, int32_t count,
                       uint8_t *out_dev, uint64_t *hist_dev) const;
    WalkArgs walk_args(const WorkSet &w, int32_t count, uint8_t *out_dev, uint64_t *hist_dev) const;
    int grid_blocks(const perm_tuning &tn) const;
    int32_t enqueue(const Launch &L, const WorkSet &w, const perm_tuning &tn, hipStream_t st, bool timed);
    int32_t run_captured(const Launch &L, hipStream_t st);
    int32_t run(const Launch &L, hipStream_t st, bool use_graph);
    int32_t run_dev(const Launch &L, hipStream_t user);
    int32_t run_host(const uint8_t *const *As, const int32_t *ns, int32_t count, bool use_range, uint64_t lo,
                     uint64_t hi, uint8_t *out_host, int64_t *tally_host);
    int32_t timing(perm_timing *t);
};

int32_t get_context(Context **out);

// Tuning cache (perm3_tuning.hip): apply the lines of a cache file that match
// the context's device (returns the classes set, or -1 if the file cannot be
// read), and the load made when a context is created.
int cache_apply(Context &c, const char *path);

// The device address of the allocation-free calls' static work set on the
// context's device (perm3_noalloc.hip), looked up once when the context is made.
int32_t noalloc_init(Context &c);
void load_default_cache(Context &c);
extern const char *const TUNE_CLASS_NAMES[PERM_TUNE_CLASSES];
bool timing_enabled();   // perm_timing_enable() state of the calling thread

}  // namespace perm3
