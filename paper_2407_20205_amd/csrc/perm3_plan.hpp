// Planning of Gray-index work: chunk lengths, task counts and the one-launch
// decision of small calls.  Pure functions of the orders and the tuning,
// shared by the plan kernels and the host runtime, and free of HIP so that a
// CPU build of the walk can include them too.
//
// The Gray range [lo, hi) of a matrix (normally [0, 2^n), Section 3) is cut
// into aligned chunks of 2^m indices, one per lane, 64 lanes to a task; each
// chunk is started by jumping to its first Gray state (Section 3.1).
#pragma once

#include <stdint.h>

#ifndef PERM3_HD
#if defined(__HIPCC__)
#define PERM3_HD __host__ __device__
#else
#define PERM3_HD
#endif
#endif

namespace perm3 {

enum WalkMode : int32_t {
    MODE_FAST = 0,     // fast walk over whole chunks in blocks of 16, candidate blocks re-walked
    MODE_DIRECT = 1,   // every index tested exactly (small n)
    MODE_NONE = 2,     // no tasks: n == 0, invalid n, or an empty range
};

// Per-matrix plan, written by the plan kernel.
struct MatMeta {
    int32_t n;
    int32_t m;          // log2 of the per-lane chunk length
    int32_t mode;       // WalkMode
    int32_t ul;         // body_log of the matrix's class (4, 5 or 6): chunks of 2^(ul+1) or more
    uint64_t ntasks;    // 64 * S chunks per task
    int64_t row_base;   // first RowW of this matrix
    uint64_t lo, hi;    // Gray index range [lo, hi)
    uint64_t c_first;   // first chunk index (lo >> m)
};

// Serving: one tick visits an explicit list of tasks over device-resident slots.
struct TickTask {
    int32_t slot;
    int32_t m;            // chunk log
    int32_t mode;         // WalkMode (FAST or DIRECT)
    int32_t nchunks;      // valid chunks in this task (1..64)
    uint64_t c_first;     // first chunk of this task
    int32_t ul;           // body_log of the class: chunks of 2^(ul+1) or more
    int32_t pad;
};

// counters[] slots
enum : int { CNT_QUEUE = 0, CNT_TOTAL_TASKS = 1, CNT_COUNT = 4 };

constexpr int SMALL_PLAN_MAX = 64;                  // calls of up to this many matrices are planned (and packed) by k_small
constexpr uint64_t SMALL_FUSED_WORK = 1ull << 28;   // ... and are walked in the same launch up to this many indices

struct RowW;

struct PlanArgs {
    const int32_t *ns;
    int32_t count;
    int32_t use_range;            // 1: matrix 0 walks [range_lo, range_hi) only (count == 1)
    uint64_t range_lo, range_hi;
    int32_t body_log, chunk_log_max, direct_max_n, direct_chunk_log_max;
    int32_t body_log_mid, mid_max_n;  // body_log for direct_max_n < n <= mid_max_n
    int32_t states_log;           // log2 of the chunks a lane walks per task
    int32_t max_tasks_log;        // at most 2^max_tasks_log tasks per matrix ...
    int32_t min_task_log;         // ... unless tasks would exceed 2^min_task_log indices
    int32_t queue_task_log;       // floor of a task, once every wave has one that long (0: none)
    int32_t waves_total, tasks_per_wave;
    MatMeta *meta;
    int32_t *order;               // [count] matrix index by decreasing n
    uint64_t *task_start;         // [count + 1] first task of order[p]
    int64_t *tally;               // [count]
    uint64_t *done;               // [count]
    uint8_t *status;              // [count] 0 ok, 1 invalid
    uint64_t *counters;           // [CNT_COUNT]
    uint8_t *out;                 // [count]
    uint64_t *hist;               // [64 * 3] or null
};

PERM3_HD inline void range_of(const PlanArgs &a, int n, uint64_t &lo, uint64_t &hi)
{
    if (a.use_range) {
        lo = a.range_lo;
        hi = a.range_hi;
    } else {
        lo = 0;
        hi = 1ull << n;
    }
}

// Chunk log that gives each persistent wave about tasks_per_wave tasks of the
// whole call's work, but tasks of at least 2^queue_task_log indices while that
// still gives every wave a task (else one task per wave): every task after a
// wave's first costs one atomic on the call's queue counter, and atomics on
// one address serialise, so short tasks in large numbers would wait on it.
PERM3_HD inline int target_chunk_log(const PlanArgs &a, double total_work)
{
    const double waves = (double)(a.waves_total > 0 ? a.waves_total : 1);
    const double want_tasks = waves * (double)(a.tasks_per_wave > 0 ? a.tasks_per_wave : 1);
    double per_task = total_work / want_tasks;
    if (a.queue_task_log > 0) {
        const double floor_task = (double)(1ull << a.queue_task_log);
        const double one_each = total_work / waves;
        const double lo = floor_task < one_each ? floor_task : one_each;
        if (per_task < lo) per_task = lo;
    }
    if (per_task < 128.0) return 0;
    return (63 - __builtin_clzll((uint64_t)per_task)) - 6 - a.states_log;
}

// The plan of a matrix of order n (invalid outside 0..63): its mode, chunk
// log, block log, Gray range and task count; row_base is filled in later.
// Pure: reads and writes no memory.
PERM3_HD inline MatMeta plan_pure(const PlanArgs &a, int n, int target_m)
{
    const bool valid = n >= 0 && n <= 63;
    MatMeta mt;
    mt.n = valid ? n : 0;
    mt.m = 0;
    mt.mode = MODE_NONE;
    mt.ntasks = 0;
    mt.row_base = 0;
    mt.lo = 0;
    mt.hi = 0;
    mt.c_first = 0;
    mt.ul = a.body_log;
    if (!valid || n == 0) return mt;
    uint64_t lo, hi;
    range_of(a, n, lo, hi);
    mt.lo = lo;
    mt.hi = hi;
    const int slog = a.states_log;
    const int ul = n <= a.mid_max_n ? a.body_log_mid : a.body_log;
    mt.ul = ul;
    const bool fast_ok = n >= ul + 7 + slog && n > a.direct_max_n;
    int m;
    if (fast_ok) {
        // a lane's int32 tally covers S chunks and a wave sums 64 lanes: S * 2^m <= 2^24
        int mmax = a.chunk_log_max < n - 6 - slog ? a.chunk_log_max : n - 6 - slog;
        if (mmax > 24 - slog) mmax = 24 - slog;
        // at most 2^max_tasks_log tasks for this matrix, and at most about
        // 2^(n/2) for a small one (a task's fixed cost, its seed and its
        // cold start, then outweighs the walk it shares out), unless its
        // tasks would then exceed 2^min_task_log indices: every task ends
        // with an atomic on the matrix's counters, and those serialise
        const int tasks_log = (n - 3) / 2 < a.max_tasks_log ? (n - 3) / 2 : a.max_tasks_log;
        const int fewer = n - 6 - slog - tasks_log;
        const int longest = a.min_task_log - 6 - slog;
        const int mfloor = fewer < longest ? fewer : longest;
        m = target_m > mfloor ? target_m : mfloor;
        if (m > mmax) m = mmax;
        if (m < ul + 1) m = ul + 1;
        mt.mode = MODE_FAST;
    } else {
        m = n - 6;
        if (m > a.direct_chunk_log_max) m = a.direct_chunk_log_max;
        if (m < 0) m = 0;
        mt.mode = MODE_DIRECT;
    }
    mt.m = m;
    if (hi > lo) {
        const uint64_t c0 = lo >> m;
        const uint64_t c1 = (hi - 1) >> m;
        mt.c_first = c0;
        const uint64_t per_task = 64ull << a.states_log;
        mt.ntasks = (c1 - c0 + per_task) / per_task;
    } else {
        mt.mode = MODE_NONE;
    }
    return mt;
}

// Sum of 2^n over the valid orders (0..63) of a call, stopping as soon as it
// passes `cap`: then cap + 1 is returned.  Two orders of 63 add up to 2^64,
// which a plain 64-bit sum would wrap to 0.  The one-launch kernel makes the
// same decision in double precision, where such a sum cannot wrap; below
// 64 * 2^28 every partial sum is exact there.
inline uint64_t capped_work(const int32_t *ns, int32_t count, uint64_t cap)
{
    uint64_t w = 0;
    for (int32_t k = 0; k < count; ++k) {
        const int32_t n = ns[k];
        if (n < 0 || n > 63) continue;
        const uint64_t add = 1ull << n;
        if (add > cap - w) return cap + 1;
        w += add;
    }
    return w;
}

// Whether a call of these orders over whole Gray ranges is walked entirely by
// the one-launch kernel: at most SMALL_PLAN_MAX matrices and SMALL_FUSED_WORK
// Gray indices in all.
inline bool small_call_fused(const int32_t *ns, int32_t count, bool use_range)
{
    return count >= 1 && count <= SMALL_PLAN_MAX && !use_range &&
           capped_work(ns, count, SMALL_FUSED_WORK) <= SMALL_FUSED_WORK;
}

// The tasks the one-launch walk makes of these orders: the same plan (one
// chunk per lane), run on the host so that a caller who knows the orders can
// size the grid to the work.
inline uint64_t small_call_tasks(const PlanArgs &a, const int32_t *ns, int32_t count)
{
    PlanArgs pf = a;
    pf.states_log = 0;
    double total_work = 0.0;
    for (int32_t k = 0; k < count; ++k) {
        if (ns[k] < 0 || ns[k] > 63) continue;
        uint64_t lo, hi;
        range_of(pf, ns[k], lo, hi);
        total_work += (double)(hi - lo);
    }
    const int target_m = target_chunk_log(pf, total_work);
    uint64_t tasks = 0;
    for (int32_t k = 0; k < count; ++k) tasks += plan_pure(pf, ns[k], target_m).ntasks;
    return tasks;
}

}  // namespace perm3
