// Internal declarations shared by the kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace perm3 {

struct RowW;

enum WalkMode : int32_t {
    MODE_FAST = 0,     // unrolled fast walk over whole chunks, exact replay of candidate blocks
    MODE_DIRECT = 1,   // every index tested exactly (small n)
    MODE_NONE = 2,     // no tasks: n == 0, invalid n, or an empty range
};

// Per-matrix plan, written by the plan kernel.
struct MatMeta {
    int32_t n;
    int32_t m;          // log2 of the per-lane chunk length
    int32_t mode;       // WalkMode
    int32_t ul;         // log2 of the unrolled block (4, 5 or 6)
    uint64_t ntasks;    // 64 * S chunks per task
    int64_t row_base;   // first RowW of this matrix
    uint64_t lo, hi;    // Gray index range [lo, hi)
    uint64_t c_first;   // first chunk index (lo >> m)
};

// counters[] slots
enum : int { CNT_QUEUE = 0, CNT_TOTAL_TASKS = 1, CNT_COUNT = 4 };

struct PlanArgs {
    const int32_t *ns;
    int32_t count;
    int32_t use_range;            // 1: matrix 0 walks [range_lo, range_hi) only (count == 1)
    uint64_t range_lo, range_hi;
    int32_t body_log, chunk_log_max, direct_max_n, direct_chunk_log_max;
    int32_t body_log_mid, mid_max_n;  // block length for direct_max_n < n <= mid_max_n
    int32_t states_log;           // log2 of the chunks a lane carries side by side
    int32_t max_tasks_log;        // at most 2^max_tasks_log tasks per matrix ...
    int32_t min_task_log;         // ... unless tasks would exceed 2^min_task_log indices
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

struct PackU8Args {
    const uint8_t *mats;
    const int64_t *offs;          // byte offset of each matrix
    const MatMeta *meta;
    int32_t count;
    RowW *rows;
    uint8_t *status;
};

struct PackPlanesArgs {
    const uint64_t *planes;       // {mag, sgn} per row
    const int64_t *row_off;       // first row of each matrix
    const MatMeta *meta;
    int32_t count;
    RowW *rows;
    uint8_t *status;
};

struct WalkArgs {
    const RowW *rows;
    const MatMeta *meta;
    const int32_t *order;
    const uint64_t *task_start;
    int32_t count;
    int64_t *tally;
    uint64_t *done;
    const uint8_t *status;
    uint64_t *counters;
    uint8_t *out;
    uint64_t *hist;
};

// Serving: one tick visits an explicit list of tasks over device-resident slots.
struct TickTask {
    int32_t slot;
    int32_t m;            // chunk log
    int32_t mode;         // WalkMode (FAST or DIRECT)
    int32_t nchunks;      // valid chunks in this task (1..64)
    uint64_t c_first;     // first chunk of this task
    int32_t ul;           // log2 of the unrolled block
    int32_t pad;
};

struct SlotInfo {
    int32_t n;
    int32_t pad;
    int64_t row_base;
};

struct TickArgs {
    const RowW *rows;
    const SlotInfo *slots;
    const TickTask *tasks;
    const uint32_t *ntasks;       // device count of tasks in this tick
    int64_t *tally;               // [max_slots]
    uint32_t *queue;              // tick work counter, reset by the finish kernel
};

struct FinishArgs {
    const int32_t *fin_slots;     // slots that complete in this tick
    const uint32_t *nfin;
    const SlotInfo *slots;
    int64_t *tally;               // read, then cleared for reuse
    uint8_t *fin_out;             // result per finishing slot
    uint32_t *queue;              // cleared for the next tick
};

hipError_t launch_plan(const PlanArgs &a, hipStream_t st);
constexpr int SMALL_PLAN_MAX = 64;   // calls of up to this many matrices are planned (and packed) by k_small
constexpr uint64_t SMALL_FUSED_WORK = 1ull << 28;   // ... and are walked in the same launch up to this many indices

// Per-matrix accumulator words of one-launch small calls (completed tasks
// and biased tally in one uint64 each): zero between calls.
struct SmallAcc {
    uint64_t *word;     // SMALL_PLAN_MAX entries
};
hipError_t launch_small(const PlanArgs &a, const PackU8Args &pk, const PackPlanesArgs &pp, const SmallAcc &acc,
                        int kind, bool allow_fused, int blocks, hipStream_t st);
uint64_t small_call_tasks(const PlanArgs &a, const int32_t *ns, int32_t count);
hipError_t launch_pack_u8(const PackU8Args &a, hipStream_t st);
hipError_t launch_pack_planes(const PackPlanesArgs &a, hipStream_t st);
hipError_t launch_walk(const WalkArgs &a, int states, int grid_blocks, hipStream_t st);
hipError_t launch_tick(const TickArgs &a, int grid_blocks, hipStream_t st);
int walk_resident_per_cu(int states);   // k_walk<states> workgroups per CU at once; 0: k_tick
hipError_t launch_finish(const FinishArgs &a, int max_fin, hipStream_t st);
hipError_t launch_slot_pack(const uint8_t *A, int n, RowW *dst, hipStream_t st);
hipError_t launch_bipedal_ops(const uint32_t *in, int count, uint32_t *out, hipStream_t st);

constexpr int WALK_BLOCK = 256;   // 4 waves, one per SIMD

// Matrices of up to 128 columns: one Gray range of one matrix with 128-bit
// indices.  The range [B + off_lo, B + off_hi) is held relative to the
// chunk-aligned base B = c0 * 2^m, so every offset fits in 64 bits even when
// the range ends at 2^128.
struct RowX;

struct WideArgs {
    const RowX *rows;             // [n]
    int32_t n, m, mode, ul;       // chunk log m, WalkMode, block log
    uint64_t c0_lo, c0_hi;        // first chunk index c0 (128-bit)
    uint64_t off_lo, off_hi;      // the range, relative to B
    uint64_t ntasks;              // 64 chunks per task
    uint64_t *queue;              // task counter, cleared by the pack kernel
    int64_t *tally;               // the range's T, cleared by the pack kernel
};

constexpr int WIDE_MAX_N = 128;

hipError_t launch_pack_wide(const uint8_t *A, int n, int vrows, RowX *rows, uint64_t *queue, int64_t *tally,
                            hipStream_t st);
hipError_t launch_walk_wide(const WideArgs &a, int grid_blocks, hipStream_t st);
int wide_resident_per_cu();             // k_walk_wide workgroups per CU at once

}  // namespace perm3

namespace perm3 {

// Matrices generated on the device for a census (perm_mod3_census).
enum CensusGen : int32_t { GEN_ENUMERATE = 0, GEN_SPLITMIX = 1 };

struct CensusArgs {
    int32_t n;
    int32_t gen;
    uint64_t key;
    uint64_t first;                 // first matrix index
    uint64_t count;                 // matrices
    unsigned long long *counts;     // [3] perm = 0, 1, 2 (added to)
};

struct GenArgs {                    // write matrices first .. first+count-1 as bytes
    int32_t n;
    int32_t gen;
    uint64_t key;
    uint64_t first;
    uint32_t count;
    uint8_t *mats;                  // count * n * n bytes
    int64_t *offs;                  // [count]
    int32_t *ns;                    // [count]
};

constexpr int CENSUS_LANE_MAX_N = 20;   // one matrix per lane up to this n

hipError_t launch_census_lanes(const CensusArgs &a, int grid_blocks, hipStream_t st);
hipError_t launch_generate(const GenArgs &a, hipStream_t st);

}  // namespace perm3
