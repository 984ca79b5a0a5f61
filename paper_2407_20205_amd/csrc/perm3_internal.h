// Internal declarations shared by the kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "perm3_plan.hpp"

namespace perm3 {

struct RowW;

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

// Per-matrix accumulator words of one-launch small calls (completed tasks
// and biased tally in one uint64 each): zero between calls.
struct SmallAcc {
    uint64_t *word;     // SMALL_PLAN_MAX entries
};
hipError_t launch_small(const PlanArgs &a, const PackU8Args &pk, const PackPlanesArgs &pp, const SmallAcc &acc,
                        int kind, bool allow_fused, int blocks, hipStream_t st);
hipError_t launch_pack_u8(const PackU8Args &a, hipStream_t st);
hipError_t launch_pack_planes(const PackPlanesArgs &a, hipStream_t st);
// defer: candidate blocks re-walked one lane each after a chunk (batches), else at once
hipError_t launch_walk(const WalkArgs &a, int states, bool defer, int grid_blocks, hipStream_t st);
hipError_t launch_tick(const TickArgs &a, int grid_blocks, hipStream_t st);
int walk_resident_per_cu(int states);   // k_walk<states> workgroups per CU at once; 0: k_tick
hipError_t launch_finish(const FinishArgs &a, int max_fin, hipStream_t st);
hipError_t launch_slot_pack(const uint8_t *A, int n, RowW *dst, hipStream_t st);
hipError_t launch_finish_tallies(const int64_t *t, int32_t count, int32_t n, uint8_t *out, hipStream_t st);
hipError_t launch_fill_u64(uint64_t *p, int64_t count, uint64_t value, hipStream_t st);
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

hipError_t launch_census_lanes(const CensusArgs &a, int cus, hipStream_t st);
hipError_t launch_generate(const GenArgs &a, hipStream_t st);

}  // namespace perm3
