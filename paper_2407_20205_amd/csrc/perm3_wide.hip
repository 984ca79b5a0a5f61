// Matrices of up to 128 columns: Gray ranges with 128-bit indices (gfx950).
//
// Section 3 keeps a row in one unsigned word per plane and notes that a
// second word would be needed past 64 columns.  Here a row is four 32-bit
// words per plane (RowX), but the walk still carries only the low word of the
// running subset sum: the zero-mask test on columns 0..31 rejects all but a
// (2/3)^32 fraction of indices, and only those have their other words formed
// from scratch (exact_term on MasksX).  So an index costs what it costs at
// n = 36, whatever the width.
//
//   k_pack_wide  phi of Section 2 over up to 128 columns, columns ordered so
//                that the low word makes a good filter; clears the range's
//                tally and task counter.
//   k_walk_wide  persistent waves over 64-chunk tasks of one range; whole
//                chunks take the fast walk, ragged ends (and small n)
//                a walk that tests every index.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>

#include "perm3.h"
#include "perm3_device.hpp"
#include "perm3_internal.h"
#include "perm3_runtime.h"
#include "perm3_walk.hpp"

namespace perm3 {

// phi on one row per thread, with the columns reordered.  T(a, b) does not
// depend on the order of the columns (each term is a product over all of
// them), so the low 32-bit word, the only one the walk carries, is given the
// columns most likely to be zero: those with the most non-zero entries among
// the first vrows rows, the rows whose Gray bit varies over the range.  A
// column with none there has the same sum at every index of the range and
// can never reject one; such columns go last.  For a uniform matrix the order
// hardly matters; for a matrix with fixed rows (a block whose rows are in
// every subset of the range) it decides how often the low word passes.
__global__ void __launch_bounds__(128) k_pack_wide(const uint8_t *A, int n, int vrows, RowX *rows,
                                                   uint64_t *queue, int64_t *tally)
{
    __shared__ int s_cnt[WIDE_MAX_N];
    __shared__ int s_pos[WIDE_MAX_N];
    const int t = threadIdx.x;
    if (t == 0) {
        *queue = 0;
        *tally = 0;
    }
    if (t < n) {
        int c = 0;
        for (int r = 0; r < vrows; ++r) c += A[r * n + t] != 0;
        s_cnt[t] = c;
    }
    __syncthreads();
    if (t < n) {
        // the column's bit: its rank by decreasing count, ties by column index
        const int c = s_cnt[t];
        int pos = 0;
        for (int j = 0; j < n; ++j) pos += (s_cnt[j] > c) || (s_cnt[j] == c && j < t);
        s_pos[t] = pos;
    }
    __syncthreads();
    if (t >= n) return;
    const int r = t;
    uint64_t mag[2] = {0, 0}, sgn[2] = {0, 0};
    for (int j = 0; j < n; ++j) {
        const uint8_t v = A[r * n + j];
        const int p = s_pos[j];
        const uint64_t bit = 1ull << (p & 63);
        if (v != 0) mag[p >> 6] |= bit;
        if (v == 2) sgn[p >> 6] |= bit;
    }
    RowX x;
    x.m_lo = (uint32_t)mag[0];
    x.s_lo = (uint32_t)sgn[0];
    x.sn_lo = (uint32_t)(sgn[0] ^ mag[0]);
    x.pad0 = 0;
    x.m_w[0] = (uint32_t)(mag[0] >> 32);
    x.m_w[1] = (uint32_t)mag[1];
    x.m_w[2] = (uint32_t)(mag[1] >> 32);
    x.pad1 = 0;
    x.s_w[0] = (uint32_t)(sgn[0] >> 32);
    x.s_w[1] = (uint32_t)sgn[1];
    x.s_w[2] = (uint32_t)(sgn[1] >> 32);
    x.pad2 = 0;
    rows[r] = x;
}

__device__ __forceinline__ int walk_task_wide(cptr<RowX> R, const WideArgs &a, const MasksX &mk, uint64_t cr)
{
    LowSums<WALK_UL> lr;
    const bool fast = a.mode == MODE_FAST;
    if (fast) load_low_sums<WALK_UL>(R, lr);
    const u128 c0 = ((u128)a.c0_hi << 64) | (u128)a.c0_lo;
    // candidate blocks noted and re-walked one lane each after the chunk, and
    // each block's closing row read a block ahead
    return walk_lane_wide<WALK_UL, true, true>(R, a.n, a.m, fast, c0, a.off_lo, a.off_hi, cr, mk, lr);
}

__global__ void __launch_bounds__(WALK_BLOCK) k_walk_wide(WideArgs a)
{
    const int lane = threadIdx.x & 63;
    const uint32_t nwaves = gridDim.x * (WALK_BLOCK / 64);
    const cptr<RowX> R = to_const(a.rows);
    const MasksX mk = masks_wide(a.n);
    for (uint64_t tau = wave_index(); tau < a.ntasks; tau = next_task64(a.queue, nwaves, lane)) {
        const uint64_t cr = tau * 64u + (uint64_t)lane;
        const int tally = walk_task_wide(R, a, mk, cr);
        const int sum = wave_sum(tally);
        if (lane == 0 && sum != 0) atomicAdd((unsigned long long *)a.tally, (unsigned long long)(long long)sum);
    }
}

hipError_t launch_pack_wide(const uint8_t *A, int n, int vrows, RowX *rows, uint64_t *queue, int64_t *tally,
                            hipStream_t st)
{
    if (n < 1 || n > WIDE_MAX_N || vrows < 0 || vrows > n) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pack_wide, dim3(1), dim3(128), 0, st, A, n, vrows, rows, queue, tally);
    return hipGetLastError();
}

int wide_resident_per_cu()
{
    static std::atomic<int> cache{0};
    int n = cache.load(std::memory_order_relaxed);
    if (n > 0) return n;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_walk_wide, WALK_BLOCK, 0) != hipSuccess || n < 1) n = 1;
    cache.store(n, std::memory_order_relaxed);
    return n;
}

hipError_t launch_walk_wide(const WideArgs &a, int grid_blocks, hipStream_t st)
{
    if (a.n < 1 || a.n > WIDE_MAX_N || a.m < 0 || a.m > 24) return hipErrorInvalidValue;
    if (a.mode == MODE_FAST && (a.m <= a.ul || a.m > a.n - 6)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_walk_wide, dim3(grid_blocks), dim3(WALK_BLOCK), 0, st, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------ host plan

// Chunk length and task count of the range [begin, begin + count), count >= 1.
WideArgs plan_wide(const perm_tuning &tn, int waves_total, int n, u128 begin, uint64_t count)
{
    WideArgs a;
    memset(&a, 0, sizeof a);
    a.n = n;
    a.ul = n <= tn.mid_max_n ? tn.body_log_mid : tn.body_log;
    int m;
    if (n >= a.ul + 7 && n > tn.direct_max_n) {
        // about tasks_per_wave tasks of 64 chunks per persistent wave
        const double per_task = (double)count / ((double)waves_total * (double)tn.tasks_per_wave);
        int target = 0;
        if (per_task >= 128.0) target = (63 - __builtin_clzll((uint64_t)per_task)) - 6;
        const int mmax = std::min(std::min(tn.chunk_log_max, n - 6), 24);
        // at most 2^max_tasks_log tasks unless they would exceed 2^min_task_log indices
        const int count_log = count > 1 ? 64 - __builtin_clzll(count - 1) : 0;   // ceil(log2 count)
        const int fewer = count_log - 6 - tn.max_tasks_log;
        const int mfloor = std::min(fewer, tn.min_task_log - 6);
        m = std::max(std::min(std::max(target, mfloor), mmax), a.ul + 1);
        a.mode = MODE_FAST;
    } else {
        m = std::max(std::min(n - 6, 10), 0);
        a.mode = MODE_DIRECT;
    }
    a.m = m;
    const u128 c0 = begin >> m;
    const u128 base = c0 << m;
    a.c0_lo = (uint64_t)c0;
    a.c0_hi = (uint64_t)(c0 >> 64);
    a.off_lo = (uint64_t)(begin - base);
    a.off_hi = a.off_lo + count;
    const uint64_t nchunks = ((a.off_hi - 1) >> m) + 1;
    a.ntasks = (nchunks + 63) / 64;
    return a;
}

}  // namespace perm3

using namespace perm3;

#define WIDE_TRY(expr)                                        \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return hip_fail(_e, #expr);     \
    } while (0)

extern "C" int32_t perm_mod3_range_tally_wide(const uint8_t *A, int32_t n, uint64_t begin_hi, uint64_t begin_lo,
                                              uint64_t count, int64_t *tally)
{
    set_error_index(-1);
    if (!tally) return set_error(PERM_EINVAL, "null tally pointer");
    if (n < 1 || n > PERM_MAX_N_WIDE) return set_error(PERM_EINVAL, "n = %d is outside [1, %d]", n, PERM_MAX_N_WIDE);
    if (!A) return set_error(PERM_EINVAL, "null matrix pointer");
    const int64_t cells = (int64_t)n * n;
    for (int64_t i = 0; i < cells; ++i)
        if (A[i] > 2) {
            set_error_index(i);
            return set_error(PERM_EDOMAIN, "entry %lld is %u; entries must be 0, 1 or 2", (long long)i,
                             (unsigned)A[i]);
        }
    if (count > PERM_WIDE_MAX_COUNT)
        return set_error(PERM_EINVAL, "count = %llu exceeds 2^62", (unsigned long long)count);
    const u128 begin = ((u128)begin_hi << 64) | (u128)begin_lo;
    // begin + count <= 2^n, written so that 2^128 is never formed
    const bool in_range = n == 128 ? (count == 0 || begin <= (u128)0 - (u128)count)
                                   : (begin <= ((u128)1 << n) && (u128)count <= ((u128)1 << n) - begin);
    if (!in_range) return set_error(PERM_EINVAL, "range [begin, begin + %llu) is not inside [0, 2^%d]",
                                    (unsigned long long)count, n);
    *tally = 0;
    if (count == 0) return PERM_OK;

    Context *c = nullptr;
    int32_t rc = get_context(&c);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(c->mu);
    const size_t mat_bytes = (size_t)cells;
    const size_t rows_at = ((mat_bytes + 255) / 256) * 256;
    const size_t tally_at = rows_at + (size_t)WIDE_MAX_N * sizeof(RowX);
    const size_t queue_at = tally_at + 64;
    // pinned staging: the matrix, then the returned tally
    const size_t h_tally_at = ((mat_bytes + 7) / 8) * 8;
    WIDE_TRY(c->d_wide.reserve(queue_at + 64));
    WIDE_TRY(c->h_wide.reserve(h_tally_at + sizeof(int64_t)));
    uint8_t *d = (uint8_t *)c->d_wide.p;
    uint8_t *h = (uint8_t *)c->h_wide.p;
    int64_t *h_tally = (int64_t *)(h + h_tally_at);
    memcpy(h, A, mat_bytes);

    const uint64_t resident = (uint64_t)c->cus * (uint64_t)std::min(c->tn(PERM_TUNE_LARGE).waves_per_simd, wide_resident_per_cu());
    WideArgs a = plan_wide(c->tn(PERM_TUNE_LARGE), (int)(4 * resident), n, begin, count);
    a.rows = (const RowX *)(d + rows_at);
    a.tally = (int64_t *)(d + tally_at);
    a.queue = (uint64_t *)(d + queue_at);
    const hipStream_t st = c->stream;
    if ((rc = c->join(st))) return rc;
    const bool timed = timing_enabled();
    if (timed) WIDE_TRY(hipEventRecord(c->ev_all0, st));
    WIDE_TRY(hipMemcpyAsync(d, h, mat_bytes, hipMemcpyHostToDevice, st));
    // rows whose Gray bit varies over the range: bits below the highest bit in
    // which the first and last index differ
    const u128 diff = begin ^ (begin + (count - 1));
    const uint64_t dh = (uint64_t)(diff >> 64), dl = (uint64_t)diff;
    const int varying = dh ? 128 - __builtin_clzll(dh) : (dl ? 64 - __builtin_clzll(dl) : 0);
    WIDE_TRY(launch_pack_wide(d, n, std::min(varying, n), (RowX *)(d + rows_at), a.queue, a.tally, st));
    if (timed) WIDE_TRY(hipEventRecord(c->ev_walk0, st));
    const uint64_t want_blocks = (a.ntasks + 3) / 4;
    const int blocks = (int)std::max<uint64_t>(1, std::min<uint64_t>(want_blocks, resident));
    WIDE_TRY(launch_walk_wide(a, blocks, st));
    if (timed) WIDE_TRY(hipEventRecord(c->ev_walk1, st));
    WIDE_TRY(hipMemcpyAsync(h_tally, a.tally, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    if (timed) WIDE_TRY(hipEventRecord(c->ev_all1, st));
    WIDE_TRY(hipStreamSynchronize(st));
    c->last_timing_valid = timed;
    c->last_launches = 2;
    c->last_graph = 0;
    *tally = *h_tally;
    return c->mark(st);
}
