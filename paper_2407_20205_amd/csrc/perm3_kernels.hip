// gfx950 kernels for perm(A) mod 3 by the bipedal Gray-code Ryser sum.
//
//   k_plan        one workgroup: per-matrix chunk size, task counts, the task
//                 order (largest n first), row offsets; clears counters.
//   k_pack_u8     phi of Section 2 on byte matrices, with validation.
//   k_pack_planes accepts caller-packed (mag, sgn) uint64 planes, validated.
//   k_walk<S>     persistent waves pull 64-chunk tasks from an atomic queue,
//                 walk them (perm3_walk.hpp), reduce each task's tally over the
//                 wavefront with DPP, add it to the matrix's int64 tally; the
//                 wave that completes a matrix's last task reduces it mod 3
//                 (Section 3: s times (-1)^n, then cmod3) and counts it in the
//                 per-n histogram.
//   k_tick        the serving form of k_walk over an explicit task list.
//   k_finish      serving: reduce finished slots' tallies mod 3.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>

#include "perm3_device.hpp"
#include "perm3_internal.h"
#include "perm3_walk.hpp"

namespace perm3 {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ Masks masks_for(int n)
{
    const uint64_t full = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
    Masks mk;
    mk.lo = (uint32_t)full;
    mk.hi = (uint32_t)(full >> 32);
    return mk;
}

// Walk one lane's chunk c (chunk length 2^m) clipped to [lo, hi): a whole
// chunk of a fast-mode matrix by walk_chunks_fast (DEFER and AHEAD choose its
// form), else every index tested exactly.
template <int UL, bool DEFER, bool AHEAD, typename RP>
__device__ __forceinline__ int walk_lane(RP R, int n, int m, int mode, uint64_t c,
                                         uint64_t lo, uint64_t hi, const LowSums<UL> &lr)
{
    const Masks mk = masks_for(n);
    const uint64_t a0 = c << m;
    const uint64_t e0 = a0 + (1ull << m);
    const uint64_t a = a0 > lo ? a0 : lo;
    const uint64_t e = e0 < hi ? e0 : hi;
    if (a >= e) return 0;
    if (a == a0 && e == e0) {
        if (mode == MODE_FAST) return walk_chunks_fast<UL, DEFER, AHEAD>(R, n, m, c, mk, lr);
        return n > 32 ? walk_chunk_direct<true>(R, n, m, c, mk) : walk_chunk_direct<false>(R, n, m, c, mk);
    }
    return n > 32 ? walk_range_direct<true>(R, n, a, e, mk) : walk_range_direct<false>(R, n, a, e, mk);
}

// ------------------------------------------------------------------ plan

template <typename T>
__device__ T block_incl_scan_1024(T v, T *sh, T &total)
{
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const T add = tid >= off ? sh[tid - off] : (T)0;
        __syncthreads();
        sh[tid] += add;
        __syncthreads();
    }
    total = sh[1023];
    const T r = sh[tid];
    __syncthreads();
    return r;
}

// The plan of matrix k with its side effects: clears the matrix's tally and
// completion count, sets its status (always for an invalid order, otherwise
// only with write_status: a packer running beside the plan owns it then), and
// writes the result of matrices that need no walk.
__device__ MatMeta plan_matrix(const PlanArgs &a, int k, int target_m, bool write_status)
{
    const int n = a.ns[k];
    const bool valid = n >= 0 && n <= 63;
    const MatMeta mt = plan_pure(a, n, target_m);
    a.tally[k] = 0;
    a.done[k] = 0;
    if (write_status || !valid) a.status[k] = valid ? 0 : 1;
    if (!valid) {
        a.out[k] = 0xFF;
    } else if (n == 0) {
        // the one subset (Gray index 0) is empty: its empty product makes
        // a term of +1, and perm of the 0 x 0 matrix is 1
        uint64_t lo, hi;
        range_of(a, 0, lo, hi);
        const long long T = lo < hi ? 1 : 0;
        a.tally[k] = T;
        const uint8_t r = finish_mod3(0, T);
        a.out[k] = r;
        if (a.hist) atomicAdd((unsigned long long *)&a.hist[r], 1ull);
    } else if (mt.mode == MODE_NONE) {
        a.out[k] = finish_mod3(n, 0);   // empty range
    }
    return mt;
}

__global__ void __launch_bounds__(1024) k_plan(PlanArgs a)
{
    __shared__ double s_dbl[1024];
    __shared__ uint64_t s_u64[1024];
    __shared__ uint32_t s_bucket[65];
    __shared__ uint32_t s_cursor[65];
    const int tid = threadIdx.x;

    if (tid < 65) s_bucket[tid] = 0;
    if (tid == 0) a.counters[CNT_QUEUE] = 0;
    __syncthreads();

    // total work and per-n bucket sizes
    double w = 0.0;
    for (int k = tid; k < a.count; k += 1024) {
        const int n = a.ns[k];
        const bool valid = n >= 0 && n <= 63;
        if (valid) {
            uint64_t lo, hi;
            range_of(a, n, lo, hi);
            w += (double)(hi - lo);
        }
        atomicAdd(&s_bucket[valid ? n : 64], 1u);
    }
    s_dbl[tid] = w;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if (tid < off) s_dbl[tid] += s_dbl[tid + off];
        __syncthreads();
    }
    const double total_work = s_dbl[0];
    if (tid == 0) {
        uint32_t off = 0;
        for (int b = 63; b >= 0; --b) {
            s_cursor[b] = off;
            off += s_bucket[b];
        }
        s_cursor[64] = off;
    }
    __syncthreads();

    const int target_m = target_chunk_log(a, total_work);
    for (int k = tid; k < a.count; k += 1024) {
        const MatMeta mt = plan_matrix(a, k, target_m, true);
        a.meta[k] = mt;
        const int n = a.ns[k];
        const bool valid = n >= 0 && n <= 63;
        const uint32_t pos = atomicAdd(&s_cursor[valid ? n : 64], 1u);
        a.order[pos] = k;
    }
    __syncthreads();

    // first task of each position in the order
    uint64_t running = 0;
    for (int base = 0; base < a.count; base += 1024) {
        const int p = base + tid;
        const uint64_t v = p < a.count ? (uint64_t)a.meta[a.order[p]].ntasks : 0;
        uint64_t tot;
        const uint64_t incl = block_incl_scan_1024<uint64_t>(v, s_u64, tot);
        if (p < a.count) a.task_start[p] = running + incl - v;
        running += tot;
    }
    if (tid == 0) {
        a.task_start[a.count] = running;
        a.counters[CNT_TOTAL_TASKS] = running;
    }

    // row offsets in matrix order
    uint64_t rrun = 0;
    for (int base = 0; base < a.count; base += 1024) {
        const int k = base + tid;
        const uint64_t v = k < a.count ? (uint64_t)a.meta[k].n : 0;
        uint64_t tot;
        const uint64_t incl = block_incl_scan_1024<uint64_t>(v, s_u64, tot);
        if (k < a.count) a.meta[k].row_base = (int64_t)(rrun + incl - v);
        rrun += tot;
    }
}

// ------------------------------------------------------------------ pack

// The walk's row record of a row with words (mag, sgn): both words split in
// 32-bit halves, with the negated row's sign word sn = sgn ^ mag beside them.
__device__ __forceinline__ RowW make_row(uint64_t mag, uint64_t sgn)
{
    RowW r;
    const uint64_t sn = sgn ^ mag;
    r.m_lo = (uint32_t)mag;
    r.s_lo = (uint32_t)sgn;
    r.sn_lo = (uint32_t)sn;
    r.pad0 = 0;
    r.m_hi = (uint32_t)(mag >> 32);
    r.s_hi = (uint32_t)(sgn >> 32);
    r.sn_hi = (uint32_t)(sn >> 32);
    r.pad1 = 0;
    return r;
}

__device__ __forceinline__ void store_row(RowW *dst, uint64_t mag, uint64_t sgn) { *dst = make_row(mag, sgn); }

// phi (Section 2): mag bit = (a != 0), sgn bit = (a == -1); element j of a
// row goes to bit n-1-j, so (1,1,0,-1) becomes (0xd, 0x1).
// phi (Section 2) of one row of n bytes: column c at bit n-1-c of the mag
// and sgn words; returns whether an entry is outside {0, 1, 2}.
__device__ __forceinline__ bool phi_row(const uint8_t *row, int n, uint64_t &mag, uint64_t &sgn)
{
    mag = 0;
    sgn = 0;
    bool bad = false;
    for (int c = 0; c < n; ++c) {
        const uint8_t x = row[c];
        const uint64_t bit = 1ull << (n - 1 - c);
        bad |= x > 2;
        if (x != 0) mag |= bit;
        if (x == 2) sgn |= bit;
    }
    return bad;
}

// The n x n bytes at src (n <= 63: at most 3969) copied into dst (4096 bytes
// of LDS) by NT cooperating threads, thread t of them, each with its 16
// loads in flight together.  A round covers NT * 16 bytes, which divides
// 4096, so every round that starts below n * n <= 4096 ends inside dst.
template <int NT>
__device__ __forceinline__ void stage_bytes(const uint8_t *src, int n, uint8_t *dst, int t)
{
    static_assert(4096 % (NT * 16) == 0, "rounds tile the 4096-byte buffer");
    const int nn = n * n;
    for (int base = 0; base < nn; base += NT * 16) {
        uint8_t v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int idx = base + t + NT * i;
            v[i] = idx < nn ? src[idx] : 0;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int idx = base + t + NT * i;
            dst[idx] = v[i];
        }
    }
}

constexpr int PACK_BLOCK = 256;

// phi of one byte matrix (1 <= n <= 63) by a PACK_BLOCK-thread block: its
// bytes read once into LDS, row r formed by thread r; the matrix's status is
// set to whether any entry is outside {0, 1, 2}.  Every thread of the block
// must call it.
__device__ void pack_block(const uint8_t *src, int n, RowW *dst, uint8_t *status)
{
    __shared__ uint8_t s_mat[4096];
    const int t = threadIdx.x;
    stage_bytes<PACK_BLOCK>(src, n, s_mat, t);
    __syncthreads();
    if (t >= 64) return;                       // n <= 63: every row is in wave 0
    uint64_t mag = 0, sgn = 0;
    const bool bad = t < n ? phi_row(s_mat + t * n, n, mag, sgn) : false;
    const bool any_bad = __any(bad) != 0;
    if (t == 0) *status = any_bad ? 1 : 0;
    if (t < n) store_row(dst + t, mag, sgn);
}

__global__ void __launch_bounds__(PACK_BLOCK) k_pack_u8(PackU8Args a)
{
    const int k = blockIdx.x;
    if (k >= a.count) return;
    const MatMeta mt = a.meta[k];
    if (mt.mode == MODE_NONE) return;
    pack_block(a.mats + a.offs[k], mt.n, a.rows + mt.row_base, a.status + k);
}

// Row r of a caller-packed matrix: its (mag, sgn) words at src[2r], src[2r+1];
// returns whether a bit at or above n is set in either.
__device__ __forceinline__ bool planes_row(const uint64_t *src, int n, int r, uint64_t &mag, uint64_t &sgn)
{
    mag = src[2 * r];
    sgn = src[2 * r + 1];
    const uint64_t high = (n >= 64) ? 0 : ~((1ull << n) - 1ull);
    return ((mag | sgn) & high) != 0;
}

__global__ void __launch_bounds__(64) k_pack_planes(PackPlanesArgs a)
{
    const int k = blockIdx.x;
    if (k >= a.count) return;
    const MatMeta mt = a.meta[k];
    if (mt.mode == MODE_NONE) return;
    const int n = mt.n;
    const int r = threadIdx.x;
    if (r >= n) return;
    uint64_t mag, sgn;
    if (planes_row(a.planes + 2 * a.row_off[k], n, r, mag, sgn)) a.status[k] = 1;
    store_row(a.rows + mt.row_base + r, mag, sgn);
}

// ------------------------------------------------------------------ small calls


// Lane j's value of a 64-bit variable, read by every lane (j wave-uniform).
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int j)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}

// Planning of up to SMALL_PLAN_MAX matrices by one wavefront: lane k plans
// matrix k and takes its rank in the task order and its prefix sums from the
// other lanes' registers (readlane over the call's matrices only), with no
// LDS round trips and no block scans.
__device__ void plan_small(const PlanArgs &a, bool write_status)
{
    const int k = threadIdx.x;
    const int count = a.count;
    const bool have = k < count;
    const int n = have ? a.ns[k] : -1;
    const bool valid = have && n >= 0 && n <= 63;
    double w = 0.0;
    if (valid) {
        uint64_t lo, hi;
        range_of(a, n, lo, hi);
        w = (double)(hi - lo);
    }
    const int key = have ? (valid ? n : -1) : -2;   // larger n first, then invalid n
    if (k == 0) a.counters[CNT_QUEUE] = 0;
    double total_work = 0.0;
    for (int j = 0; j < count; ++j) total_work += __longlong_as_double((long long)readlane64((uint64_t)__double_as_longlong(w), j));
    const int target_m = target_chunk_log(a, total_work);
    MatMeta mt;
    if (have) mt = plan_matrix(a, k, target_m, write_status);
    const uint64_t ntasks = have ? mt.ntasks : 0;
    const int rows = have ? mt.n : 0;
    int rank = 0;
    uint64_t first = 0, total_tasks = 0;
    int64_t row_base = 0;
    for (int j = 0; j < count; ++j) {
        const int kj = __builtin_amdgcn_readlane(key, j);
        const uint64_t tj = readlane64(ntasks, j);
        const bool before = kj > key || (kj == key && j < k);
        rank += before ? 1 : 0;
        if (before) first += tj;
        total_tasks += tj;
        if (j < k) row_base += __builtin_amdgcn_readlane(rows, j);
    }
    if (have) {
        mt.row_base = row_base;
        a.meta[k] = mt;
        a.order[rank] = k;
        a.task_start[rank] = first;
    }
    if (k == 0) {
        a.task_start[count] = total_tasks;
        a.counters[CNT_TOTAL_TASKS] = total_tasks;
    }
}

// phi (Section 2) of byte matrix j with its validation: the matrix (at most
// 63 x 63 bytes) is read once with coalesced byte loads, all in flight
// together, into LDS, and lane r forms row r from there.  Its first row is
// the sum of the earlier matrices' orders (invalid orders count 0, as in the
// plan).  This block alone writes the matrix's status when its order is valid.
__device__ void pack_small(const PlanArgs &a, const PackU8Args &pk, int j)
{
    __shared__ long long s_base;
    const int t = threadIdx.x;
    const int n = a.ns[j];
    if (n < 0 || n > 63) return;                  // the plan marks it invalid
    if (n == 0) {
        if (t == 0) pk.status[j] = 0;
        return;
    }
    if (t < 64) {
        const int ni = t < j ? a.ns[t] : 0;
        const long long base = wave_sum_i64(ni >= 0 && ni <= 63 ? ni : 0);
        if (t == 0) s_base = base;
    }
    __syncthreads();
    pack_block(pk.mats + pk.offs[j], n, pk.rows + s_base, pk.status + j);
}

// The same for caller-packed planes: wave 0 of the block, row r by lane r.
__device__ void pack_small_planes(const PlanArgs &a, const PackPlanesArgs &pp, int j)
{
    const int t = threadIdx.x;
    if (t >= 64) return;
    const int n = a.ns[j];
    if (n < 0 || n > 63) return;                  // the plan marks it invalid
    const int ni = t < j ? a.ns[t] : 0;
    const long long base = wave_sum_i64(ni >= 0 && ni <= 63 ? ni : 0);
    uint64_t mag = 0, sgn = 0;
    const bool bad = t < n ? planes_row(pp.planes + 2 * pp.row_off[j], n, t, mag, sgn) : false;
    const bool any_bad = __any(bad) != 0;
    if (t == 0) pp.status[j] = any_bad ? 1 : 0;
    if (t < n) store_row(pp.rows + base + t, mag, sgn);
}

// ------------------------------------------------------------------ walk

// One task of one matrix: the lane's S chunks c + 64 s, one after another,
// in blocks of 2^WALK_UL indices; candidate blocks re-walked together after
// each chunk (DEFER) or each at once; each block's closing row read a block
// ahead (AHEAD) or at its start.
template <int S, bool DEFER, bool AHEAD, typename RP>
__device__ __forceinline__ int walk_task(RP R, const MatMeta &mt, uint64_t c)
{
    LowSums<WALK_UL> lr;
    if (mt.mode == MODE_FAST) load_low_sums<WALK_UL>(R, lr);
    int tally = 0;
#pragma unroll
    for (int q = 0; q < S; ++q)
        tally += walk_lane<WALK_UL, DEFER, AHEAD>(R, mt.n, mt.m, mt.mode, c + 64u * (uint64_t)q, mt.lo, mt.hi, lr);
    return tally;
}

// DEFER: candidate blocks noted and re-walked one lane each (batches, whose
// small matrices hold candidates in one block of tens), else re-walked by the
// whole wave at once (one large matrix, where they are rare: the leaner walk).
template <int S, bool DEFER>
__global__ void __launch_bounds__(WALK_BLOCK) k_walk(WalkArgs a)
{
    const int lane = threadIdx.x & 63;
    const uint64_t total = a.counters[CNT_TOTAL_TASKS];
    const uint32_t nwaves = gridDim.x * (WALK_BLOCK / 64);
    const cptr<uint64_t> task_start = to_const(a.task_start);
    // A wave's tasks come in increasing order (its own index first, then the
    // queue's), so the position holding the next task is at or after the
    // last one: gallop forward from there, then bisect.
    int pos = 0;
    for (uint64_t tau = wave_index(); tau < total; tau = next_task64(&a.counters[CNT_QUEUE], nwaves, lane)) {
        // position p in the order whose tasks contain tau: the largest p with
        // task_start[p] <= tau (matrices without tasks share their successor's start)
        int lo = pos, hi = pos + 1, step = 1;
        while (hi < a.count && task_start[hi] <= tau) {
            lo = hi;
            hi = lo + step;
            step <<= 1;
        }
        if (hi > a.count) hi = a.count;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (task_start[mid] <= tau) lo = mid; else hi = mid;
        }
        pos = lo;
        const int k = to_const(a.order)[lo];
        const MatMeta mt = load_const(a.meta, k);
        const uint64_t q = tau - task_start[lo];

        int tally = 0;
        if (to_const(a.status)[k] == 0) {
            const cptr<RowW> R = to_const(a.rows) + mt.row_base;
            const uint64_t c = mt.c_first + q * (64u * S) + (uint64_t)lane;
            tally = walk_task<S, DEFER, true>(R, mt, c);
        }
        const int sum = wave_sum(tally);

        if (lane == 0) {
            if (sum != 0) atomicAdd((unsigned long long *)&a.tally[k], (unsigned long long)(long long)sum);
            __threadfence();
            const uint64_t prev = atomicAdd((unsigned long long *)&a.done[k], 1ull);
            if (prev + 1 == mt.ntasks) {
                __threadfence();
                const long long T = __hip_atomic_load((long long *)&a.tally[k], __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                if (a.status[k] != 0) {
                    a.out[k] = 0xFF;
                } else {
                    const uint8_t r = finish_mod3(mt.n, T);
                    a.out[k] = r;
                    if (a.hist) atomicAdd((unsigned long long *)&a.hist[3 * mt.n + r], 1ull);
                }
            }
        }
    }
}

// ------------------------------------------------------------------ one-launch small calls

// A call of up to SMALL_PLAN_MAX byte matrices with at most SMALL_FUSED_WORK
// Gray indices in all is planned, packed and walked by one launch: every wave
// plans the whole call in registers (lane k holds matrix k), takes tasks
// tau = wave, wave + waves, ... in rank order, packs its task's matrix into
// its own LDS (one coalesced read of the bytes) and walks it from there.  No
// result of another kernel is waited on, so the chain of dependent memory
// reads is short.  The per-matrix accumulator words are left at zero by the
// wave that completes each matrix, ready for the next call.  A larger call is
// planned and packed here into the work buffers, and k_walk follows.

struct SmallLds {
    uint8_t bytes[64 * 64];
    RowW rows[64];
};
typedef const __attribute__((address_space(3))) RowW *lds_rows;

__device__ __forceinline__ double readlane_f64(double v, int j)
{
    return __longlong_as_double((long long)readlane64((uint64_t)__double_as_longlong(v), j));
}

__device__ __forceinline__ MatMeta readlane_meta(const MatMeta &v, int j)
{
    MatMeta r;
    r.n = __builtin_amdgcn_readlane(v.n, j);
    r.m = __builtin_amdgcn_readlane(v.m, j);
    r.mode = __builtin_amdgcn_readlane(v.mode, j);
    r.ul = __builtin_amdgcn_readlane(v.ul, j);
    r.ntasks = readlane64(v.ntasks, j);
    r.row_base = (int64_t)readlane64((uint64_t)v.row_base, j);
    r.lo = readlane64(v.lo, j);
    r.hi = readlane64(v.hi, j);
    r.c_first = readlane64(v.c_first, j);
    return r;
}

// Order the wave's LDS accesses: the rows one lane writes are read by others.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// phi (Section 2) of the n x n byte matrix at src into the wave's LDS rows;
// returns whether any entry is outside {0, 1, 2} (wave-uniform).
__device__ bool pack_lds(const uint8_t *src, int n, SmallLds &L, int lane)
{
    stage_bytes<64>(src, n, L.bytes, lane);
    wave_lds_sync();
    uint64_t mag = 0, sgn = 0;
    const bool bad = lane < n ? phi_row(L.bytes + lane * n, n, mag, sgn) : false;
    if (lane < n) L.rows[lane] = make_row(mag, sgn);
    const bool any_bad = __any(bad) != 0;
    wave_lds_sync();
    return any_bad;
}

// Caller-packed planes into the wave's LDS rows; returns whether a bit at or
// above n is set (wave-uniform).
__device__ bool pack_lds_planes(const uint64_t *src, int n, SmallLds &L, int lane)
{
    uint64_t mag = 0, sgn = 0;
    const bool bad = lane < n ? planes_row(src, n, lane, mag, sgn) : false;
    if (lane < n) L.rows[lane] = make_row(mag, sgn);
    const bool any_bad = __any(bad) != 0;
    wave_lds_sync();
    return any_bad;
}

// kind 0: byte matrices (pk); kind 1: caller-packed planes (pp).
__global__ void __launch_bounds__(WALK_BLOCK) k_small(PlanArgs a, PackU8Args pk, PackPlanesArgs pp, SmallAcc acc,
                                                      int kind, int allow_fused)
{
    static_assert(WALK_BLOCK == PACK_BLOCK, "one block shape for both roles");
    // a small call is latency-bound: beside the waves of a long walk on the
    // same SIMDs (a serving tick), these waves issue first
    __builtin_amdgcn_s_setprio(3);
    __shared__ SmallLds lds[WALK_BLOCK / 64];
    const int lane = threadIdx.x & 63;
    const int count = a.count;
    const bool have = lane < count;
    const int n = have ? a.ns[lane] : -1;
    const int64_t off = have ? (kind == 0 ? pk.offs[lane] : pp.row_off[lane]) : 0;
    const bool valid = have && n >= 0 && n <= 63;
    double w = 0.0;
    if (valid) {
        uint64_t lo, hi;
        range_of(a, n, lo, hi);
        w = (double)(hi - lo);
    }
    double total_work = 0.0;
    for (int j = 0; j < count; ++j) total_work += readlane_f64(w, j);
    if (!(allow_fused && total_work <= (double)SMALL_FUSED_WORK)) {
        // block 0 plans; block 1 + j packs matrix j and owns its status
        if (blockIdx.x == 0) {
            if (threadIdx.x < 64) plan_small(a, false);
        } else if ((int)blockIdx.x <= count) {
            if (kind == 0)
                pack_small(a, pk, blockIdx.x - 1);
            else
                pack_small_planes(a, pp, blockIdx.x - 1);
        }
        return;
    }

    // one chunk per lane: carrying several side by side pays only on long tasks
    PlanArgs pf = a;
    pf.states_log = 0;
    const int target_m = target_chunk_log(pf, total_work);
    const MatMeta mt = plan_pure(pf, valid ? n : -1, target_m);
    const uint64_t ntasks = have ? mt.ntasks : 0;
    const int key = have ? (valid ? n : -1) : -2;   // larger n first
    uint64_t first = 0, total = 0;
    for (int j = 0; j < count; ++j) {
        const int kj = __builtin_amdgcn_readlane(key, j);
        const uint64_t tj = readlane64(ntasks, j);
        if (kj > key || (kj == key && j < lane)) first += tj;
        total += tj;
    }
    const uint32_t wi = wave_index();
    if (wi == 0) {
        // matrices with no tasks: an invalid order, or n = 0 (one empty
        // subset, a term of +1: perm of the 0 x 0 matrix is 1)
        if (have && ntasks == 0) {
            if (!valid) {
                a.out[lane] = 0xFF;
            } else {
                const uint8_t r = finish_mod3(0, 1);
                a.out[lane] = r;
                if (a.hist) atomicAdd((unsigned long long *)&a.hist[r], 1ull);
            }
        }
        if (lane == 0) a.counters[CNT_TOTAL_TASKS] = 0;   // nothing left for a k_walk that follows
    }

    SmallLds &L = lds[threadIdx.x >> 6];
    const lds_rows R = (lds_rows)L.rows;
    const uint32_t nwaves = gridDim.x * (WALK_BLOCK / 64);
    int packed = -1;
    bool bad = false;
    for (uint64_t tau = wi; tau < total; tau += nwaves) {
        const bool mine = ntasks > 0 && first <= tau && tau < first + ntasks;
        const int k = __builtin_amdgcn_readfirstlane(__builtin_ctzll(__ballot(mine)));
        const MatMeta m = readlane_meta(mt, k);
        const uint64_t q = tau - readlane64(first, k);
        if (k != packed) {
            const int64_t ok = (int64_t)readlane64((uint64_t)off, k);
            bad = kind == 0 ? pack_lds(pk.mats + ok, m.n, L, lane) : pack_lds_planes(pp.planes + 2 * ok, m.n, L, lane);
            packed = k;
        }
        int tally = 0;
        if (!bad) {
            const uint64_t c = m.c_first + q * 64u + (uint64_t)lane;
            tally = walk_task<1, true, false>(R, m, c);
        }
        const int sum = wave_sum(tally);
        if (lane == 0) {
            bool last = m.ntasks == 1;
            long long T = sum;
            if (!last) {
                // one word per matrix: completed tasks from bit 40 up, and below
                // them the tally plus a bias of 64 * 2^m per task (a task's sum
                // is at least minus its index count, so no addend is negative;
                // the biased total stays under 2^31 because the call walks at
                // most 2^28 indices); one atomic per task, and the wave that
                // completes the matrix reads its total from the returned value
                const uint64_t bias = 64ull << m.m;
                const uint64_t add = (1ull << 40) + (uint64_t)((long long)sum + (long long)bias);
                const uint64_t now = atomicAdd((unsigned long long *)&acc.word[k], (unsigned long long)add) + add;
                if ((now >> 40) == m.ntasks) {
                    T = (long long)(now & ((1ull << 40) - 1)) - (long long)(m.ntasks * bias);
                    __hip_atomic_store((unsigned long long *)&acc.word[k], 0ull, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    last = true;
                }
            }
            if (last) {
                if (bad) {
                    a.out[k] = 0xFF;
                } else {
                    const uint8_t r = finish_mod3(m.n, T);
                    a.out[k] = r;
                    if (a.hist) atomicAdd((unsigned long long *)&a.hist[3 * m.n + r], 1ull);
                }
            }
        }
    }
}

// ------------------------------------------------------------------ serving

__global__ void __launch_bounds__(WALK_BLOCK) k_tick(TickArgs a)
{
    const int lane = threadIdx.x & 63;
    const uint32_t total = *a.ntasks;
    const uint32_t nwaves = gridDim.x * (WALK_BLOCK / 64);
    for (uint32_t tau = wave_index(); tau < total; tau = next_task(a.queue, nwaves, lane)) {
        const TickTask tk = load_const(a.tasks, tau);
        const SlotInfo si = load_const(a.slots, tk.slot);
        const cptr<RowW> R = to_const(a.rows) + si.row_base;
        MatMeta mt;
        mt.n = si.n;
        mt.m = tk.m;
        mt.mode = tk.mode;
        mt.lo = 0;
        mt.hi = 1ull << si.n;
        int tally = 0;
        if (lane < tk.nchunks) {
            const uint64_t c = tk.c_first + (uint64_t)lane;
            tally = walk_task<1, true, true>(R, mt, c);
        }
        const int sum = wave_sum(tally);
        if (lane == 0 && sum != 0)
            atomicAdd((unsigned long long *)&a.tally[tk.slot], (unsigned long long)(long long)sum);
    }
}

__global__ void k_finish(FinishArgs a)
{
    const uint32_t nf = *a.nfin;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *a.queue = 0;
    if (i >= nf) return;
    const int slot = a.fin_slots[i];
    const int n = a.slots[slot].n;
    const long long T = a.tally[slot];
    a.fin_out[i] = finish_mod3(n, T);
    a.tally[slot] = 0;
}

// Pack one matrix into a serving slot.
__global__ void __launch_bounds__(64) k_slot_pack(const uint8_t *A, int n, RowW *dst)
{
    const int r = threadIdx.x;
    if (r >= n) return;
    uint64_t mag = 0, sgn = 0;
    for (int j = 0; j < n; ++j) {
        const uint8_t v = A[r * n + j];
        const uint64_t bit = 1ull << (n - 1 - j);
        if (v != 0) mag |= bit;
        if (v == 2) sgn |= bit;
    }
    store_row(dst + r, mag, sgn);
}

// ((-1)^n times the sum of the tallies) mod 3: eq. (2) finished over pieces
// of the Gray range walked separately (Section 3.1), for example the shards
// of a long run.  One wavefront.
__global__ void __launch_bounds__(64) k_finish_tallies(const int64_t *t, int32_t count, int32_t n, uint8_t *out)
{
    long long s = 0;
    for (int32_t i = threadIdx.x; i < count; i += 64) s += t[i];
    s = wave_sum_i64(s);
    if (threadIdx.x == 0) *out = finish_mod3(n, s);
}

// ------------------------------------------------------------------ self-check

// Theorem 2.1 on individual 32-bit words, through the same device functions
// the walk uses.
__global__ void k_bipedal_ops(const uint32_t *in, int count, uint32_t *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint32_t m1 = in[4 * i], s1 = in[4 * i + 1], m2 = in[4 * i + 2], s2 = in[4 * i + 3];
    uint32_t am = m1, as = s1;
    bip_add(am, as, m2, s2);
    uint32_t bm = m1, bs = s1;
    bip_sub(bm, bs, m2, s2);
    // the walk's subtraction: add the negated row (sgn xor mag)
    uint32_t nm = m1, ns = s1;
    bip_add(nm, ns, m2, s2 ^ m2);
    out[8 * i + 0] = am;
    out[8 * i + 1] = as;
    out[8 * i + 2] = bm;
    out[8 * i + 3] = bs;
    out[8 * i + 4] = m1 & m2;   // multiplication
    out[8 * i + 5] = s1 ^ s2;
    out[8 * i + 6] = nm;        // subtraction as the walk performs it
    out[8 * i + 7] = ns;
}

// p[0 .. count) = value: clears counters and accumulator words with a kernel,
// which a stream capture records as a kernel node.
__global__ void k_fill_u64(uint64_t *p, int64_t count, uint64_t value)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// ------------------------------------------------------------------ launchers

hipError_t launch_plan(const PlanArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_small(const PlanArgs &a, const PackU8Args &pk, const PackPlanesArgs &pp, const SmallAcc &acc,
                        int kind, bool allow_fused, int blocks, hipStream_t st)
{
    if (a.count < 1 || a.count > SMALL_PLAN_MAX || blocks < a.count + 1 || (kind != 0 && kind != 1))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_small, dim3(blocks), dim3(WALK_BLOCK), 0, st, a, pk, pp, acc, kind, allow_fused ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_pack_u8(const PackU8Args &a, hipStream_t st)
{
    if (a.count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_u8, dim3(a.count), dim3(PACK_BLOCK), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_pack_planes(const PackPlanesArgs &a, hipStream_t st)
{
    if (a.count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_planes, dim3(a.count), dim3(64), 0, st, a);
    return hipGetLastError();
}

// Workgroups of a kernel that fit on one CU at once.  A persistent wave's first
// task is its own index, so a workgroup that is not resident at launch would
// start its first task only when an earlier one exits, at the end of the run:
// the walk grids are capped at this count.
template <typename K>
static int resident_per_cu(std::atomic<int> &cache, K kernel)
{
    int n = cache.load(std::memory_order_relaxed);
    if (n > 0) return n;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, WALK_BLOCK, 0) != hipSuccess || n < 1) n = 1;
    cache.store(n, std::memory_order_relaxed);
    return n;
}

// the fewer of the two forms (with and without deferred re-walks), so that a
// plan made for the grid holds for either
int walk_resident_per_cu(int states)
{
    static std::atomic<int> c1{0}, c2{0}, c4{0}, d1{0}, d2{0}, d4{0}, ct{0};
    switch (states) {
    case 1: return std::min(resident_per_cu(c1, k_walk<1, false>), resident_per_cu(d1, k_walk<1, true>));
    case 2: return std::min(resident_per_cu(c2, k_walk<2, false>), resident_per_cu(d2, k_walk<2, true>));
    case 4: return std::min(resident_per_cu(c4, k_walk<4, false>), resident_per_cu(d4, k_walk<4, true>));
    default: return resident_per_cu(ct, k_tick);   // 0: the serving tick
    }
}

hipError_t launch_walk(const WalkArgs &a, int states, bool defer, int grid_blocks, hipStream_t st)
{
    const dim3 g(grid_blocks), b(WALK_BLOCK);
    switch (states * 2 + (defer ? 1 : 0)) {
    case 2: hipLaunchKernelGGL((k_walk<1, false>), g, b, 0, st, a); break;
    case 3: hipLaunchKernelGGL((k_walk<1, true>), g, b, 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_walk<2, false>), g, b, 0, st, a); break;
    case 5: hipLaunchKernelGGL((k_walk<2, true>), g, b, 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_walk<4, false>), g, b, 0, st, a); break;
    case 9: hipLaunchKernelGGL((k_walk<4, true>), g, b, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_tick(const TickArgs &a, int grid_blocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_tick, dim3(grid_blocks), dim3(WALK_BLOCK), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_finish(const FinishArgs &a, int max_fin, hipStream_t st)
{
    const int blocks = max_fin > 0 ? (max_fin + 255) / 256 : 1;
    hipLaunchKernelGGL(k_finish, dim3(blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_slot_pack(const uint8_t *A, int n, RowW *dst, hipStream_t st)
{
    hipLaunchKernelGGL(k_slot_pack, dim3(1), dim3(64), 0, st, A, n, dst);
    return hipGetLastError();
}

hipError_t launch_finish_tallies(const int64_t *t, int32_t count, int32_t n, uint8_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_finish_tallies, dim3(1), dim3(64), 0, st, t, count, n, out);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t *p, int64_t count, uint64_t value, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 1024);
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, st, p, count, value);
    return hipGetLastError();
}

hipError_t launch_bipedal_ops(const uint32_t *in, int count, uint32_t *out, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bipedal_ops, dim3((count + 63) / 64), dim3(64), 0, st, in, count, out);
    return hipGetLastError();
}

}  // namespace perm3
