// Device helpers shared by the walk kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "perm3_internal.h"

namespace perm3 {

// Read-only data seen through the constant address space: wave-uniform loads
// from it become scalar loads into SGPRs.
#define PERM3_CONST __attribute__((address_space(4)))
template <typename T>
using cptr = const PERM3_CONST T *;

template <typename T>
__device__ __forceinline__ cptr<T> to_const(const T *p)
{
    return reinterpret_cast<cptr<T>>(reinterpret_cast<uintptr_t>(p));
}

// p[i] copied out word by word (wave-uniform i: scalar loads).
template <typename T>
__device__ __forceinline__ T load_const(const T *p, int64_t i)
{
    static_assert(sizeof(T) % 4 == 0, "word-sized records");
    const cptr<uint32_t> w = reinterpret_cast<cptr<uint32_t>>(reinterpret_cast<uintptr_t>(p + i));
    T v;
    uint32_t *d = reinterpret_cast<uint32_t *>(&v);
#pragma unroll
    for (size_t k = 0; k < sizeof(T) / 4; ++k) d[k] = w[k];
    return v;
}

// Sum over the 64 lanes of a wavefront: an inclusive scan inside each row of
// 16 lanes with DPP row shifts, then the four row totals read as scalars.
// Every lane must be active.
__device__ __forceinline__ int wave_sum(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);   // row_shr:8
    return __builtin_amdgcn_readlane(v, 15) + __builtin_amdgcn_readlane(v, 31) +
           __builtin_amdgcn_readlane(v, 47) + __builtin_amdgcn_readlane(v, 63);
}

// The same for 64-bit values, by butterfly shuffles.  Every lane must be active.
__device__ __forceinline__ long long wave_sum_i64(long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// r = ((-1)^n * T) mod 3 in {0, 1, 2} (2 stands for -1).
__device__ __forceinline__ uint8_t finish_mod3(int n, long long T)
{
    long long p = (n & 1) ? -T : T;
    long long r = p % 3;
    if (r < 0) r += 3;
    return (uint8_t)r;
}

// The index of this wavefront in the grid (wave-uniform).
__device__ __forceinline__ uint32_t wave_index()
{
    return blockIdx.x * (WALK_BLOCK / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Task scheduling shared by k_walk and k_tick: wave w first takes task w
// with no atomic, then draws grid-size + counter; a wave whose first task is
// past the end leaves at once, so small jobs touch the counter once per
// active wave instead of once per launched wave.
__device__ __forceinline__ uint32_t next_task(uint32_t *queue, uint32_t nwaves, int lane)
{
    uint32_t t = 0;
    if (lane == 0) t = atomicAdd(queue, 1u);
    return nwaves + __builtin_amdgcn_readfirstlane(t);
}

__device__ __forceinline__ uint64_t next_task64(uint64_t *queue, uint32_t nwaves, int lane)
{
    uint64_t t = 0;
    if (lane == 0) t = atomicAdd((unsigned long long *)queue, 1ull);
    return (uint64_t)nwaves + uniform64(t);
}

}  // namespace perm3
