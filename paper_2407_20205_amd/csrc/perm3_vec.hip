// Bitsliced vectors over F_3 in device memory (gfx950): the operations of
// Theorem 2.1 beyond the permanent's addition.
//
// A vector of len elements is ceil(len / 64) words; word w is the pair
// planes[2w] = mag, planes[2w + 1] = sgn, and element e sits at bit e mod 64
// of word e / 64 (least significant first).  phi of Section 2 maps 0 -> (0,0),
// 1 -> (1,0), -1 -> (1,1); (0,1) is a second zero (Definition 2.1).  Bits at
// and above len in the last word are zero after a pack.
//
//   k_f3_pack    bytes {0,1,2} (2 = -1) -> planes; counts bytes > 2 (packed as 0)
//   k_f3_unpack  planes -> bytes, psi of Section 2
//   k_f3_op      add, sub, mul, div by Theorem 2.1's formulas as printed, and
//                negation; one 16-byte word pair per lane
//   k_f3_dot     sum over e of a_e b_e as an integer: the product word of
//                Theorem 2.1, then popcounts of its +1 and -1 elements
//
// All four stream once through HBM; each is bound by its bytes moved.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "perm3.h"
#include "perm3_device.hpp"
#include "perm3_internal.h"
#include "perm3_runtime.h"

namespace perm3 {

constexpr int VEC_BLOCK = 256;

struct alignas(16) WordPair {
    uint64_t mag, sgn;
};
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Every byte is touched once, so loads and stores are marked non-temporal
// (streamed past the caches): 3-8% more bandwidth than plain accesses.
__device__ __forceinline__ WordPair ld_nt(const WordPair *p)
{
    const u64x2 v = __builtin_nontemporal_load(reinterpret_cast<const u64x2 *>(p));
    WordPair r;
    r.mag = v.x;
    r.sgn = v.y;
    return r;
}

__device__ __forceinline__ void st_nt(WordPair *p, WordPair r)
{
    u64x2 v;
    v.x = r.mag;
    v.y = r.sgn;
    __builtin_nontemporal_store(v, reinterpret_cast<u64x2 *>(p));
}

__device__ __forceinline__ uint64_t grid_waves() { return (uint64_t)gridDim.x * (VEC_BLOCK / 64); }
__device__ __forceinline__ uint64_t my_wave() { return (uint64_t)blockIdx.x * (VEC_BLOCK / 64) + (threadIdx.x >> 6); }

// phi, 1024 elements per wave and step: lane l reads 16 bytes (elements
// 16 l .. 16 l + 15), forms their 16 mag and 16 sgn bits, and lanes 4k .. 4k+3
// join their pieces into word k of the step.
template <bool ALIGNED>
__global__ void __launch_bounds__(VEC_BLOCK) k_f3_pack(const uint8_t *v, int64_t len, WordPair *planes,
                                                       unsigned long long *invalid)
{
    const int lane = threadIdx.x & 63;
    const uint64_t steps = ((uint64_t)len + 1023) / 1024;
    uint32_t bad = 0;
    for (uint64_t st = my_wave(); st < steps; st += grid_waves()) {
        const int64_t e0 = (int64_t)st * 1024 + 16 * lane;
        uint8_t b[16];
        if (ALIGNED && e0 + 16 <= len) {
            const u32x4 q = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(v + e0));
            const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int i = 0; i < 16; ++i) b[i] = (uint8_t)(w[i >> 2] >> (8 * (i & 3)));
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i) b[i] = e0 + i < len ? v[e0 + i] : 0;
        }
        uint32_t piece = 0;   // mag bits 0..15, sgn bits 16..31
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            bad += b[i] > 2;
            piece |= (uint32_t)(b[i] == 1 || b[i] == 2) << i;
            piece |= (uint32_t)(b[i] == 2) << (16 + i);
        }
        const uint32_t p1 = __shfl_down(piece, 1);
        const uint32_t p2 = __shfl_down(piece, 2);
        const uint32_t p3 = __shfl_down(piece, 3);
        const int64_t w = (int64_t)st * 16 + (lane >> 2);
        if ((lane & 3) == 0 && w * 64 < len) {
            WordPair o;
            o.mag = (uint64_t)(piece & 0xffffu) | ((uint64_t)(p1 & 0xffffu) << 16) |
                    ((uint64_t)(p2 & 0xffffu) << 32) | ((uint64_t)(p3 & 0xffffu) << 48);
            o.sgn = (uint64_t)(piece >> 16) | ((uint64_t)(p1 >> 16) << 16) | ((uint64_t)(p2 >> 16) << 32) |
                    ((uint64_t)(p3 >> 16) << 48);
            st_nt(planes + w, o);
        }
    }
    if (invalid) {
        const long long total = wave_sum_i64((long long)bad);
        if (lane == 0 && total) atomicAdd(invalid, (unsigned long long)total);
    }
}

// psi: lane l writes the 16 bytes of elements 16 l .. 16 l + 15 of the step
// from its word's 16-bit pieces (four lanes read each word pair).
template <bool ALIGNED>
__global__ void __launch_bounds__(VEC_BLOCK) k_f3_unpack(const WordPair *planes, int64_t len, uint8_t *v)
{
    const int lane = threadIdx.x & 63;
    const uint64_t steps = ((uint64_t)len + 1023) / 1024;
    for (uint64_t st = my_wave(); st < steps; st += grid_waves()) {
        const int64_t e0 = (int64_t)st * 1024 + 16 * lane;
        if (e0 >= len) continue;
        const WordPair p = ld_nt(planes + (int64_t)st * 16 + (lane >> 2));
        const int sh = 16 * (lane & 3);
        const uint32_t m = (uint32_t)(p.mag >> sh) & 0xffffu;
        const uint32_t s = (uint32_t)(p.sgn >> sh) & 0xffffu;
        uint8_t b[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) b[i] = ((m >> i) & 1u) ? (((s >> i) & 1u) ? 2 : 1) : 0;
        if (ALIGNED && e0 + 16 <= len) {
            u32x4 q;
            q.x = b[0] | (b[1] << 8) | (b[2] << 16) | ((uint32_t)b[3] << 24);
            q.y = b[4] | (b[5] << 8) | (b[6] << 16) | ((uint32_t)b[7] << 24);
            q.z = b[8] | (b[9] << 8) | (b[10] << 16) | ((uint32_t)b[11] << 24);
            q.w = b[12] | (b[13] << 8) | (b[14] << 16) | ((uint32_t)b[15] << 24);
            __builtin_nontemporal_store(q, reinterpret_cast<u32x4 *>(v + e0));
        } else {
            for (int i = 0; i < 16 && e0 + i < len; ++i) v[e0 + i] = b[i];
        }
    }
}

// Theorem 2.1 on one word pair, the formulas as printed.
__device__ __forceinline__ WordPair f3_apply(int op, WordPair a, WordPair b)
{
    const uint64_t m1 = a.mag, s1 = a.sgn, m2 = b.mag, s2 = b.sgn;
    WordPair r;
    switch (op) {
    case PERM_F3_ADD: {
        const uint64_t x = m2 & (m1 ^ s1 ^ s2);
        r.mag = x | (m1 ^ m2);
        r.sgn = x ^ s1;
        break;
    }
    case PERM_F3_SUB: {
        const uint64_t x = m1 & (s1 ^ s2);
        r.mag = x | (m1 ^ m2);
        r.sgn = x ^ (m2 ^ s2);
        break;
    }
    case PERM_F3_MUL:
        r.mag = m1 & m2;
        r.sgn = s1 ^ s2;
        break;
    case PERM_F3_DIV:
        r.mag = m1;
        r.sgn = s1 ^ s2;
        break;
    default:   // PERM_F3_NEG: every non-zero element changes sign
        r.mag = m1;
        r.sgn = s1 ^ m1;
        break;
    }
    return r;
}

// Four independent word pairs per lane and iteration (a grid-stride apart, so
// each load instruction of a wave stays contiguous) keep more bytes in flight.
template <int OP>
__global__ void __launch_bounds__(VEC_BLOCK) k_f3_op(const WordPair *a, const WordPair *b, WordPair *out,
                                                     int64_t words)
{
    const uint64_t stride = (uint64_t)gridDim.x * VEC_BLOCK;
    const uint64_t W = (uint64_t)words;
    uint64_t w = (uint64_t)blockIdx.x * VEC_BLOCK + threadIdx.x;
    for (; w + 3 * stride < W; w += 4 * stride) {
        WordPair x[4], y[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            x[k] = ld_nt(a + w + k * stride);
            y[k] = OP == PERM_F3_NEG ? x[k] : ld_nt(b + w + k * stride);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) st_nt(out + w + k * stride, f3_apply(OP, x[k], y[k]));
    }
    for (; w < W; w += stride) {
        const WordPair x = ld_nt(a + w);
        st_nt(out + w, f3_apply(OP, x, OP == PERM_F3_NEG ? x : ld_nt(b + w)));
    }
}

__global__ void k_f3_zero(long long *p) { *p = 0; }

// sum_e a_e b_e over the integers (each product in {-1,0,1}); a lane's int32
// partial stays exact for up to 2^24 words per lane (the host keeps it so).
__global__ void __launch_bounds__(VEC_BLOCK) k_f3_dot(const WordPair *a, const WordPair *b, int64_t words,
                                                      long long *sum)
{
    const uint64_t stride = (uint64_t)gridDim.x * VEC_BLOCK;
    const uint64_t W = (uint64_t)words;
    int acc = 0;
    uint64_t w = (uint64_t)blockIdx.x * VEC_BLOCK + threadIdx.x;
    for (; w + 3 * stride < W; w += 4 * stride) {
        WordPair x[4], y[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            x[k] = ld_nt(a + w + k * stride);
            y[k] = ld_nt(b + w + k * stride);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const WordPair p = f3_apply(PERM_F3_MUL, x[k], y[k]);
            acc += __popcll(p.mag & ~p.sgn) - __popcll(p.mag & p.sgn);
        }
    }
    for (; w < W; w += stride) {
        const WordPair p = f3_apply(PERM_F3_MUL, ld_nt(a + w), ld_nt(b + w));
        acc += __popcll(p.mag & ~p.sgn) - __popcll(p.mag & p.sgn);
    }
    const long long t = wave_sum_i64(acc);
    if ((threadIdx.x & 63) == 0 && t) atomicAdd((unsigned long long *)sum, (unsigned long long)t);
}

int vec_grid(int cus, uint64_t units_per_block)
{
    const uint64_t want = units_per_block ? units_per_block : 1;
    return (int)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)cus * 16));
}

}  // namespace perm3

using namespace perm3;

#define VEC_TRY(expr)                                         \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return hip_fail(_e, #expr);     \
    } while (0)

static int32_t vec_device(int *cus)
{
    Context *c = nullptr;
    const int32_t rc = get_context(&c);
    if (rc) return rc;
    *cus = c->cus;
    return PERM_OK;
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

extern "C" {

int32_t perm_f3_pack(const uint8_t *v_dev, int64_t len, uint64_t *planes_dev, uint64_t *invalid_dev, void *stream)
{
    set_error_index(-1);
    if (len < 0 || len > PERM_F3_MAX_LEN) return set_error(PERM_EINVAL, "len = %lld out of range", (long long)len);
    if (len == 0) return PERM_OK;
    if (!v_dev || !planes_dev) return set_error(PERM_EINVAL, "null pointer argument");
    if (!aligned16(planes_dev)) return set_error(PERM_EINVAL, "planes must be 16-byte aligned");
    int cus = 0;
    int32_t rc = vec_device(&cus);
    if (rc) return rc;
    const hipStream_t st = (hipStream_t)stream;
    const int grid = vec_grid(cus, ((uint64_t)len + 4095) / 4096);
    if (aligned16(v_dev))
        hipLaunchKernelGGL(k_f3_pack<true>, dim3(grid), dim3(VEC_BLOCK), 0, st, v_dev, len, (WordPair *)planes_dev,
                           (unsigned long long *)invalid_dev);
    else
        hipLaunchKernelGGL(k_f3_pack<false>, dim3(grid), dim3(VEC_BLOCK), 0, st, v_dev, len, (WordPair *)planes_dev,
                           (unsigned long long *)invalid_dev);
    VEC_TRY(hipGetLastError());
    return PERM_OK;
}

int32_t perm_f3_unpack(const uint64_t *planes_dev, int64_t len, uint8_t *v_dev, void *stream)
{
    set_error_index(-1);
    if (len < 0 || len > PERM_F3_MAX_LEN) return set_error(PERM_EINVAL, "len = %lld out of range", (long long)len);
    if (len == 0) return PERM_OK;
    if (!v_dev || !planes_dev) return set_error(PERM_EINVAL, "null pointer argument");
    if (!aligned16(planes_dev)) return set_error(PERM_EINVAL, "planes must be 16-byte aligned");
    int cus = 0;
    int32_t rc = vec_device(&cus);
    if (rc) return rc;
    const hipStream_t st = (hipStream_t)stream;
    const int grid = vec_grid(cus, ((uint64_t)len + 4095) / 4096);
    if (aligned16(v_dev))
        hipLaunchKernelGGL(k_f3_unpack<true>, dim3(grid), dim3(VEC_BLOCK), 0, st, (const WordPair *)planes_dev, len,
                           v_dev);
    else
        hipLaunchKernelGGL(k_f3_unpack<false>, dim3(grid), dim3(VEC_BLOCK), 0, st, (const WordPair *)planes_dev, len,
                           v_dev);
    VEC_TRY(hipGetLastError());
    return PERM_OK;
}

int32_t perm_f3_op(int32_t op, const uint64_t *a_dev, const uint64_t *b_dev, uint64_t *out_dev, int64_t words,
                   void *stream)
{
    set_error_index(-1);
    if (op < PERM_F3_ADD || op > PERM_F3_NEG) return set_error(PERM_EINVAL, "unknown operation %d", op);
    if (words < 0 || words > PERM_F3_MAX_LEN / 64)
        return set_error(PERM_EINVAL, "words = %lld out of range", (long long)words);
    if (words == 0) return PERM_OK;
    if (!a_dev || !out_dev || (op != PERM_F3_NEG && !b_dev)) return set_error(PERM_EINVAL, "null pointer argument");
    if (!aligned16(a_dev) || !aligned16(out_dev) || (b_dev && !aligned16(b_dev)))
        return set_error(PERM_EINVAL, "planes must be 16-byte aligned");
    int cus = 0;
    int32_t rc = vec_device(&cus);
    if (rc) return rc;
    const hipStream_t st = (hipStream_t)stream;
    const int grid = vec_grid(cus, ((uint64_t)words + VEC_BLOCK * 4 - 1) / (VEC_BLOCK * 4));
    const WordPair *a = (const WordPair *)a_dev, *b = (const WordPair *)b_dev;
    WordPair *o = (WordPair *)out_dev;
    switch (op) {
    case PERM_F3_ADD: hipLaunchKernelGGL(k_f3_op<PERM_F3_ADD>, dim3(grid), dim3(VEC_BLOCK), 0, st, a, b, o, words); break;
    case PERM_F3_SUB: hipLaunchKernelGGL(k_f3_op<PERM_F3_SUB>, dim3(grid), dim3(VEC_BLOCK), 0, st, a, b, o, words); break;
    case PERM_F3_MUL: hipLaunchKernelGGL(k_f3_op<PERM_F3_MUL>, dim3(grid), dim3(VEC_BLOCK), 0, st, a, b, o, words); break;
    case PERM_F3_DIV: hipLaunchKernelGGL(k_f3_op<PERM_F3_DIV>, dim3(grid), dim3(VEC_BLOCK), 0, st, a, b, o, words); break;
    default: hipLaunchKernelGGL(k_f3_op<PERM_F3_NEG>, dim3(grid), dim3(VEC_BLOCK), 0, st, a, a, o, words); break;
    }
    VEC_TRY(hipGetLastError());
    return PERM_OK;
}

int32_t perm_f3_dot(const uint64_t *a_dev, const uint64_t *b_dev, int64_t words, int64_t *sum_dev, void *stream)
{
    set_error_index(-1);
    if (words < 0 || words > PERM_F3_MAX_LEN / 64)
        return set_error(PERM_EINVAL, "words = %lld out of range", (long long)words);
    if (!sum_dev) return set_error(PERM_EINVAL, "null pointer argument");
    if (words > 0 && (!a_dev || !b_dev)) return set_error(PERM_EINVAL, "null pointer argument");
    if ((a_dev && !aligned16(a_dev)) || (b_dev && !aligned16(b_dev)))
        return set_error(PERM_EINVAL, "planes must be 16-byte aligned");
    int cus = 0;
    int32_t rc = vec_device(&cus);
    if (rc) return rc;
    const hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_f3_zero, dim3(1), dim3(1), 0, st, (long long *)sum_dev);
    VEC_TRY(hipGetLastError());
    if (words == 0) return PERM_OK;
    // at most 2^24 words per lane, so a lane's int32 partial stays exact
    const uint64_t min_blocks = ((uint64_t)words + ((uint64_t)VEC_BLOCK << 24) - 1) / ((uint64_t)VEC_BLOCK << 24);
    const int grid = (int)std::max<uint64_t>(min_blocks, (uint64_t)vec_grid(cus, ((uint64_t)words + 1023) / 1024));
    hipLaunchKernelGGL(k_f3_dot, dim3(grid), dim3(VEC_BLOCK), 0, st, (const WordPair *)a_dev, (const WordPair *)b_dev,
                       words, (long long *)sum_dev);
    VEC_TRY(hipGetLastError());
    return PERM_OK;
}

}  // extern "C"
