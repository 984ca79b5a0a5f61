// Census kernels: perm mod 3 over many matrices made on the device.
//
// Generators (a matrix is n x n bytes in {0,1,2}, entry k in row-major order):
//   GEN_ENUMERATE  matrix t has entry k = the k-th base-3 digit of t (least
//                  significant first), so t = 0 .. 3^(n*n)-1 lists every
//                  matrix over F_3 once (the exact counts z(n) of Table 3);
//   GEN_SPLITMIX   entry k of matrix t is floor(3 x / 2^64) for x the
//                  (t*n*n + k + 1)-th output of SplitMix64 seeded with `key`
//                  (Steele, Lea and Flood, 2014): state s_q = key + q * 0x9E3779B97F4A7C15,
//                  output = mix(s_q) (uniform random matrices, Table 4).
//
// k_census_lanes: one matrix at a time per lane for n <= CENSUS_LANE_MAX_N,
// each lane over a run of consecutive matrices.  The lane walks all 2^n - 1
// Gray steps of its matrix with every index tested (the
// rows sit in LDS, one column of words per lane; all lanes flip the same row
// at the same step), forms ((-1)^n T) mod 3, and the wave counts results 0,
// 1 and 2 with ballots.  Larger n: k_generate writes the matrices and the
// batch walk takes them.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "perm3_internal.h"
#include "perm3_walk.hpp"

namespace perm3 {

constexpr uint64_t SPLITMIX_GAMMA = 0x9E3779B97F4A7C15ull;

// SplitMix64's output function of state z
__device__ __forceinline__ uint64_t splitmix_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t splitmix_out(uint64_t key, uint64_t q)
{
    return splitmix_mix(key + q * SPLITMIX_GAMMA);
}

// floor(3 x / 2^64): the high word of 3x = 2x + x
__device__ __forceinline__ uint32_t trit_of(uint64_t x)
{
    const uint64_t lo2 = x << 1;
    const uint64_t sum = lo2 + x;
    return (uint32_t)(x >> 63) + (sum < x ? 1u : 0u);
}

// Entry k of matrix t.  For enumeration the caller passes the running quotient
// (t / 3^k) and gets the next one back.
__device__ __forceinline__ uint32_t census_entry(int gen, uint64_t key, uint64_t t, int nn, int k, uint64_t &rest)
{
    if (gen == GEN_ENUMERATE) {
        const uint64_t q = rest / 3u;
        const uint32_t d = (uint32_t)(rest - 3u * q);
        rest = q;
        return d;
    }
    return trit_of(splitmix_out(key, t * (uint64_t)nn + (uint64_t)k + 1u));
}

constexpr int CENSUS_BLOCK = 256;
constexpr int CENSUS_UL = 4;   // the lane walk's blocks are 2^4 Gray steps

// The lanes' rows in LDS, sized to the call's n: row i of lane tid's matrix
// at [i * CENSUS_BLOCK + tid] (mag words, then the sgn words after n rows).
#define CROW(a, i) (a)[(i) * CENSUS_BLOCK + tid]

// The Ryser tally T of the lane's matrix: the Gray walk over all subsets from
// the empty one, every index tested.
__device__ int census_walk_plain(int n, uint32_t mask, int tid, const uint32_t *s_m, const uint32_t *s_s)
{
    uint32_t ml = 0, sl = 0;
    int tally = 0;
    const uint32_t steps = (1u << n) - 1u;
    for (uint32_t i = 1; i <= steps; ++i) {
        const int tr = __builtin_ctz(i);
        const uint32_t rm = CROW(s_m, tr), rs0 = CROW(s_s, tr);
        const bool leave = (i >> (tr + 1)) & 1u;
        bip_add(ml, sl, rm, leave ? (rs0 ^ rm) : rs0);
        if (ml == mask) {
            const int par = (__builtin_popcount(sl) + (int)(i & 1u)) & 1;
            tally += par ? -1 : 1;
        }
    }
    return tally;
}

// The same walk for n > CENSUS_UL in unrolled blocks of 16 steps: the rows
// flipped inside a block (0..3) sit in VGPRs, the row of the step closing the
// block is read from LDS once per block, and every index is still tested,
// without branches (small n makes hits far too common to skip blocks).
__device__ int census_walk_blocks(int n, uint32_t mask, int tid, const uint32_t *s_m, const uint32_t *s_s)
{
    constexpr int U = 1 << CENSUS_UL;
    uint32_t vm[CENSUS_UL], vs[CENSUS_UL], vsn[CENSUS_UL];
#pragma unroll
    for (int t = 0; t < CENSUS_UL; ++t) {
        vm[t] = CROW(s_m, t);
        vs[t] = CROW(s_s, t);
        vsn[t] = vs[t] ^ vm[t];
    }
    const uint32_t nblocks = 1u << (n - CENSUS_UL);
    uint32_t ml = 0, sl = 0;
    int tally = 0;
    for (uint32_t b = 0; b < nblocks; ++b) {
        // the step closing block b enters index 16 (b + 1); the last block has none
        const uint32_t jb = b + 1;
        const bool closing = jb < nblocks;
        const int tb = closing ? CENSUS_UL + __builtin_ctz(jb) : 0;   // a row of the matrix either way
        const int sh = closing ? tb - CENSUS_UL + 1 : 0;
        const bool leave_b = closing && ((jb >> sh) & 1u);
        const uint32_t bm = closing ? CROW(s_m, tb) : 0u;
        const uint32_t bs0 = closing ? CROW(s_s, tb) : 0u;
        const uint32_t bs = leave_b ? (bs0 ^ bm) : bs0;
#pragma unroll
        for (int k = 1; k <= U; ++k) {
            uint32_t rm, rs;
            if (k < U) {
                const int t = __builtin_ctz(k);
                rm = vm[t];
                // the step into 16 b + k leaves the subset when bit t+1 of the index is set
                const bool leave = t + 1 < CENSUS_UL ? ((k >> (t + 1)) & 1) != 0 : (b & 1u) != 0;
                rs = leave ? vsn[t] : vs[t];
            } else {
                rm = bm;
                rs = bs;
            }
            bip_add(ml, sl, rm, rs);
            // the index 16 b + k has the parity of k
            const int odd = (__builtin_popcount(sl) + k) & 1;
            const int term = odd ? -1 : 1;
            const bool exists = k < U || closing;   // the last block ends at index 2^n - 1
            tally += exists && ml == mask ? term : 0;
        }
    }
    return tally;
}

__global__ void __launch_bounds__(CENSUS_BLOCK) k_census_lanes(CensusArgs a)
{
    extern __shared__ uint32_t s_rows[];
    const int n = a.n;
    uint32_t *s_m = s_rows, *s_s = s_rows + n * CENSUS_BLOCK;
    const int nn = n * n;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    // each lane takes a run of consecutive matrices: after the first, the next
    // matrix comes from the last by a base-3 increment of its entries
    // (enumeration) or by carrying on with the generator's state (SplitMix64)
    const uint64_t lanes = (uint64_t)gridDim.x * CENSUS_BLOCK;
    const uint64_t per = (a.count + lanes - 1) / lanes;
    const uint64_t begin = ((uint64_t)blockIdx.x * CENSUS_BLOCK + tid) * per;
    const uint32_t mask = (1u << n) - 1u;
    unsigned long long c0 = 0, c1 = 0, c2 = 0;
    uint64_t x = 0;   // SplitMix64 state of the lane's next entry
    for (uint64_t r = 0; r < per; ++r) {
        const uint64_t idx = begin + r;
        const bool active = idx < a.count;
        if (active && (r == 0 || a.gen != GEN_ENUMERATE)) {
            // the matrix from scratch, packed by phi: element j of row i at bit n-1-j
            const uint64_t t = a.first + idx;
            uint64_t rest = t;
            if (r == 0) x = a.key + (t * (uint64_t)nn + 1u) * SPLITMIX_GAMMA;
            for (int i = 0; i < n; ++i) {
                uint32_t mag = 0, sgn = 0;
                for (int j = 0; j < n; ++j) {
                    uint32_t v;
                    if (a.gen == GEN_ENUMERATE) {
                        const uint64_t q = rest / 3u;
                        v = (uint32_t)(rest - 3u * q);
                        rest = q;
                    } else {
                        v = trit_of(splitmix_mix(x));
                        x += SPLITMIX_GAMMA;
                    }
                    const uint32_t bit = 1u << (n - 1 - j);
                    mag |= v != 0 ? bit : 0u;
                    sgn |= v == 2 ? bit : 0u;
                }
                CROW(s_m, i) = mag;
                CROW(s_s, i) = sgn;
            }
        } else if (active) {
            // t = t_prev + 1: add 1 to the base-3 number whose digit k is entry k
            // (row-major); a digit 2 (-1) becomes 0 and carries
            for (int i = 0; i < n; ++i) {
                uint32_t m = CROW(s_m, i), sg = CROW(s_s, i);
                bool carry = true;
                for (int j = 0; j < n && carry; ++j) {
                    const uint32_t bit = 1u << (n - 1 - j);
                    if (!(m & bit)) {
                        m |= bit;                  // 0 -> 1
                        carry = false;
                    } else if (!(sg & bit)) {
                        sg |= bit;                 // 1 -> 2
                        carry = false;
                    } else {
                        m &= ~bit;                 // 2 -> 0
                        sg &= ~bit;
                    }
                }
                CROW(s_m, i) = m;
                CROW(s_s, i) = sg;
                if (!carry) break;
            }
        }
        const int tally = n > CENSUS_UL ? census_walk_blocks(n, mask, tid, s_m, s_s) : census_walk_plain(n, mask, tid, s_m, s_s);
        const int p = (n & 1) ? -tally : tally;
        int res = p % 3;
        if (res < 0) res += 3;
        const unsigned long long b0 = __ballot(active && res == 0);
        const unsigned long long b1 = __ballot(active && res == 1);
        const unsigned long long b2 = __ballot(active && res == 2);
        if (lane == 0) {
            c0 += __popcll(b0);
            c1 += __popcll(b1);
            c2 += __popcll(b2);
        }
    }
    if (lane == 0) {
        if (c0) atomicAdd(&a.counts[0], c0);
        if (c1) atomicAdd(&a.counts[1], c1);
        if (c2) atomicAdd(&a.counts[2], c2);
    }
}

__global__ void __launch_bounds__(256) k_generate(GenArgs a)
{
    const uint32_t idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= a.count) return;
    const int n = a.n;
    const int nn = n * n;
    const uint64_t t = a.first + idx;
    uint64_t rest = t;
    uint8_t *dst = a.mats + (uint64_t)idx * nn;
    for (int k = 0; k < nn; ++k) dst[k] = (uint8_t)census_entry(a.gen, a.key, t, nn, k, rest);
    a.offs[idx] = (int64_t)idx * nn;
    a.ns[idx] = n;
}

hipError_t launch_census_lanes(const CensusArgs &a, int grid_blocks, hipStream_t st)
{
    if (a.n < 1 || a.n > CENSUS_LANE_MAX_N) return hipErrorInvalidValue;
    const size_t lds = 2u * (size_t)a.n * CENSUS_BLOCK * sizeof(uint32_t);   // at most 40 KiB
    hipLaunchKernelGGL(k_census_lanes, dim3(grid_blocks), dim3(CENSUS_BLOCK), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_generate(const GenArgs &a, hipStream_t st)
{
    if (a.count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_generate, dim3((a.count + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace perm3
