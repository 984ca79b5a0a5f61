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
// Gray steps of its matrix (the rows sit in LDS, one column of words per lane;
// all lanes flip the same row at the same step), with every index tested for
// small n (k_census_lanes) and, from CENSUS_FILTER_MIN_N on, a block of 16
// indices tested at once and re-walked exactly only when it holds a candidate
// (k_census_filtered); it forms ((-1)^n T) mod 3, and the wave counts results
// 0, 1 and 2 with ballots.
// Larger n: k_generate writes the matrices and the batch walk takes them.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

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
    // the row closing block b is read one block ahead (rows 4 .. n-1 exist: n > 4)
    uint32_t next_m = CROW(s_m, CENSUS_UL), next_s = CROW(s_s, CENSUS_UL);
    for (uint32_t b = 0; b < nblocks; ++b) {
        // the step closing block b enters index 16 (b + 1); the last block has none
        const uint32_t jb = b + 1;
        const bool closing = jb < nblocks;
        const int tb = closing ? CENSUS_UL + __builtin_ctz(jb) : CENSUS_UL;
        const int sh = tb - CENSUS_UL + 1;
        const bool leave_b = closing && ((jb >> sh) & 1u);
        const uint32_t bm = closing ? next_m : 0u;
        const uint32_t bs0 = closing ? next_s : 0u;
        if (jb + 1 < nblocks) {
            const int tn = CENSUS_UL + __builtin_ctz(jb + 1);
            next_m = CROW(s_m, tn);
            next_s = CROW(s_s, tn);
        }
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

// From this n on (SplitMix64 matrices) the lanes test a block's 16 indices at
// once and re-walk only the blocks that hold a candidate.  Below it an index is
// a candidate so often ((2/3)^n) that the re-walks cost more than testing
// every index (n = 8 breaks even, n = 7 loses 6%, n = 9 gains 11%).
constexpr int CENSUS_FILTER_MIN_N = 9;
// A wave's list of candidate blocks: re-walked 64 at a time, one per lane.
constexpr int CENSUS_CAND_CAP = 128;

struct CensusCand {
    uint32_t ml, sl;   // the Gray state at the block's first index, 16 b
    uint32_t tag;      // the lane whose matrix it is, from bit 26; the block b below
};

// The filtered lanes keep rows 0..3 of their matrix in registers (another
// lane's come by a shuffle) and rows 4..n-1 in LDS: row i of lane tid at
// [(i - 4) * CENSUS_BLOCK + tid].
#define FROW(a, i, who) (a)[((i) - CENSUS_UL) * CENSUS_BLOCK + (who)]

// The exact walk of entries list[0 .. cnt) (cnt <= 64), lane j taking entry j:
// indices 16 b .. 16 b + 15 from the saved state at 16 b, with rows 0..3 of the
// lane the block belongs to (from that lane's registers), every index tested.
// Each entry's tally is added to that lane's word in s_tally.  Every lane of
// the wave calls it.
__device__ __forceinline__ void census_flush(uint32_t mask, int wave_base, int lane,
                                             const uint32_t (&r_m)[CENSUS_UL], const uint32_t (&r_s)[CENSUS_UL],
                                             const CensusCand *list, uint32_t cnt, int *s_tally)
{
    PERM3_WAVE_LDS_SYNC();
    // entries at and above cnt are stale but inside the list: read, never used
    const CensusCand e = list[lane];
    const int src_lane = (int)(e.tag >> 26);
    uint32_t vm[CENSUS_UL], vs[CENSUS_UL], vsn[CENSUS_UL];
#pragma unroll
    for (int t = 0; t < CENSUS_UL; ++t) {
        vm[t] = PERM3_SHFL32(r_m[t], src_lane);
        vs[t] = PERM3_SHFL32(r_s[t], src_lane);
        vsn[t] = vs[t] ^ vm[t];
    }
    if ((uint32_t)lane < cnt) {
        const uint32_t b = e.tag & ((1u << 26) - 1u);
        uint32_t ml = e.ml, sl = e.sl;
        // the index 16 b + k has the parity of k
        int part = ml == mask ? ((__builtin_popcount(sl) & 1) ? -1 : 1) : 0;
#pragma unroll
        for (int k = 1; k < (1 << CENSUS_UL); ++k) {
            const int t = __builtin_ctz(k);
            const bool leave = t + 1 < CENSUS_UL ? ((k >> (t + 1)) & 1) != 0 : (b & 1u) != 0;
            bip_add(ml, sl, vm[t], leave ? vsn[t] : vs[t]);
            const int odd = (__builtin_popcount(sl) + k) & 1;
            part += ml == mask ? (odd ? -1 : 1) : 0;
        }
        if (part) atomicAdd(&s_tally[wave_base + src_lane], part);
    }
    PERM3_WAVE_LDS_SYNC();
}

// The Ryser tally of the lane's matrix for CENSUS_FILTER_MIN_N <= n, in
// blocks of 16 Gray indices: the subset sums of block b are H_b + L_k, with
// H_b the block's sum over rows 4..n-1 (one Gray step from block to block,
// its row read from LDS one block ahead) and L_k the sums of the lane's rows
// 0..3 over g(k), the same for every block (an odd block meets them in
// reverse order).  A block holds a non-zero term only if the largest mag
// word of its 16 states equals the mask of n columns (the rows have no bit at
// or above n), and the mag word of H + L_k takes two 3-input ops by Theorem
// 2.1.  Such a block is noted (the Gray state at its first index: H_b, plus
// row 3 when b is odd) in the wave's list; once 64 are noted, the wave
// re-walks them exactly, one per lane, whichever lane's matrix each belongs
// to.  The lane's tally is left in s_tally[tid] once the wave is through.
__device__ __forceinline__ void census_walk_filtered(int n, uint32_t mask, int tid, bool active,
                                                     const uint32_t (&r_m)[CENSUS_UL],
                                                     const uint32_t (&r_s)[CENSUS_UL], const uint32_t *s_m,
                                                     const uint32_t *s_s, CensusCand *list, int *s_tally)
{
    constexpr int U = 1 << CENSUS_UL;
    const int lane = tid & 63;
    const int wave_base = tid & ~63;
    LowSums<CENSUS_UL> lr;
    {
        uint32_t mm = 0, ss = 0;
        lr.p[0] = 0;
#pragma unroll
        for (int k = 1; k < U; ++k) {
            const int t = __builtin_ctz(k);
            const bool leave = ((k >> (t + 1)) & 1) != 0;
            bip_add(mm, ss, r_m[t], leave ? (r_s[t] ^ r_m[t]) : r_s[t]);
            uint64_t pk = ((uint64_t)mm << 32) | ss;   // {s_L low, m_L high}, as the main walk
            PERM3_PIN_PAIR(pk);
            lr.p[k] = pk;
        }
    }
    s_tally[tid] = 0;
    const uint32_t nblocks = 1u << (n - CENSUS_UL);
    uint64_t hp = 0;   // H_0: the empty subset
    PERM3_PIN_PAIR(hp);
    uint32_t ncand = 0;
    // the row of the step into block b + 1 is read from LDS one block ahead
    uint32_t next_m = FROW(s_m, CENSUS_UL, tid), next_s = FROW(s_s, CENSUS_UL, tid);
    for (uint32_t b = 0; b < nblocks; ++b) {
        const uint32_t jb = b + 1;
        const bool closing = jb < nblocks;
        const int tb = closing ? CENSUS_UL + __builtin_ctz(jb) : CENSUS_UL;
        const bool leave_b = closing && ((jb >> (tb - CENSUS_UL + 1)) & 1u);
        const uint32_t bm = closing ? next_m : 0u;
        const uint32_t bs0 = closing ? next_s : 0u;
        if (jb + 1 < nblocks) {
            const int tn = CENSUS_UL + __builtin_ctz(jb + 1);
            next_m = FROW(s_m, tn, tid);
            next_s = FROW(s_s, tn, tid);
        }
        const uint32_t bs = leave_b ? (bs0 ^ bm) : bs0;
        uint32_t mh = (uint32_t)hp, sh = (uint32_t)(hp >> 32);
        uint32_t v[U];
        v[0] = mh;
#pragma unroll
        for (int k = 1; k < U; ++k) {
            const uint32_t sl = (uint32_t)lr.p[k], ml = (uint32_t)(lr.p[k] >> 32);
            v[k] = PERM3_BITOP3(PERM3_BITOP3(mh, sh, sl, TT_XOR3), mh, ml, TT_AC_OR_BXC);
        }
        const uint32_t acc = max_tree<U>(v);
        const bool cand = active && acc == mask;
        const uint64_t cands = PERM3_BALLOT(cand);
        if (cands) {
            if (cand) {
                CensusCand e;
                e.ml = mh;
                e.sl = sh;
                if (b & 1u) bip_add(e.ml, e.sl, r_m[CENSUS_UL - 1], r_s[CENSUS_UL - 1]);
                e.tag = ((uint32_t)lane << 26) | b;
                list[ncand + PERM3_RANK(cands)] = e;
            }
            ncand += (uint32_t)__builtin_popcountll(cands);
            if (ncand >= 64) {
                ncand -= 64;
                census_flush(mask, wave_base, lane, r_m, r_s, list + ncand, 64, s_tally);
            }
        }
        bip_add(mh, sh, bm, bs);   // the last block adds a zero row: H stays put
        hp = ((uint64_t)sh << 32) | mh;
        PERM3_PIN_PAIR(hp);
    }
    if (ncand) census_flush(mask, wave_base, lane, r_m, r_s, list, ncand, s_tally);
}

// One row of a SplitMix64 matrix, packed by phi (element j at bit n-1-j),
// continuing the generator's state x.
__device__ __forceinline__ void splitmix_row(int n, uint64_t &x, uint32_t &mag, uint32_t &sgn)
{
    mag = 0;
    sgn = 0;
    for (int j = 0; j < n; ++j) {
        const uint32_t v = trit_of(splitmix_mix(x));
        x += SPLITMIX_GAMMA;
        const uint32_t bit = 1u << (n - 1 - j);
        mag |= v != 0 ? bit : 0u;
        sgn |= v == 2 ? bit : 0u;
    }
}

// k_census_lanes for SplitMix64 matrices with CENSUS_FILTER_MIN_N <= n <=
// CENSUS_LANE_MAX_N, through the filtered walk.
__global__ void __launch_bounds__(CENSUS_BLOCK) k_census_filtered(CensusArgs a)
{
    extern __shared__ uint32_t s_rows[];
    __shared__ CensusCand s_cand[CENSUS_BLOCK / 64][CENSUS_CAND_CAP];
    __shared__ int s_tally[CENSUS_BLOCK];
    const int n = a.n;
    const int nr = n - CENSUS_UL;
    uint32_t *s_m = s_rows, *s_s = s_rows + nr * CENSUS_BLOCK;
    const int nn = n * n;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const uint64_t lanes = (uint64_t)gridDim.x * CENSUS_BLOCK;
    const uint64_t per = (a.count + lanes - 1) / lanes;
    const uint64_t begin = ((uint64_t)blockIdx.x * CENSUS_BLOCK + tid) * per;
    const uint32_t mask = (1u << n) - 1u;
    unsigned long long c0 = 0, c1 = 0, c2 = 0;
    uint32_t r_m[CENSUS_UL] = {0, 0, 0, 0}, r_s[CENSUS_UL] = {0, 0, 0, 0};
    uint64_t x = 0;
    for (uint64_t r = 0; r < per; ++r) {
        const uint64_t idx = begin + r;
        const bool active = idx < a.count;
        if (active) {
            // matrix t's entries are outputs t n^2 + 1 .. (t+1) n^2: a lane's
            // run of consecutive matrices continues one stream
            if (r == 0) x = a.key + ((a.first + idx) * (uint64_t)nn + 1u) * SPLITMIX_GAMMA;
#pragma unroll
            for (int i = 0; i < CENSUS_UL; ++i) splitmix_row(n, x, r_m[i], r_s[i]);
            for (int i = CENSUS_UL; i < n; ++i) {
                uint32_t mag, sgn;
                splitmix_row(n, x, mag, sgn);
                FROW(s_m, i, tid) = mag;
                FROW(s_s, i, tid) = sgn;
            }
        }
        census_walk_filtered(n, mask, tid, active, r_m, r_s, s_m, s_s, s_cand[tid >> 6], s_tally);
        const int tally = s_tally[tid];
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
        // every lane's reads of this matrix's rows are done before it writes the next
        PERM3_WAVE_LDS_SYNC();
    }
    if (lane == 0) {
        if (c0) atomicAdd(&a.counts[0], c0);
        if (c1) atomicAdd(&a.counts[1], c1);
        if (c2) atomicAdd(&a.counts[2], c2);
    }
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

// ---------------------------------------------------------------- enumeration, 27 matrices a lane

// Enumerated matrices come in groups of 27: matrices 27 g .. 27 g + 26 share
// every base-3 digit but their three lowest (entries 0, 1 and 2 of row 0),
// which run through all 27 combinations.  So a lane holds a group
// bit-sliced: bit q of a word belongs to matrix 27 g + q, entry k of all 27
// is one (mag, sgn) word pair (a fixed pattern for k < 3, all ones or all
// zeros from digit k - 3 of g otherwise), and each column sum of the Gray
// walk is one word pair as well.  A Gray step adds or subtracts one row to
// the n column sums (n Theorem 2.1 operations), a term needs every column
// sum non-zero (an AND over the n mag words) and its sign is the parity of
// the negative ones (an XOR over the n sgn words) and of the index, and the
// 27 tallies mod 3 are kept as one more word pair.  One step costs about 4n
// word operations for 27 matrices.
constexpr int SLICE = 27;

// mag and sgn patterns of base-3 digit r (r < 3) over q = 0 .. 26
__host__ __device__ constexpr uint32_t slice_pattern(int r, bool sgn)
{
    uint32_t w = 0;
    for (int q = 0; q < SLICE; ++q) {
        const int d = (r == 0 ? q : (r == 1 ? q / 3 : q / 9)) % 3;
        if (sgn ? d == 2 : d != 0) w |= 1u << q;
    }
    return w;
}

// Theorem 2.1 subtraction in three 3-input ops: x = m1 & (s1 ^ s2),
// mag = x | (m1 ^ m2), sgn = x ^ m2 ^ s2.
constexpr uint32_t TT_A_AND_BXC = (0xF0 & (0xCC ^ 0xAA)) & 0xFF;
constexpr uint32_t TT_A_OR_BXC = (0xF0 | (0xCC ^ 0xAA)) & 0xFF;
__device__ __forceinline__ void f3_sub(uint32_t &m1, uint32_t &s1, uint32_t m2, uint32_t s2)
{
    const uint32_t x = PERM3_BITOP3(m1, s1, s2, TT_A_AND_BXC);
    const uint32_t mo = PERM3_BITOP3(x, m1, m2, TT_A_OR_BXC);
    s1 = PERM3_BITOP3(x, m2, s2, TT_XOR3);
    m1 = mo;
}

constexpr uint32_t TT_AND3 = (0xF0 & 0xCC & 0xAA) & 0xFF;

// k_census_lanes for the enumeration generator (n = N <= 6), a group of 27
// matrices per lane step: counts of perm = 0, 1, 2 over matrices
// first .. first + count - 1.
template <int N>
__global__ void __launch_bounds__(CENSUS_BLOCK) k_census_sliced(CensusArgs a)
{
    constexpr int NN = N * N;
    constexpr int ND = NN > 3 ? NN - 3 : 0;     // digits of the group number g
    const int lane = threadIdx.x & 63;
    const uint64_t g_first = a.first / SLICE;
    const uint64_t g_last = (a.first + a.count - 1) / SLICE;
    const uint64_t groups = g_last - g_first + 1;
    const uint64_t lanes = (uint64_t)gridDim.x * CENSUS_BLOCK;
    const uint64_t per = (groups + lanes - 1) / lanes;
    const uint64_t g0 = g_first + ((uint64_t)blockIdx.x * CENSUS_BLOCK + threadIdx.x) * per;
    const uint64_t g1 = g0 + per < g_last + 1 ? g0 + per : g_last + 1;
    unsigned long long c0 = 0, c1 = 0, c2 = 0;
    // digit d of g as bit d of dm (digit != 0) and of ds (digit == 2)
    uint64_t dm = 0, ds = 0;
    {
        uint64_t rest = g0;
        for (int d = 0; d < ND; ++d) {
            const uint64_t q = rest / 3u;
            const uint32_t v = (uint32_t)(rest - 3u * q);
            rest = q;
            dm |= (uint64_t)(v != 0) << d;
            ds |= (uint64_t)(v == 2) << d;
        }
    }
    for (uint64_t g = g0; g < g1; ++g) {
        // entry words: k < 3 a fixed pattern, else all ones or zeros from digit k - 3
        uint32_t em[NN], es[NN];
#pragma unroll
        for (int k = 0; k < NN; ++k) {
            if (k < 3) {
                em[k] = slice_pattern(k, false);
                es[k] = slice_pattern(k, true);
            } else {
                const int d = k - 3;
                const uint32_t wm = (uint32_t)(dm >> (d & 32)), ws = (uint32_t)(ds >> (d & 32));
                em[k] = (uint32_t)(-(int32_t)((wm >> (d & 31)) & 1u));
                es[k] = (uint32_t)(-(int32_t)((ws >> (d & 31)) & 1u));
            }
        }
        // the Gray walk over all 2^N subsets of rows from the empty one; the
        // column sums start at zero and index 0's term is 0
        uint32_t cm[N], cs[N];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            cm[j] = 0;
            cs[j] = 0;
        }
        uint32_t tm = 0, ts = 0;
#pragma unroll
        for (int i = 1; i < (1 << N); ++i) {
            const int t = __builtin_ctz(i);
            const bool leave = (i >> (t + 1)) & 1;    // row t leaves the subset
#pragma unroll
            for (int j = 0; j < N; ++j) {
                if (leave)
                    f3_sub(cm[j], cs[j], em[t * N + j], es[t * N + j]);
                else
                    bip_add(cm[j], cs[j], em[t * N + j], es[t * N + j]);
            }
            // every column sum non-zero, and the parity of the negative ones
            uint32_t hit = cm[0], sx = cs[0];
            int j = 1;
#pragma unroll
            for (; j + 1 < N; j += 2) {
                hit = PERM3_BITOP3(hit, cm[j], cm[j + 1], TT_AND3);
                sx = PERM3_BITOP3(sx, cs[j], cs[j + 1], TT_XOR3);
            }
            if (j < N) {
                hit &= cm[j];
                sx ^= cs[j];
            }
            // the term is (-1)^(negative sums + i): add it to the tallies mod 3
            const uint32_t neg = (i & 1) ? ~sx : sx;
            bip_add(tm, ts, hit, hit & neg);
        }
        // perm = (-1)^N T; the valid matrices of the group
        const uint64_t base = g * SLICE;
        const uint64_t lo = a.first > base ? a.first - base : 0;
        const uint64_t end = a.first + a.count;
        const uint64_t hi = end < base + SLICE ? end - base : SLICE;
        const uint32_t valid = (uint32_t)(((1ull << hi) - 1ull) & ~((1ull << lo) - 1ull));
        const uint32_t minus = (N & 1) ? (tm & ~ts) : (tm & ts);
        c0 += (unsigned long long)__builtin_popcount(valid & ~tm);
        c2 += (unsigned long long)__builtin_popcount(valid & minus);
        c1 += (unsigned long long)__builtin_popcount(valid & tm & ~minus);
        // g + 1: digits 2 roll over to 0 up to the first digit below 2, which grows
        const uint64_t twos = dm & ds;
        const int c = __builtin_ctzll(~twos);
        const uint64_t below = c >= 64 ? ~0ull : ((1ull << c) - 1ull);
        dm &= ~below;
        ds &= ~below;
        if (c < 64) {
            const uint64_t bit = 1ull << c;
            if (dm & bit)
                ds |= bit;
            else
                dm |= bit;
        }
    }
    // the wave's counts to its first lane, then one atomic each
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        c0 += (unsigned long long)__shfl_xor((long long)c0, off);
        c1 += (unsigned long long)__shfl_xor((long long)c1, off);
        c2 += (unsigned long long)__shfl_xor((long long)c2, off);
    }
    if (lane == 0) {
        if (c0) atomicAdd(&a.counts[0], c0);
        if (c1) atomicAdd(&a.counts[1], c1);
        if (c2) atomicAdd(&a.counts[2], c2);
    }
}

hipError_t launch_census_lanes(const CensusArgs &a, int cus, hipStream_t st)
{
    if (a.n < 1 || a.n > CENSUS_LANE_MAX_N) return hipErrorInvalidValue;
    if (a.gen == GEN_ENUMERATE) {
        if (a.n > 6) return hipErrorInvalidValue;
        const void *ks[6] = {(const void *)k_census_sliced<1>, (const void *)k_census_sliced<2>,
                             (const void *)k_census_sliced<3>, (const void *)k_census_sliced<4>,
                             (const void *)k_census_sliced<5>, (const void *)k_census_sliced<6>};
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ks[a.n - 1], CENSUS_BLOCK, 0);
        if (e != hipSuccess) return e;
        if (per_cu < 1) per_cu = 1;
        const uint64_t groups = (a.first + a.count - 1) / SLICE - a.first / SLICE + 1;
        const uint64_t want = (groups + CENSUS_BLOCK - 1) / CENSUS_BLOCK;
        const int blocks = (int)std::min<uint64_t>(want, (uint64_t)cus * per_cu);
        switch (a.n) {
        case 1: hipLaunchKernelGGL(k_census_sliced<1>, dim3(blocks), dim3(CENSUS_BLOCK), 0, st, a); break;
        case 2: hipLaunchKernelGGL(k_census_sliced<2>, dim3(blocks), dim3(CENSUS_BLOCK), 0, st, a); break;
        case 3: hipLaunchKernelGGL(k_census_sliced<3>, dim3(blocks), dim3(CENSUS_BLOCK), 0, st, a); break;
        case 4: hipLaunchKernelGGL(k_census_sliced<4>, dim3(blocks), dim3(CENSUS_BLOCK), 0, st, a); break;
        case 5: hipLaunchKernelGGL(k_census_sliced<5>, dim3(blocks), dim3(CENSUS_BLOCK), 0, st, a); break;
        default: hipLaunchKernelGGL(k_census_sliced<6>, dim3(blocks), dim3(CENSUS_BLOCK), 0, st, a); break;
        }
        return hipGetLastError();
    }
    const bool filtered = a.gen == GEN_SPLITMIX && a.n >= CENSUS_FILTER_MIN_N;
    const int rows = filtered ? a.n - CENSUS_UL : a.n;
    const size_t lds = 2u * (size_t)rows * CENSUS_BLOCK * sizeof(uint32_t);   // at most 32 KiB
    // every lane takes an equal run of matrices, so the grid is what stays
    // resident at once (LDS bounds it for large n)
    int per_cu = 0;
    hipError_t e = filtered ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_census_filtered, CENSUS_BLOCK, lds)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_census_lanes, CENSUS_BLOCK, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    const uint64_t want = (a.count + CENSUS_BLOCK - 1) / CENSUS_BLOCK;
    const int blocks = (int)std::min<uint64_t>(want, (uint64_t)cus * per_cu);
    if (filtered)
        hipLaunchKernelGGL(k_census_filtered, dim3(blocks), dim3(CENSUS_BLOCK), lds, st, a);
    else
        hipLaunchKernelGGL(k_census_lanes, dim3(blocks), dim3(CENSUS_BLOCK), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_generate(const GenArgs &a, hipStream_t st)
{
    if (a.count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_generate, dim3((a.count + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace perm3
