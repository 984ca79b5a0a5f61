// Per-lane Gray-code walk over bipedal rows (gfx950 device code).
//
// A matrix row over F_3 is held as two F_2^n words (mag, sgn) under phi
// (Section 2).  Columns beyond bit 31 live in a second 32-bit "hi" word, so
// n <= 63 uses at most two words per plane.  Each row is stored as
//     { m_lo, s_lo, sn_lo, -, m_hi, s_hi, sn_hi, - }
// where sn = s xor m is the sgn word of the NEGATED row: subtracting a row is
// adding its negation, and negating a bipedal vector flips sgn exactly where
// mag is set (every zero, (0,0) or (0,1), stays a zero).  Matrices of up to
// 128 columns (two 64-bit words per plane, the widest case Section 3 names)
// use RowX and 128-bit Gray indices; the walk itself only ever carries the
// low word, so its cost per index does not grow with the width.
//
// Gray order (Section 3, RBC footnote): index i has subset g(i) = i ^ (i >> 1);
// the step into i flips row t = ctz(i), which leaves the subset (subtract)
// when bit t of g(i-1) is set, i.e. when bit t+1 of i is set.  The Ryser term
// of index i is (-1)^|g(i)| times the product of the column sums; |g(i)| has
// the parity of i, and the product is non-zero exactly when every mag bit is
// set, in which case it is (-1)^popcount(sgn) (Section 3).
#pragma once

#include <stdint.h>

#ifndef PERM3_FN
#define PERM3_FN __device__ __forceinline__
#endif
#ifndef PERM3_BITOP3
#define PERM3_BITOP3(a, b, c, tt) __builtin_amdgcn_bitop3_b32((a), (b), (c), (tt))
#endif
// A value every active lane of the wave holds alike, made a scalar so that
// the row it indexes is read with scalar loads.
#ifndef PERM3_UNIFORM
#define PERM3_UNIFORM(x) __builtin_amdgcn_readfirstlane(x)
#endif
// Wave-level primitives of the deferred re-walks: a ballot over the active
// lanes, this lane's index, the number of set bits of a lane mask below this
// lane, a 32-bit value read from another lane, and the ordering of a wave's
// LDS accesses (entries one lane writes are read by another).
#ifndef PERM3_BALLOT
#define PERM3_BALLOT(p) ((uint64_t)__ballot(p))
#define PERM3_LANE() ((int)__lane_id())
#define PERM3_RANK(mask) \
    ((uint32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)((mask) >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)(mask), 0u)))
#define PERM3_SHFL32(v, src) ((uint32_t)__shfl((int)(v), (src)))
#define PERM3_WAVE_LDS_SYNC()                                  \
    do {                                                       \
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront"); \
        __builtin_amdgcn_wave_barrier();                       \
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront"); \
    } while (0)
#endif

namespace perm3 {

struct RowW {
    uint32_t m_lo, s_lo, sn_lo, pad0;
    uint32_t m_hi, s_hi, sn_hi, pad1;
};

// A row of a matrix with up to 128 columns: the walk's low word as in RowW,
// then the mag and sgn words of columns 32 .. 127.
struct RowX {
    uint32_t m_lo, s_lo, sn_lo, pad0;
    uint32_t m_w[3], pad1;
    uint32_t s_w[3], pad2;
};

typedef unsigned __int128 u128;

// Truth-table immediates for v_bitop3_b32(A, B, C): bit (4A + 2B + C) of the
// immediate is the output, so A = 0xF0, B = 0xCC, C = 0xAA as bit patterns.
constexpr uint32_t TT_XOR3 = 0xF0 ^ 0xCC ^ 0xAA;                  // A ^ B ^ C
constexpr uint32_t TT_AC_OR_BXC = ((0xF0 & 0xAA) | (0xCC ^ 0xAA)) & 0xFF;  // (A & C) | (B ^ C)
constexpr uint32_t TT_AC_XOR_B = ((0xF0 & 0xAA) ^ 0xCC) & 0xFF;            // (A & C) ^ B

// Theorem 2.1, addition: with x = m2 & (m1 ^ s1 ^ s2),
//   mag+ = x | (m1 ^ m2),  sgn+ = x ^ s1.
// Three 3-input ops; the row words (m2, s2) are wave-uniform, so each op
// reads at most one scalar register.
PERM3_FN void bip_add(uint32_t &m1, uint32_t &s1, uint32_t m2, uint32_t s2)
{
    const uint32_t y = PERM3_BITOP3(m1, s1, s2, TT_XOR3);     // m1 ^ s1 ^ s2
    const uint32_t mo = PERM3_BITOP3(y, m1, m2, TT_AC_OR_BXC); // (m2 & y) | (m1 ^ m2)
    s1 = PERM3_BITOP3(y, s1, m2, TT_AC_XOR_B);                // (m2 & y) ^ s1
    m1 = mo;
}

// Theorem 2.1, subtraction, as printed (used by the self-check kernel; the
// walk subtracts by adding the negated row instead).
PERM3_FN void bip_sub(uint32_t &m1, uint32_t &s1, uint32_t m2, uint32_t s2)
{
    const uint32_t x = m1 & (s1 ^ s2);
    const uint32_t mo = x | (m1 ^ m2);
    s1 = x ^ (m2 ^ s2);
    m1 = mo;
}

struct Masks {
    uint32_t lo, hi;   // all-ones over the n columns, split into words
};

struct MasksX {
    uint32_t lo;       // columns 0 .. 31
    uint32_t w[3];     // columns 32 .. 127, word by word
    int nw;            // how many of w[] the matrix uses
};

// The Ryser term of Gray index i whose subset sum has low words (ml, sl):
// zero unless every column sum is non-zero.  The high words are not carried
// by the fast walk; when the low words pass, they are formed here from
// scratch by summing the rows of g(i) (rare: a (2/3)^32 event per index).
template <typename RP>
PERM3_FN int exact_term(RP R, int n, uint64_t i, uint32_t ml, uint32_t sl, Masks mk)
{
    if (ml != mk.lo) return 0;
    uint32_t mh = 0, sh = 0;
    if (n > 32) {
        const uint64_t g = i ^ (i >> 1);
        for (int k = 0; k < n; ++k)
            if ((g >> k) & 1u) bip_add(mh, sh, R[k].m_hi, R[k].s_hi);
        if (mh != mk.hi) return 0;
    }
    const int par = (__builtin_popcount(sl & mk.lo) + __builtin_popcount(sh & mk.hi) + (int)(i & 1u)) & 1;
    return par ? -1 : 1;
}

// The same for a matrix of up to 128 columns and a 128-bit Gray index: the
// words beyond the low one are formed from scratch one at a time, each tested
// before the next is built, from the rows of g(i) (visited by their set bits).
template <typename RP>
PERM3_FN int exact_term(RP R, int n, u128 i, uint32_t ml, uint32_t sl, const MasksX &mk)
{
    if (ml != mk.lo) return 0;
    const u128 g = i ^ (i >> 1);
    const uint64_t g0 = (uint64_t)g, g1 = (uint64_t)(g >> 64);
    int par = __builtin_popcount(sl & mk.lo) + (int)((uint32_t)i & 1u);
    for (int w = 0; w < mk.nw; ++w) {
        uint32_t mw = 0, sw = 0;
        for (uint64_t x = g0; x; x &= x - 1) {
            const int k = __builtin_ctzll(x);
            bip_add(mw, sw, R[k].m_w[w], R[k].s_w[w]);
        }
        for (uint64_t x = g1; x; x &= x - 1) {
            const int k = 64 + __builtin_ctzll(x);
            bip_add(mw, sw, R[k].m_w[w], R[k].s_w[w]);
        }
        if (mw != mk.w[w]) return 0;
        par += __builtin_popcount(sw & mk.w[w]);
    }
    (void)n;
    return (par & 1) ? -1 : 1;
}

// Low words of the subset sum of g(i0): jump straight to a Gray state
// (Section 3.1).  O(n) word operations per lane.
template <typename RP, typename I>
PERM3_FN void seed_lo(RP R, int n, I i0, uint32_t &ml, uint32_t &sl)
{
    const I g = i0 ^ (i0 >> 1);
    ml = 0;
    sl = 0;
    for (int k = 0; k < n; ++k) {
        const uint32_t sel = 0u - (uint32_t)((g >> k) & 1u);
        bip_add(ml, sl, R[k].m_lo & sel, R[k].s_lo & sel);
    }
}

// Static rows of the unrolled block: t = 0 .. UL-1, wave-uniform.
template <int UL>
struct StaticRows {
    uint32_t m[UL], s[UL], sn[UL];
};

template <int UL, typename RP>
PERM3_FN void load_static_rows(RP R, StaticRows<UL> &sr)
{
#pragma unroll
    for (int t = 0; t < UL; ++t) {
        sr.m[t] = R[t].m_lo;
        sr.s[t] = R[t].s_lo;
        sr.sn[t] = R[t].sn_lo;
    }
}

// A wave-uniform word moved into a vector register.  bitop3 with a scalar
// operand issues more slowly than with three vector operands on gfx950, so
// the rows the block adds are kept in VGPRs.
#ifndef PERM3_TO_VGPR
#define PERM3_TO_VGPR(x) perm3::to_vgpr(x)
PERM3_FN uint32_t to_vgpr(uint32_t x)
{
    uint32_t v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(x));
    return v;
}
#endif

// Exact re-walk of Gray indices ia+1 .. ib (ia itself already counted) for
// the lanes whose block held a candidate, from the low words (ml, sl) of the
// subset sum at ia; the high words are formed only where the low words pass.
// Indices ia+1 .. ib lie in one aligned chunk above its first index, so the
// flipped row and its direction come from the low 64 bits of i.  The loop
// stops on reaching ib rather than on i > ib: ib may be the largest index
// the type holds (the last index below 2^128).
template <typename RP, typename I, typename MK>
PERM3_FN int rewalk_exact(RP R, int n, I ia, I ib, uint32_t ml, uint32_t sl, const MK &mk)
{
    int tally = 0;
    for (I i = ia; i != ib;) {
        ++i;
        const uint64_t il = (uint64_t)i;
        const int t = __builtin_ctzll(il);
        const bool leave = (il >> (t + 1)) & 1u;
        bip_add(ml, sl, R[t].m_lo, leave ? R[t].sn_lo : R[t].s_lo);
        tally += exact_term(R, n, i, ml, sl, mk);
    }
    return tally;
}

// Exact re-walk of a block backwards: (ml, sl) is the low-word state at
// Gray index ib; indices ib, ib-1, .. ia+1 are tested, each step undone by
// adding back what the step into it removed (or removing what it added).  An
// undone step may leave a zero as (0,1) where the forward walk had (0,0); the
// test reads only mag and, where every mag bit is set, sgn, and neither
// depends on how a zero is represented.
//
// All lanes of a wave walk their chunks in step, so within a block every
// active lane is at the same offset: the flipped row and its direction (a
// block never contains the chunk's middle step, the only one whose direction
// differs between lanes) are wave-uniform and the rows come in by scalar
// loads.
template <typename RP, typename I, typename MK>
PERM3_FN int rewalk_back(RP R, int n, I ia, I ib, uint32_t ml, uint32_t sl, const MK &mk)
{
    int tally = 0;
    for (I i = ib; i != ia; --i) {
        tally += exact_term(R, n, i, ml, sl, mk);
        const uint32_t il = (uint32_t)i;                 // offsets within a chunk fit 32 bits
        const int t = PERM3_UNIFORM(__builtin_ctz(il));
        const bool left = PERM3_UNIFORM((il >> (t + 1)) & 1u);   // the step into i removed row t
        bip_add(ml, sl, R[t].m_lo, left ? R[t].s_lo : R[t].sn_lo);
    }
    return tally;
}

// Candidate blocks of a wave, re-walked later all together (one lane per
// block) instead of each by the whole wave at once: an entry holds the lane
// whose chunk it is (bits 26..31), whether the block ends on a boundary step
// (bit 25) and the block number (bits 0..24; blocks per chunk are at most
// 2^(24-4)).  Up to CAND_CAP entries per wave, in LDS; the walk kernels run
// 4 waves per workgroup.
constexpr uint32_t CAND_CAP = 128;
constexpr int CAND_WAVES = 4;

#ifndef PERM3_CAND_LIST
PERM3_FN uint32_t *cand_list()
{
    __shared__ uint32_t lists[CAND_WAVES][CAND_CAP];
    return lists[threadIdx.x >> 6];
}
#define PERM3_CAND_LIST() perm3::cand_list()
#endif

PERM3_FN uint64_t shfl_from(uint64_t v, int src)
{
    const uint32_t lo = PERM3_SHFL32((uint32_t)v, src);
    const uint32_t hi = PERM3_SHFL32((uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

PERM3_FN u128 shfl_from(u128 v, int src)
{
    const uint64_t lo = shfl_from((uint64_t)v, src);
    const uint64_t hi = shfl_from((uint64_t)(v >> 64), src);
    return ((u128)hi << 64) | lo;
}

// The exact terms of one candidate block, walked forward from the Gray state
// at its first index ia (a multiple of U = 2^UL): indices ia+1 .. ia+U-1 and,
// when the block closes on a boundary step (inner), ia+U.  Lanes re-walk
// different blocks side by side, all at the same offset k, so the row flipped
// at k < U is t = ctz(k) for every lane and comes in by a scalar load; its
// direction is bit t+1 of k, except at t = UL-1 where it is the parity of the
// lane's block number.  Only the closing step's row depends on the lane
// (t = UL + ctz(b+1)).
template <int UL, typename RP, typename I, typename MK>
PERM3_FN int rewalk_block(RP R, int n, I ia, uint32_t b, bool inner, uint32_t ml, uint32_t sl, const MK &mk)
{
    constexpr uint32_t U = 1u << UL;
    int tally = 0;
#pragma nounroll
    for (uint32_t k = 1; k < U; ++k) {
        const int t = PERM3_UNIFORM(__builtin_ctz(k));
        const bool leave = t < UL - 1 ? ((k >> (t + 1)) & 1u) != 0 : (b & 1u) != 0;
        bip_add(ml, sl, R[t].m_lo, leave ? R[t].sn_lo : R[t].s_lo);
        tally += exact_term(R, n, ia + (I)k, ml, sl, mk);
    }
    if (inner) {
        const uint32_t jb = b + 1;
        const int t = UL + __builtin_ctz(jb);
        const bool leave = ((jb >> (t + 1 - UL)) & 1u) != 0;
        bip_add(ml, sl, R[t].m_lo, leave ? R[t].sn_lo : R[t].s_lo);
        tally += exact_term(R, n, ia + (I)U, ml, sl, mk);
    }
    return tally;
}

// The exact terms of the candidate blocks a wave noted, list[0 .. ncand):
// every active lane takes entries in turn, jumps to the Gray state at its
// block's first index (Section 3.1) and re-walks the block (rewalk_block).
// A block then costs one lane instead of the whole wave.
template <int UL, int S, typename RP, typename I, typename MK>
PERM3_FN int flush_candidates(RP R, int n, int m, I c, const MK &mk, const uint32_t *list, uint32_t ncand)
{
    constexpr uint32_t U = 1u << UL;
    PERM3_WAVE_LDS_SYNC();
    const uint64_t act = PERM3_BALLOT(true);
    const uint32_t nact = (uint32_t)__builtin_popcountll(act);
    const uint32_t me = PERM3_RANK(act);
    int tally = 0;
    for (uint32_t base = 0; base < ncand; base += nact) {
        const uint32_t j = base + me;
        const uint32_t e = j < ncand ? list[j] : 0u;
        const I ce = shfl_from(c, (int)(e >> 26));   // every active lane takes part
        if (j < ncand) {
            const uint32_t b = e & 0x1FFFFFFu;
            const bool inner = ((e >> 25) & 1u) != 0;
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const I ia = ((ce + (I)(64u * q)) << m) + (I)(b * U);
                uint32_t ml, sl;
                seed_lo(R, n, ia, ml, sl);
                tally += rewalk_block<UL>(R, n, ia, b, inner, ml, sl, mk);
            }
        }
    }
    return tally;
}

// Fast walk of S whole aligned chunks c + 64 s (s = 0 .. S-1) of length
// 2^m, m > UL, carried side by side in one lane.
//
// Each chunk is cut into nb = 2^(m-UL) blocks of 2^UL indices.  Inside a
// block the flipped row t = ctz(offset) and its direction are compile-time
// constants except for the middle step (t = UL-1, direction = parity of the
// block number), so each index costs the three bitop3 of the addition, with
// the rows held in vector registers.  The step into the next block flips a
// row t >= UL chosen at run time; its row and direction are wave-uniform.
// The one step of a chunk whose direction differs between lanes (t = m-1,
// entering the second half; the row leaves the subset when the chunk index
// is odd) sits between the two halves' loops.  The last block of each half
// adds a zero row instead of a boundary step, which keeps the block body
// free of branches.  Chunks 64 apart have the same parity, so the S states
// take exactly the same row operations: S independent dependency chains.
//
// Candidates are found a block at a time: with bits >= n of every row zero,
// each low mag word is <= mk.lo, so the block's maximum equals mk.lo exactly
// when some index in it has all its low columns non-zero (one 3-input max
// per two states, or per two steps when S = 1).  Only then is the block
// walked again exactly: noted in the wave's candidate list and re-walked by
// one lane after the chunk (flush_candidates), or, when the list is full,
// at once by the whole wave, backwards from its end state (rewalk_back), so
// the block keeps no copy of the state it started from.
//
// AHEAD: the row of the step closing a block is loaded one block ahead, so
// that its load has a whole block to land; else at the block's start, where
// the wave waits for it.  Which is faster depends on how the register
// allocator then lays out the rest, so the caller picks: the persistent walk
// reads ahead (one matrix 2.7% faster; a batch 2.2% faster once re-tuned, 2.8%
// slower under its old tuning), so do the serving ticks (p99 6% lower) and the
// 128-column walk, there together with the deferred re-walks (8.5% faster on
// uniform matrices; either change alone made it slower); the one-launch small
// calls keep their code.
//
// The chunk index c is a uint64_t for n <= 63 and a u128 for wider matrices
// (with MasksX); only the seed and the exact terms see its high bits.
template <int UL, int S, bool DEFER, bool AHEAD, typename RP, typename I, typename MK>
PERM3_FN int walk_chunks_fast(RP R, int n, int m, I c, const MK &mk, const StaticRows<UL> &sr)
{
    static_assert(S == 1 || S == 2 || S == 4, "1, 2 or 4 states per lane");
    constexpr uint32_t U = 1u << UL;
    uint32_t ml[S], sl[S];
    int tally = 0;
#pragma unroll
    for (int q = 0; q < S; ++q) {
        const I i0 = (c + (I)(64u * q)) << m;
        seed_lo(R, n, i0, ml[q], sl[q]);
        tally += exact_term(R, n, i0, ml[q], sl[q], mk);
    }
    // static rows as vector registers
    uint32_t vm[UL], vs[UL], vsn[UL];
#pragma unroll
    for (int t = 0; t < UL; ++t) {
        vm[t] = PERM3_TO_VGPR(sr.m[t]);
        vs[t] = PERM3_TO_VGPR(sr.s[t]);
        vsn[t] = PERM3_TO_VGPR(sr.sn[t]);
    }
    uint32_t *const list = DEFER ? PERM3_CAND_LIST() : nullptr;
    const uint32_t lane_tag = (uint32_t)PERM3_LANE() << 26;
    uint32_t ncand = 0;
    const uint32_t half = 1u << (m - UL - 1);
    // The row added by the step into block j of a half ending at bend (a zero
    // row when j = bend; t = UL + ctz(j) <= m < n is in range even unused).
    auto closing_row = [&](uint32_t j, uint32_t bend, uint32_t &rm, uint32_t &rs) {
        const bool in = j < bend;
        const int t = UL + __builtin_ctz(j);
        const bool leave = (j >> (t + 1 - UL)) & 1u;
        rm = in ? R[t].m_lo : 0u;
        rs = in ? (leave ? R[t].sn_lo : R[t].s_lo) : 0u;
    };
    for (uint32_t h = 0; h < 2; ++h) {
        const uint32_t bend = (h + 1) * half;
        uint32_t next_m = 0, next_s = 0;
        if (AHEAD) closing_row(h * half + 1, bend, next_m, next_s);
        for (uint32_t b = h * half; b < bend; ++b) {
            // boundary step into block b+1 when it lies in this half (t < m-1)
            const uint32_t jb = b + 1;
            const bool inner = jb < bend;
            uint32_t bm, bs;
            if (AHEAD) {
                bm = PERM3_TO_VGPR(next_m);
                bs = PERM3_TO_VGPR(next_s);
                closing_row(jb + 1, bend, next_m, next_s);
            } else {
                const int tb = UL + __builtin_ctz(jb);      // <= m < n: in range even when unused
                const bool leave = (jb >> (tb + 1 - UL)) & 1u;
                bm = PERM3_TO_VGPR(inner ? R[tb].m_lo : 0u);
                bs = PERM3_TO_VGPR(inner ? (leave ? R[tb].sn_lo : R[tb].s_lo) : 0u);
            }
            uint32_t acc = 0;
#pragma unroll
            for (int k = 1; k <= (int)U; ++k) {
                uint32_t rm, rs;
                if (k < (int)U) {
                    const int t = __builtin_ctz(k);
                    rm = vm[t];
                    if (t < UL - 1)
                        rs = ((k >> (t + 1)) & 1) ? vsn[t] : vs[t];
                    else
                        rs = (b & 1u) ? vsn[t] : vs[t];
                } else {
                    rm = bm;
                    rs = bs;
                }
#pragma unroll
                for (int q = 0; q < S; ++q) bip_add(ml[q], sl[q], rm, rs);
                if (S == 1) {
                    acc = k == 1 ? ml[0] : (acc > ml[0] ? acc : ml[0]);
                } else {
                    // max(max(acc, a), b): one v_max3_u32 per pair of states
#pragma unroll
                    for (int q = 0; q < S; q += 2) {
                        const uint32_t x = acc > ml[q] ? acc : ml[q];
                        acc = x > ml[q + 1] ? x : ml[q + 1];
                    }
                }
            }
            const bool cand = acc == mk.lo;
            if (!DEFER) {
                if (cand) {
                    const uint32_t last = b * U + U - (inner ? 0u : 1u);
#pragma unroll
                    for (int q = 0; q < S; ++q) {
                        const I i0 = (c + (I)(64u * q)) << m;
                        tally += rewalk_back(R, n, i0 + b * U, i0 + last, ml[q], sl[q], mk);
                    }
                }
                continue;
            }
            const uint64_t cands = PERM3_BALLOT(cand);
            if (cands) {
                const uint32_t nc = (uint32_t)__builtin_popcountll(cands);
                if (ncand + nc <= CAND_CAP) {
                    if (cand) list[ncand + PERM3_RANK(cands)] = lane_tag | (inner ? 1u << 25 : 0u) | b;
                    ncand += nc;
                } else if (cand) {
                    const uint32_t last = b * U + U - (inner ? 0u : 1u);
#pragma unroll
                    for (int q = 0; q < S; ++q) {
                        const I i0 = (c + (I)(64u * q)) << m;
                        tally += rewalk_back(R, n, i0 + b * U, i0 + last, ml[q], sl[q], mk);
                    }
                }
            }
        }
        if (h == 0) {
            // offset L/2 flips row m-1
            const bool odd = (c & 1u) != 0;
            const uint32_t rm = R[m - 1].m_lo, rs = odd ? R[m - 1].sn_lo : R[m - 1].s_lo;
#pragma unroll
            for (int q = 0; q < S; ++q) {
                bip_add(ml[q], sl[q], rm, rs);
                tally += exact_term(R, n, ((c + (I)(64u * q)) << m) + (I)((uint64_t)half << UL), ml[q], sl[q], mk);
            }
        }
    }
    if (DEFER && ncand) tally += flush_candidates<UL, S>(R, n, m, c, mk, list, ncand);
    return tally;
}

// All-ones over the n columns of a matrix with up to 128 columns, word by word.
PERM3_FN MasksX masks_wide(int n)
{
    MasksX mk;
    mk.lo = n >= 32 ? 0xffffffffu : ((1u << n) - 1u);
    mk.nw = (n + 31) / 32 - 1;
    for (int w = 0; w < 3; ++w) {
        const int cols = n - 32 * (w + 1);
        mk.w[w] = cols >= 32 ? 0xffffffffu : (cols <= 0 ? 0u : ((1u << cols) - 1u));
    }
    return mk;
}

// One lane's chunk of a range of 128-bit Gray indices.  Chunk cr (counted
// from c0) covers [B + cr 2^m, B + (cr+1) 2^m) with B = c0 2^m, and the range
// is [B + off_lo, B + off_hi); offsets stay below 2^64, so a range may end at
// 2^128.  A whole chunk of a fast-mode matrix takes the unrolled walk; a
// ragged end (or a small matrix) is seeded at its first index and tests every
// index on the low word, forming the other words only where it passes.
template <int UL, bool DEFER, bool AHEAD, typename RP>
PERM3_FN int walk_lane_wide(RP R, int n, int m, bool fast, u128 c0, uint64_t off_lo, uint64_t off_hi,
                            uint64_t cr, const MasksX &mk, const StaticRows<UL> &sr)
{
    const uint64_t oa0 = cr << m;
    const uint64_t oe0 = oa0 + (1ull << m);
    const uint64_t oa = oa0 > off_lo ? oa0 : off_lo;
    const uint64_t oe = oe0 < off_hi ? oe0 : off_hi;
    if (oa >= oe) return 0;
    if (fast && oa == oa0 && oe == oe0) return walk_chunks_fast<UL, 1, DEFER, AHEAD>(R, n, m, c0 + cr, mk, sr);
    const u128 base = c0 << m;
    const u128 ia = base + oa;
    uint32_t ml, sl;
    seed_lo(R, n, ia, ml, sl);
    return exact_term(R, n, ia, ml, sl, mk) + rewalk_exact(R, n, ia, base + (oe - 1), ml, sl, mk);
}

// Exact walk of the whole aligned chunk c of length 2^m, both words carried
// and every index tested (small matrices).  The offset j within the chunk is
// the loop counter, the same in every lane walking a whole chunk, so the
// flipped row t = ctz(j) is wave-uniform and read with scalar loads; only the
// middle step (t = m-1, whose direction is the chunk index's parity) selects
// the row's sign word per lane.
template <bool HI, typename RP>
PERM3_FN int walk_chunk_direct(RP R, int n, int m, uint64_t c, Masks mk)
{
    const uint64_t a = c << m;
    const uint64_t g = a ^ (a >> 1);
    uint32_t ml = 0, sl = 0, mh = 0, sh = 0;
    for (int k = 0; k < n; ++k) {
        const uint32_t sel = 0u - (uint32_t)((g >> k) & 1u);
        bip_add(ml, sl, R[k].m_lo & sel, R[k].s_lo & sel);
        if (HI) bip_add(mh, sh, R[k].m_hi & sel, R[k].s_hi & sel);
    }
    int tally = 0;
    if (ml == mk.lo && (!HI || mh == mk.hi)) {
        const int par = (__builtin_popcount(sl & mk.lo) + (HI ? __builtin_popcount(sh & mk.hi) : 0) + (int)(a & 1u)) & 1;
        tally += par ? -1 : 1;
    }
    const bool odd = (c & 1u) != 0;
    const uint32_t len = 1u << m;
    for (uint32_t j = 1; j < len; ++j) {
        const int t = __builtin_ctz(j);
        const bool leave = t + 1 < m ? ((j >> (t + 1)) & 1u) != 0 : odd;
        bip_add(ml, sl, R[t].m_lo, leave ? R[t].sn_lo : R[t].s_lo);
        if (HI) bip_add(mh, sh, R[t].m_hi, leave ? R[t].sn_hi : R[t].s_hi);
        if (ml == mk.lo && (!HI || mh == mk.hi)) {
            const int par = (__builtin_popcount(sl & mk.lo) + (HI ? __builtin_popcount(sh & mk.hi) : 0) + (int)(j & 1u)) & 1;
            tally += par ? -1 : 1;
        }
    }
    return tally;
}

// Exact walk of an arbitrary range [a, e) with both words carried and every
// index tested: ragged ends of a range, and checks.
template <bool HI, typename RP>
PERM3_FN int walk_range_direct(RP R, int n, uint64_t a, uint64_t e, Masks mk)
{
    if (a >= e) return 0;
    const uint64_t g = a ^ (a >> 1);
    uint32_t ml = 0, sl = 0, mh = 0, sh = 0;
    for (int k = 0; k < n; ++k) {
        if ((g >> k) & 1u) {
            bip_add(ml, sl, R[k].m_lo, R[k].s_lo);
            if (HI) bip_add(mh, sh, R[k].m_hi, R[k].s_hi);
        }
    }
    int tally = 0;
    uint64_t i = a;
    for (;;) {
        if (ml == mk.lo && (!HI || mh == mk.hi)) {
            const int par = (__builtin_popcount(sl & mk.lo) + (HI ? __builtin_popcount(sh & mk.hi) : 0) +
                             (int)(i & 1u)) & 1;
            tally += par ? -1 : 1;
        }
        if (++i >= e) break;
        const int t = __builtin_ctzll(i);
        const bool leave = (i >> (t + 1)) & 1u;
        bip_add(ml, sl, R[t].m_lo, leave ? R[t].sn_lo : R[t].s_lo);
        if (HI) bip_add(mh, sh, R[t].m_hi, leave ? R[t].sn_hi : R[t].s_hi);
    }
    return tally;
}

}  // namespace perm3
