// Per-lane Gray-code walk over bipedal rows (gfx950 device code).
//
// A matrix row over F_3 is held as two F_2^n words (mag, sgn) under phi
// (Section 2).  Columns beyond bit 31 live in a second 32-bit "hi" word, so
// n <= 63 uses at most two words per plane.  Each row is stored as
//     { m_lo, s_lo, sn_lo, -, m_hi, s_hi, sn_hi, - }
// where sn = s xor m is the sgn word of the NEGATED row: subtracting a row is
// adding its negation, and negating a bipedal vector flips sgn exactly where
// mag is set (every zero, (0,0) or (0,1), stays a zero).
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

namespace perm3 {

struct RowW {
    uint32_t m_lo, s_lo, sn_lo, pad0;
    uint32_t m_hi, s_hi, sn_hi, pad1;
};

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

// The Ryser term of Gray index i whose subset sum has low words (ml, sl):
// zero unless every column sum is non-zero.  The high words are not carried
// by the fast walk; when the low words pass, they are formed here from
// scratch by summing the rows of g(i) (rare: a (2/3)^32 event per index).
PERM3_FN int exact_term(const RowW *__restrict__ R, int n, uint64_t i, uint32_t ml, uint32_t sl,
                        Masks mk)
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

// Low words of the subset sum of g(i0): jump straight to a Gray state
// (Section 3.1).  O(n) word operations per lane.
PERM3_FN void seed_lo(const RowW *__restrict__ R, int n, uint64_t i0, uint32_t &ml, uint32_t &sl)
{
    const uint64_t g = i0 ^ (i0 >> 1);
    ml = 0;
    sl = 0;
    for (int k = 0; k < n; ++k) {
        const uint32_t sel = 0u - (uint32_t)((g >> k) & 1u);
        bip_add(ml, sl, R[k].m_lo & sel, R[k].s_lo & sel);
    }
}

// Exact re-walk of one block of the fast walk, for the lanes whose block
// contained a candidate.  Starts from the state at chunk offset b*2^UL and
// visits offsets b*2^UL + 1 .. jend with an exact test of every index.
template <int UL>
PERM3_FN int replay_block(const RowW *__restrict__ R, int n, uint64_t i0, uint32_t b, uint32_t nb,
                          uint32_t ml, uint32_t sl, Masks mk)
{
    int tally = 0;
    const uint32_t jend = (b + 1 < nb) ? ((b + 1) << UL) : (((b + 1) << UL) - 1);
    for (uint32_t j = (b << UL) + 1; j <= jend; ++j) {
        const uint64_t i = i0 + j;
        const int t = __builtin_ctz(j);
        const bool leave = (i >> (t + 1)) & 1u;
        bip_add(ml, sl, R[t].m_lo, leave ? R[t].sn_lo : R[t].s_lo);
        tally += exact_term(R, n, i, ml, sl, mk);
    }
    return tally;
}

// Static rows of the unrolled block: t = 0 .. UL-1, wave-uniform.
template <int UL>
struct StaticRows {
    uint32_t m[UL], s[UL], sn[UL];
};

// Fast walk of one whole aligned chunk [c*2^m, (c+1)*2^m), m > UL.
//
// The chunk is cut into nb = 2^(m-UL) blocks of 2^UL indices.  Inside a
// block the flipped row t = ctz(offset) and its direction are compile-time
// constants except for the middle step (t = UL-1, direction = parity of the
// block number), so the rows sit in scalar registers and each index costs
// the three bitop3 of the addition.  The step into the next block flips a
// row t >= UL chosen at run time (t = m-1 once per chunk, with a direction
// given by the chunk's parity).
//
// Candidates are found a block at a time: with bits >= n of every row zero,
// each low mag word is <= mk.lo, so the block's maximum equals mk.lo exactly
// when some index in it has all its low columns non-zero.  Only then is the
// block re-walked exactly (replay_block).
template <int UL>
PERM3_FN int walk_chunk_fast(const RowW *__restrict__ R, int n, int m, uint64_t c, Masks mk,
                             const StaticRows<UL> &sr)
{
    const uint64_t i0 = c << m;
    uint32_t ml, sl;
    seed_lo(R, n, i0, ml, sl);
    int tally = exact_term(R, n, i0, ml, sl, mk);
    const uint32_t nb = 1u << (m - UL);
    const bool codd = (c & 1u) != 0;
    for (uint32_t b = 0; b < nb; ++b) {
        const uint32_t m0 = ml, s0 = sl;
        uint32_t acc = 0;
#pragma unroll
        for (int k = 1; k < (1 << UL); ++k) {
            const int t = __builtin_ctz(k);
            uint32_t rs;
            if (t < UL - 1)
                rs = ((k >> (t + 1)) & 1) ? sr.sn[t] : sr.s[t];
            else
                rs = (b & 1u) ? sr.sn[t] : sr.s[t];
            bip_add(ml, sl, sr.m[t], rs);
            acc = k == 1 ? ml : (acc > ml ? acc : ml);
        }
        if (b + 1 < nb) {
            const uint32_t jb = b + 1;
            const int t = UL + __builtin_ctz(jb);
            const uint32_t bm = R[t].m_lo, bs = R[t].s_lo, bsn = R[t].sn_lo;
            bool leave;
            if (t + 1 < m)
                leave = (jb >> (t + 1 - UL)) & 1u;
            else
                leave = codd;
            bip_add(ml, sl, bm, leave ? bsn : bs);
            acc = acc > ml ? acc : ml;
        }
        if (acc == mk.lo) tally += replay_block<UL>(R, n, i0, b, nb, m0, s0, mk);
    }
    return tally;
}

// Exact walk of an arbitrary range [a, e) with both words carried and every
// index tested: small matrices, ragged ends of a range, and checks.
template <bool HI>
PERM3_FN int walk_range_direct(const RowW *__restrict__ R, int n, uint64_t a, uint64_t e, Masks mk)
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
