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

// Candidate blocks of a wave, re-walked later all together (one lane per
// block) instead of each by the whole wave at once: an entry holds the lane
// whose chunk it is (bits 26..31) and the block number (bits 0..25; blocks
// per chunk are at most 2^(24-4)).  Up to CAND_CAP entries per wave, in LDS;
// the walk kernels run 4 waves per workgroup.
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

// The exact terms of indices ia+1 .. ia+U-1 of one candidate block, walked
// forward from the Gray state at its first index ia (a multiple of
// U = 2^UL; ia itself is tested by the caller).  Lanes re-walk different
// blocks side by side, all at the same offset k, so the row flipped at k is
// t = ctz(k) for every lane and comes in by a scalar load; its direction is
// bit t+1 of k, except at t = UL-1 where it is bit UL of ia, the parity of
// the lane's block number b.
template <int UL, typename RP, typename I, typename MK>
PERM3_FN int rewalk_block(RP R, int n, I ia, uint32_t b, uint32_t ml, uint32_t sl, const MK &mk)
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
    return tally;
}

// ------------------------------------------------------------------ fast walk
//
// Write an index of an aligned chunk as i = i0 + b 2^UL + k with k < 2^UL.
// The low UL bits of g(i) are g(k), with bit UL-1 flipped when the block
// number b is odd, and the bits above are those of g(i >> UL).  So the
// subset sum at i is H_b + L, where H_b sums the rows UL .. n-1 of g(i) (one
// sum per block, moved by one Gray step from block to block) and L sums rows
// 0 .. UL-1 of the low bits.  Flipping bit UL-1 of g(k) gives g of
// k xor (2^UL - 1), so an odd block meets the same low sums as an even one,
// in reverse order: every block's states are exactly {H_b + L_k : k < 2^UL},
// with L_k the sum of the rows of g(k), the same for every block, chunk and
// lane of a matrix.
//
// The states of a block are then independent of each other (no dependency
// chain through the block), and the candidate test needs only their mag
// words: by Theorem 2.1 the mag word of H + L_k is (m_L & y) | (m_H ^ m_L)
// with y = m_H ^ s_H ^ s_L, two 3-input ops per index where a Gray step that
// must also carry sgn takes three.  A block with a candidate is walked again
// exactly, index by index in Gray order.
//
// Block length: 2^4.  The 2^UL - 1 word pairs L_k stay in vector registers
// (a scalar operand makes bitop3 issue more slowly, and 62 scalar words
// spill); with 2^5-index blocks they hold 62 VGPRs and the walk drops to 5
// waves per SIMD, which made the 36 x 36 walk slower (4.73 against 4.35 ms
// for 2^4 on one box).  Forming y as u ^ s_L with u = m_H ^ s_H taken once
// per block saves an op per block but measured 17% slower (4.35 against
// 3.72 ms): the 3-input form is what the SIMDs issue fastest.
constexpr int WALK_UL = 4;

// L_k, k < 2^UL: the low words of the sum of rows g(k) (k = 0 is zero),
// built by a Gray walk over rows 0 .. UL-1 on the scalar unit, each word
// moved into a vector register as soon as it is formed (held there for the
// whole task, so the scalar words are never all live at once).
template <int UL>
struct LowSums {
    uint64_t p[1u << UL];   // mag word << 32 | sgn word
};

// A 64-bit value held in one register pair: an even-aligned pair of VGPRs,
// its low word in an even register bank and its high word in an odd one.  A
// 3-input op whose three sources share one bank issues at about half rate on
// gfx950, and the allocator left to itself put m_H, s_H and a third operand
// in one bank for 6 of the 44 ops of a block (the 36 x 36 walk 13% slower
// than with the words spread).  With H = {m_H low, s_H high} and
// L_k = {s_L low, m_L high}, the op forming y reads m_H and s_H from banks
// of both parities, and the op forming the mag word reads m_H (even) and
// m_L (odd): no op of a block can have all its sources in one bank.
#ifndef PERM3_PIN_PAIR
#define PERM3_PIN_PAIR(x) asm("" : "+v"(x))
#endif

template <int UL, typename RP>
PERM3_FN void load_low_sums(RP R, LowSums<UL> &lr)
{
    constexpr uint32_t U = 1u << UL;
    uint32_t mm = 0, ss = 0;
    lr.p[0] = 0;
#pragma unroll
    for (uint32_t k = 1; k < U; ++k) {
        const int t = __builtin_ctz(k);
        const bool leave = ((k >> (t + 1)) & 1u) != 0;
        const uint32_t rm = R[t].m_lo, rs = leave ? R[t].sn_lo : R[t].s_lo;
        // Theorem 2.1's addition on wave-uniform words (scalar ALU)
        const uint32_t x = rm & (mm ^ ss ^ rs);
        const uint32_t mo = x | (mm ^ rm);
        ss = x ^ ss;
        mm = mo;
        uint64_t pk = ((uint64_t)PERM3_TO_VGPR(mm) << 32) | PERM3_TO_VGPR(ss);
        PERM3_PIN_PAIR(pk);
        lr.p[k] = pk;
    }
}

// The exact terms of the candidate blocks a wave noted (entries: lane in
// bits 26..31, block number below), one lane per entry: jump to the Gray
// state at the block's first index (Section 3.1), test it, and walk the
// block's other 2^UL - 1 indices (rewalk_block).
template <int UL, typename RP, typename I, typename MK>
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
            const uint32_t b = e & 0x3FFFFFFu;
            const I ia = (ce << m) + (I)(b * U);
            uint32_t ml, sl;
            seed_lo(R, n, ia, ml, sl);
            tally += exact_term(R, n, ia, ml, sl, mk) + rewalk_block<UL>(R, n, ia, b, ml, sl, mk);
        }
    }
    return tally;
}

// The largest of N words, by rounds of 3-input maxima (one v_max3_u32 each):
// a tree, so that the block's maxima do not form one dependency chain (16
// words: five, then two, then one; the 36 x 36 walk 2.4% faster than folding
// them one pair at a time into a running maximum).
template <int N>
PERM3_FN uint32_t max_tree(const uint32_t *v)
{
    if constexpr (N == 1) {
        return v[0];
    } else if constexpr (N == 2) {
        return v[0] > v[1] ? v[0] : v[1];
    } else {
        constexpr int M = (N + 2) / 3;
        uint32_t w[M];
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const int j = 3 * i;
            uint32_t x = v[j];
            if (j + 1 < N) x = x > v[j + 1] ? x : v[j + 1];
            if (j + 2 < N) x = x > v[j + 2] ? x : v[j + 2];
            w[i] = x;
        }
        return max_tree<M>(w);
    }
}

// Fast walk of the whole aligned chunk c of length 2^m, m > UL, in blocks
// of 2^UL indices (above).  H starts as the state at the chunk's first index
// (whose low m-1 Gray bits are zero) and takes the steps between blocks: the
// row t = UL + ctz(b+1) into block b+1, wave-uniform, and between the two
// halves the chunk's middle step (row m-1, which leaves the subset when the
// chunk index is odd, the one step whose direction differs between lanes).
// The last block of each half adds a zero row instead, which keeps the block
// body free of branches.
//
// Candidates are found a block at a time: with bits >= n of every row zero,
// each low mag word is <= mk.lo, so the block's maximum equals mk.lo exactly
// when some index in it has all its low columns non-zero (one 3-input max
// per two states).  Only then is the block walked again exactly: with DEFER
// noted in the wave's candidate list and re-walked by one lane after the
// chunk (flush_candidates), or at once when the list is full; without DEFER
// at once by the whole wave, from H_b plus row UL-1 when b is odd (the state
// at the block's first index).
//
// AHEAD: the row of the step closing a block is loaded one block ahead, so
// that its load has a whole block to land; else at the block's start.
//
// The chunk index c is a uint64_t for n <= 63 and a u128 for wider matrices
// (with MasksX); only the seed and the exact terms see its high bits.
template <int UL, bool DEFER, bool AHEAD, typename RP, typename I, typename MK>
PERM3_FN int walk_chunks_fast(RP R, int n, int m, I c, const MK &mk, const LowSums<UL> &lr)
{
    constexpr uint32_t U = 1u << UL;
    const I i0 = c << m;
    uint32_t m0, s0;
    seed_lo(R, n, i0, m0, s0);
    uint64_t hp = ((uint64_t)s0 << 32) | m0;   // H as a register pair
    PERM3_PIN_PAIR(hp);
    uint32_t *const list = DEFER ? PERM3_CAND_LIST() : nullptr;
    const uint32_t lane_tag = (uint32_t)PERM3_LANE() << 26;
    uint32_t ncand = 0;
    int tally = 0;
    const uint32_t half = 1u << (m - UL - 1);
    // the row added by the step into block j of a half ending at bend (a zero
    // row when j = bend; t = UL + ctz(j) <= m < n is in range even unused)
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
            uint32_t bm, bs;
            if (AHEAD) {
                bm = PERM3_TO_VGPR(next_m);
                bs = PERM3_TO_VGPR(next_s);
                closing_row(b + 2, bend, next_m, next_s);
            } else {
                uint32_t rm, rs;
                closing_row(b + 1, bend, rm, rs);
                bm = PERM3_TO_VGPR(rm);
                bs = PERM3_TO_VGPR(rs);
            }
            uint32_t mh = (uint32_t)hp, sh = (uint32_t)(hp >> 32);
            auto mag_of = [&](uint32_t k) {
                const uint32_t sl = (uint32_t)lr.p[k], ml = (uint32_t)(lr.p[k] >> 32);
                return PERM3_BITOP3(PERM3_BITOP3(mh, sh, sl, TT_XOR3), mh, ml, TT_AC_OR_BXC);
            };
            // the block's mag words (k = 0 is H itself), folded as a tree
            uint32_t v[U];
            v[0] = mh;
#pragma unroll
            for (uint32_t k = 1; k < U; ++k) v[k] = mag_of(k);
            uint32_t acc;
            if constexpr (U == 16) {
                // written out: the scheduler orders the block's ops from this
                // form as measured (max_tree<16> computes the same maxima,
                // but its schedule walked the 36 x 36 2.4% slower)
                auto mx3 = [](uint32_t a, uint32_t b, uint32_t c) {
                    const uint32_t x = a > b ? a : b;
                    return x > c ? x : c;
                };
                uint32_t t[5];
#pragma unroll
                for (int q = 0; q < 5; ++q) t[q] = mx3(v[3 * q], v[3 * q + 1], v[3 * q + 2]);
                acc = mx3(mx3(t[0], t[1], t[2]), mx3(t[3], t[4], v[15]), 0u);
            } else {
                acc = max_tree<(int)U>(v);
            }
            const bool cand = acc == mk.lo;
            bool now = false;
            if (DEFER) {
                const uint64_t cands = PERM3_BALLOT(cand);
                if (cands) {
                    const uint32_t nc = (uint32_t)__builtin_popcountll(cands);
                    if (ncand + nc <= CAND_CAP) {
                        if (cand) list[ncand + PERM3_RANK(cands)] = lane_tag | b;
                        ncand += nc;
                    } else {
                        now = cand;
                    }
                }
            } else {
                now = cand;
            }
            if (now) {
                const I ia = i0 + (I)(b * U);
                uint32_t ml = mh, sl = sh;
                if (b & 1u) bip_add(ml, sl, R[UL - 1].m_lo, R[UL - 1].s_lo);
                tally += exact_term(R, n, ia, ml, sl, mk) + rewalk_block<UL>(R, n, ia, b, ml, sl, mk);
            }
            bip_add(mh, sh, bm, bs);
            hp = ((uint64_t)sh << 32) | mh;
            PERM3_PIN_PAIR(hp);
        }
        if (h == 0) {
            // offset L/2 flips row m-1
            const bool odd = (c & 1u) != 0;
            uint32_t mh = (uint32_t)hp, sh = (uint32_t)(hp >> 32);
            bip_add(mh, sh, R[m - 1].m_lo, odd ? R[m - 1].sn_lo : R[m - 1].s_lo);
            hp = ((uint64_t)sh << 32) | mh;
            PERM3_PIN_PAIR(hp);
        }
    }
    if (DEFER && ncand) tally += flush_candidates<UL>(R, n, m, c, mk, list, ncand);
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
// 2^128.  A whole chunk of a fast-mode matrix takes the fast walk; a
// ragged end (or a small matrix) is seeded at its first index and tests every
// index on the low word, forming the other words only where it passes.
template <int UL, bool DEFER, bool AHEAD, typename RP>
PERM3_FN int walk_lane_wide(RP R, int n, int m, bool fast, u128 c0, uint64_t off_lo, uint64_t off_hi,
                            uint64_t cr, const MasksX &mk, const LowSums<UL> &lr)
{
    const uint64_t oa0 = cr << m;
    const uint64_t oe0 = oa0 + (1ull << m);
    const uint64_t oa = oa0 > off_lo ? oa0 : off_lo;
    const uint64_t oe = oe0 < off_hi ? oe0 : off_hi;
    if (oa >= oe) return 0;
    if (fast && oa == oa0 && oe == oe0) return walk_chunks_fast<UL, DEFER, AHEAD>(R, n, m, c0 + cr, mk, lr);
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
