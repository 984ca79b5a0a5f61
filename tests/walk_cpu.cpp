// CPU build of the device walk and the planning helpers, for tests under
// AddressSanitizer and UndefinedBehaviorSanitizer.
//
// The walk templates (paper_2407_20205_amd/csrc/perm3_walk.hpp) and the plan
// functions (perm3_plan.hpp) are compiled here as plain C++: the 3-input
// table op is evaluated bit by bit from its truth table, wave-uniform values
// are plain values, and a "wave" is one lane.  Rows are packed here with phi
// (Section 2).  Commands come one per line on stdin and each prints one line:
//
//   fused <count> <n_1> .. <n_count>        -> <fused 0/1> <capped work>
//   target <work> <waves> <tasks_per_wave> <states_log> <queue_task_log> -> target chunk log
//   plan <n> <lo> <hi> <target_m> <tuning 10 ints> -> <mode> <m> <ul> <c_first> <ntasks>
//   chunks <UL> <S> <n> <m> <c> <digits>    -> T over chunks c + 64 q, q < S (walk_chunks_fast,
//                                              its four forms checked against each other)
//   direct <n> <m> <c> <digits>             -> T over chunk c (walk_chunk_direct)
//   range <n> <a> <e> <digits>              -> T(a, e) (walk_range_direct)
//   rewalk <n> <a> <b> <digits>             -> T(a, b + 1) by seed + rewalk_exact forward, then
//                                              T over the aligned blocks of 2^4, 2^5, 2^6
//                                              holding a (rewalk_block; 0 where n <= UL)
//   wide <UL> <n> <c0_hi> <c0_lo> <m> <fast> <off_lo> <off_hi> <cr> <digits>
//                                           -> T of one lane's piece of a 128-bit range
//
// <digits> is the matrix row-major as n*n characters '0', '1', '2' (2 = -1).
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <iostream>
#include <sstream>
#include <string>
#include <vector>

static inline uint32_t cpu_bitop3(uint32_t a, uint32_t b, uint32_t c, uint32_t tt)
{
    uint32_t r = 0;
    for (int k = 0; k < 8; ++k) {
        if (!((tt >> k) & 1u)) continue;
        const uint32_t x = (k & 4) ? a : ~a;
        const uint32_t y = (k & 2) ? b : ~b;
        const uint32_t z = (k & 1) ? c : ~c;
        r |= x & y & z;
    }
    return r;
}

#define PERM3_FN static inline
#define PERM3_BITOP3(a, b, c, tt) cpu_bitop3((a), (b), (c), (tt))
#define PERM3_UNIFORM(x) (x)
#define PERM3_TO_VGPR(x) (x)
#define PERM3_PIN_PAIR(x) ((void)(x))
// a wave of one lane
#define PERM3_BALLOT(p) ((uint64_t)((p) ? 1u : 0u))
#define PERM3_LANE() 0
#define PERM3_RANK(mask) 0u
#define PERM3_SHFL32(v, src) ((uint32_t)(v))
#define PERM3_WAVE_LDS_SYNC() \
    do {                      \
    } while (0)
static uint32_t g_cand_list[128];
#define PERM3_CAND_LIST() g_cand_list

#include "perm3_plan.hpp"
#include "perm3_walk.hpp"

using namespace perm3;

static bool read_matrix(const std::string &digits, int n, std::vector<uint8_t> &A)
{
    if ((int)digits.size() != n * n) return false;
    A.resize((size_t)n * n);
    for (int k = 0; k < n * n; ++k) {
        const char ch = digits[k];
        if (ch < '0' || ch > '2') return false;
        A[k] = (uint8_t)(ch - '0');
    }
    return true;
}

// phi (Section 2) of each row: element j at bit n-1-j of (mag, sgn), with
// the negated row's sign word beside them, split into 32-bit words.
static std::vector<RowW> pack_rows(const std::vector<uint8_t> &A, int n)
{
    std::vector<RowW> rows((size_t)(n > 0 ? n : 1));
    for (int r = 0; r < n; ++r) {
        uint64_t mag = 0, sgn = 0;
        for (int j = 0; j < n; ++j) {
            const uint8_t v = A[(size_t)r * n + j];
            const uint64_t bit = 1ull << (n - 1 - j);
            if (v) mag |= bit;
            if (v == 2) sgn |= bit;
        }
        const uint64_t sn = sgn ^ mag;
        RowW w;
        w.m_lo = (uint32_t)mag;
        w.s_lo = (uint32_t)sgn;
        w.sn_lo = (uint32_t)sn;
        w.pad0 = 0;
        w.m_hi = (uint32_t)(mag >> 32);
        w.s_hi = (uint32_t)(sgn >> 32);
        w.sn_hi = (uint32_t)(sn >> 32);
        w.pad1 = 0;
        rows[r] = w;
    }
    return rows;
}

// Rows of up to 128 columns: column j at bit j of the 128-bit planes (any
// column order gives the same T); the low 32 columns form the walk's word.
static std::vector<RowX> pack_rows_wide(const std::vector<uint8_t> &A, int n)
{
    std::vector<RowX> rows((size_t)n);
    for (int r = 0; r < n; ++r) {
        uint32_t m[4] = {0, 0, 0, 0}, s[4] = {0, 0, 0, 0};
        for (int j = 0; j < n; ++j) {
            const uint8_t v = A[(size_t)r * n + j];
            if (v) m[j / 32] |= 1u << (j % 32);
            if (v == 2) s[j / 32] |= 1u << (j % 32);
        }
        RowX x;
        memset(&x, 0, sizeof x);
        x.m_lo = m[0];
        x.s_lo = s[0];
        x.sn_lo = s[0] ^ m[0];
        for (int w = 0; w < 3; ++w) {
            x.m_w[w] = m[w + 1];
            x.s_w[w] = s[w + 1];
        }
        rows[r] = x;
    }
    return rows;
}

static Masks masks_of(int n)
{
    const uint64_t full = n >= 64 ? ~0ull : ((1ull << n) - 1ull);
    Masks mk;
    mk.lo = (uint32_t)full;
    mk.hi = (uint32_t)(full >> 32);
    return mk;
}

template <int UL, int S>
static long long chunks_ul_s(const RowW *R, int n, int m, uint64_t c)
{
    LowSums<UL> lr;
    load_low_sums<UL>(R, lr);
    // every form of the fast walk over the chunks c + 64 q, q < S: candidate
    // blocks noted and re-walked after the chunk or at once, each block's
    // closing row read a block ahead or at its start
    long long deferred = 0, direct = 0, ahead = 0, both = 0;
    for (int q = 0; q < S; ++q) {
        const uint64_t cq = c + 64u * (uint64_t)q;
        deferred += walk_chunks_fast<UL, true, false>(R, n, m, cq, masks_of(n), lr);
        direct += walk_chunks_fast<UL, false, false>(R, n, m, cq, masks_of(n), lr);
        ahead += walk_chunks_fast<UL, false, true>(R, n, m, cq, masks_of(n), lr);
        both += walk_chunks_fast<UL, true, true>(R, n, m, cq, masks_of(n), lr);
    }
    if (deferred != direct || ahead != direct || both != direct) {
        printf("error\n");
        exit(1);
    }
    return deferred;
}

static long long chunks(int ul, int s, const RowW *R, int n, int m, uint64_t c)
{
    switch (ul * 10 + s) {
    case 41: return chunks_ul_s<4, 1>(R, n, m, c);
    case 42: return chunks_ul_s<4, 2>(R, n, m, c);
    case 44: return chunks_ul_s<4, 4>(R, n, m, c);
    case 51: return chunks_ul_s<5, 1>(R, n, m, c);
    case 52: return chunks_ul_s<5, 2>(R, n, m, c);
    case 54: return chunks_ul_s<5, 4>(R, n, m, c);
    case 61: return chunks_ul_s<6, 1>(R, n, m, c);
    case 62: return chunks_ul_s<6, 2>(R, n, m, c);
    case 64: return chunks_ul_s<6, 4>(R, n, m, c);
    default: fprintf(stderr, "bad UL/S\n"); exit(2);
    }
}

template <int UL>
static long long wide_ul(const RowX *R, int n, int m, bool fast, u128 c0, uint64_t off_lo, uint64_t off_hi,
                         uint64_t cr)
{
    LowSums<UL> lr;
    load_low_sums<UL>(R, lr);
    // the kernel's form (deferred re-walks, rows read ahead) against the plain one
    const long long deferred =
        walk_lane_wide<UL, true, true>(R, n, m, fast, c0, off_lo, off_hi, cr, masks_wide(n), lr);
    const long long direct =
        walk_lane_wide<UL, false, false>(R, n, m, fast, c0, off_lo, off_hi, cr, masks_wide(n), lr);
    if (deferred != direct) {
        printf("error\n");
        exit(1);
    }
    return deferred;
}

// The exact terms of the aligned block of 2^UL indices at ia: its first index
// and rewalk_block over the rest.
template <int UL>
static long long block_ul(const RowW *R, int n, uint64_t ia, const Masks &mk)
{
    uint32_t ml, sl;
    seed_lo(R, n, ia, ml, sl);
    return exact_term(R, n, ia, ml, sl, mk) + rewalk_block<UL>(R, n, ia, (uint32_t)(ia >> UL), ml, sl, mk);
}

int main()
{
    std::string line;
    while (std::getline(std::cin, line)) {
        std::istringstream in(line);
        std::string cmd;
        if (!(in >> cmd)) continue;
        if (cmd == "fused") {
            int count = 0;
            in >> count;
            std::vector<int32_t> ns((size_t)(count > 0 ? count : 1));
            for (int k = 0; k < count; ++k) in >> ns[k];
            printf("%d %llu\n", small_call_fused(ns.data(), count, false) ? 1 : 0,
                   (unsigned long long)capped_work(ns.data(), count, SMALL_FUSED_WORK));
        } else if (cmd == "target") {
            double work = 0;
            PlanArgs a;
            memset(&a, 0, sizeof a);
            in >> work >> a.waves_total >> a.tasks_per_wave >> a.states_log >> a.queue_task_log;
            printf("%d\n", target_chunk_log(a, work));
        } else if (cmd == "plan") {
            int n, target_m;
            unsigned long long lo, hi;
            PlanArgs a;
            memset(&a, 0, sizeof a);
            in >> n >> lo >> hi >> target_m >> a.body_log >> a.chunk_log_max >> a.direct_max_n >>
                a.direct_chunk_log_max >> a.body_log_mid >> a.mid_max_n >> a.states_log >> a.max_tasks_log >>
                a.min_task_log >> a.tasks_per_wave;
            a.use_range = 1;
            a.range_lo = lo;
            a.range_hi = hi;
            const MatMeta mt = plan_pure(a, n, target_m);
            printf("%d %d %d %llu %llu\n", mt.mode, mt.m, mt.ul, (unsigned long long)mt.c_first,
                   (unsigned long long)mt.ntasks);
        } else if (cmd == "chunks" || cmd == "direct" || cmd == "range" || cmd == "rewalk") {
            int ul = 5, s = 1, n = 0, m = 0;
            unsigned long long c = 0, a = 0, e = 0;
            if (cmd == "chunks") in >> ul >> s >> n >> m >> c;
            if (cmd == "direct") in >> n >> m >> c;
            if (cmd == "range" || cmd == "rewalk") in >> n >> a >> e;
            std::string digits;
            in >> digits;
            std::vector<uint8_t> A;
            if (n < 1 || n > 63 || !read_matrix(digits, n, A)) {
                printf("error\n");
                continue;
            }
            const std::vector<RowW> rows = pack_rows(A, n);
            const RowW *R = rows.data();
            const Masks mk = masks_of(n);
            if (cmd == "chunks") {
                printf("%lld\n", chunks(ul, s, R, n, m, c));
            } else if (cmd == "direct") {
                printf("%d\n", n > 32 ? walk_chunk_direct<true>(R, n, m, c, mk) : walk_chunk_direct<false>(R, n, m, c, mk));
            } else if (cmd == "range") {
                printf("%d\n", n > 32 ? walk_range_direct<true>(R, n, a, e, mk) : walk_range_direct<false>(R, n, a, e, mk));
            } else {
                // forward: state at a, then every index a+1 .. e
                uint32_t ml, sl;
                seed_lo(R, n, (uint64_t)a, ml, sl);
                const int fwd = exact_term(R, n, (uint64_t)a, ml, sl, mk) + rewalk_exact(R, n, (uint64_t)a, (uint64_t)e, ml, sl, mk);
                // the aligned block of 2^UL around a, UL = 4, 5, 6 (each within range when n > UL)
                long long blk[3] = {0, 0, 0};
                if (n > 4) blk[0] = block_ul<4>(R, n, (uint64_t)a & ~15ull, mk);
                if (n > 5) blk[1] = block_ul<5>(R, n, (uint64_t)a & ~31ull, mk);
                if (n > 6) blk[2] = block_ul<6>(R, n, (uint64_t)a & ~63ull, mk);
                printf("%d %lld %lld %lld\n", fwd, blk[0], blk[1], blk[2]);
            }
        } else if (cmd == "wide") {
            int ul, n, m, fast;
            unsigned long long c0_hi, c0_lo, off_lo, off_hi, cr;
            std::string digits;
            in >> ul >> n >> c0_hi >> c0_lo >> m >> fast >> off_lo >> off_hi >> cr >> digits;
            std::vector<uint8_t> A;
            if (n < 1 || n > 128 || !read_matrix(digits, n, A)) {
                printf("error\n");
                continue;
            }
            const std::vector<RowX> rows = pack_rows_wide(A, n);
            const u128 c0 = ((u128)c0_hi << 64) | (u128)c0_lo;
            long long t = 0;
            switch (ul) {
            case 4: t = wide_ul<4>(rows.data(), n, m, fast != 0, c0, off_lo, off_hi, cr); break;
            case 5: t = wide_ul<5>(rows.data(), n, m, fast != 0, c0, off_lo, off_hi, cr); break;
            case 6: t = wide_ul<6>(rows.data(), n, m, fast != 0, c0, off_lo, off_hi, cr); break;
            default: printf("error\n"); continue;
            }
            printf("%lld\n", t);
        } else {
            printf("error\n");
        }
        fflush(stdout);
    }
    return 0;
}
