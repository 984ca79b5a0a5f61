/*
 * CPU oracle for perm(A) mod 3 -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load this code.  It shares nothing with the GPU library: no headers, no
 * helpers, no tables.  It is deliberately plain and slow.
 *
 * What it computes (Scheinerman, "Fast computation of permanents over F_3
 * via F_2 arithmetic"):
 *
 *   perm(A) = sum over permutations sigma of prod_i a_{i,sigma(i)}   (eq. 1)
 *
 * reached through Ryser's identity (eq. 2), read over ROW subsets S as the
 * paper's own code does (eq. 2 printed over column subsets is the same
 * number because perm(A) = perm(A^T)):
 *
 *   perm(A) = (-1)^n * sum_S (-1)^|S| * prod_cols ( sum_{k in S} A[k][col] ).
 *
 * The subsets are visited in reflected-binary Gray-code order (Section 3,
 * footnote on the RBC): Gray index i has state g(i) = i xor (i >> 1), and the
 * step into index i flips row ctz(i).  A row is subtracted when it leaves
 * the subset (its bit is set in the previous state) and added when it
 * enters.  Elements are kept UNPACKED, one int per column, reduced to the
 * centred residues {-1, 0, 1} after every update (the cmod3 of Section 3),
 * so every column product is in {-1, 0, 1}.
 *
 * Matrix entries are bytes in {0,1,2}; 2 is read as -1.  Results are in
 * {0,1,2}.  A partial tally T(a,b) is the exact signed integer
 *     T(a,b) = sum_{a <= i < b} (-1)^|g(i)| * prod_cols v_col(g(i))
 * with v(S) the centred column sums of the rows in S; T is additive over
 * ranges and perm(A) mod 3 = (-1)^n T(0, 2^n) mod 3.  A block of
 * consecutive Gray indices starts by jumping straight to state g(a)
 * (Section 3.1).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define ORACLE_MAX_N 63

/* cmod3 (Section 3): mod(x,3) mapped to {-1,0,1}. */
static int centred_mod3(int64_t x)
{
    int64_t a = x % 3;
    if (a < 0) a += 3;
    return a == 2 ? -1 : (int)a;
}

/* Entry of A as an element of F_3 in {-1,0,1}. */
static int entry(const uint8_t *A, int n, int row, int col)
{
    return A[row * n + col] == 2 ? -1 : (int)A[row * n + col];
}

static int popcount64(uint64_t x)
{
    int c = 0;
    while (x) { c += (int)(x & 1u); x >>= 1; }
    return c;
}

static int trailing_zeros64(uint64_t x)
{
    int t = 0;
    while (!(x & 1u)) { x >>= 1; ++t; }
    return t;
}

/* Reject anything the definition does not cover. */
static int valid_input(const uint8_t *A, int n)
{
    if (n < 0 || n > ORACLE_MAX_N) return 0;
    if (n > 0 && A == NULL) return 0;
    for (int k = 0; k < n * n; ++k)
        if (A[k] > 2) return 0;
    return 1;
}

/*
 * One Ryser term by its definition, no Gray walk: the subset is g(i), the
 * column sums are formed from scratch, and the sign is (-1)^|S| counted on
 * the subset itself.
 */
int oracle_term(const uint8_t *A, int n, uint64_t i)
{
    if (!valid_input(A, n)) return 0;
    uint64_t S = i ^ (i >> 1);
    int prod = 1;
    for (int col = 0; col < n; ++col) {
        int64_t sum = 0;
        for (int k = 0; k < n; ++k)
            if ((S >> k) & 1u) sum += entry(A, n, k, col);
        prod *= centred_mod3(sum);
    }
    return (popcount64(S) & 1) ? -prod : prod;
}

/*
 * T(a,b) by a Gray-code walk over unpacked centred residues, the way the
 * paper's plain Ryser routine walks (with its cmod3 reduction).  Returns 0 and
 * sets *ok = 0 on invalid input or a range outside [0, 2^n].
 */
int64_t oracle_range_tally(const uint8_t *A, int n, uint64_t a, uint64_t b, int *ok)
{
    if (ok) *ok = 0;
    if (!valid_input(A, n)) return 0;
    uint64_t total = (uint64_t)1 << n;
    if (a > b || b > total) return 0;
    if (ok) *ok = 1;
    if (a == b) return 0;

    /* the matrix as centred residues, E[k][col] in {-1,0,1} */
    int E[ORACLE_MAX_N][ORACLE_MAX_N];
    for (int k = 0; k < n; ++k)
        for (int col = 0; col < n; ++col)
            E[k][col] = entry(A, n, k, col);

    int v[ORACLE_MAX_N];
    /* jump to state g(a): add every row whose bit is set */
    uint64_t x = a ^ (a >> 1);
    for (int col = 0; col < n; ++col) {
        int64_t sum = 0;
        for (int k = 0; k < n; ++k)
            if ((x >> k) & 1u) sum += E[k][col];
        v[col] = centred_mod3(sum);
    }

    int64_t s = 0;
    for (uint64_t i = a; i < b; ++i) {
        if (i > a) {
            int t = trailing_zeros64(i);
            int leaving = (int)((x >> t) & 1u);   /* row t is in the subset: remove it */
            x ^= (uint64_t)1 << t;
            for (int col = 0; col < n; ++col)
                v[col] = centred_mod3(leaving ? v[col] - E[t][col] : v[col] + E[t][col]);
        }
        int prod = 1;
        for (int col = 0; col < n; ++col) prod *= v[col];
        if (popcount64(x) & 1) s -= prod; else s += prod;
    }
    return s;
}

/* ------------------------------------------------------------------ */
/* Threaded whole-range tally: the paper's parallel scheme (Section 3.1) of
 * independent blocks of consecutive Gray indices, partial sums added.     */

typedef struct {
    const uint8_t *A;
    int n;
    uint64_t a, b;
    int64_t out;
    int ok;
} oracle_job;

static void *oracle_job_run(void *p)
{
    oracle_job *j = (oracle_job *)p;
    j->out = oracle_range_tally(j->A, j->n, j->a, j->b, &j->ok);
    return NULL;
}

int64_t oracle_range_tally_mt(const uint8_t *A, int n, uint64_t a, uint64_t b,
                              int nthreads, int *ok)
{
    if (ok) *ok = 0;
    if (!valid_input(A, n)) return 0;
    uint64_t total = (uint64_t)1 << n;
    if (a > b || b > total) return 0;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    uint64_t len = b - a;
    if (len < (uint64_t)nthreads * 4096u) nthreads = 1;

    oracle_job jobs[256];
    pthread_t th[256];
    for (int k = 0; k < nthreads; ++k) {
        jobs[k].A = A; jobs[k].n = n;
        jobs[k].a = a + len * (uint64_t)k / (uint64_t)nthreads;
        jobs[k].b = a + len * (uint64_t)(k + 1) / (uint64_t)nthreads;
        jobs[k].out = 0; jobs[k].ok = 0;
    }
    int started = 0;
    for (int k = 1; k < nthreads; ++k) {
        if (pthread_create(&th[k], NULL, oracle_job_run, &jobs[k]) != 0) break;
        started = k;
    }
    oracle_job_run(&jobs[0]);
    for (int k = started + 1; k < nthreads; ++k)
        oracle_job_run(&jobs[k]);   /* threads that failed to start run inline */
    for (int k = 1; k <= started; ++k) pthread_join(th[k], NULL);

    int64_t s = 0;
    int all_ok = 1;
    for (int k = 0; k < nthreads; ++k) { s += jobs[k].out; all_ok &= jobs[k].ok; }
    if (ok) *ok = all_ok;
    return s;
}

/* perm(A) mod 3 in {0,1,2}; -1 on invalid input.  For n = 0 the only subset is
 * the empty one and its empty product is 1, so perm of the 0x0 matrix is 1. */
int oracle_perm_mod3(const uint8_t *A, int n, int nthreads)
{
    if (!valid_input(A, n)) return -1;
    int ok = 0;
    int64_t T = oracle_range_tally_mt(A, n, 0, (uint64_t)1 << n, nthreads, &ok);
    if (!ok) return -1;
    int64_t p = (n & 1) ? -T : T;          /* the (-1)^n of eq. 2 */
    int r = centred_mod3(p);
    return r < 0 ? 2 : r;
}

/*
 * z(n) of Section 4: how many of the 3^(n*n) matrices over F_3 have
 * permanent 0, by visiting every one of them.  n <= 4 (3^16 matrices).
 * Also returns the counts of permanent 1 and permanent -1 (= 2).
 */
int oracle_count_by_value(int n, uint64_t counts[3])
{
    counts[0] = counts[1] = counts[2] = 0;
    if (n < 1 || n > 4) return -1;
    int cells = n * n;
    uint8_t A[16];
    memset(A, 0, sizeof A);
    for (;;) {
        int r = oracle_perm_mod3(A, n, 1);
        counts[r] += 1;
        int k = 0;                        /* next matrix: base-3 odometer */
        while (k < cells && A[k] == 2) { A[k] = 0; ++k; }
        if (k == cells) break;
        A[k] += 1;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Census over generated matrices (the counts of Table 3, the Monte Carlo
 * study of Table 4).  Matrix t, entry k (row-major):
 *   generator 0: the k-th base-3 digit of t, least significant first;
 *   generator 1: floor(3 x / 2^64) for x the (t*n*n + k + 1)-th output of
 *                SplitMix64 seeded with key (state key + q * gamma, gamma =
 *                0x9E3779B97F4A7C15, then the generator's mixing function). */

static uint64_t splitmix64_output(uint64_t key, uint64_t q)
{
    uint64_t z = key + q * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t oracle_splitmix64(uint64_t key, uint64_t q) { return splitmix64_output(key, q); }

int oracle_census(int n, int generator, uint64_t key, uint64_t first, uint64_t count, uint64_t counts[3])
{
    counts[0] = counts[1] = counts[2] = 0;
    if (n < 1 || n > ORACLE_MAX_N || (generator != 0 && generator != 1)) return -1;
    uint8_t A[ORACLE_MAX_N * ORACLE_MAX_N];
    const int cells = n * n;
    for (uint64_t t = first; t < first + count; ++t) {
        uint64_t rest = t;
        for (int k = 0; k < cells; ++k) {
            if (generator == 0) {
                A[k] = (uint8_t)(rest % 3);
                rest /= 3;
            } else {
                unsigned __int128 x = splitmix64_output(key, t * (uint64_t)cells + (uint64_t)k + 1);
                A[k] = (uint8_t)((x * 3) >> 64);
            }
        }
        int r = oracle_perm_mod3(A, n, 1);
        if (r < 0) return -1;
        counts[r] += 1;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Matrices of up to 128 columns, Gray indices of up to 128 bits.
 *
 * Section 3 stops at n <= 64, where a row and a Gray index each fit one
 * 64-bit word, and notes that larger n would take a second word.  The sums
 * are the same: T(a, b) over Gray indices a <= i < b with the state
 * g(i) = i xor (i >> 1) now a 128-bit row set.  Only ranges are offered: the
 * whole sum for n >= 64 has 2^64 terms or more.                           */

#define ORACLE_MAX_N_WIDE 128
#define ORACLE_WIDE_MAX_COUNT ((uint64_t)1 << 62)

typedef unsigned __int128 oracle_u128;

static int valid_input_wide(const uint8_t *A, int n)
{
    if (n < 1 || n > ORACLE_MAX_N_WIDE || A == NULL) return 0;
    for (int k = 0; k < n * n; ++k)
        if (A[k] > 2) return 0;
    return 1;
}

static int popcount128(oracle_u128 x)
{
    return popcount64((uint64_t)x) + popcount64((uint64_t)(x >> 64));
}

static int trailing_zeros128(oracle_u128 x)
{
    int t = 0;
    while (!(x & 1u)) { x >>= 1; ++t; }
    return t;
}

/* [a, a + count) inside [0, 2^n], without forming 2^128. */
static int range_fits_wide(int n, oracle_u128 a, uint64_t count)
{
    if (count > ORACLE_WIDE_MAX_COUNT) return 0;
    if (n == 128) return count == 0 || a <= (oracle_u128)0 - (oracle_u128)count;
    oracle_u128 total = (oracle_u128)1 << n;
    return a <= total && (oracle_u128)count <= total - a;
}

/* One term by its definition at the 128-bit Gray index hi * 2^64 + lo. */
int oracle_term_wide(const uint8_t *A, int n, uint64_t i_hi, uint64_t i_lo)
{
    if (!valid_input_wide(A, n)) return 0;
    oracle_u128 i = ((oracle_u128)i_hi << 64) | i_lo;
    oracle_u128 S = i ^ (i >> 1);
    int prod = 1;
    for (int col = 0; col < n; ++col) {
        int64_t sum = 0;
        for (int k = 0; k < n; ++k)
            if ((S >> k) & 1u) sum += entry(A, n, k, col);
        prod *= centred_mod3(sum);
    }
    return (popcount128(S) & 1) ? -prod : prod;
}

/* T over [a, a + count), a = a_hi * 2^64 + a_lo: the Gray walk of
 * oracle_range_tally on 128-bit indices.  *ok = 0 on invalid input. */
int64_t oracle_range_tally_wide(const uint8_t *A, int n, uint64_t a_hi, uint64_t a_lo, uint64_t count,
                                int *ok)
{
    if (ok) *ok = 0;
    if (!valid_input_wide(A, n)) return 0;
    oracle_u128 a = ((oracle_u128)a_hi << 64) | a_lo;
    if (!range_fits_wide(n, a, count)) return 0;
    if (ok) *ok = 1;
    if (count == 0) return 0;

    int E[ORACLE_MAX_N_WIDE][ORACLE_MAX_N_WIDE];   /* 64 KB of stack */
    for (int k = 0; k < n; ++k)
        for (int col = 0; col < n; ++col)
            E[k][col] = entry(A, n, k, col);

    int v[ORACLE_MAX_N_WIDE];
    oracle_u128 state = a ^ (a >> 1);
    for (int col = 0; col < n; ++col) {
        int64_t sum = 0;
        for (int k = 0; k < n; ++k)
            if ((state >> k) & 1u) sum += E[k][col];
        v[col] = centred_mod3(sum);
    }

    int64_t s = 0;
    for (uint64_t step = 0; step < count; ++step) {
        oracle_u128 i = a + step;
        if (step > 0) {
            int t = trailing_zeros128(i);
            int out = (int)((state >> t) & 1u);     /* row t leaves the subset */
            state ^= (oracle_u128)1 << t;
            for (int col = 0; col < n; ++col)
                v[col] = centred_mod3(out ? v[col] - E[t][col] : v[col] + E[t][col]);
        }
        int prod = 1;
        for (int col = 0; col < n; ++col) prod *= v[col];
        s += (popcount128(state) & 1) ? -prod : prod;
    }
    return s;
}

typedef struct {
    const uint8_t *A;
    int n;
    oracle_u128 a;
    uint64_t count;
    int64_t out;
    int ok;
} oracle_wide_job;

static void *oracle_wide_job_run(void *p)
{
    oracle_wide_job *j = (oracle_wide_job *)p;
    j->out = oracle_range_tally_wide(j->A, j->n, (uint64_t)(j->a >> 64), (uint64_t)j->a, j->count, &j->ok);
    return NULL;
}

/* The same split over host threads into consecutive blocks (Section 3.1). */
int64_t oracle_range_tally_wide_mt(const uint8_t *A, int n, uint64_t a_hi, uint64_t a_lo, uint64_t count,
                                   int nthreads, int *ok)
{
    if (ok) *ok = 0;
    if (!valid_input_wide(A, n)) return 0;
    oracle_u128 a = ((oracle_u128)a_hi << 64) | a_lo;
    if (!range_fits_wide(n, a, count)) return 0;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (count < (uint64_t)nthreads * 4096u) nthreads = 1;

    oracle_wide_job jobs[256];
    pthread_t th[256];
    for (int k = 0; k < nthreads; ++k) {
        uint64_t b0 = (uint64_t)((oracle_u128)count * (uint64_t)k / (uint64_t)nthreads);
        uint64_t b1 = (uint64_t)((oracle_u128)count * (uint64_t)(k + 1) / (uint64_t)nthreads);
        jobs[k].A = A; jobs[k].n = n;
        jobs[k].a = a + b0;
        jobs[k].count = b1 - b0;
        jobs[k].out = 0; jobs[k].ok = 0;
    }
    int started = 0;
    for (int k = 1; k < nthreads; ++k) {
        if (pthread_create(&th[k], NULL, oracle_wide_job_run, &jobs[k]) != 0) break;
        started = k;
    }
    oracle_wide_job_run(&jobs[0]);
    for (int k = started + 1; k < nthreads; ++k)
        oracle_wide_job_run(&jobs[k]);
    for (int k = 1; k <= started; ++k) pthread_join(th[k], NULL);

    int64_t s = 0;
    int all_ok = 1;
    for (int k = 0; k < nthreads; ++k) { s += jobs[k].out; all_ok &= jobs[k].ok; }
    if (ok) *ok = all_ok;
    return s;
}

/* ------------------------------------------------------------------ */
/* Vectors over F_3 (Section 2 and Theorem 2.1 beyond the permanent): the
 * definitions, on unpacked values.  A vector is bytes in {0,1,2} (2 = -1).
 * Its bipedal form is ceil(len/64) word pairs, planes[2w] = mag and
 * planes[2w+1] = sgn, element e at bit e mod 64 of word e / 64.           */

/* The element of F_3 named by 0, 1 or -1 as a byte. */
static uint8_t f3_byte(int x)
{
    int r = centred_mod3(x);
    return r < 0 ? 2 : (uint8_t)r;
}

static int f3_value(uint8_t b) { return b == 2 ? -1 : (int)b; }

/* phi of Section 2: 0 -> (0,0), 1 -> (1,0), -1 -> (1,1).  Bytes > 2 are left
 * as (0,0) and counted; the count is returned. */
int64_t oracle_f3_phi(const uint8_t *v, int64_t len, uint64_t *planes)
{
    int64_t words = (len + 63) / 64, bad = 0;
    for (int64_t w = 0; w < 2 * words; ++w) planes[w] = 0;
    for (int64_t e = 0; e < len; ++e) {
        uint64_t bit = (uint64_t)1 << (e % 64);
        if (v[e] > 2) { ++bad; continue; }
        if (v[e] != 0) planes[2 * (e / 64)] |= bit;        /* magnitude: non-zero */
        if (v[e] == 2) planes[2 * (e / 64) + 1] |= bit;    /* sign: -1 */
    }
    return bad;
}

/* psi of Section 2: magnitude 0 is 0 whatever the sign bit; else the sign bit
 * chooses between 1 and -1. */
void oracle_f3_psi(const uint64_t *planes, int64_t len, uint8_t *v)
{
    for (int64_t e = 0; e < len; ++e) {
        int m = (int)((planes[2 * (e / 64)] >> (e % 64)) & 1u);
        int s = (int)((planes[2 * (e / 64) + 1] >> (e % 64)) & 1u);
        v[e] = m ? (s ? 2 : 1) : 0;
    }
}

/* out_e = a_e op b_e in F_3; op 0 add, 1 subtract, 2 multiply, 3 divide,
 * 4 negate a.  Division multiplies by the inverse found from its definition
 * (the y with b y = 1); where b_e = 0 the quotient is undefined and out_e is
 * 0xFF.  Returns -1 for an unknown op or an entry > 2. */
int oracle_f3_op(int op, const uint8_t *a, const uint8_t *b, int64_t len, uint8_t *out)
{
    if (op < 0 || op > 4) return -1;
    for (int64_t e = 0; e < len; ++e) {
        if (a[e] > 2 || (op != 4 && b[e] > 2)) return -1;
        int x = f3_value(a[e]);
        int y = op == 4 ? 0 : f3_value(b[e]);
        switch (op) {
        case 0: out[e] = f3_byte(x + y); break;
        case 1: out[e] = f3_byte(x - y); break;
        case 2: out[e] = f3_byte(x * y); break;
        case 3: {
            int inv = 0;
            for (int c = -1; c <= 1; ++c)
                if (centred_mod3(y * c) == 1) inv = c;
            out[e] = inv ? f3_byte(x * inv) : 0xFF;
            break;
        }
        default: out[e] = f3_byte(-x); break;
        }
    }
    return 0;
}

/* sum over e of a_e * b_e as integers in {-1,0,1} (the F_3 dot product is
 * this mod 3). */
int64_t oracle_f3_dot(const uint8_t *a, const uint8_t *b, int64_t len)
{
    int64_t s = 0;
    for (int64_t e = 0; e < len; ++e) s += (int64_t)f3_value(a[e]) * f3_value(b[e]);
    return s;
}
