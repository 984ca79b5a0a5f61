/*
 * A plain C99 user of libperm3 through include/perm3.h alone (test
 * infrastructure).  With no argument it calls only what needs no GPU (the
 * version, status names, argument checks and the host phi packer of
 * Section 2) and prints "host ok".  With "gpu" it also computes permanents
 * whose values are fixed by closed forms and prints "gpu ok".  It exits
 * non-zero at the first mismatch.
 */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "perm3.h"

static int fails = 0;

#define EXPECT(cond)                                                   \
    do {                                                               \
        if (!(cond)) {                                                 \
            fprintf(stderr, "line %d: %s failed\n", __LINE__, #cond); \
            ++fails;                                                   \
        }                                                              \
    } while (0)

static void host_checks(void)
{
    /* the worked example of Section 2: (1, 1, 0, -1) packs to (0xd, 0x1) */
    const uint8_t row[16] = {1, 1, 0, 2, 0, 1, 0, 0, 2, 2, 1, 0, 0, 0, 0, 1};
    uint64_t planes[8];
    EXPECT(strstr(perm_version(), "gfx950") != NULL);
    EXPECT(strcmp(perm_strerror(PERM_OK), "ok") == 0);
    EXPECT(perm_mod3_pack(row, 4, planes) == PERM_OK);
    EXPECT(planes[0] == 0x0d && planes[1] == 0x01);   /* first row of the 4 x 4 matrix */
    /* argument checks return before any device work */
    uint8_t out = 0;
    EXPECT(perm_mod3(row, 64, &out) == PERM_EINVAL);
    EXPECT(perm_mod3(row, 4, NULL) == PERM_EINVAL);
    const uint8_t bad[4] = {0, 1, 3, 2};
    EXPECT(perm_mod3(bad, 2, &out) == PERM_EDOMAIN);
    EXPECT(perm_last_error_index() == 2);
    int64_t t = 0;
    EXPECT(perm_mod3_range_tally(row, 4, 3, 2, &t) == PERM_EINVAL);
    EXPECT(perm_mod3_range_tally_wide(row, 129, 0, 0, 1, &t) == PERM_EINVAL);
    EXPECT(perm_f3_op(99, NULL, NULL, NULL, 1, NULL) == PERM_EINVAL);
}

static void gpu_checks(void)
{
    uint8_t A[64 * 64];
    uint8_t out = 7;
    int64_t t = 0;
    /* perm(I_n) = 1, perm(2 I_n) = 2^n mod 3, perm(J_n) = n! mod 3 */
    for (int n = 1; n <= 40; n += 13) {
        memset(A, 0, sizeof A);
        for (int i = 0; i < n; ++i) A[i * n + i] = 1;
        EXPECT(perm_mod3(A, n, &out) == PERM_OK && out == 1);
        for (int i = 0; i < n; ++i) A[i * n + i] = 2;
        EXPECT(perm_mod3(A, n, &out) == PERM_OK && out == ((n & 1) ? 2 : 1));
        /* T(0, 2^n) of I_n is (-1)^n: one non-zero term, the full subset */
        for (int i = 0; i < n; ++i) A[i * n + i] = 1;
        EXPECT(perm_mod3_range_tally(A, n, 0, 1ull << n, &t) == PERM_OK && t == ((n & 1) ? -1 : 1));
    }
    memset(A, 1, sizeof A);
    EXPECT(perm_mod3(A, 2, &out) == PERM_OK && out == 2);    /* 2! = 2 */
    EXPECT(perm_mod3(A, 3, &out) == PERM_OK && out == 0);    /* 3! = 6 */
    /* the empty matrix */
    EXPECT(perm_mod3(NULL, 0, &out) == PERM_OK && out == 1);
    /* a batch through host pointers */
    const uint8_t *as[3] = {A, A, A};
    const int32_t ns[3] = {2, 3, 4};
    uint8_t outs[3] = {9, 9, 9};
    EXPECT(perm_mod3_batch(as, ns, 3, outs) == PERM_OK && outs[0] == 2 && outs[1] == 0 && outs[2] == 0);
}

int main(int argc, char **argv)
{
    host_checks();
    if (fails) return 1;
    printf("host ok\n");
    if (argc > 1 && strcmp(argv[1], "gpu") == 0) {
        gpu_checks();
        if (fails) return 1;
        printf("gpu ok\n");
    }
    return 0;
}
