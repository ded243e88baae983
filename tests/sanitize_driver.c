/*
 * Exercises the CPU oracle (oracle/oracle.c) and the workload generator
 * (workload/gen.c) built with AddressSanitizer and UndefinedBehaviorSanitizer:
 * every entry point on small profiles of both id widths, weighted and not,
 * both weight modes, truncated and full ballots, and the invalid inputs the
 * oracle rejects.  Exits non-zero on any failed check (the sanitizers abort
 * on their own findings).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_pairwise(const void *, int, int64_t, int32_t, int32_t, const uint32_t *, int64_t *);
int oracle_pairwise_rows(const void *, int, int64_t, int32_t, int32_t, const uint32_t *, const int32_t *, int64_t,
                         int64_t *);
int oracle_pairwise_cols(const void *, int, int64_t, int32_t, int32_t, const uint32_t *, const int32_t *, int64_t,
                         int64_t *);
int oracle_weights(const int64_t *, int32_t, int, int64_t *);
int oracle_closure(const int64_t *, int32_t, int64_t *);
int oracle_rank(const int64_t *, int32_t, int32_t *, uint8_t *, int32_t *);
int oracle_widest_from(const int64_t *, int32_t, int32_t, int64_t *);
int oracle_widest_to(const int64_t *, int32_t, int32_t, int64_t *);
int oracle_set_threads(int);
int gen_permutation(uint64_t, uint64_t, int32_t, int32_t *);
int gen_mallows(uint64_t, uint64_t, int64_t, int32_t, double, const int32_t *, int32_t, int32_t, int32_t, int32_t, int,
                void *);
int gen_pl_zipf(uint64_t, uint64_t, int64_t, int32_t, double, const int32_t *, int32_t, int32_t, int, void *);
int gen_mallows_topk(uint64_t, uint64_t, int64_t, int32_t, double, const int32_t *, int32_t, int32_t, int, void *);
int gen_uniform_int(uint64_t, uint64_t, int64_t, int64_t, int64_t, int64_t *);
int gen_uniform_real(uint64_t, uint64_t, int64_t, double, double, double *);
int gen_uniform_ballots(uint64_t, uint64_t, int64_t, int32_t, int32_t, int32_t, int, void *);

static int failures = 0;
#define CHECK(cond, what)                                        \
    do {                                                         \
        if (!(cond)) {                                           \
            fprintf(stderr, "check failed: %s (%s)\n", what, #cond); \
            ++failures;                                          \
        }                                                        \
    } while (0)

/* The whole oracle path on one profile. */
static void run_profile(const void *b, int dtype32, int64_t n, int32_t L, int32_t m, const uint32_t *w) {
    int64_t *d = malloc(sizeof(int64_t) * m * m), *wt = malloc(sizeof(int64_t) * m * m);
    int64_t *p = malloc(sizeof(int64_t) * m * m), *row = malloc(sizeof(int64_t) * m * 2);
    int32_t *beaten = malloc(sizeof(int32_t) * m), *order = malloc(sizeof(int32_t) * m);
    uint8_t *win = malloc(m);
    int32_t sel[2] = {0, m - 1};
    CHECK(oracle_pairwise(b, dtype32, n, L, m, w, d) == 0, "pairwise");
    CHECK(oracle_pairwise_rows(b, dtype32, n, L, m, w, sel, 2, row) == 0, "pairwise_rows");
    for (int32_t y = 0; y < m; ++y) CHECK(row[y] == d[y] && row[m + y] == d[(int64_t)(m - 1) * m + y], "rows agree");
    CHECK(oracle_pairwise_cols(b, dtype32, n, L, m, w, sel, 2, row) == 0, "pairwise_cols");
    for (int32_t x = 0; x < m; ++x) CHECK(row[x] == d[(int64_t)x * m], "cols agree");
    for (int mode = 0; mode < 2; ++mode) {
        CHECK(oracle_weights(d, m, mode, wt) == 0, "weights");
        CHECK(oracle_closure(wt, m, p) == 0, "closure");
        const int ranked = oracle_rank(p, m, beaten, win, order);  /* the number of winners */
        int nwin = 0;
        for (int32_t x = 0; x < m; ++x) nwin += win[x];
        CHECK(ranked >= 1 && ranked == nwin, "rank: winners");
        for (int32_t s = 0; s < m; s += (m > 7 ? m / 3 : 1)) {
            CHECK(oracle_widest_from(wt, m, s, row) == 0, "widest_from");
            for (int32_t x = 0; x < m; ++x) CHECK(row[x] == p[(int64_t)s * m + x], "row of p");
            CHECK(oracle_widest_to(wt, m, s, row) == 0, "widest_to");
            for (int32_t x = 0; x < m; ++x) CHECK(row[x] == p[(int64_t)x * m + s], "column of p");
        }
    }
    free(d), free(wt), free(p), free(row), free(beaten), free(order), free(win);
}

int main(void) {
    oracle_set_threads(2);
    const int32_t ms[] = {1, 2, 5, 33, 70};
    for (int i = 0; i < 5; ++i) {
        const int32_t m = ms[i];
        const int64_t n = 37;
        int32_t *perm = malloc(sizeof(int32_t) * m);
        uint16_t *b16 = malloc(sizeof(uint16_t) * n * m);
        int32_t *b32 = malloc(sizeof(int32_t) * n * m);
        uint32_t *w = malloc(sizeof(uint32_t) * n);
        for (int64_t v = 0; v < n; ++v) w[v] = (uint32_t)(v % 5);
        CHECK(gen_permutation(7, i, m, perm) == 0, "permutation");
        CHECK(gen_mallows(7, i, n, m, 0.8, perm, m, 3, 1, m / 2, 0, b16) == 0, "mallows u16");
        run_profile(b16, 0, n, m, m, NULL);
        run_profile(b16, 0, n, m, m, w);
        CHECK(gen_mallows(7, i, n, m, 1.0, perm, m, 0, 0, 0, 1, b32) == 0, "mallows i32");
        run_profile(b32, 1, n, m, m, NULL);
        const int32_t k = m < 4 ? m : 4;
        CHECK(gen_pl_zipf(7, i, n, m, 1.1, perm, k, k, 0, b16) == 0, "pl_zipf");
        run_profile(b16, 0, n, k, m, NULL);
        CHECK(gen_mallows_topk(7, i, n, m, 0.9, perm, k, k, 1, b32) == 0, "mallows_topk");
        run_profile(b32, 1, n, k, m, w);
        CHECK(gen_uniform_ballots(7, i, n, m, m, 0, 0, b16) == 0, "uniform");
        run_profile(b16, 0, n, m, m, NULL);
        /* a repeated id and an id out of range are rejected */
        if (m >= 2) {
            int64_t *d = malloc(sizeof(int64_t) * m * m);
            int32_t bad[2] = {1, 1};
            CHECK(oracle_pairwise(bad, 1, 1, 2, m, NULL, d) < 0, "repeated id rejected");
            bad[0] = m;
            CHECK(oracle_pairwise(bad, 1, 1, 2, m, NULL, d) < 0, "id out of range rejected");
            free(d);
        }
        free(perm), free(b16), free(b32), free(w);
    }
    int64_t iv[16];
    double rv[16];
    CHECK(gen_uniform_int(3, 1, 16, -5, 5, iv) == 0, "uniform_int");
    for (int i = 0; i < 16; ++i) CHECK(iv[i] >= -5 && iv[i] <= 5, "uniform_int range");
    CHECK(gen_uniform_real(3, 2, 16, 0.5, 1.0, rv) == 0, "uniform_real");
    for (int i = 0; i < 16; ++i) CHECK(rv[i] >= 0.5 && rv[i] <= 1.0, "uniform_real range");
    CHECK(gen_mallows(7, 0, 4, 3, 0.5, NULL, 3, 0, 0, 0, 0, rv) < 0, "null reference order rejected");
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("sanitized oracle and generator: all checks passed\n");
    return 0;
}
