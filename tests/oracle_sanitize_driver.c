/*
 * Driver for sanitizer builds of the CPU oracle (test infrastructure only):
 * linked with oracle.c under AddressSanitizer + UndefinedBehaviorSanitizer, or
 * under ThreadSanitizer, it runs the oracle's pthread pool on small inputs
 * whose answers are closed forms, with caps, enumeration, several thread counts
 * and a time limit.  Exit status 0 means every answer matched; the sanitizers
 * report memory, undefined-behaviour or data-race errors on stderr.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t count;
    int32_t outcome;
    int32_t threads;
    uint64_t tasks;
    uint64_t groups;
    uint64_t rows;
    double seconds;
} orc_result;

int orc_check_graph(int32_t n, const int64_t *row_ptr, const int32_t *col, int32_t check_symmetry);
int orc_match(int32_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *glabels, int32_t k,
              int32_t m, const int32_t *edges, const int32_t *qlabels, const int32_t *order, uint64_t cap,
              double time_limit_s, int32_t nthreads, int32_t *rows, uint64_t rows_cap, orc_result *out);

static int failures = 0;

static void expect(const char *what, uint64_t got, uint64_t want) {
    if (got != want) {
        fprintf(stderr, "MISMATCH %s: got %llu want %llu\n", what, (unsigned long long)got, (unsigned long long)want);
        ++failures;
    }
}

/* K_n: row v lists every other vertex in ascending order */
static void complete(int32_t n, int64_t **rp, int32_t **col) {
    *rp = malloc(sizeof(int64_t) * (size_t)(n + 1));
    *col = malloc(sizeof(int32_t) * (size_t)n * (size_t)(n - 1) + 1);
    int64_t at = 0;
    for (int32_t v = 0; v < n; ++v) {
        (*rp)[v] = at;
        for (int32_t w = 0; w < n; ++w)
            if (w != v) (*col)[at++] = w;
    }
    (*rp)[n] = at;
}

/* a x b grid, vertex (i, j) = i * b + j */
static void grid(int32_t a, int32_t b, int64_t **rp, int32_t **col) {
    const int32_t n = a * b;
    *rp = malloc(sizeof(int64_t) * (size_t)(n + 1));
    *col = malloc(sizeof(int32_t) * (size_t)n * 4);
    int64_t at = 0;
    for (int32_t i = 0; i < a; ++i)
        for (int32_t j = 0; j < b; ++j) {
            (*rp)[i * b + j] = at;
            if (i > 0) (*col)[at++] = (i - 1) * b + j;
            if (j > 0) (*col)[at++] = i * b + j - 1;
            if (j + 1 < b) (*col)[at++] = i * b + j + 1;
            if (i + 1 < a) (*col)[at++] = (i + 1) * b + j;
        }
    (*rp)[n] = at;
}

static uint64_t falling(uint64_t n, int k) {
    uint64_t r = 1;
    for (int i = 0; i < k; ++i) r *= n - (uint64_t)i;
    return r;
}

int main(void) {
    orc_result r;
    int32_t zero[64] = {0};
    /* cliques and paths in K_12: n! / (n - k)! for any connected k-vertex query */
    int64_t *rp;
    int32_t *col;
    const int32_t n = 12;
    complete(n, &rp, &col);
    expect("check K12", (uint64_t)orc_check_graph(n, rp, col, 1), 0);
    const int32_t tri[] = {0, 1, 1, 2, 0, 2};
    const int32_t path5[] = {0, 1, 1, 2, 2, 3, 3, 4};
    for (int32_t threads = 1; threads <= 8; threads *= 2) {
        orc_match(n, rp, col, zero, 3, 3, tri, zero, NULL, 0, 0.0, threads, NULL, 0, &r);
        expect("triangles in K12", r.count, falling(12, 3));
        orc_match(n, rp, col, zero, 5, 4, path5, zero, NULL, 0, 0.0, threads, NULL, 0, &r);
        expect("5-paths in K12", r.count, falling(12, 5));
        orc_match(n, rp, col, zero, 5, 4, path5, zero, NULL, 1000, 0.0, threads, NULL, 0, &r);
        expect("capped 5-paths", r.count, 1000);
        expect("capped outcome", (uint64_t)r.outcome, 1);
    }
    /* enumeration: every row injective */
    int32_t *rows = malloc(sizeof(int32_t) * 3 * 1320);
    orc_match(n, rp, col, zero, 3, 3, tri, zero, NULL, 0, 0.0, 4, rows, 1320, &r);
    expect("enumerated rows", r.rows, 1320);
    for (uint64_t i = 0; i < r.rows; ++i) {
        const int32_t *x = rows + 3 * i;
        if (x[0] == x[1] || x[1] == x[2] || x[0] == x[2]) ++failures;
    }
    free(rows);
    /* a time limit the search cannot meet ends it with a lower bound */
    const int32_t path8[] = {0, 1, 1, 2, 2, 3, 3, 4, 4, 5, 5, 6, 6, 7};
    orc_match(n, rp, col, zero, 8, 7, path8, zero, NULL, 0, 1e-4, 4, NULL, 0, &r);
    if (r.outcome != 2 && r.count != falling(12, 8)) ++failures;
    free(rp);
    free(col);
    /* 4-cycles in a 5 x 7 grid: 8 (a - 1)(b - 1) */
    grid(5, 7, &rp, &col);
    const int32_t c4[] = {0, 1, 1, 2, 2, 3, 0, 3};
    for (int32_t threads = 1; threads <= 4; threads *= 2) {
        orc_match(35, rp, col, zero, 4, 4, c4, zero, NULL, 0, 0.0, threads, NULL, 0, &r);
        expect("4-cycles in a 5x7 grid", r.count, 8 * 4 * 6);
        orc_match(35, rp, col, zero, 3, 3, tri, zero, NULL, 0, 0.0, threads, NULL, 0, &r);
        expect("triangles in a grid", r.count, 0);
    }
    free(rp);
    free(col);
    if (failures) fprintf(stderr, "%d failures\n", failures);
    else printf("sanitizer driver ok\n");
    return failures ? 1 : 0;
}
