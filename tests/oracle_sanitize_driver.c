/*
 * Drives every entry point of the CPU oracle on small problems, for the
 * AddressSanitizer / UndefinedBehaviorSanitizer build of the CPU test tier
 * (tests/test_oracle_sanitizers.py).  Exits non-zero on a wrong result; the
 * sanitizers abort on a memory or undefined-behaviour error.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

static double urand(unsigned *s) {
    *s = *s * 1103515245u + 12345u;
    return ((*s >> 8) & 0xffff) / 32768.0 - 1.0;
}

static void exercise(int nx, int ny, int nz, int levels, int order, int use_theta, int sweeps) {
    unsigned seed = (unsigned)(nx * 131 + ny * 17 + nz * 7 + levels * 3 + order);
    int64_t n0 = (int64_t)nx * ny * nz;
    double *theta = NULL;
    if (use_theta) {
        theta = malloc((size_t)n0 * sizeof(double));
        for (int64_t i = 0; i < n0; ++i) theta[i] = 2.0 * urand(&seed);
    }
    ora_hier *h = ora_create(nx, ny, nz, levels, order, theta);
    CHECK(h != NULL);
    if (!h) { free(theta); return; }
    CHECK(ora_set_sweeps(h, sweeps) == 0);
    for (int l = 0; l < levels; ++l) {
        int64_t n = ora_n(h, l), nnz = ora_nnz(h, l);
        int64_t *rp = malloc((size_t)(n + 1) * sizeof(int64_t));
        int32_t *col = malloc((size_t)nnz * sizeof(int32_t));
        double *val = malloc((size_t)nnz * sizeof(double));
        int32_t *colour = malloc((size_t)n * sizeof(int32_t));
        ora_get_crs(h, l, rp, col, val);
        ora_get_colours(h, l, colour);
        CHECK(rp[n] == nnz);
        double *x = malloc((size_t)n * sizeof(double)), *y = malloc((size_t)n * sizeof(double));
        double *z = calloc((size_t)n, sizeof(double));
        float *r32 = malloc((size_t)n * sizeof(float)), *z32 = calloc((size_t)n, sizeof(float));
        for (int64_t i = 0; i < n; ++i) { x[i] = urand(&seed); r32[i] = (float)x[i]; }
        ora_spmv(h, l, x, y);
        for (int k = 0; k < ora_ncolours(h, l); ++k) ora_colour_pass(h, l, k, x, z);
        ora_sgs(h, l, x, z);
        ora_sgs_lex(h, l, x, z);
        ora_sgs32(h, l, r32, z32);
        for (int64_t i = 0; i < n; ++i) CHECK(isfinite(z[i]) && isfinite(z32[i]));
        if (l + 1 < levels) {
            int64_t nc = ora_n(h, l + 1);
            int64_t *f2c = malloc((size_t)nc * sizeof(int64_t));
            double *rc = malloc((size_t)nc * sizeof(double));
            ora_get_f2c(h, l, f2c);
            for (int64_t j = 0; j < nc; ++j) CHECK(f2c[j] >= 0 && f2c[j] < n);
            ora_restrict(h, l, x, z, rc);
            ora_prolong_add(h, l, rc, z);
            free(f2c);
            free(rc);
        }
        ora_vcycle(h, l, x, y);
        ora_vcycle_lex(h, l, x, y);
        free(rp); free(col); free(val); free(colour); free(x); free(y); free(z); free(r32); free(z32);
    }
    double *b = malloc((size_t)n0 * sizeof(double)), *xs = malloc((size_t)n0 * sizeof(double));
    double *ones = malloc((size_t)n0 * sizeof(double)), *hist = malloc(200 * sizeof(double));
    for (int64_t i = 0; i < n0; ++i) ones[i] = 1.0;
    ora_spmv(h, 0, ones, b);
    for (int pre = 0; pre <= 3; ++pre) {
        memset(xs, 0, (size_t)n0 * sizeof(double));
        int it = -1;
        int st = ora_pcg(h, b, xs, 200, 1e-10, pre, hist, &it);
        CHECK(st == 0);
        CHECK(it >= 0 && it <= 200);
        if (!use_theta)
            for (int64_t i = 0; i < n0; ++i) CHECK(fabs(xs[i] - 1.0) < 1e-6);
    }
    double *lam = malloc((size_t)n0 * sizeof(double)), *g = malloc((size_t)n0 * sizeof(double));
    for (int64_t i = 0; i < n0; ++i) lam[i] = urand(&seed);
    if (theta) ora_theta_grad(n0, lam, xs, theta, g);
    CHECK(isfinite(ora_dot(n0, lam, xs)));
    ora_vcycle32(h, b, xs);
    free(b); free(xs); free(ones); free(hist); free(lam); free(g); free(theta);
    ora_destroy(h);
}

int main(void) {
    /* invalid problems are rejected without touching memory */
    CHECK(ora_create(6, 6, 6, 3, 0, NULL) == NULL);
    CHECK(ora_create(0, 4, 4, 1, 0, NULL) == NULL);
    CHECK(ora_create(4, 4, 4, 1, 2, NULL) == NULL);
    CHECK(ora_create(4, 4, 4, ORA_MAX_LEVELS + 1, 0, NULL) == NULL);
    ora_hier *h = ora_create(4, 4, 4, 2, 0, NULL);
    CHECK(h && ora_set_sweeps(h, 0) == -1);
    ora_destroy(h);
    ora_destroy(NULL);
    exercise(1, 1, 1, 1, 0, 0, 1);
    exercise(5, 1, 3, 1, 1, 1, 1);
    exercise(6, 5, 4, 1, 0, 1, 2);
    exercise(8, 8, 8, 4, 0, 0, 1);
    exercise(8, 8, 8, 4, 1, 1, 1);
    exercise(16, 8, 8, 3, 1, 0, 2);
    exercise(16, 16, 8, 4, 0, 1, 1);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer run ok\n");
    return 0;
}
