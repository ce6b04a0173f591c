/* Runs every exported function of the FP64 oracle (oracle/ell_oracle.c,
 * included here as one translation unit) on small grids, one-column-wide and
 * single-column ones included, under AddressSanitizer and UBSan.  Checks a
 * few facts on the way (A 1 = V, finite results, convergence) and prints
 * "oracle-ok".  Built by tests/test_sanitize.py. */
#include "../../oracle/ell_oracle.c"

#include <stdio.h>

static int failures = 0;
#define CHECK(cond)                                                    \
    do {                                                               \
        if (!(cond)) {                                                 \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            failures++;                                                \
        }                                                              \
    } while (0)

static double frand(unsigned *s) {
    *s = *s * 1664525u + 1013904223u;
    return ((*s >> 8) & 0xffff) / 65536.0 - 0.5;
}

static void run(int nx, int ny, int nz, int levels, int nu_coarse, unsigned seed) {
    size_t n = (size_t)nx * ny * nz;
    double *dz = malloc(sizeof(double) * nz), *lam = malloc(sizeof(double) * nz);
    for (int k = 0; k < nz; k++) {
        dz[k] = 1e-3 * (k + 1) * (k + 1);
        lam[k] = 1.0 + 0.5 * k;
    }
    orc_geom g = {nx, ny, nz, 1.0 / nx, 1.0 / ny, 0.05, dz, lam};
    double *x = malloc(sizeof(double) * n), *y = malloc(sizeof(double) * n);
    double *z = malloc(sizeof(double) * n), *w = malloc(sizeof(double) * n);
    for (size_t c = 0; c < n; c++) x[c] = 1.0;
    orc_apply(&g, x, y);
    for (int k = 0; k < nz; k++)
        for (size_t c = (size_t)k * nx * ny; c < (size_t)(k + 1) * nx * ny; c++)
            CHECK(fabs(y[c] - g.hx * g.hy * dz[k]) <= 1e-12 * g.hx * g.hy * dz[k]);
    for (size_t c = 0; c < n; c++) x[c] = frand(&seed);
    orc_apply_abs(&g, x, z);
    orc_apply(&g, x, y);
    for (size_t c = 0; c < n; c++) CHECK(fabs(y[c]) <= z[c] * (1 + 1e-14));
    memcpy(w, x, sizeof(double) * n);
    orc_smooth_colour(&g, 0, 1.0, y, w);
    orc_smooth_colour(&g, 1, 0.8, y, w);
    orc_residual(&g, y, w, z);
    for (size_t c = 0; c < n; c++) CHECK(isfinite(w[c]) && isfinite(z[c]));
    if (nx % 2 == 0 && ny % 2 == 0) {
        size_t nc = n / 4;
        double *bc = malloc(sizeof(double) * nc);
        orc_restrict(&g, z, bc);
        orc_prolong_add(&g, 0, bc, w);
        orc_prolong_add(&g, 1, bc, w);
        for (size_t c = 0; c < n; c++) CHECK(isfinite(w[c]));
        free(bc);
    }
    orc_mg mg = {g, levels, 1, 1, nu_coarse, 1.0, 0};
    CHECK(orc_num_levels(&mg) >= 1);
    CHECK(orc_vcycle(&mg, y, z) == 0);
    orc_opts o = {1e-8, 0.0, 200, 1, 0};
    orc_stats st;
    memset(w, 0, sizeof(double) * n);
    CHECK(orc_pcg(&mg, &o, x, w, &st) == 0);
    CHECK(st.status == 0 && st.iters > 0 && st.r_norm < 1e-8 * st.r0_norm);
    o.flexible = 0;
    o.rel_to_rhs = 1;
    CHECK(orc_pcg(&mg, &o, x, w, &st) == 0 && st.status == 0);   /* warm start */
    memset(w, 0, sizeof(double) * n);
    o.maxiter = 400;
    CHECK(orc_mg_solve(&mg, &o, x, w, &st) == 0 && st.status == 0);
    orc_mg bad = mg;
    bad.n_levels = 40;
    CHECK(orc_vcycle(&bad, y, z) == -1 && orc_pcg(&bad, &o, x, w, &st) == -1);
    free(dz); free(lam); free(x); free(y); free(z); free(w);
}

int main(void) {
    run(8, 8, 6, 0, 1, 1u);
    run(8, 4, 5, 2, 3, 2u);
    run(1, 4, 3, 0, 1, 3u);
    run(4, 1, 3, 0, 1, 4u);
    run(1, 1, 7, 0, 1, 5u);
    run(16, 16, 4, 3, 5, 6u);
    {
        double a[5] = {4, 5, 6, 5, 4}, b[5] = {-1, -1, -1, -1, 0}, c[5] = {0, -1, -1, -1, -1};
        double f[5] = {1, 2, 3, 4, 5}, u[5], s[5] = {1, 1, 1, 1, 1}, Tz[6] = {0, 2, 3, 2, 1, 0};
        double wv[5], work[10];
        orc_thomas_plain(5, a, b, c, f, u);
        for (int i = 0; i < 5; i++) {
            double r = a[i] * u[i] - f[i];
            if (i < 4) r += b[i] * u[i + 1];
            if (i > 0) r += c[i] * u[i - 1];
            CHECK(fabs(r) < 1e-12);
        }
        orc_column_solve(5, s, Tz, f, wv, work);
        for (int k = 0; k < 5; k++) {
            double r = (s[k] + Tz[k] + Tz[k + 1]) * wv[k] - f[k];
            if (k > 0) r -= Tz[k] * wv[k - 1];
            if (k < 4) r -= Tz[k + 1] * wv[k + 1];
            CHECK(fabs(r) < 1e-12);
        }
    }
    orc_set_num_threads(2);
    CHECK(orc_num_threads() >= 1);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle-ok\n");
    return 0;
}
