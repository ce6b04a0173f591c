/* Host-side checks of the C ABI under AddressSanitizer and UBSan: descriptor
 * validation, schedule records, tuning keys, NULL and invalid arguments of
 * every entry point, and grid or batch creation failing cleanly on a host
 * without a GPU.  Built from the host half of the library by
 * tests/test_sanitize.py; prints "abi-ok" when every check held. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "ell.h"

static int failures = 0;
#define CHECK(cond)                                                    \
    do {                                                               \
        if (!(cond)) {                                                 \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            failures++;                                                \
        }                                                              \
    } while (0)

static double dz[300], lam[300];

static ell_grid_desc base(void) {
    ell_grid_desc d;
    memset(&d, 0, sizeof d);
    d.nx = 32; d.ny = 32; d.nz = 16;
    d.hx = 1.0 / 32; d.hy = 1.0 / 32; d.omega2 = 1e-2;
    d.dz = dz; d.lambda2 = lam;
    d.n_levels = 0; d.nu_pre = 1; d.nu_post = 1; d.nu_coarse = 1;
    d.rho = 1.0; d.prolong = 0; d.precision = ELL_FP64;
    return d;
}

int main(void) {
    for (int k = 0; k < 300; k++) { dz[k] = 1.0 / 16; lam[k] = 1e4; }
    ell_grid_desc d = base();
    CHECK(ell_grid_bytes(&d) > 5u * 32 * 32 * 16 * 8);
    d.precision = ELL_FP32_PRECOND;
    CHECK(ell_grid_bytes(&d) > 0);
    d = base(); d.nx = 1; d.ny = 1;
    CHECK(ell_grid_bytes(&d) > 0);
    d = base(); d.nz = 300;
    CHECK(ell_grid_bytes(&d) > 0);

    /* every invalid descriptor: 0 bytes and a message */
    for (int v = 0; v < 15; v++) {
        d = base();
        switch (v) {
            case 0: d.nx = 33; break;
            case 1: d.ny = 3; break;
            case 2: d.nz = 0; break;
            case 3: d.hx = 0.0; break;
            case 4: d.hy = NAN; break;
            case 5: d.rho = 2.0; break;
            case 6: d.n_levels = 7; break;
            case 7: d.prolong = 2; break;
            case 8: d.precision = 5; break;
            case 9: d.omega2 = -1.0; break;
            case 10: d.dz = NULL; break;
            case 11: d.nu_pre = -1; break;
            case 12: d.nu_coarse = 5000; break;
            case 13: d.nx = 1 << 16; d.ny = 1 << 16; break;
            case 14: d.lambda2 = NULL; break;
        }
        CHECK(ell_grid_bytes(&d) == 0);
        CHECK(strlen(ell_last_error()) > 0);
    }
    {
        double bad[16];
        for (int k = 0; k < 16; k++) bad[k] = 1.0 / 16;
        bad[15] = 0.0;
        d = base(); d.dz = bad;
        CHECK(ell_grid_bytes(&d) == 0);
        bad[15] = INFINITY;
        CHECK(ell_grid_bytes(&d) == 0);
        d = base(); bad[15] = NAN; d.lambda2 = bad;
        CHECK(ell_grid_bytes(&d) == 0);
    }
    CHECK(ell_grid_bytes(NULL) == 0);

    /* schedule records: heuristic, set, get, reject invalid, clear */
    {
        ell_schedule s0, s1, s2;
        d = base(); d.nx = 64; d.ny = 64; d.nz = 128; d.hx = d.hy = 1.0 / 64; d.n_levels = 4;
        CHECK(ell_schedule_get(&d, &s0) == ELL_OK);
        s1 = s0;
        s1.apply_tile = 0; s1.apply_nseg = 2;
        CHECK(ell_schedule_set(&d, &s1) == ELL_OK);
        CHECK(ell_schedule_get(&d, &s2) == ELL_OK);
        CHECK(s2.apply_tile == 0 && s2.apply_nseg == 2);
        s1.apply_nseg = 3;
        CHECK(ell_schedule_set(&d, &s1) == ELL_ERR_INVALID);
        s1.apply_nseg = 2; s1.smooth_nseg[2] = 5;
        CHECK(ell_schedule_set(&d, &s1) == ELL_ERR_INVALID);
        CHECK(ell_schedule_set(&d, NULL) == ELL_OK);
        CHECK(ell_schedule_get(&d, &s2) == ELL_OK);
        CHECK(memcmp(&s0, &s2, sizeof s0) == 0);
        CHECK(ell_schedule_get(NULL, &s2) != ELL_OK);
        CHECK(ell_schedule_get(&d, NULL) != ELL_OK);
    }

    /* tuning keys: in range accepted, out of range rejected */
    CHECK(ell_set_tuning(ELL_TUNE_FUSED_DOT, 1) == ELL_OK);
    CHECK(ell_set_tuning(-1, 0) == ELL_ERR_INVALID);
    CHECK(ell_set_tuning(1000, 0) == ELL_ERR_INVALID);

    /* NULL handles and arguments */
    {
        ell_grid *g = (ell_grid *)0;
        ell_solve_stats st;
        CHECK(ell_grid_create(NULL, &g) == ELL_ERR_INVALID && g == NULL);
        d = base();
        CHECK(ell_grid_create(&d, NULL) == ELL_ERR_INVALID);
        CHECK(ell_grid_destroy(NULL) == ELL_OK);
        CHECK(ell_grid_levels(NULL) == ELL_ERR_INVALID);
        CHECK(ell_apply_A(NULL, NULL, NULL, 0) == ELL_ERR_INVALID);
        CHECK(ell_vcycle(NULL, NULL, NULL, 0) == ELL_ERR_INVALID);
        CHECK(ell_pcg_solve(NULL, NULL, NULL, NULL, &st, 0) == ELL_ERR_INVALID);
        CHECK(ell_mg_solve(NULL, NULL, NULL, NULL, &st, 0) == ELL_ERR_INVALID);
        CHECK(ell_level_elems(NULL, 0) == 0);
        CHECK(ell_level_smooth(NULL, 0, 0, 0, NULL, NULL, 0) != ELL_OK);
        CHECK(ell_profile_enable(NULL, 0, 4) != ELL_OK);
        CHECK(ell_batch_submit(NULL, 0, NULL, NULL, NULL, NULL, NULL) != ELL_OK);
        CHECK(ell_batch_poll(NULL, 1, NULL) != ELL_OK);
        CHECK(ell_batch_destroy(NULL) == ELL_OK || ell_batch_destroy(NULL) == ELL_ERR_INVALID);

        /* without a GPU: creation fails with a message and no grid */
        int rc = ell_grid_create(&d, &g);
        CHECK(rc < 0 && g == NULL && strlen(ell_last_error()) > 0);
        ell_batch *b = (ell_batch *)0;
        rc = ell_batch_create((size_t)1 << 30, &b);
        if (rc == ELL_OK) {
            CHECK(ell_batch_grid(b, &d, &g) < 0 && g == NULL);
            CHECK(ell_batch_destroy(b) == ELL_OK);
        } else {
            CHECK(rc < 0 && b == NULL);
        }
    }
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("abi-ok\n");
    return 0;
}
