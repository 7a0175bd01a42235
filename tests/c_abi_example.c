/*
 * A plain C99 caller of liblbm.so through include/lbm.h (built and run by
 * tests/test_c_header.py).  On a machine with a GPU it runs a small D3Q19
 * box for a few steps and checks that mass is conserved; without one it
 * checks the host-only calls and that lbm_create reports LBM_ENODEV.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "lbm.h"

int main(void)
{
    int32_t D = 0, Q = 0, two_n = 0, c[39 * 3];
    double T0 = 0.0, w[39], wsum = 0.0;
    if (lbm_lattice_table(LBM_D3Q19, &D, &Q, &T0, &two_n, c, w) != LBM_OK) return 1;
    for (int i = 0; i < Q; ++i) wsum += w[i];
    if (D != 3 || Q != 19 || two_n != 4 || fabs(T0 - 1.0 / 3.0) > 1e-15 || fabs(wsum - 1.0) > 1e-15) return 2;
    if (lbm_lattice_table(42, NULL, NULL, NULL, NULL, NULL, NULL) != LBM_EINVAL) return 3;
    if (lbm_last_error()[0] == '\0') return 4;

    const int64_t dims[3] = {16, 8, 4};
    lbm_t h = NULL;
    lbm_status st = lbm_create(&h, LBM_D3Q19, dims, 0.6, LBM_FP32);
    if (st == LBM_ENODEV) {
        printf("c abi example: no GPU (%s)\n", lbm_last_error());
        return 0;
    }
    if (st != LBM_OK) return 5;
    const int64_t n = dims[0] * dims[1] * dims[2];
    double* rho = malloc(sizeof(double) * (size_t)n);
    double* u = malloc(sizeof(double) * (size_t)(3 * n));
    for (int64_t s = 0; s < n; ++s) {
        rho[s] = 1.0 + 0.01 * sin(0.1 * (double)s);
        u[s] = 0.02 * cos(0.3 * (double)s);
        u[n + s] = 0.01;
        u[2 * n + s] = -0.01;
    }
    double before[4], after[4];
    int bad = lbm_init(h, rho, u, 0) != LBM_OK || lbm_totals(h, before) != LBM_OK || lbm_step(h, 10) != LBM_OK ||
              lbm_totals(h, after) != LBM_OK || lbm_moments(h, rho, u, 0) != LBM_OK;
    lbm_info info;
    bad = bad || lbm_get_info(h, &info) != LBM_OK || info.t != 10 || info.nsites != n;
    bad = bad || fabs(after[0] - before[0]) > 1e-6 * before[0];
    printf("c abi example: mass %.9f -> %.9f after %lld steps\n", before[0], after[0], (long long)info.t);
    free(rho);
    free(u);
    if (lbm_destroy(h) != LBM_OK) bad = 1;
    return bad ? 6 : 0;
}
