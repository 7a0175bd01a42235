/*
 * Exercise every entry point of the CPU oracle (oracle/lbm_oracle.c) on small
 * inputs, for a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitizers.py).  Any out-of-bounds access, leak or
 * undefined operation makes the sanitizer runtime report and exit non-zero;
 * a failing return code of the oracle makes this driver exit 2.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct oracle_sim oracle_sim;
int oracle_lattice(int lat, int* D, int* Q, double* T0, int* two_n, int* c_out, double* w_out);
int oracle_hermite(int lat, int n, double* out);
int oracle_feq(int lat, int K, int mode, double rho, const double* u, double* out);
int oracle_fneq(int lat, int K, int mode, const double* u, const double* Pi, double* out);
int oracle_fq(int lat, int K, const double* u, const double* Qt, double* out);
int oracle_collide(int lat, int kind, int mode, int Keq, int Kneq, double tau, double theta, const double* f,
                   double* out);
oracle_sim* oracle_sim_create(int lat, long nx, long ny, long nz, double tau, int Keq, int Kneq, int kind, int mode,
                              double theta);
void oracle_sim_destroy(oracle_sim* s);
int oracle_sim_init(oracle_sim* s, const double* rho, const double* u);
int oracle_sim_step(oracle_sim* s, long n);
int oracle_sim_moments(const oracle_sim* s, double* rho, double* u);
int oracle_sim_totals(const oracle_sim* s, double* out);
int oracle_sim_get(const oracle_sim* s, double* out);
int oracle_sim_set(oracle_sim* s, const double* in);

#define CHECK(call)                                                        \
    do {                                                                   \
        int rc_ = (call);                                                  \
        if (rc_ != 0) {                                                    \
            fprintf(stderr, "%s returned %d (line %d)\n", #call, rc_, __LINE__); \
            exit(2);                                                       \
        }                                                                  \
    } while (0)

static unsigned rng_state = 12345u;
static double rnd(double a)  /* uniform in [-a, a) */
{
    rng_state = rng_state * 1664525u + 1013904223u;
    return a * (2.0 * (double)(rng_state >> 8) / 16777216.0 - 1.0);
}

static long ipow(long b, int e)
{
    long r = 1;
    while (e-- > 0) r *= b;
    return r;
}

int main(void)
{
    /* D2Q9, D3Q19, D3Q39, D3Q15 and their highest Hermite order K = 2N - 1 */
    const int lats[4] = {0, 1, 2, 3};
    const int kmax[4] = {3, 3, 5, 3};
    for (int li = 0; li < 4; ++li) {
        const int lat = lats[li];
        int D = 0, Q = 0, two_n = 0, c[39 * 3];
        double T0 = 0.0, w[39];
        CHECK(oracle_lattice(lat, &D, &Q, &T0, &two_n, c, w));
        for (int n = 0; n <= kmax[li] + 1; ++n) {
            double* H = (double*)malloc(sizeof(double) * (size_t)Q * (size_t)ipow(D, n));
            CHECK(oracle_hermite(lat, n, H));
            free(H);
        }
        double u[3] = {rnd(0.05), rnd(0.05), D == 3 ? rnd(0.05) : 0.0};
        double Pi[9], Qt[27], out[39], f[39], g[39];
        for (int k = 0; k < 9; ++k) Pi[k] = rnd(1e-3);
        for (int k = 0; k < 27; ++k) Qt[k] = rnd(1e-4);
        for (int K = 2; K <= kmax[li]; ++K) {
            for (int mode = 0; mode < 2; ++mode) {
                if (mode == 1 && K > 4) continue; /* the printed closed forms stop at K = 4 */
                CHECK(oracle_feq(lat, K, mode, 1.0 + rnd(0.01), u, out));
                CHECK(oracle_fneq(lat, K, mode, u, Pi, out));
            }
            if (K >= 3) CHECK(oracle_fq(lat, K, u, Qt, out));
        }
        CHECK(oracle_feq(lat, kmax[li], 0, 1.0, u, f));
        for (int i = 0; i < Q; ++i) f[i] += rnd(1e-3) * w[i];
        for (int kind = 0; kind < 3; ++kind)
            for (int mode = 0; mode < 2; ++mode) {
                const int K = (mode == 1 && kmax[li] > 4) ? 4 : kmax[li];
                const double theta = (kind == 0 && K >= 3) ? 0.5 : 0.0;
                CHECK(oracle_collide(lat, kind, mode, K, K, 0.6, theta, f, g));
            }
        /* periodic boxes, including sides shorter than the longest velocity */
        const long boxes[4][3] = {{1, 1, 1}, {2, 3, 2}, {5, 3, 4}, {7, 2, 3}};
        for (int b = 0; b < 4; ++b) {
            const long nx = boxes[b][0], ny = boxes[b][1], nz = D == 2 ? 1 : boxes[b][2];
            const long n = nx * ny * nz;
            double* rho = (double*)malloc(sizeof(double) * (size_t)n);
            double* uu = (double*)malloc(sizeof(double) * (size_t)(n * D));
            double* pop = (double*)malloc(sizeof(double) * (size_t)(n * Q));
            double tot[4];
            for (long s = 0; s < n; ++s) rho[s] = 1.0 + rnd(0.01);
            for (long s = 0; s < n * D; ++s) uu[s] = rnd(0.05);
            for (int mode = 0; mode < 2; ++mode)
                for (int kind = 0; kind < 3; ++kind) {
                    const int K = (mode == 1 && kmax[li] > 4) ? 4 : kmax[li];
                    const double theta = (kind == 0 && mode == 0 && K >= 3) ? 0.25 : 0.0;
                    oracle_sim* sim = oracle_sim_create(lat, nx, ny, nz, 0.7, K, K, kind, mode, theta);
                    if (!sim) {
                        fprintf(stderr, "oracle_sim_create failed: lattice %d box %d mode %d kind %d\n", lat, b,
                                mode, kind);
                        return 2;
                    }
                    CHECK(oracle_sim_init(sim, rho, uu));
                    CHECK(oracle_sim_step(sim, 3));
                    CHECK(oracle_sim_moments(sim, rho, uu));
                    CHECK(oracle_sim_totals(sim, tot));
                    CHECK(oracle_sim_get(sim, pop));
                    CHECK(oracle_sim_set(sim, pop));
                    CHECK(oracle_sim_step(sim, 1));
                    oracle_sim_destroy(sim);
                    if (!isfinite(tot[0])) {
                        fprintf(stderr, "non-finite mass\n");
                        return 2;
                    }
                }
            free(rho);
            free(uu);
            free(pop);
        }
    }
    /* invalid arguments are refused, not crashed on */
    if (oracle_sim_create(1, 0, 1, 1, 0.6, 3, 3, 0, 0, 0.0) != NULL) return 2;
    if (oracle_fneq(1, 1, 0, (const double[3]){0, 0, 0}, (const double[9]){0}, (double[39]){0}) == 0) return 2;
    if (oracle_lattice(9, NULL, NULL, NULL, NULL, NULL, NULL) == 0) return 2;
    printf("oracle sanitizer driver: ok\n");
    return 0;
}
