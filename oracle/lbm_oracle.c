/*
 * lbm_oracle.c -- plain FP64 CPU oracle for the filtered, Galilean-invariant
 * lattice Boltzmann time step of Chen, Zhang & Gopalakrishnan,
 * "Filtered Lattice Boltzmann Collision Formulation Enforcing Isotropy and
 * Galilean Invariance" (arXiv:2002.02503).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the independent reference the GPU
 * library is checked against.  Only the test suite, the package smoke check
 * and the CPU-baseline leg of the benchmark may load it.  The product library
 * never links, includes or calls it; the two share no code, no tables and no
 * headers.
 *
 * Arithmetic is IEEE double precision throughout (build without fast-math).
 * The code is deliberately plain: it builds the Hermite tensors of the paper
 * as dense arrays and contracts them, one site at a time.
 *
 * Readings of the paper used here (the paper is silent or ambiguous):
 *   R1  Both Hermite expansions -- the equilibrium (eq. hermite) and the
 *       filtered non-equilibrium part (eq. hermite-coll) -- are truncated at
 *       the same order K.  The default is K = 3 on the 2N = 4 lattices
 *       (D2Q9, D3Q19; the rule n <= 2N-1) and K = 4 on D3Q39 (the printed
 *       closed form eq. filter-2nd).  Keq and Kneq can be set apart for the
 *       comparator operators.
 *   R2  Pi^neq (eq. coeff-2 / eq. Pi_def) is taken with the truncated
 *       equilibrium the collision itself uses.
 *   R3  Streaming is written in pull form: f_i(x, t+1) = f'_i(x - c_i, t),
 *       which is eq. lbe read from the arrival site.  Every axis is periodic.
 *       The stored state is the post-collision population.
 *   R4  The energy-flux term of eq. pq has weight theta (default 0).  Its
 *       compact form eq. filter-Q is read with f^eq / rho in place of f^eq,
 *       as in eq. filter-coll, so that at u = 0 it reduces to the theta term
 *       of eq. filter2.  Its Hermite expansion follows from the generating
 *       function exp(xi.t - t.t/2) of the H^(n) exactly as eq. hermite-coll
 *       follows from eq. filter-coll (three t-derivatives instead of two):
 *           fhat^q_i = (w_i / 6 T0^{3/2}) sum_{n>=3} H^(n)(xi_i) (V^[n-3] Qt) / (n-3)!
 *       and it is truncated at the same order K.  Qt is the relative energy
 *       flux eq. Q_def, computed literally with c' = c - u.
 *   R5  Lattice weights and T0 are not printed in the paper.  D2Q9 and
 *       D3Q15 and D3Q19 use T0 = 1/3 (stated in the section on isotropy) with
 *       the standard shell weights; D3Q39 uses T0 = 2/3 and the six shell
 *       weights that satisfy the isotropy condition eq. iso through 6th
 *       order (the test suite re-derives them from eq. iso).
 *
 * Parity pins live in the test suite: isotropy (eq. iso), Hermite
 * orthogonality, exact low moments, the printed closed forms, the K -> infinity
 * compact forms, u = 0 reduction, fixed points, conservation, viscous decay.
 */

#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_QMAX 39
#define OR_NMAX 10 /* highest Hermite order the tensor tables are built to */

enum { OR_D2Q9 = 0, OR_D3Q19 = 1, OR_D3Q39 = 2, OR_D3Q15 = 3, OR_NLAT = 4 };
enum { OR_KIND_FILTERED = 0, OR_KIND_BGK = 1, OR_KIND_NONE = 2 };
enum { OR_MODE_LITERAL = 0, OR_MODE_CLOSED = 1 };
enum { OR_OK = 0, OR_EINVAL = -1, OR_ENOMEM = -2 };

/* ------------------------------------------------------------------------ */
/* Lattices (section "Basic Filtered Collision Formulation", eq. iso).       */
/* A lattice is a union of shells: all integer vectors whose sorted absolute */
/* components equal a given triple share one weight.                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    int m[3];   /* sorted absolute components, largest first */
    double w;   /* weight of every vector in the shell */
} shell_t;

typedef struct {
    int D, Q, two_n;
    double T0;
    int c[OR_QMAX][3];
    double w[OR_QMAX];
} lattice_t;

static int lattice_make(int lat, lattice_t* L)
{
    static const shell_t d2q9[] = {
        {{0, 0, 0}, 4.0 / 9.0}, {{1, 0, 0}, 1.0 / 9.0}, {{1, 1, 0}, 1.0 / 36.0}};
    static const shell_t d3q19[] = {
        {{0, 0, 0}, 1.0 / 3.0}, {{1, 0, 0}, 1.0 / 18.0}, {{1, 1, 0}, 1.0 / 36.0}};
    static const shell_t d3q15[] = {
        {{0, 0, 0}, 2.0 / 9.0}, {{1, 0, 0}, 1.0 / 9.0}, {{1, 1, 1}, 1.0 / 72.0}};
    static const shell_t d3q39[] = {
        {{0, 0, 0}, 1.0 / 12.0},  {{1, 0, 0}, 1.0 / 12.0},  {{1, 1, 1}, 1.0 / 27.0},
        {{2, 0, 0}, 2.0 / 135.0}, {{2, 2, 0}, 1.0 / 432.0}, {{3, 0, 0}, 1.0 / 1620.0}};
    const shell_t* sh;
    int nsh;
    memset(L, 0, sizeof(*L));
    switch (lat) {
    case OR_D2Q9:  sh = d2q9;  nsh = 3; L->D = 2; L->T0 = 1.0 / 3.0; L->two_n = 4; break;
    case OR_D3Q19: sh = d3q19; nsh = 3; L->D = 3; L->T0 = 1.0 / 3.0; L->two_n = 4; break;
    case OR_D3Q39: sh = d3q39; nsh = 6; L->D = 3; L->T0 = 2.0 / 3.0; L->two_n = 6; break;
    case OR_D3Q15: sh = d3q15; nsh = 3; L->D = 3; L->T0 = 1.0 / 3.0; L->two_n = 4; break;
    default: return OR_EINVAL;
    }
    int zr = (L->D == 3) ? 3 : 0;
    int q = 0;
    for (int z = -zr; z <= zr; ++z)
        for (int y = -3; y <= 3; ++y)
            for (int x = -3; x <= 3; ++x) {
                int a[3] = {abs(x), abs(y), abs(z)};
                /* sort descending */
                for (int p = 0; p < 2; ++p)
                    for (int r = 0; r < 2 - p; ++r)
                        if (a[r] < a[r + 1]) { int tmp = a[r]; a[r] = a[r + 1]; a[r + 1] = tmp; }
                for (int s = 0; s < nsh; ++s) {
                    if (a[0] == sh[s].m[0] && a[1] == sh[s].m[1] && a[2] == sh[s].m[2]) {
                        L->c[q][0] = x; L->c[q][1] = y; L->c[q][2] = z;
                        L->w[q] = sh[s].w;
                        ++q;
                        break;
                    }
                }
            }
    L->Q = q;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Hermite tensors H^(n)(xi_i), xi_i = c_i / sqrt(T0) (eq. hermite), built by */
/* the recursion eq. recurG:                                                   */
/*   H^(n+1)_{a1..a(n+1)} = xi_{a(n+1)} H^(n)_{a1..an}                         */
/*                          - sum_k delta_{a(n+1) ak} H^(n-1)_{a1..(no ak)..an} */
/* A rank-n tensor is a dense array of D^n entries; the multi-index           */
/* (a1, ..., an) is stored at sum_m a_m D^(n-m) (a1 most significant).          */
/* ------------------------------------------------------------------------ */

typedef struct {
    int built_to;                 /* highest order present, -1 if none */
    double* H[OR_NMAX + 1];       /* H[n][i * D^n + idx] */
} hermite_t;

static long ipow(int b, int e)
{
    long r = 1;
    while (e-- > 0) r *= b;
    return r;
}

static int hermite_build(const lattice_t* L, int nmax, hermite_t* out)
{
    const int D = L->D, Q = L->Q;
    const double s = 1.0 / sqrt(L->T0);
    memset(out, 0, sizeof(*out));
    out->built_to = -1;
    for (int n = 0; n <= nmax; ++n) {
        out->H[n] = (double*)malloc(sizeof(double) * (size_t)Q * (size_t)ipow(D, n));
        if (!out->H[n]) return OR_ENOMEM;
    }
    int digits[OR_NMAX + 2];
    for (int i = 0; i < Q; ++i) {
        double xi[3] = {L->c[i][0] * s, L->c[i][1] * s, L->c[i][2] * s};
        out->H[0][i] = 1.0;
        for (int n = 0; n < nmax; ++n) {
            const long szn = ipow(D, n), szn1 = ipow(D, n + 1);
            const long szm = (n >= 1) ? ipow(D, n - 1) : 0;
            for (long idx = 0; idx < szn1; ++idx) {
                /* digits[0..n] = a1..a(n+1) */
                long rem = idx;
                for (int p = n; p >= 0; --p) { digits[p] = (int)(rem % D); rem /= D; }
                const int last = digits[n];
                double val = xi[last] * out->H[n][i * szn + idx / D];
                for (int k = 0; k < n; ++k) {
                    if (digits[k] != last) continue;
                    long sub = 0;
                    for (int p = 0; p < n; ++p)
                        if (p != k) sub = sub * D + digits[p];
                    val -= out->H[n - 1][i * szm + sub];
                }
                out->H[n + 1][i * szn1 + idx] = val;
            }
        }
    }
    out->built_to = nmax;
    return OR_OK;
}

static void hermite_free(hermite_t* h)
{
    for (int n = 0; n <= OR_NMAX; ++n) free(h->H[n]);
    memset(h, 0, sizeof(*h));
    h->built_to = -1;
}

/* Process-wide cache of the tensor tables, one per lattice. */
static lattice_t g_lat[OR_NLAT];
static hermite_t g_herm[OR_NLAT];
static int g_ready[OR_NLAT];
static pthread_mutex_t g_lock = PTHREAD_MUTEX_INITIALIZER;

static int tables_get(int lat, int nmax, const lattice_t** L, const hermite_t** H)
{
    if (lat < 0 || lat >= OR_NLAT || nmax < 0 || nmax > OR_NMAX) return OR_EINVAL;
    int rc = OR_OK;
    pthread_mutex_lock(&g_lock);
    if (!g_ready[lat]) {
        rc = lattice_make(lat, &g_lat[lat]);
        if (rc == OR_OK) { g_herm[lat].built_to = -1; g_ready[lat] = 1; }
    }
    if (rc == OR_OK && g_herm[lat].built_to < nmax) {
        hermite_free(&g_herm[lat]);
        rc = hermite_build(&g_lat[lat], nmax, &g_herm[lat]);
    }
    pthread_mutex_unlock(&g_lock);
    if (rc != OR_OK) return rc;
    *L = &g_lat[lat];
    *H = &g_herm[lat];
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Per-site pieces.  `ws` is caller scratch of at least 2 * D^K doubles.      */
/* ------------------------------------------------------------------------ */

/* V^[n]: direct product of V with itself n times, dense D^n array. */
static void outer_power(const double* V, int D, int n, double* out)
{
    out[0] = 1.0;
    long sz = 1;
    for (int m = 0; m < n; ++m) {
        for (long idx = sz - 1; idx >= 0; --idx) {
            const double v = out[idx];
            for (int a = D - 1; a >= 0; --a) out[idx * D + a] = v * V[a];
        }
        sz *= D;
    }
}

/* eq. hermite truncated at order K:
 *   f^eq_i = w_i rho sum_{n=0}^{K} H^(n)(xi_i) . V^[n] / n!,   V = u / sqrt(T0). */
static void feq_literal(const lattice_t* L, const hermite_t* H, int K, double rho,
                        const double* u, double* feq, double* ws)
{
    const int D = L->D, Q = L->Q;
    double V[3];
    for (int a = 0; a < D; ++a) V[a] = u[a] / sqrt(L->T0);
    for (int i = 0; i < Q; ++i) feq[i] = 0.0;
    double nfact = 1.0;
    for (int n = 0; n <= K; ++n) {
        if (n > 0) nfact *= n;
        const long sz = ipow(D, n);
        outer_power(V, D, n, ws);
        for (int i = 0; i < Q; ++i) {
            const double* Hn = H->H[n] + i * sz;
            double acc = 0.0;
            for (long idx = 0; idx < sz; ++idx) acc += Hn[idx] * ws[idx];
            feq[i] += acc / nfact;
        }
    }
    for (int i = 0; i < Q; ++i) feq[i] *= L->w[i] * rho;
}

/* eq. hermite-coll truncated at order K:
 *   fhat_i = (w_i / 2 T0) sum_{n=2}^{K} H^(n)(xi_i) : (V^[n-2] Pi) / (n-2)!
 * where the last two indices of H^(n) contract with Pi. */
static void fneq_literal(const lattice_t* L, const hermite_t* H, int K, const double* u,
                         const double* Pi, double* fneq, double* ws)
{
    const int D = L->D, Q = L->Q;
    double V[3];
    for (int a = 0; a < D; ++a) V[a] = u[a] / sqrt(L->T0);
    for (int i = 0; i < Q; ++i) fneq[i] = 0.0;
    double mfact = 1.0; /* (n-2)! */
    for (int n = 2; n <= K; ++n) {
        if (n > 2) mfact *= (n - 2);
        const long szv = ipow(D, n - 2), sz = ipow(D, n);
        double* Vn = ws;
        double* T = ws + szv;
        outer_power(V, D, n - 2, Vn);
        for (long idx = 0; idx < szv; ++idx)
            for (int b = 0; b < D; ++b)
                for (int g = 0; g < D; ++g) T[(idx * D + b) * D + g] = Vn[idx] * Pi[b * 3 + g];
        for (int i = 0; i < Q; ++i) {
            const double* Hn = H->H[n] + i * sz;
            double acc = 0.0;
            for (long idx = 0; idx < sz; ++idx) acc += Hn[idx] * T[idx];
            fneq[i] += acc / mfact;
        }
    }
    for (int i = 0; i < Q; ++i) fneq[i] *= L->w[i] / (2.0 * L->T0);
}

/* Energy-flux part of eq. pq (reading R4), truncated at order K:
 *   fhat^q_i = (w_i / 6 T0^{3/2}) sum_{n=3}^{K} H^(n)(xi_i) (V^[n-3] Qt) / (n-3)!
 * where the last three indices of H^(n) contract with Qt (3x3x3, row-major,
 * only the leading D x D x D block is read).  Empty for K < 3. */
static void fq_literal(const lattice_t* L, const hermite_t* H, int K, const double* u,
                       const double* Qt, double* fq, double* ws)
{
    const int D = L->D, Q = L->Q;
    double V[3];
    for (int a = 0; a < D; ++a) V[a] = u[a] / sqrt(L->T0);
    for (int i = 0; i < Q; ++i) fq[i] = 0.0;
    double mfact = 1.0; /* (n-3)! */
    for (int n = 3; n <= K; ++n) {
        if (n > 3) mfact *= (n - 3);
        const long szv = ipow(D, n - 3), sz = ipow(D, n);
        double* Vn = ws;
        double* T = ws + szv;
        outer_power(V, D, n - 3, Vn);
        for (long idx = 0; idx < szv; ++idx)
            for (int a = 0; a < D; ++a)
                for (int b = 0; b < D; ++b)
                    for (int g = 0; g < D; ++g)
                        T[((idx * D + a) * D + b) * D + g] = Vn[idx] * Qt[(a * 3 + b) * 3 + g];
        for (int i = 0; i < Q; ++i) {
            const double* Hn = H->H[n] + i * sz;
            double acc = 0.0;
            for (long idx = 0; idx < sz; ++idx) acc += Hn[idx] * T[idx];
            fq[i] += acc / mfact;
        }
    }
    for (int i = 0; i < Q; ++i) fq[i] *= L->w[i] / (6.0 * L->T0 * sqrt(L->T0));
}

/* Relative non-equilibrium energy flux eq. Q_def, literally:
 *   Qt = sum_i c'_i c'_i c'_i (f_i - f^eq_i),  c'_i = c_i - u. */
static void qtilde_literal(const lattice_t* L, const double* f, const double* feq, const double* u,
                           double* Qt)
{
    const int D = L->D;
    for (int k = 0; k < 27; ++k) Qt[k] = 0.0;
    for (int i = 0; i < L->Q; ++i) {
        const double d = f[i] - feq[i];
        double cp[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < D; ++a) cp[a] = L->c[i][a] - u[a];
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b)
                for (int g = 0; g < D; ++g) Qt[(a * 3 + b) * 3 + g] += cp[a] * cp[b] * cp[g] * d;
    }
}

/* Scalar form of eq. hermite: H^(n)(xi) . V^[n] equals the probabilists'
 * Hermite polynomial He_n(a; v) with a = xi . V, v = V . V, generated by
 * He_{n+1} = a He_n - n v He_{n-1}.  Used by the closed-form mode. */
static void feq_closed(const lattice_t* L, int K, double rho, const double* u, double* feq)
{
    const int D = L->D, Q = L->Q;
    double uu = 0.0;
    for (int a = 0; a < D; ++a) uu += u[a] * u[a];
    const double v = uu / L->T0;
    for (int i = 0; i < Q; ++i) {
        double cu = 0.0;
        for (int a = 0; a < D; ++a) cu += L->c[i][a] * u[a];
        const double a = cu / L->T0;
        double hm1 = 0.0, h = 1.0, sum = 1.0, fact = 1.0;
        for (int n = 0; n < K; ++n) {
            const double hn1 = a * h - n * v * hm1;
            hm1 = h;
            h = hn1;
            fact *= (n + 1);
            sum += h / fact;
        }
        feq[i] = L->w[i] * rho * sum;
    }
}

/* The paper's printed closed forms of the filtered non-equilibrium part:
 *   K = 2: eq. filter-Pi   (w/2T0) [cc/T0 - I] : Pi
 *   K = 3: eq. filter-1st  (w/2T0) [(1 + c.u/T0)(cc/T0 - I) - (cu + uc)/T0] : Pi
 *   K = 4: eq. filter-2nd  (w/2T0) [(1 + c.u/T0 + (c.u)^2/2T0^2 - u^2/2T0)(cc/T0 - I)
 *                                   - (1 + c.u/T0)(cu + uc)/T0 + uu/T0] : Pi        */
static int fneq_closed(const lattice_t* L, int K, const double* u, const double* Pi, double* fneq)
{
    if (K < 2 || K > 4) return OR_EINVAL;
    const int D = L->D, Q = L->Q;
    const double T0 = L->T0;
    double trPi = 0.0, uu = 0.0, uPiu = 0.0;
    for (int a = 0; a < D; ++a) {
        trPi += Pi[a * 3 + a];
        uu += u[a] * u[a];
        for (int b = 0; b < D; ++b) uPiu += u[a] * Pi[a * 3 + b] * u[b];
    }
    for (int i = 0; i < Q; ++i) {
        const int* c = L->c[i];
        double cu = 0.0, cPic = 0.0, cPiu = 0.0;
        for (int a = 0; a < D; ++a) {
            cu += c[a] * u[a];
            for (int b = 0; b < D; ++b) {
                cPic += c[a] * Pi[a * 3 + b] * c[b];
                cPiu += c[a] * Pi[a * 3 + b] * u[b];
            }
        }
        const double ccI = cPic / T0 - trPi;   /* [cc/T0 - I] : Pi   */
        const double cuuc = 2.0 * cPiu / T0;   /* (cu + uc)/T0 : Pi  */
        double br;
        if (K == 2) {
            br = ccI;
        } else if (K == 3) {
            br = (1.0 + cu / T0) * ccI - cuuc;
        } else {
            br = (1.0 + cu / T0 + cu * cu / (2.0 * T0 * T0) - uu / (2.0 * T0)) * ccI
               - (1.0 + cu / T0) * cuuc + uPiu / T0;
        }
        fneq[i] = L->w[i] / (2.0 * T0) * br;
    }
    return OR_OK;
}

/* ρ = sum f, ρu = sum c f (eq. mme). */
static void moments(const lattice_t* L, const double* f, double* rho, double* u)
{
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < L->Q; ++i) {
        r += f[i];
        for (int a = 0; a < L->D; ++a) j[a] += L->c[i][a] * f[i];
    }
    *rho = r;
    for (int a = 0; a < 3; ++a) u[a] = (a < L->D) ? j[a] / r : 0.0;
}

typedef struct {
    int kind, mode, Keq, Kneq;
    double tau, theta;
} collide_cfg;

/* One collision at one site.
 *   filtered: eq. post-1 with the truncated eq. hermite-coll,
 *             f' = f^eq + (1 - 1/tau) fhat^neq, with Pi^neq = sum c c (f - f^eq)
 *             (eq. coeff-2, equal to eq. Pi_def); with theta != 0 the
 *             energy-flux part of eq. pq is added: fhat^neq + theta fhat^q.
 *   bgk:      eq. BGK, f' = f - (f - f^eq)/tau.
 *   none:     f' = f (streaming only; used to pin the streaming half).      */
static int collide(const lattice_t* L, const hermite_t* H, const collide_cfg* cfg,
                   const double* f, double* fout, double* ws)
{
    const int D = L->D, Q = L->Q;
    if (cfg->kind == OR_KIND_NONE) {
        for (int i = 0; i < Q; ++i) fout[i] = f[i];
        return OR_OK;
    }
    double rho, u[3], feq[OR_QMAX];
    moments(L, f, &rho, u);
    if (cfg->mode == OR_MODE_LITERAL) feq_literal(L, H, cfg->Keq, rho, u, feq, ws);
    else feq_closed(L, cfg->Keq, rho, u, feq);
    if (cfg->kind == OR_KIND_BGK) {
        for (int i = 0; i < Q; ++i) fout[i] = f[i] - (f[i] - feq[i]) / cfg->tau;
        return OR_OK;
    }
    double Pi[9] = {0};
    for (int i = 0; i < Q; ++i) {
        const double d = f[i] - feq[i];
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) Pi[a * 3 + b] += L->c[i][a] * L->c[i][b] * d;
    }
    double fneq[OR_QMAX];
    if (cfg->mode == OR_MODE_LITERAL) {
        fneq_literal(L, H, cfg->Kneq, u, Pi, fneq, ws);
    } else {
        int rc = fneq_closed(L, cfg->Kneq, u, Pi, fneq);
        if (rc != OR_OK) return rc;
    }
    if (cfg->theta != 0.0) {
        double Qt[27], fq[OR_QMAX];
        qtilde_literal(L, f, feq, u, Qt);
        fq_literal(L, H, cfg->Kneq, u, Qt, fq, ws);
        for (int i = 0; i < Q; ++i) fneq[i] += cfg->theta * fq[i];
    }
    const double om = 1.0 - 1.0 / cfg->tau;
    for (int i = 0; i < Q; ++i) fout[i] = feq[i] + om * fneq[i];
    return OR_OK;
}

static size_t scratch_len(const lattice_t* L, int K)
{
    return 2 * (size_t)ipow(L->D, K < 2 ? 2 : K) + 16;
}

/* ------------------------------------------------------------------------ */
/* Exported single-site functions (used by the pin tests).                   */
/* ------------------------------------------------------------------------ */

int oracle_lattice(int lat, int* D, int* Q, double* T0, int* two_n, int* c_out, double* w_out)
{
    lattice_t L;
    int rc = lattice_make(lat, &L);
    if (rc != OR_OK) return rc;
    if (D) *D = L.D;
    if (Q) *Q = L.Q;
    if (T0) *T0 = L.T0;
    if (two_n) *two_n = L.two_n;
    for (int i = 0; i < L.Q; ++i) {
        if (c_out) for (int a = 0; a < 3; ++a) c_out[i * 3 + a] = L.c[i][a];
        if (w_out) w_out[i] = L.w[i];
    }
    return OR_OK;
}

/* out: Q * D^n doubles, velocity-major. */
int oracle_hermite(int lat, int n, double* out)
{
    const lattice_t* L;
    const hermite_t* H;
    int rc = tables_get(lat, n, &L, &H);
    if (rc != OR_OK) return rc;
    memcpy(out, H->H[n], sizeof(double) * (size_t)L->Q * (size_t)ipow(L->D, n));
    return OR_OK;
}

int oracle_feq(int lat, int K, int mode, double rho, const double* u, double* out)
{
    const lattice_t* L;
    const hermite_t* H;
    if (K < 0) return OR_EINVAL;
    int rc = tables_get(lat, K, &L, &H);
    if (rc != OR_OK) return rc;
    if (mode == OR_MODE_CLOSED) { feq_closed(L, K, rho, u, out); return OR_OK; }
    double* ws = (double*)malloc(sizeof(double) * scratch_len(L, K));
    if (!ws) return OR_ENOMEM;
    feq_literal(L, H, K, rho, u, out, ws);
    free(ws);
    return OR_OK;
}

/* Pi: 3x3 row-major (only the leading D x D block is read). */
int oracle_fneq(int lat, int K, int mode, const double* u, const double* Pi, double* out)
{
    const lattice_t* L;
    const hermite_t* H;
    if (K < 2) return OR_EINVAL;
    int rc = tables_get(lat, K, &L, &H);
    if (rc != OR_OK) return rc;
    if (mode == OR_MODE_CLOSED) return fneq_closed(L, K, u, Pi, out);
    double* ws = (double*)malloc(sizeof(double) * scratch_len(L, K));
    if (!ws) return OR_ENOMEM;
    fneq_literal(L, H, K, u, Pi, out, ws);
    free(ws);
    return OR_OK;
}

/* Qt: 3x3x3 row-major (only the leading D x D x D block is read). */
int oracle_fq(int lat, int K, const double* u, const double* Qt, double* out)
{
    const lattice_t* L;
    const hermite_t* H;
    if (K < 3) return OR_EINVAL;
    int rc = tables_get(lat, K, &L, &H);
    if (rc != OR_OK) return rc;
    double* ws = (double*)malloc(sizeof(double) * scratch_len(L, K));
    if (!ws) return OR_ENOMEM;
    fq_literal(L, H, K, u, Qt, out, ws);
    free(ws);
    return OR_OK;
}

int oracle_collide(int lat, int kind, int mode, int Keq, int Kneq, double tau, double theta,
                   const double* f, double* out)
{
    const lattice_t* L;
    const hermite_t* H;
    if (Keq < 0 || Kneq < 2 || !(tau > 0.0) || !isfinite(theta)) return OR_EINVAL;
    int kmax = Keq > Kneq ? Keq : Kneq;
    int rc = tables_get(lat, kmax, &L, &H);
    if (rc != OR_OK) return rc;
    collide_cfg cfg = {kind, mode, Keq, Kneq, tau, theta};
    double* ws = (double*)malloc(sizeof(double) * scratch_len(L, kmax));
    if (!ws) return OR_ENOMEM;
    rc = collide(L, H, &cfg, f, out, ws);
    free(ws);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Periodic simulation: the lattice Boltzmann equation eq. lbe / eq. lbe-reg */
/* on an nx * ny * nz box.  Populations are stored site-major: f[s * Q + i],  */
/* s = (z * ny + y) * nx + x.                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    const lattice_t* L;
    const hermite_t* H;
    collide_cfg cfg;
    long nx, ny, nz, nsites;
    long t;
    double* f;  /* current post-collision state */
    double* g;  /* next state */
} oracle_sim;

static long wrap(long v, long n) { return ((v % n) + n) % n; }

oracle_sim* oracle_sim_create(int lat, long nx, long ny, long nz, double tau,
                              int Keq, int Kneq, int kind, int mode, double theta)
{
    if (nx < 1 || ny < 1 || nz < 1 || !(tau > 0.0) || Keq < 0 || Kneq < 2) return NULL;
    if (!isfinite(theta)) return NULL;
    if (kind < OR_KIND_FILTERED || kind > OR_KIND_NONE) return NULL;
    if (mode == OR_MODE_CLOSED && kind == OR_KIND_FILTERED && (Kneq < 2 || Kneq > 4)) return NULL;
    const lattice_t* L;
    const hermite_t* H;
    int kmax = Keq > Kneq ? Keq : Kneq;
    if (tables_get(lat, kmax, &L, &H) != OR_OK) return NULL;
    if (L->D == 2 && nz != 1) return NULL;
    oracle_sim* s = (oracle_sim*)calloc(1, sizeof(oracle_sim));
    if (!s) return NULL;
    s->L = L;
    s->H = H;
    s->cfg.kind = kind;
    s->cfg.mode = mode;
    s->cfg.Keq = Keq;
    s->cfg.Kneq = Kneq;
    s->cfg.tau = tau;
    s->cfg.theta = theta;
    s->nx = nx; s->ny = ny; s->nz = nz;
    s->nsites = nx * ny * nz;
    s->f = (double*)calloc((size_t)s->nsites * L->Q, sizeof(double));
    s->g = (double*)calloc((size_t)s->nsites * L->Q, sizeof(double));
    if (!s->f || !s->g) { free(s->f); free(s->g); free(s); return NULL; }
    return s;
}

void oracle_sim_destroy(oracle_sim* s)
{
    if (!s) return;
    free(s->f);
    free(s->g);
    free(s);
}

/* rho[s], u[a * nsites + s] (x fastest).  f := f^eq_Keq(rho, u), t := 0. */
int oracle_sim_init(oracle_sim* s, const double* rho, const double* u)
{
    const lattice_t* L = s->L;
    const int D = L->D, Q = L->Q;
    int rc = OR_OK;
#pragma omp parallel
    {
        double* ws = (double*)malloc(sizeof(double) * scratch_len(L, s->cfg.Keq));
#pragma omp for schedule(static)
        for (long k = 0; k < s->nsites; ++k) {
            double uk[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < D; ++a) uk[a] = u[a * s->nsites + k];
            if (s->cfg.mode == OR_MODE_LITERAL) feq_literal(L, s->H, s->cfg.Keq, rho[k], uk, s->f + k * Q, ws);
            else feq_closed(L, s->cfg.Keq, rho[k], uk, s->f + k * Q);
        }
        free(ws);
    }
    s->t = 0;
    return rc;
}

/* n time steps: pull the post-collision populations along -c_i (eq. lbe,
 * read at the arrival site), then collide (eq. lbe-reg / eq. post-1). */
int oracle_sim_step(oracle_sim* s, long n)
{
    const lattice_t* L = s->L;
    const int Q = L->Q;
    int err = OR_OK;
    for (long step = 0; step < n; ++step) {
#pragma omp parallel
        {
            double* ws = (double*)malloc(sizeof(double) * scratch_len(L, s->cfg.Keq > s->cfg.Kneq ? s->cfg.Keq : s->cfg.Kneq));
            double fin[OR_QMAX], fout[OR_QMAX];
#pragma omp for collapse(2) schedule(static)
            for (long z = 0; z < s->nz; ++z)
                for (long y = 0; y < s->ny; ++y)
                    for (long x = 0; x < s->nx; ++x) {
                        for (int i = 0; i < Q; ++i) {
                            const long xs = wrap(x - L->c[i][0], s->nx);
                            const long ys = wrap(y - L->c[i][1], s->ny);
                            const long zs = wrap(z - L->c[i][2], s->nz);
                            fin[i] = s->f[((zs * s->ny + ys) * s->nx + xs) * Q + i];
                        }
                        int rc = collide(L, s->H, &s->cfg, fin, fout, ws);
                        if (rc != OR_OK) {
#pragma omp atomic write
                            err = rc;
                        }
                        double* dst = s->g + ((z * s->ny + y) * s->nx + x) * Q;
                        for (int i = 0; i < Q; ++i) dst[i] = fout[i];
                    }
            free(ws);
        }
        double* tmp = s->f;
        s->f = s->g;
        s->g = tmp;
        s->t += 1;
    }
    return err;
}

/* rho and u of the stored state (eq. mme); u[a * nsites + s]. */
int oracle_sim_moments(const oracle_sim* s, double* rho, double* u)
{
    const lattice_t* L = s->L;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < s->nsites; ++k) {
        double r, uk[3];
        moments(L, s->f + k * L->Q, &r, uk);
        rho[k] = r;
        for (int a = 0; a < L->D; ++a) u[a * s->nsites + k] = uk[a];
    }
    return OR_OK;
}

/* Global mass and momentum [sum rho, sum rho u_a], summed in site order. */
int oracle_sim_totals(const oracle_sim* s, double* out)
{
    const lattice_t* L = s->L;
    for (int a = 0; a < 4; ++a) out[a] = 0.0;
    for (long k = 0; k < s->nsites; ++k)
        for (int i = 0; i < L->Q; ++i) {
            const double v = s->f[k * L->Q + i];
            out[0] += v;
            for (int a = 0; a < L->D; ++a) out[1 + a] += L->c[i][a] * v;
        }
    return OR_OK;
}

/* Raw populations f[s * Q + i]. */
int oracle_sim_get(const oracle_sim* s, double* out)
{
    memcpy(out, s->f, sizeof(double) * (size_t)s->nsites * s->L->Q);
    return OR_OK;
}

int oracle_sim_set(oracle_sim* s, const double* in)
{
    memcpy(s->f, in, sizeof(double) * (size_t)s->nsites * s->L->Q);
    return OR_OK;
}

long oracle_sim_time(const oracle_sim* s) { return s->t; }

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
