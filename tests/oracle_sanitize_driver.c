/* Host driver for the oracle built with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitize.py): calls every
 * oracle entry point on small inputs (powers of two and other N, the
 * Bluestein route, Z-string terms, the XY mixer) and checks the invariants
 * that need no reference: unit norm after an evolution, the adjoint against
 * brute-force differences, the inverse transform undoing the forward one.
 * Prints "ok" and returns 0, or names the failed check and returns 1. */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef double complex cplx;

void oracle_init_uniform(int64_t N, cplx *psi);
void oracle_phase(int64_t N, cplx *psi, const double *q, double gamma);
void oracle_mix_x(int n, cplx *psi, double t);
void oracle_dft(int64_t N, const cplx *in, cplx *out, int sign);
void oracle_fft(int64_t N, cplx *x, int sign);
void oracle_bluestein(int64_t N, cplx *x, int sign);
void oracle_mix_circulant(int64_t N, cplx *psi, const double *lambda, double t);
void oracle_mix_complete(int64_t N, cplx *psi, double t);
void oracle_circulant_eigenvalues(int64_t N, const double *w, double *lam_re, double *lam_im);
void oracle_expectation(int64_t N, const cplx *psi, const double *q, double *f, double *norm);
int oracle_evolve(int kind, int64_t N, const double *q, const double *lambda, int p, const double *gammas,
                  const double *ts, cplx *psi, double *f, double *norm);
int oracle_grad(int kind, int64_t N, const double *q, const double *lambda, int p, const double *gammas,
                const double *ts, double *f, double *dgammas, double *dts);
int oracle_grad_bruteforce(int kind, int64_t N, const double *q, const double *lambda, int p,
                           const double *gammas, const double *ts, double *dgammas, double *dts);
int oracle_evolve_terms(int64_t N, const double *q, int n_terms, const uint64_t *S, const double *c, int p,
                        const double *gammas, const double *ts, cplx *psi, double *f, double *norm);
int oracle_grad_terms(int64_t N, const double *q, int n_terms, const uint64_t *S, const double *c, int p,
                      const double *gammas, const double *ts, double *f, double *dgammas, double *dts);
int oracle_parity_ring_pairs(int m, const int *ring, int *pairs);
int oracle_evolve_xy(int n, const double *q, const cplx *psi0, int n_pairs, const int *pairs, int p,
                     const double *gammas, const double *ts, cplx *psi, double *f, double *norm);
int oracle_grad_xy(int n, const double *q, const cplx *psi0, int n_pairs, const int *pairs, int p,
                   const double *gammas, const double *ts, double *f, double *dgammas, double *dts);

static int fails = 0;

static void check(int ok, const char *what, double v)
{
    if (!ok) {
        printf("FAILED %s (%.3e)\n", what, v);
        ++fails;
    }
}

static double urand(uint64_t *s)
{
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*s >> 11) * (1.0 / 9007199254740992.0);
}

static double max_rel(const double *a, const double *b, int n)
{
    double d = 0.0, m = 0.0;
    for (int i = 0; i < n; ++i) {
        d = fmax(d, fabs(a[i] - b[i]));
        m = fmax(m, fabs(b[i]));
    }
    return d / (m > 0.0 ? m : 1.0);
}

int main(void)
{
    uint64_t seed = 12345;
    const int p = 3;
    double g[3], t[3];
    for (int i = 0; i < p; ++i) {
        g[i] = 3.0 * urand(&seed);
        t[i] = 3.0 * urand(&seed);
    }
    /* kinds over powers of two and other N (the latter through Bluestein) */
    const int64_t sizes[] = {2, 3, 8, 30, 64, 100, 128};
    for (unsigned si = 0; si < sizeof(sizes) / sizeof(sizes[0]); ++si) {
        const int64_t N = sizes[si];
        double *q = malloc(N * sizeof(double)), *lam = malloc(N * sizeof(double));
        double *w = malloc(N * sizeof(double)), *lre = malloc(N * sizeof(double)), *lim = malloc(N * sizeof(double));
        cplx *psi = malloc(N * sizeof(cplx)), *x = malloc(N * sizeof(cplx)), *y = malloc(N * sizeof(cplx));
        for (int64_t j = 0; j < N; ++j) {
            q[j] = 4.0 * urand(&seed) - 1.0;
            w[j] = 0.0;
            x[j] = urand(&seed) + I * urand(&seed);
        }
        w[1 % N] += 1.0;
        w[(N - 1) % N] += 1.0; /* ring weights: the eigenvalues are real */
        oracle_circulant_eigenvalues(N, w, lre, lim);
        for (int64_t j = 0; j < N; ++j)
            lam[j] = lre[j];
        const int pow2 = (N & (N - 1)) == 0;
        for (int kind = pow2 ? 0 : 1; kind <= 2; ++kind) {
            double f, nrm, dg[3], dt[3], bg[3], bt[3];
            check(oracle_evolve(kind, N, q, lam, p, g, t, psi, &f, &nrm) == 0, "evolve status", 0.0);
            check(fabs(nrm - 1.0) < 1e-12, "evolve norm", nrm - 1.0);
            check(oracle_grad(kind, N, q, lam, p, g, t, &f, dg, dt) == 0, "grad status", 0.0);
            check(oracle_grad_bruteforce(kind, N, q, lam, p, g, t, bg, bt) == 0, "bruteforce status", 0.0);
            check(max_rel(dg, bg, p) < 1e-6 && max_rel(dt, bt, p) < 1e-6, "adjoint vs differences",
                  max_rel(dg, bg, p));
        }
        /* transforms: forward then inverse returns N x */
        for (int64_t j = 0; j < N; ++j)
            y[j] = x[j];
        if (pow2) {
            oracle_fft(N, y, -1);
            oracle_fft(N, y, +1);
        } else {
            oracle_bluestein(N, y, -1);
            oracle_bluestein(N, y, +1);
        }
        double e = 0.0;
        for (int64_t j = 0; j < N; ++j)
            e = fmax(e, cabs(y[j] / (double)N - x[j]));
        check(e < 1e-12, "transform round trip", e);
        oracle_dft(N, x, y, -1);
        oracle_mix_circulant(N, x, lam, 0.4);
        oracle_mix_complete(N, x, -0.3);
        double f, nrm;
        oracle_expectation(N, x, q, &f, &nrm);
        free(q), free(lam), free(w), free(lre), free(lim), free(psi), free(x), free(y);
    }
    /* Z-string terms (n = 5) and the XY mixer on a ring of 5 */
    {
        const int n = 5;
        const int64_t N = 1 << n;
        double q[32], c[4] = {0.5, -1.0, 0.25, 2.0}, gg[12], f, nrm, dg[12], dt[3];
        uint64_t S[4] = {3, 6, 17, 31};
        cplx psi[32], psi0[32];
        for (int j = 0; j < 32; ++j)
            q[j] = urand(&seed);
        for (int j = 0; j < 12; ++j)
            gg[j] = urand(&seed);
        check(oracle_evolve_terms(N, q, 4, S, c, p, gg, t, psi, &f, &nrm) == 0, "terms evolve", 0.0);
        check(fabs(nrm - 1.0) < 1e-12, "terms norm", nrm - 1.0);
        check(oracle_grad_terms(N, q, 4, S, c, p, gg, t, &f, dg, dt) == 0, "terms grad", 0.0);
        int ring[5] = {0, 1, 2, 3, 4}, pairs[2 * 8];
        const int np = oracle_parity_ring_pairs(5, ring, pairs);
        check(np > 0 && np <= 8, "ring pairs", (double)np);
        for (int j = 0; j < 32; ++j)
            psi0[j] = (__builtin_popcount(j) == 2) ? 1.0 / sqrt(10.0) : 0.0;
        check(oracle_evolve_xy(n, q, psi0, np, pairs, p, g, t, psi, &f, &nrm) == 0, "xy evolve", 0.0);
        check(fabs(nrm - 1.0) < 1e-12, "xy norm", nrm - 1.0);
        check(oracle_grad_xy(n, q, psi0, np, pairs, p, g, t, &f, dg, dt) == 0, "xy grad", 0.0);
        oracle_init_uniform(N, psi);
        oracle_phase(N, psi, q, 0.3);
        oracle_mix_x(n, psi, 0.7);
    }
    if (fails)
        return 1;
    printf("ok\n");
    return 0;
}
