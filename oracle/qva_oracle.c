/*
 * qva_oracle.c -- plain, slow, double-precision CPU reference of the QVA
 * state evolution and its expectation value.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  It shares no code with the GPU path and is called only by
 * the tests, the smoke check and the CPU-baseline leg of the benchmark.
 *
 * What it computes (paper, Sec. 2.1 eqs. variational_generic, objective_generic,
 * phase_shift_generic, mixing_generic; Sec. 2.3.1 eqs. phase_shift_qaoa,
 * mixing_qaoa, qaoa_initial_state, qaoa; Sec. 2.4.2 eqs. qwoa_initial_state,
 * qwoa_mixer, qwoa; Sec. 3):
 *
 *   f(gamma, t) = <psi_p| Q |psi_p>,
 *   psi_p = U_W(t_p) U_Q(gamma_p) ... U_W(t_1) U_Q(gamma_1) psi_0,
 *   U_Q(gamma) = diag(exp(-i gamma q_j)),  U_W(t) = exp(-i t W),
 *   psi_0 = N^(-1/2) (1, ..., 1).
 *
 * W is either the hypercube adjacency sum_i X_i (QAOA; U_W is then the product
 * of independent single-qubit rotations exp(-i t X_i)), or a circulant with
 * eigenvalues lambda_m, applied as F^-1 diag(exp(-i t lambda_m)) F with F the
 * unnormalised DFT (Sec. 3, circulant eigensystem), or the complete graph's
 * adjacency J - I, applied from its definition (closed form, no transform).
 *
 * Extended QAOA (Sec. 2.3.2, eqs. phase_shift_qaoa_ex, qaoa_ex): one angle per
 * Z-string term of Q.  QAOAz (Sec. 2.4.1, eqs. parity_terms, qaoaz_mixers,
 * qaoaz): the parity mixer as an ordered product of two-qubit XY rotations,
 * from a given initial state.
 *
 * Readings of the paper taken here (each one listed with its reason in the
 * design notes): W_X = sum_i X_i (hypercube, the figure of Sec. 2.3.1);
 * psi_0 normalised by 1/sqrt(N); layer 1 acts first and U_Q precedes U_W in a
 * layer; exp(-i t W) for the circulant too (the sign of Sec. 2.1); qubit i is
 * bit i of the basis index.
 *
 * Everything is double / double complex, straightforward loops, library
 * cos/sin/cexp, pairwise summation for every sum over the state.  No blocking,
 * fusion or reordering beyond what the definitions state.
 *
 * Threads (OpenMP, only for timing on many cores): loops whose iterations are
 * independent and each write their own elements -- elementwise maps, the
 * pairs of one rotation, the butterflies of one FFT stage -- are split over
 * threads.  Every sum stays a single-threaded pairwise sum, so the results are
 * bit-identical at any thread count.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* pi to double precision (M_PI is not part of strict C11). */
static const double PI = 3.14159265358979323846264338327950288;

enum { ORACLE_MIX_X = 0, ORACLE_MIX_CIRCULANT = 1, ORACLE_MIX_COMPLETE = 2 };

/* Number of threads for the parallel loops (1 without OpenMP). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
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

/* ---------------------------------------------------------------------- */
/* Pairwise (recursive halving) summation.                                 */
/* ---------------------------------------------------------------------- */

static double pairwise_sum(const double *x, int64_t n)
{
    if (n <= 8) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i)
            s += x[i];
        return s;
    }
    int64_t h = n / 2;
    return pairwise_sum(x, h) + pairwise_sum(x + h, n - h);
}

/* Sum of term(j) for j in [lo, hi), by recursive halving; term given as a
 * callback over the state arrays so that no N-sized temporary is needed. */
typedef double (*term_fn)(int64_t j, const void *ctx);

static double pairwise_sum_fn(term_fn term, const void *ctx, int64_t lo, int64_t hi)
{
    if (hi - lo <= 8) {
        double s = 0.0;
        for (int64_t j = lo; j < hi; ++j)
            s += term(j, ctx);
        return s;
    }
    int64_t mid = lo + (hi - lo) / 2;
    return pairwise_sum_fn(term, ctx, lo, mid) + pairwise_sum_fn(term, ctx, mid, hi);
}

/* ---------------------------------------------------------------------- */
/* Initial state (eq. qaoa_initial_state, eq. qwoa_initial_state).          */
/* ---------------------------------------------------------------------- */

void oracle_init_uniform(int64_t N, cplx *psi)
{
    double a = 1.0 / sqrt((double)N);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j)
        psi[j] = a;
}

/* ---------------------------------------------------------------------- */
/* Phase shift (eq. phase_shift_generic; Sec. 3 diagonal action):           */
/*   psi_j <- exp(-i gamma q_j) psi_j.                                     */
/* ---------------------------------------------------------------------- */

void oracle_phase(int64_t N, cplx *psi, const double *q, double gamma)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j)
        psi[j] *= cexp(-I * gamma * q[j]);
}

/* ---------------------------------------------------------------------- */
/* Extended QAOA phase (eq. phase_shift_qaoa_ex):                           */
/*   U_Qext(gamma) = prod_e exp(-i gamma_e Sigma_e),                        */
/* with Sigma_e = c_e Z^{S_e} a term of a Pauli decomposition of Q: for a   */
/* diagonal Q every term is a Z string, on the qubits set in the mask S_e,  */
/* so Sigma_e(j) = c_e (-1)^popcount(j & S_e).  The terms commute and the   */
/* product is exp(-i sum_e gamma_e Sigma_e(j)) on basis state j.            */
/* ---------------------------------------------------------------------- */

static double zterm(int64_t j, uint64_t S, double c)
{
    return (__builtin_popcountll((uint64_t)j & S) & 1) ? -c : c;
}

void oracle_phase_terms(int64_t N, cplx *psi, int n_terms, const uint64_t *S, const double *c,
                        const double *gamma)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        double ph = 0.0;
        for (int e = 0; e < n_terms; ++e)
            ph += gamma[e] * zterm(j, S[e], c[e]);
        psi[j] *= cexp(-I * ph);
    }
}

/* ---------------------------------------------------------------------- */
/* Hypercube mixer (eq. mixing_qaoa with W_X = sum_i X_i).                  */
/* The X_i commute, so exp(-i t sum_i X_i) = prod_i exp(-i t X_i), and      */
/* exp(-i t X) = cos t I - i sin t X acts on each pair (j, j ^ 2^i).        */
/* ---------------------------------------------------------------------- */

void oracle_mix_x(int n, cplx *psi, double t)
{
    int64_t N = (int64_t)1 << n;
    double c = cos(t), s = sin(t);
    for (int i = 0; i < n; ++i) {
        int64_t bit = (int64_t)1 << i;
        /* iteration j (bit i clear) alone touches the pair (j, j | bit) */
        #pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < N; ++j) {
            if (j & bit)
                continue;
            cplx a = psi[j], b = psi[j | bit];
            psi[j] = c * a - I * s * b;
            psi[j | bit] = -I * s * a + c * b;
        }
    }
}

/* W_X psi = sum_i X_i psi:  (W psi)_j = sum_i psi_{j ^ 2^i}. */
void oracle_apply_hypercube(int n, const cplx *psi, cplx *out)
{
    int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        cplx acc = 0.0;
        for (int i = 0; i < n; ++i)
            acc += psi[j ^ ((int64_t)1 << i)];
        out[j] = acc;
    }
}

/* ---------------------------------------------------------------------- */
/* Discrete Fourier transform (Sec. 3, circulant eigensystem).              */
/* F_{mj} = exp(sign * 2 pi i j m / N), unnormalised.  The forward          */
/* transform uses sign = -1, the inverse sign = +1 (and a 1/N elsewhere).   */
/* ---------------------------------------------------------------------- */

static int log2_exact(int64_t N);

static cplx root_of_unity(int64_t k, int64_t N, int sign)
{
    /* exp(sign * 2 pi i k / N) computed directly from the reduced integer
     * k mod N, never by recurrence. */
    int64_t r = k % N;
    if (r < 0)
        r += N;
    double ang = 2.0 * PI * (double)r / (double)N;
    return cos(ang) + (double)sign * I * sin(ang);
}

/* Naive O(N^2) DFT: out_m = sum_j in_j exp(sign 2 pi i j m / N). */
void oracle_dft(int64_t N, const cplx *in, cplx *out, int sign)
{
    double *re = malloc(sizeof(double) * (size_t)N);
    double *im = malloc(sizeof(double) * (size_t)N);
    for (int64_t m = 0; m < N; ++m) {
        for (int64_t j = 0; j < N; ++j) {
            /* (j*m) mod N without overflow for N <= 2^31 */
            int64_t k = (int64_t)(((uint64_t)j * (uint64_t)m) % (uint64_t)N);
            cplx v = in[j] * root_of_unity(k, N, sign);
            re[j] = creal(v);
            im[j] = cimag(v);
        }
        out[m] = pairwise_sum(re, N) + I * pairwise_sum(im, N);
    }
    free(re);
    free(im);
}

/* Iterative radix-2 Cooley-Tukey (decimation in time) for N = 2^k:         */
/* bit-reverse the input, then log2 N stages of butterflies.  The twiddle   */
/* table holds exp(sign 2 pi i k / N) for k < N/2, each entry computed       */
/* directly.  In place.                                                      */
void oracle_fft(int64_t N, cplx *x, int sign)
{
    if (N <= 1)
        return;
    int lg = 0;
    while (((int64_t)1 << lg) < N)
        ++lg;
    /* bit reversal permutation (iteration j alone swaps the pair j < r) */
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        int64_t r = 0;
        for (int b = 0; b < lg; ++b)
            if (j & ((int64_t)1 << b))
                r |= (int64_t)1 << (lg - 1 - b);
        if (r > j) {
            cplx tmp = x[j];
            x[j] = x[r];
            x[r] = tmp;
        }
    }
    cplx *w = malloc(sizeof(cplx) * (size_t)(N / 2));
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < N / 2; ++k)
        w[k] = root_of_unity(k, N, sign);
    for (int64_t len = 2; len <= N; len <<= 1) {
        int64_t half = len / 2;
        int64_t step = N / len; /* twiddle for butterfly k is w[k * step] */
        /* the N/2 butterflies of a stage, b = (block, k): block start
         * (b / half) * len, offset k = b % half; each owns its two elements */
        #pragma omp parallel for schedule(static)
        for (int64_t b = 0; b < N / 2; ++b) {
            const int64_t start = (b / half) * len, k = b % half;
            cplx u = x[start + k];
            cplx v = x[start + k + half] * w[k * step];
            x[start + k] = u + v;
            x[start + k + half] = u - v;
        }
    }
    free(w);
}

/* Bluestein's chirp-z transform: the same sum as oracle_dft for any N       */
/* (here N < 2^31), through three radix-2 FFTs of a power of two M >= 2N-1.  */
/* With u_k = exp(sign i pi k^2 / N), jm = (j^2 + m^2 - (m-j)^2) / 2 gives    */
/*   out_m = u_m sum_j (x_j u_j) conj(u_{m-j}),                               */
/* a linear convolution, done cyclically in length M with conj(u_k) placed   */
/* at k and M - k.  k^2 is reduced mod 2N exactly before the angle.  In place. */
void oracle_bluestein(int64_t N, cplx *x, int sign)
{
    int64_t M = 1;
    while (M < 2 * N - 1)
        M <<= 1;
    cplx *u = malloc(sizeof(cplx) * (size_t)N);
    cplx *a = calloc((size_t)M, sizeof(cplx));
    cplx *v = calloc((size_t)M, sizeof(cplx));
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < N; ++k) {
        const int64_t r = (int64_t)(((uint64_t)k * (uint64_t)k) % (uint64_t)(2 * N));
        u[k] = cexp((double)sign * I * PI * (double)r / (double)N);
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j)
        a[j] = x[j] * u[j];
    v[0] = conj(u[0]);
#pragma omp parallel for schedule(static)
    for (int64_t k = 1; k < N; ++k)
        v[k] = v[M - k] = conj(u[k]);
    oracle_fft(M, a, -1);
    oracle_fft(M, v, -1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i)
        a[i] *= v[i];
    oracle_fft(M, a, +1);
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < N; ++m)
        x[m] = u[m] * a[m] / (double)M;
    free(u);
    free(a);
    free(v);
}

/* Forward/inverse transform used by the circulant mixer: naive DFT for     */
/* small N, the radix-2 FFT for larger powers of two, Bluestein otherwise.   */
static void transform(int64_t N, cplx *x, int sign)
{
    if (N <= 4096) {
        cplx *tmp = malloc(sizeof(cplx) * (size_t)N);
        oracle_dft(N, x, tmp, sign);
        memcpy(x, tmp, sizeof(cplx) * (size_t)N);
        free(tmp);
    } else if (log2_exact(N) >= 0) {
        oracle_fft(N, x, sign);
    } else {
        oracle_bluestein(N, x, sign);
    }
}

/* ---------------------------------------------------------------------- */
/* Circulant mixer (eq. mixing_generic with a circulant W; Sec. 3):         */
/*   psi <- F^-1 diag(exp(-i t lambda_m)) F psi,  F^-1 = conj(F)/N.        */
/* ---------------------------------------------------------------------- */

void oracle_mix_circulant(int64_t N, cplx *psi, const double *lambda, double t)
{
    transform(N, psi, -1);
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < N; ++m)
        psi[m] *= cexp(-I * t * lambda[m]);
    transform(N, psi, +1);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j)
        psi[j] /= (double)N;
}

/* W psi for a circulant W = F^-1 diag(lambda) F. */
void oracle_apply_circulant(int64_t N, const cplx *psi, const double *lambda, cplx *out)
{
    memcpy(out, psi, sizeof(cplx) * (size_t)N);
    transform(N, out, -1);
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < N; ++m)
        out[m] *= lambda[m];
    transform(N, out, +1);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j)
        out[j] /= (double)N;
}

/* ---------------------------------------------------------------------- */
/* Complete-graph mixer (the QWOA default W; Sec. 3 eigenvalues N - 1 once,  */
/* -1 otherwise), from its definition W = J - I with J the all-ones matrix:  */
/*   W psi = S 1 - psi,  S = sum_j psi_j;                                    */
/*   J^2 = N J  =>  exp(-i t W) = e^{i t} (I + (e^{-i t N} - 1)/N J).        */
/* For N a power of two t N is exact; otherwise it is rounded once.         */
/* ---------------------------------------------------------------------- */

static double term_re(int64_t j, const void *c) { return creal(((const cplx *)c)[j]); }
static double term_im(int64_t j, const void *c) { return cimag(((const cplx *)c)[j]); }

static cplx state_sum(int64_t N, const cplx *psi)
{
    return pairwise_sum_fn(term_re, psi, 0, N) + I * pairwise_sum_fn(term_im, psi, 0, N);
}

void oracle_mix_complete(int64_t N, cplx *psi, double t)
{
    const cplx S = state_sum(N, psi);
    const cplx c = (cexp(-I * (t * (double)N)) - 1.0) / (double)N;
    const cplx e = cexp(I * t);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j)
        psi[j] = e * (psi[j] + c * S);
}

void oracle_apply_complete(int64_t N, const cplx *psi, cplx *out)
{
    const cplx S = state_sum(N, psi);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j)
        out[j] = S - psi[j];
}

/* Eigenvalues of the circulant whose first row is w (Sec. 3):              */
/*   lambda_m = w_0 + w_{N-1} omega^m + w_{N-2} omega^{2m} + ...            */
/*            = sum_l w_{(N-l) mod N} omega^{l m},  omega = exp(2 pi i / N). */
/* Naive O(N^2); the imaginary part is returned too (zero for symmetric w). */
void oracle_circulant_eigenvalues(int64_t N, const double *w, double *lam_re, double *lam_im)
{
    double *re = malloc(sizeof(double) * (size_t)N);
    double *im = malloc(sizeof(double) * (size_t)N);
    for (int64_t m = 0; m < N; ++m) {
        for (int64_t l = 0; l < N; ++l) {
            int64_t k = (int64_t)(((uint64_t)l * (uint64_t)m) % (uint64_t)N);
            cplx v = w[(N - l) % N] * root_of_unity(k, N, +1);
            re[l] = creal(v);
            im[l] = cimag(v);
        }
        lam_re[m] = pairwise_sum(re, N);
        lam_im[m] = pairwise_sum(im, N);
    }
    free(re);
    free(im);
}

/* ---------------------------------------------------------------------- */
/* Expectation value (eq. objective_generic): f = sum_j |psi_j|^2 q_j, and  */
/* the norm sum_j |psi_j|^2.                                                 */
/* ---------------------------------------------------------------------- */

struct expect_ctx {
    const cplx *psi;
    const double *q;
};

static double term_prob_q(int64_t j, const void *c)
{
    const struct expect_ctx *x = c;
    double a = creal(x->psi[j]), b = cimag(x->psi[j]);
    return (a * a + b * b) * x->q[j];
}

static double term_prob(int64_t j, const void *c)
{
    const struct expect_ctx *x = c;
    double a = creal(x->psi[j]), b = cimag(x->psi[j]);
    return a * a + b * b;
}

void oracle_expectation(int64_t N, const cplx *psi, const double *q, double *f, double *norm)
{
    struct expect_ctx ctx = {psi, q};
    if (f)
        *f = pairwise_sum_fn(term_prob_q, &ctx, 0, N);
    if (norm)
        *norm = pairwise_sum_fn(term_prob, &ctx, 0, N);
}

/* <a|b> = sum_j conj(a_j) b_j, pairwise over real and imaginary parts.     */
struct inner_ctx {
    const cplx *a, *b;
    const double *w; /* optional diagonal weight */
};

static double term_inner_re(int64_t j, const void *c)
{
    const struct inner_ctx *x = c;
    double v = creal(conj(x->a[j]) * x->b[j]);
    return x->w ? v * x->w[j] : v;
}

static double term_inner_im(int64_t j, const void *c)
{
    const struct inner_ctx *x = c;
    double v = cimag(conj(x->a[j]) * x->b[j]);
    return x->w ? v * x->w[j] : v;
}

static cplx inner(int64_t N, const cplx *a, const cplx *b, const double *w)
{
    struct inner_ctx ctx = {a, b, w};
    return pairwise_sum_fn(term_inner_re, &ctx, 0, N) + I * pairwise_sum_fn(term_inner_im, &ctx, 0, N);
}

/* ---------------------------------------------------------------------- */
/* The layered evolution (eqs. qaoa and qwoa).                               */
/* ---------------------------------------------------------------------- */

static int log2_exact(int64_t N)
{
    int n = 0;
    while (((int64_t)1 << n) < N)
        ++n;
    return ((int64_t)1 << n) == N ? n : -1;
}

static void apply_mixer(int kind, int64_t N, cplx *psi, const double *lambda, double t)
{
    if (kind == ORACLE_MIX_X)
        oracle_mix_x(log2_exact(N), psi, t);
    else if (kind == ORACLE_MIX_COMPLETE)
        oracle_mix_complete(N, psi, t);
    else
        oracle_mix_circulant(N, psi, lambda, t);
}

static void apply_W(int kind, int64_t N, const cplx *psi, const double *lambda, cplx *out)
{
    if (kind == ORACLE_MIX_X)
        oracle_apply_hypercube(log2_exact(N), psi, out);
    else if (kind == ORACLE_MIX_COMPLETE)
        oracle_apply_complete(N, psi, out);
    else
        oracle_apply_circulant(N, psi, lambda, out);
}

static int check_args(int kind, int64_t N)
{
    if (N < 1)
        return -1;
    if (kind == ORACLE_MIX_X && log2_exact(N) < 0)
        return -1;
    if (kind == ORACLE_MIX_CIRCULANT && N >= ((int64_t)1 << 31))
        return -1;
    if (kind != ORACLE_MIX_X && kind != ORACLE_MIX_CIRCULANT && kind != ORACLE_MIX_COMPLETE)
        return -1;
    return 0;
}

/* psi (N complex, caller-allocated) receives psi_p; f and norm its         */
/* expectation and squared norm.  Returns 0, or -1 on bad arguments.         */
int oracle_evolve(int kind, int64_t N, const double *q, const double *lambda, int p,
                  const double *gammas, const double *ts, cplx *psi, double *f, double *norm)
{
    if (check_args(kind, N) || p < 0)
        return -1;
    oracle_init_uniform(N, psi);
    for (int k = 0; k < p; ++k) {
        oracle_phase(N, psi, q, gammas[k]);
        apply_mixer(kind, N, psi, lambda, ts[k]);
    }
    oracle_expectation(N, psi, q, f, norm);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Gradient by the adjoint method.                                           */
/* With psi_p = U_2p ... U_1 psi_0, U_l = exp(-i theta_l H_l):               */
/*   df/dtheta_l = 2 Re <psi_p| Q U_2p..U_{l+1} (-i H_l) |phi_l>            */
/*               = 2 Im <chi_l| H_l |phi_l>,                                 */
/* phi_l = U_l..U_1 psi_0,  chi_l = U_{l+1}^dag .. U_2p^dag Q psi_p.        */
/* Both are walked backwards from phi = psi_p, chi = Q psi_p by applying    */
/* U_l^dag = exp(+i theta_l H_l), i.e. the same operator at -theta_l.       */
/* ---------------------------------------------------------------------- */

int oracle_grad(int kind, int64_t N, const double *q, const double *lambda, int p,
                const double *gammas, const double *ts, double *f, double *dgammas, double *dts)
{
    if (check_args(kind, N) || p < 0)
        return -1;
    cplx *phi = malloc(sizeof(cplx) * (size_t)N);
    cplx *chi = malloc(sizeof(cplx) * (size_t)N);
    cplx *wphi = malloc(sizeof(cplx) * (size_t)N);
    oracle_evolve(kind, N, q, lambda, p, gammas, ts, phi, f, NULL);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j)
        chi[j] = q[j] * phi[j];
    for (int k = p - 1; k >= 0; --k) {
        /* mixer parameter t_k: H = W, evaluated on the state after U_W(t_k) */
        apply_W(kind, N, phi, lambda, wphi);
        dts[k] = 2.0 * cimag(inner(N, chi, wphi, NULL));
        apply_mixer(kind, N, phi, lambda, -ts[k]);
        apply_mixer(kind, N, chi, lambda, -ts[k]);
        /* phase parameter gamma_k: H = Q, on the state after U_Q(gamma_k) */
        dgammas[k] = 2.0 * cimag(inner(N, chi, phi, q));
        oracle_phase(N, phi, q, -gammas[k]);
        oracle_phase(N, chi, q, -gammas[k]);
    }
    free(phi);
    free(chi);
    free(wphi);
    return 0;
}

/* Extended QAOA (eq. qaoa_ex): hypercube mixer, per-term phases; gammas is */
/* p x n_terms (layer-major), q the observable.  Returns 0 or -1.            */
int oracle_evolve_terms(int64_t N, const double *q, int n_terms, const uint64_t *S, const double *c, int p,
                        const double *gammas, const double *ts, cplx *psi, double *f, double *norm)
{
    if (log2_exact(N) < 0 || p < 0 || n_terms < 0)
        return -1;
    oracle_init_uniform(N, psi);
    for (int k = 0; k < p; ++k) {
        oracle_phase_terms(N, psi, n_terms, S, c, gammas + (size_t)k * n_terms);
        oracle_mix_x(log2_exact(N), psi, ts[k]);
    }
    oracle_expectation(N, psi, q, f, norm);
    return 0;
}

/* Im <chi| Sigma_e |phi>, pairwise. */
struct zterm_ctx {
    const cplx *chi, *phi;
    uint64_t S;
    double c;
};

static double term_zinner(int64_t j, const void *ctx)
{
    const struct zterm_ctx *x = ctx;
    return zterm(j, x->S, x->c) * cimag(conj(x->chi[j]) * x->phi[j]);
}

/* Adjoint gradient of the extended QAOA: dts[k] as for QAOA, and          */
/* dgammas[k * n_terms + e] = 2 Im <chi_l| Sigma_e |phi_l> at the phase of   */
/* layer k (the terms commute with U_Qext, so one state pair serves all e).  */
int oracle_grad_terms(int64_t N, const double *q, int n_terms, const uint64_t *S, const double *c, int p,
                      const double *gammas, const double *ts, double *f, double *dgammas, double *dts)
{
    if (log2_exact(N) < 0 || p < 0 || n_terms < 0)
        return -1;
    const int n = log2_exact(N);
    cplx *phi = malloc(sizeof(cplx) * (size_t)N);
    cplx *chi = malloc(sizeof(cplx) * (size_t)N);
    cplx *wphi = malloc(sizeof(cplx) * (size_t)N);
    double *neg = malloc(sizeof(double) * (size_t)(n_terms > 0 ? n_terms : 1));
    oracle_evolve_terms(N, q, n_terms, S, c, p, gammas, ts, phi, f, NULL);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j)
        chi[j] = q[j] * phi[j];
    for (int k = p - 1; k >= 0; --k) {
        oracle_apply_hypercube(n, phi, wphi);
        dts[k] = 2.0 * cimag(inner(N, chi, wphi, NULL));
        oracle_mix_x(n, phi, -ts[k]);
        oracle_mix_x(n, chi, -ts[k]);
        for (int e = 0; e < n_terms; ++e) {
            struct zterm_ctx ctx = {chi, phi, S[e], c[e]};
            dgammas[(size_t)k * n_terms + e] = 2.0 * pairwise_sum_fn(term_zinner, &ctx, 0, N);
            neg[e] = -gammas[(size_t)k * n_terms + e];
        }
        oracle_phase_terms(N, phi, n_terms, S, c, neg);
        oracle_phase_terms(N, chi, n_terms, S, c, neg);
    }
    free(phi);
    free(chi);
    free(wphi);
    free(neg);
    return 0;
}

/* Independent gradient by direct differentiation of the product: for each  */
/* parameter, insert (-i H_l) right after U_l, finish the evolution, and    */
/* take df/dtheta_l = 2 Re <psi_p| Q |psi'_l>.  O(p^2) operator applications, */
/* no adjoint walk.  For small test sizes.                                   */
int oracle_grad_bruteforce(int kind, int64_t N, const double *q, const double *lambda, int p,
                           const double *gammas, const double *ts, double *dgammas, double *dts)
{
    if (check_args(kind, N) || p < 0)
        return -1;
    cplx *psi = malloc(sizeof(cplx) * (size_t)N);
    cplx *d = malloc(sizeof(cplx) * (size_t)N);
    cplx *tmp = malloc(sizeof(cplx) * (size_t)N);
    double f;
    oracle_evolve(kind, N, q, lambda, p, gammas, ts, psi, &f, NULL);
    for (int l = 0; l < 2 * p; ++l) {
        int layer = l / 2, is_mixer = l % 2;
        oracle_init_uniform(N, d);
        for (int m = 0; m < 2 * p; ++m) {
            int lm = m / 2;
            if (m % 2 == 0)
                oracle_phase(N, d, q, gammas[lm]);
            else
                apply_mixer(kind, N, d, lambda, ts[lm]);
            if (m == l) {
                if (is_mixer) {
                    apply_W(kind, N, d, lambda, tmp);
                } else {
                    for (int64_t j = 0; j < N; ++j)
                        tmp[j] = q[j] * d[j];
                }
                for (int64_t j = 0; j < N; ++j)
                    d[j] = -I * tmp[j];
            }
        }
        double g = 2.0 * creal(inner(N, psi, d, q));
        if (is_mixer)
            dts[layer] = g;
        else
            dgammas[layer] = g;
    }
    free(psi);
    free(d);
    free(tmp);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* QAOAz parity mixer (Sec. 2.4.1, eqs. parity_terms and qaoaz_mixers).     */
/* On a qubit pair (a, b), X_a X_b + Y_a Y_b maps the basis state with bit  */
/* a = 0, bit b = 1 to twice the state with the two bits swapped (and back) */
/* and annihilates the states where the bits agree.  So                     */
/*   exp(-i t (X_a X_b + Y_a Y_b)) = cos 2t - i sin 2t sigma_x              */
/* on each {01, 10} pair of amplitudes and the identity on the rest.  The   */
/* mixer is a product of such factors; `pairs` lists them in the order they */
/* act, first factor first (pairs[2i], pairs[2i + 1] are factor i's qubits).*/
/* ---------------------------------------------------------------------- */

static void xy_rotate(int n, cplx *psi, int a, int b, double t)
{
    const int64_t N = (int64_t)1 << n, ma = (int64_t)1 << a, mb = (int64_t)1 << b;
    const double c = cos(2.0 * t), s = sin(2.0 * t);
    /* iteration j (bit a set, bit b clear) alone touches the pair (j, k) */
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        if ((j & ma) && !(j & mb)) {
            const int64_t k = j ^ ma ^ mb;
            const cplx u = psi[j], v = psi[k];
            psi[j] = c * u - I * s * v;
            psi[k] = c * v - I * s * u;
        }
    }
}

/* out <- (X_a X_b + Y_a Y_b) psi */
static void xy_apply(int n, const cplx *psi, int a, int b, cplx *out)
{
    const int64_t N = (int64_t)1 << n, ma = (int64_t)1 << a, mb = (int64_t)1 << b;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        const int ba = (j & ma) != 0, bb = (j & mb) != 0;
        out[j] = ba != bb ? 2.0 * psi[j ^ ma ^ mb] : 0.0;
    }
}

static int check_pairs(int n, int n_pairs, const int *pairs)
{
    if (n < 1 || n > 40 || n_pairs < 0)
        return -1;
    for (int i = 0; i < n_pairs; ++i) {
        const int a = pairs[2 * i], b = pairs[2 * i + 1];
        if (a < 0 || b < 0 || a >= n || b >= n || a == b)
            return -1;
    }
    return 0;
}

void oracle_mix_xy(int n, cplx *psi, double t, int n_pairs, const int *pairs)
{
    for (int i = 0; i < n_pairs; ++i)
        xy_rotate(n, psi, pairs[2 * i], pairs[2 * i + 1], t);
}

/* The factors of U_parity (eq. qaoaz_mixers) for a ring of m qubits         */
/* ring[0..m-1], written 1-based as r_1..r_m in eq. parity_terms:            */
/*   B_odd:  (r_a, r_{a+1}) for odd a <= m - 1;                              */
/*   B_even: (r_a, r_{a+1}) for even a <= m, r_{m+1} read cyclically as r_1; */
/*   B_last: (r_m, r_1) when m is odd.                                       */
/* The factors of one B act on disjoint pairs and commute; the three B act   */
/* in the order odd, even, last.  Writes 2 ints per factor, returns the      */
/* count (at most m + 1).                                                    */
int oracle_parity_ring_pairs(int m, const int *ring, int *pairs)
{
    int c = 0;
    for (int a = 1; a <= m - 1; a += 2) {
        pairs[2 * c] = ring[a - 1];
        pairs[2 * c + 1] = ring[a];
        ++c;
    }
    for (int a = 2; a <= m; a += 2) {
        pairs[2 * c] = ring[a - 1];
        pairs[2 * c + 1] = ring[a % m];
        ++c;
    }
    if (m % 2 == 1 && m >= 3) {
        pairs[2 * c] = ring[m - 1];
        pairs[2 * c + 1] = ring[0];
        ++c;
    }
    return c;
}

/* QAOAz evolution (eq. qaoaz): psi_p = prod_k U_parity(t_k) U_Q(gamma_k)    */
/* psi0, from the given psi0 (a state of the constrained subspace).          */
int oracle_evolve_xy(int n, const double *q, const cplx *psi0, int n_pairs, const int *pairs, int p,
                     const double *gammas, const double *ts, cplx *psi, double *f, double *norm)
{
    if (check_pairs(n, n_pairs, pairs) || p < 0)
        return -1;
    const int64_t N = (int64_t)1 << n;
    memcpy(psi, psi0, sizeof(cplx) * (size_t)N);
    for (int k = 0; k < p; ++k) {
        oracle_phase(N, psi, q, gammas[k]);
        oracle_mix_xy(n, psi, ts[k], n_pairs, pairs);
    }
    oracle_expectation(N, psi, q, f, norm);
    return 0;
}

/* Adjoint gradient of the QAOAz expectation.  Every factor of a layer's     */
/* mixer carries the same t_k, so dts[k] sums 2 Im <chi|H_i|phi> over the    */
/* layer's factors, each taken with the states at that factor (walked back   */
/* factor by factor); dgammas[k] = 2 Im <chi|Q|phi> at the phase.            */
int oracle_grad_xy(int n, const double *q, const cplx *psi0, int n_pairs, const int *pairs, int p,
                   const double *gammas, const double *ts, double *f, double *dgammas, double *dts)
{
    if (check_pairs(n, n_pairs, pairs) || p < 0)
        return -1;
    const int64_t N = (int64_t)1 << n;
    cplx *phi = malloc(sizeof(cplx) * (size_t)N);
    cplx *chi = malloc(sizeof(cplx) * (size_t)N);
    cplx *hphi = malloc(sizeof(cplx) * (size_t)N);
    oracle_evolve_xy(n, q, psi0, n_pairs, pairs, p, gammas, ts, phi, f, NULL);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j)
        chi[j] = q[j] * phi[j];
    for (int k = p - 1; k >= 0; --k) {
        double dt = 0.0;
        for (int i = n_pairs - 1; i >= 0; --i) {
            const int a = pairs[2 * i], b = pairs[2 * i + 1];
            xy_apply(n, phi, a, b, hphi);
            dt += 2.0 * cimag(inner(N, chi, hphi, NULL));
            xy_rotate(n, phi, a, b, -ts[k]);
            xy_rotate(n, chi, a, b, -ts[k]);
        }
        dts[k] = dt;
        dgammas[k] = 2.0 * cimag(inner(N, chi, phi, q));
        oracle_phase(N, phi, q, -gammas[k]);
        oracle_phase(N, chi, q, -gammas[k]);
    }
    free(phi);
    free(chi);
    free(hphi);
    return 0;
}
