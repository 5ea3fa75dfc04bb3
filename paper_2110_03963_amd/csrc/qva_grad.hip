// qva_grad.hip -- adjoint gradient of f = <psi_p|Q|psi_p> over all 2p angles.
//
// With psi_p = U_2p ... U_1 psi_0 and U_l = exp(-i theta_l H_l),
//   df/dtheta_l = 2 Im <chi_l| H_l |phi_l>,
// phi_l = U_l ... U_1 psi_0 and chi_l = U_{l+1}^dag ... U_2p^dag Q psi_p.
// Both are walked back from phi = psi_p, chi = Q psi_p by applying the
// inverse of every forward pass in reverse order (the state is uncomputed,
// never stored per layer).  Each pass accumulates the inner products whose
// operands it holds:
//   hypercube mixer: <chi|X_i|phi> = sum over pairs (j, j^2^i) of
//     conj(chi_j) phi_{j^2^i} + conj(chi_{j^2^i}) phi_j, in the pass that
//     rotates qubit i (the other rotations of the layer commute with X_i and
//     leave it unchanged);
//   circulant mixer: <chi|W|phi> = (1/N) sum_m conj(chi^_m) lambda_m phi^_m,
//     in the low-group pass where both spectra are present;
//   phase: <chi|Q|phi> = sum_j q_j conj(chi_j) phi_j, in the pass that
//     undoes the phase; with one angle per Z-string term (extended QAOA),
//     <chi|Sigma_e|phi> for every term e, read off a Walsh-Hadamard transform
//     of conj(chi_j) phi_j over each tile.
// Each (parameter, qubit group, tile) partial is written by exactly one pass
// and reduced afterwards in a fixed order, so results are deterministic.
#include "qva_passes.h"

// Two vectors plus per-element twiddles need more than the 256 registers a
// wave gets at two waves per SIMD; at one wave per SIMD the overflow stays
// in accumulation registers instead of scratch memory.
#ifndef QVA_GRADF_WAVES
#define QVA_GRADF_WAVES 1
#endif
#ifndef QVA_GRADX_WAVES
#define QVA_GRADX_WAVES 2
#endif

namespace qva {
namespace {

using namespace tile;
using namespace passes;

// ------------------------------------------------ hypercube-mixer passes
template <int C, int MODE>
__global__ __launch_bounds__(kThreads, QVA_GRADX_WAVES) void gradx_kernel(GradPassParams P)
{
    __shared__ double2 lds[1 << kTileBits];
    __shared__ double red[4 * (kThreads / 64)];
    gradx_tile<C, MODE>(P, C == 3 ? paired_tile(blockIdx.x) : (int64_t)blockIdx.x, lds, red);
}

// The extended-QAOA phase passes hold the Z-string angles beside both
// vectors: at one wave per SIMD they stay in registers (two waves spill
// about 140 registers and run 10% slower).
#ifndef QVA_GRADZ_WAVES
#define QVA_GRADZ_WAVES 1
#endif
template <int C, int MODE>
__global__ __launch_bounds__(kThreads, QVA_GRADZ_WAVES) void gradxz_kernel(GradPassParams P)
{
    __shared__ double2 lds[1 << kTileBits];
    __shared__ double red[4 * (kThreads / 64)];
    gradx_tile<C, MODE>(P, C == 3 ? paired_tile(blockIdx.x) : (int64_t)blockIdx.x, lds, red);
}

// Per-term slots of an extended-QAOA phase from the values its backward pass
// stored (GMODE_ZSLOT).
template <int C>
__global__ __launch_bounds__(kThreads, 2) void zslot_kernel(GradPassParams P)
{
    __shared__ double2 lds[1 << kTileBits];
    zslot_tile<C>(P, blockIdx.x, lds);
}

// ------------------------------------------------ circulant-mixer passes
// TAB: low-group root table (C = 0 only; see digit_twiddles).
template <int C, int L, bool TAB>
__device__ __forceinline__ void digit_twiddle2(double2 (&p)[kRegs], double2 (&x)[kRegs], const TileMap& g,
                                               int t, bool inv, const double2* tab)
{
    digit_twiddles<C, L, TAB>(g, t, [&](int r, double2 tw) {
        const double2 w = make_double2(tw.x, inv ? -tw.y : tw.y);
        p[r] = cmul(p[r], w);
        x[r] = cmul(x[r], w);
    }, tab);
}

template <int C, int L, bool TAB>
__device__ __forceinline__ void dif_digit2(double2 (&p)[kRegs], double2 (&x)[kRegs], const TileMap& g, int t,
                                           const double2* tab)
{
    constexpr int LO = digit_lo<C, L>(), W = digit_w<C, L>();
    if constexpr (W > 0) {
        local_dif<LO, W>(p);
        local_dif<LO, W>(x);
        digit_twiddle2<C, L, TAB>(p, x, g, t, false, tab);
    }
}

template <int C, int L, bool TAB>
__device__ __forceinline__ void dit_digit2(double2 (&p)[kRegs], double2 (&x)[kRegs], const TileMap& g, int t,
                                           const double2* tab)
{
    constexpr int LO = digit_lo<C, L>(), W = digit_w<C, L>();
    if constexpr (W > 0) {
        digit_twiddle2<C, L, TAB>(p, x, g, t, true, tab);
        local_dit<LO, W>(p);
        local_dit<LO, W>(x);
    }
}

template <int C, bool TAB = false>
__device__ __forceinline__ void dif_tile2(double2 (&p)[kRegs], double2 (&x)[kRegs], double2* lds,
                                          const TileMap& g, int t, const double2* tab = nullptr)
{
    dif_digit2<C, LA, TAB>(p, x, g, t, tab);
    if constexpr (C < 8) {
        exchange2<LA, LB>(p, x, lds, t);
        dif_digit2<C, LB, TAB>(p, x, g, t, tab);
        if constexpr (C == 0) {
            exchange2<LB, LC>(p, x, lds, t);
            dif_digit2<C, LC, TAB>(p, x, g, t, tab);
        } else if constexpr (C == 3) {
            exchange2<LB, LA3>(p, x, lds, t);
            dif_digit2<C, LA3, false>(p, x, g, t, tab);
        }
    }
}

template <int C, bool TAB = false>
__device__ __forceinline__ void dit_tile2(double2 (&p)[kRegs], double2 (&x)[kRegs], double2* lds,
                                          const TileMap& g, int t, const double2* tab = nullptr)
{
    if constexpr (C < 8) {
        if constexpr (C == 0) {
            dit_digit2<C, LC, TAB>(p, x, g, t, tab);
            exchange2<LC, LB>(p, x, lds, t);
        } else if constexpr (C == 3) {
            dit_digit2<C, LA3, false>(p, x, g, t, tab);
            exchange2<LA3, LB>(p, x, lds, t);
        }
        dit_digit2<C, LB, TAB>(p, x, g, t, tab);
        exchange2<LB, LA>(p, x, lds, t);
    }
    dit_digit2<C, LA, TAB>(p, x, g, t, tab);
}

// lambda_m at bit-reversed position pos (see the forward low-group pass);
// u: ring_lambda_base of the tile and thread when the kind is the ring.
__device__ __forceinline__ double lambda_at(const GradPassParams& P, int64_t tile, int t, int r, double2 u)
{
    if (P.lambda_kind == FFT_LAMBDA_TILED)
        return ld_nt(P.lam + (tile << kTileBits) + r * kThreads + t);
    if (P.lambda_kind == FFT_LAMBDA_RING)
        return ring_lambda(u, r);
    const int64_t pos = (tile << kTileBits) | elem<LC>(t, r);
    const uint64_t m = __brevll((uint64_t)pos) >> (64 - P.n);
    if (P.lambda_kind == FFT_LAMBDA_NATURAL)
        return P.lam[m];
    return m == 0 ? (double)((int64_t(1) << P.n) - 1) : -1.0;
}

// lambda_j of the Bluestein passes (natural order, j < nb): the ring's
// 2 cos(2 pi j / N), or the caller's array.
__device__ __forceinline__ double blu_lambda(const GradPassParams& P, int64_t j)
{
    if (P.lambda_kind == FFT_LAMBDA_RING) {
        double s, c;
        sincospi_red((double)(2 * j) / (double)P.nb, &s, &c);
        return 2.0 * c;
    }
    return P.lam[j];
}

// Top-group passes of the adjoint through Bluestein's transform.  Both
// vectors live in padded buffers of M amplitudes in the convolution form of
// the forward: a state psi is x = conj(w) psi (j < N, zero above), and the
// first convolution of a mixer gives S = x * w, with F psi = conj(w) S, so
// <chi|W|phi> = (1/N) sum_{m < N} conj(S_chi,m) lambda_m S_phi,m and
// <chi|Q|phi> = sum_{j < N} q_j conj(x_chi,j) x_phi,j (the chirps cancel).
// The inverse of a mixer is the forward's pipeline with +t.
template <int C, int MODE>
__device__ __forceinline__ void gradb_tile(const GradPassParams& P, int64_t tile, double2* lds, double* red)
{
    const int t = threadIdx.x;
    const TileMap g = tile_map(tile, P.k, C);
    const double invNb = 1.0 / (double)P.nb;
    double2 p[kRegs], x[kRegs];
    if constexpr (MODE == GMODE_B_TURN) {
        load_tile<dif_last<C>()>(p, P.phi, g, t);
        dit_tile<C>(p, lds, g, t);
        double f = 0.0, nr = 0.0;
#pragma unroll
        for (int r = 0; r < kRegs; ++r) {
            const int64_t j = g(elem<LA>(t, r));
            if (j < P.nb) {
                const double qj = ld_nt(P.q + j);
                p[r] = make_double2(p[r].x * invNb, p[r].y * invNb);
                const double a = p[r].x * p[r].x + p[r].y * p[r].y;
                f = fma(a, qj, f);
                nr += a;
                x[r] = make_double2(qj * p[r].x, qj * p[r].y);
            } else {
                p[r] = x[r] = make_double2(0.0, 0.0);
            }
        }
        double fv[2] = {f, nr};
        block_sum_k<2>(fv, red);
        if (t == 0)
            P.fpart[tile] = make_double2(fv[0], fv[1]);
    } else {
        const double ang = MODE == GMODE_B_LAM ? angle_value(P.t1) : angle_value(P.gamma);
        load2<dif_last<C>()>(p, x, P, g, t);
        dit_tile2<C>(p, x, lds, g, t);
        double acc = 0.0;
#pragma unroll
        for (int r = 0; r < kRegs; ++r) {
            const int64_t j = g(elem<LA>(t, r));
            if (j < P.nb) {
                double h;
                if constexpr (MODE == GMODE_B_LAM) {
                    h = blu_lambda(P, j);
                } else {
                    h = ld_nt(P.q + j);
                    p[r] = make_double2(p[r].x * invNb, p[r].y * invNb);
                    x[r] = make_double2(x[r].x * invNb, x[r].y * invNb);
                }
                acc = fma(h, x[r].x * p[r].y - x[r].y * p[r].x, acc);
                const double2 u = expmi(-ang * h);  // the inverse factor exp(+i ang h)
                p[r] = cmul(p[r], u);
                x[r] = cmul(x[r], u);
            } else {
                p[r] = x[r] = make_double2(0.0, 0.0);
            }
            QVA_SCHED_FENCE();
        }
        if constexpr (MODE == GMODE_B_LAM)
            write_slots(P, acc * invNb, 0.0, 0.0, red, tile);
        else
            write_slots(P, 0.0, acc, 0.0, red, tile);
        if constexpr (MODE == GMODE_B_FINAL)
            return;
    }
    dif_tile2<C>(p, x, lds, g, t);
    store2<dif_last<C>()>(p, x, P, g, t);
}

template <int C, int MODE>
__global__ __launch_bounds__(kThreads, QVA_GRADF_WAVES) void gradb_kernel(GradPassParams P)
{
    __shared__ double2 lds[1 << kTileBits];
    __shared__ double red[4 * (kThreads / 64)];
    gradb_tile<C, MODE>(P, blockIdx.x, lds, red);
}

template <int C, int MODE>
__global__ __launch_bounds__(kThreads, QVA_GRADF_WAVES) void gradf_kernel(GradPassParams P)
{
    __shared__ double2 lds[1 << kTileBits];
    __shared__ double red[4 * (kThreads / 64)];
    const int t = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const TileMap g = tile_map(tile, P.k, C);
    const double invN = ldexp(1.0, -P.n);
    const double tt = (MODE == GMODE_LOWDIAG) ? angle_value(P.t1) : 0.0;
    const double gam = (MODE == GMODE_BOUND || MODE == GMODE_FINAL) ? angle_value(P.gamma) : 0.0;
    double2 p[kRegs], x[kRegs];

    if constexpr (MODE == GMODE_TURN) {
        load_tile<dif_last<C>()>(p, P.phi, g, t);
        dit_tile<C>(p, lds, g, t);
        double qq[kRegs];
#pragma unroll
        for (int r = 0; r < kRegs; ++r)
            qq[r] = ld_nt(P.q + g(elem<LA>(t, r)));
        double f = 0.0, nr = 0.0;
#pragma unroll
        for (int r = 0; r < kRegs; ++r) {
            p[r] = make_double2(p[r].x * invN, p[r].y * invN);
            const double a = p[r].x * p[r].x + p[r].y * p[r].y;
            f = fma(a, qq[r], f);
            nr += a;
            x[r] = make_double2(qq[r] * p[r].x, qq[r] * p[r].y);
        }
        double fv[2] = {f, nr};
        block_sum_k<2>(fv, red);
        if (t == 0)
            P.fpart[blockIdx.x] = make_double2(fv[0], fv[1]);
        dif_tile2<C>(p, x, lds, g, t);
        store2<dif_last<C>()>(p, x, P, g, t);
    } else if constexpr (MODE == GMODE_LOWDIAG) {
        load2<LA>(p, x, P, g, t);
        dif_tile2<C, true>(p, x, lds, g, t, P.tw);
        double a1 = 0.0;
        const double2 u = P.lambda_kind == FFT_LAMBDA_RING ? ring_lambda_base(tile, t, P.n) : make_double2(0.0, 0.0);
        if (P.lambda_kind == FFT_LAMBDA_RING) {
            // registers r and r + 1 (r even): ring eigenvalues of opposite
            // sign, one exponential for both (as in the forward pass)
#pragma unroll
            for (int r = 0; r < kRegs; r += 2) {
                const double lam = ring_lambda(u, r);
                a1 = fma(lam, x[r].x * p[r].y - x[r].y * p[r].x, a1);
                a1 = fma(-lam, x[r + 1].x * p[r + 1].y - x[r + 1].y * p[r + 1].x, a1);
                const double2 dd = expmi(-tt * lam), dc = make_double2(dd.x, -dd.y);
                p[r] = cmul(p[r], dd);
                x[r] = cmul(x[r], dd);
                p[r + 1] = cmul(p[r + 1], dc);
                x[r + 1] = cmul(x[r + 1], dc);
                QVA_SCHED_FENCE();
            }
        } else {
#pragma unroll
            for (int r = 0; r < kRegs; ++r) {
                const double lam = lambda_at(P, tile, t, r, u);
                a1 = fma(lam, x[r].x * p[r].y - x[r].y * p[r].x, a1);
                // exp(+i t lambda): the inverse diagonal
                const double2 d = P.lambda_kind == FFT_LAMBDA_COMPLETE
                                      ? complete_diag(tile == 0 && elem<LC>(t, r) == 0, -tt, P.n)
                                      : expmi(-tt * lam);
                p[r] = cmul(p[r], d);
                x[r] = cmul(x[r], d);
                QVA_SCHED_FENCE();
            }
        }
        write_slots(P, a1 * invN, 0.0, 0.0, red, tile);
        dit_tile2<C, true>(p, x, lds, g, t, P.tw);
        store2<LA>(p, x, P, g, t);
    } else {  // GMODE_BOUND, GMODE_FINAL
        load2<dif_last<C>()>(p, x, P, g, t);
        dit_tile2<C>(p, x, lds, g, t);
        const double ag = unphase2<LA, true>(p, x, P.q, g, t, gam, invN);
        if constexpr (MODE == GMODE_BOUND) {
            write_slots(P, 0.0, ag, 0.0, red, tile);
            dif_tile2<C>(p, x, lds, g, t);
            store2<dif_last<C>()>(p, x, P, g, t);
        } else {
            write_slots(P, 0.0, ag, 0.0, red, tile);
        }
    }
}

// ------------------------------------------------ whole state in one workgroup
// phi and chi both in LDS (n <= 12).  Same walk, plain radix-2 loops.
__device__ double small_unrotate_x(double2* ph, double2* ch, int n, double tt)
{
    double c, s;
    inv_cs(tt, c, s);
    const int N = 1 << n;
    double acc = 0.0;
    for (int i = 0; i < n; ++i) {
        const int bit = 1 << i;
        for (int m = threadIdx.x; m < N / 2; m += blockDim.x) {
            const int j = ((m >> i) << (i + 1)) | (m & (bit - 1));
            double2 a = ph[j], b = ph[j | bit], ca = ch[j], cb = ch[j | bit];
            acc += im_pair(a, b, ca, cb);
            rot_pair(a, b, c, s);
            rot_pair(ca, cb, c, s);
            ph[j] = a;
            ph[j | bit] = b;
            ch[j] = ca;
            ch[j | bit] = cb;
        }
        __syncthreads();
    }
    return acc;
}

__device__ void small_rotate_x(double2* s, int n, double tt)
{
    double sn, c;
    sincos_red(tt, &sn, &c);
    const int N = 1 << n;
    for (int i = 0; i < n; ++i) {
        const int bit = 1 << i;
        for (int m = threadIdx.x; m < N / 2; m += blockDim.x) {
            const int j = ((m >> i) << (i + 1)) | (m & (bit - 1));
            rot_pair(s[j], s[j | bit], c, sn);
        }
        __syncthreads();
    }
}

__device__ void small_dft(double2* s, int n, bool inverse)
{
    const int N = 1 << n;
    for (int it = 0; it < n; ++it) {
        const int st = inverse ? it : n - 1 - it;
        const int h = 1 << st;
        for (int m = threadIdx.x; m < N / 2; m += blockDim.x) {
            const int j = ((m >> st) << (st + 1)) | (m & (h - 1));
            double sn, cs;
            sincospi_red(ldexp((double)(j & (h - 1)), -st), &sn, &cs);
            const double2 w = make_double2(cs, inverse ? sn : -sn);
            const double2 a = s[j];
            double2 b = s[j + h];
            if (!inverse) {
                s[j] = make_double2(a.x + b.x, a.y + b.y);
                s[j + h] = cmul(make_double2(a.x - b.x, a.y - b.y), w);
            } else {
                b = cmul(b, w);
                s[j] = make_double2(a.x + b.x, a.y + b.y);
                s[j + h] = make_double2(a.x - b.x, a.y - b.y);
            }
        }
        __syncthreads();
    }
}

__device__ double small_lambda(const SmallGradParams& P, int j)
{
    const int n = P.n;
    const unsigned m = __brev((unsigned)j) >> (32 - n);
    if (P.lambda_kind == FFT_LAMBDA_NATURAL)
        return P.lam[m];
    if (P.lambda_kind == FFT_LAMBDA_RING)
        return ring_lambda_m(m, n);
    return m == 0 ? (double)((1 << n) - 1) : -1.0;
}

// exp(-i tt W) on s (circulant); with chi given, also returns
// Im sum conj(chi^) lambda phi^ / N before the diagonal (s = phi).
__device__ double small_circ(double2* s, double2* c2, const SmallGradParams& P, double tt)
{
    const int n = P.n, N = 1 << n;
    small_dft(s, n, false);
    if (c2)
        small_dft(c2, n, false);
    double acc = 0.0;
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
        const double lam = small_lambda(P, j);
        const double2 d = P.lambda_kind == FFT_LAMBDA_COMPLETE ? complete_diag(lam != -1.0, tt, n)
                                                               : expmi(tt * lam);
        if (c2) {
            acc = fma(lam, c2[j].x * s[j].y - c2[j].y * s[j].x, acc);
            c2[j] = cmul(c2[j], d);
        }
        s[j] = cmul(s[j], d);
    }
    __syncthreads();
    small_dft(s, n, true);
    if (c2)
        small_dft(c2, n, true);
    const double invN = ldexp(1.0, -n);
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
        s[j] = make_double2(s[j].x * invN, s[j].y * invN);
        if (c2)
            c2[j] = make_double2(c2[j].x * invN, c2[j].y * invN);
    }
    __syncthreads();
    return acc * invN;
}

__global__ __launch_bounds__(kThreads) void small_grad_kernel(SmallGradParams P)
{
    __shared__ double2 ph[1 << kTileBits];
    __shared__ double2 ch[1 << kTileBits];
    __shared__ double red[2 * (kThreads / 64)];
    const int n = P.n, N = 1 << n;
    const int t = threadIdx.x;
    const bool circ = P.circulant;
    const double a0 = 1.0 / sqrt((double)N);
    for (int j = t; j < N; j += blockDim.x)
        ph[j] = make_double2(a0, 0.0);
    __syncthreads();
    for (int L = 0; L < P.p; ++L) {
        if (P.n_terms > 0) {
            const double* row = P.gammas + (int64_t)L * P.n_terms;
            for (int j = t; j < N; j += blockDim.x)
                ph[j] = cmul(ph[j], expmi(zterm_angle(j, P.terms, P.n_terms, row)));
        } else {
            const double gam = P.gammas[L];
            for (int j = t; j < N; j += blockDim.x)
                ph[j] = cmul(ph[j], expmi(gam * P.q[j]));
        }
        __syncthreads();
        if (circ)
            small_circ(ph, nullptr, P, P.ts[L]);
        else
            small_rotate_x(ph, n, P.ts[L]);
    }
    double f = 0.0, nr = 0.0;
    for (int j = t; j < N; j += blockDim.x) {
        const double a = ph[j].x * ph[j].x + ph[j].y * ph[j].y;
        f = fma(a, P.q[j], f);
        nr += a;
        ch[j] = make_double2(P.q[j] * ph[j].x, P.q[j] * ph[j].y);
    }
    const double2 tot = block_sum2(f, nr, red);
    if (t == 0)
        P.out_f[0] = tot.x;
    __syncthreads();
    for (int L = P.p - 1; L >= 0; --L) {
        const double tt = P.ts[L];
        const double at = circ ? small_circ(ph, ch, P, -tt) : small_unrotate_x(ph, ch, n, tt);
        if (P.n_terms > 0) {
            // extended QAOA: Im(conj(chi_j) phi_j) of the thread's states, the
            // inverse phase, then one block sum per term (two at a time)
            const int E = P.n_terms;
            const double* row = P.gammas + (int64_t)L * E;
            double dj[kRegs];  // N <= kRegs * kThreads
#pragma unroll
            for (int i = 0; i < kRegs; ++i) {
                const int j = t + i * kThreads;
                dj[i] = 0.0;
                if (j < N) {
                    dj[i] = ch[j].x * ph[j].y - ch[j].y * ph[j].x;
                    const double2 u = expmi(-zterm_angle(j, P.terms, E, row));
                    ph[j] = cmul(ph[j], u);
                    ch[j] = cmul(ch[j], u);
                }
            }
            const double2 ts_sum = block_sum2(at, 0.0, red);
            if (t == 0)
                P.dts[L] = 2.0 * ts_sum.x;
            for (int e = 0; e < E; e += 2) {
                double a[2] = {0.0, 0.0};
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if (e + h >= E)
                        continue;
                    const uint64_t S = P.terms[e + h].support;
#pragma unroll
                    for (int i = 0; i < kRegs; ++i) {
                        const int j = t + i * kThreads;
                        if (j < N)
                            a[h] += (__popcll((uint64_t)j & S) & 1) ? -dj[i] : dj[i];
                    }
                    a[h] *= P.terms[e + h].coef;
                }
                const double2 sm = block_sum2(a[0], a[1], red);
                if (t == 0) {
                    P.dgammas[(int64_t)L * E + e] = 2.0 * sm.x;
                    if (e + 1 < E)
                        P.dgammas[(int64_t)L * E + e + 1] = 2.0 * sm.y;
                }
            }
            __syncthreads();
            continue;
        }
        double ag = 0.0;
        const double gam = P.gammas[L];
        for (int j = t; j < N; j += blockDim.x) {
            const double qj = P.q[j];
            ag = fma(qj, ch[j].x * ph[j].y - ch[j].y * ph[j].x, ag);
            const double2 u = expmi(-gam * qj);
            ph[j] = cmul(ph[j], u);
            ch[j] = cmul(ch[j], u);
        }
        const double2 sums = block_sum2(at, ag, red);
        if (t == 0) {
            P.dts[L] = 2.0 * sums.x;
            P.dgammas[L] = 2.0 * sums.y;
        }
        __syncthreads();
    }
}

// ------------------------------------------------ fixed-order reductions
// block s: out[s] = sum over tiles of slots[s * tiles + i]
__global__ __launch_bounds__(256) void slot_reduce_kernel(const double* slots, int64_t tiles, double* out)
{
    __shared__ double red[2 * (256 / 64)];
    const double* base = slots + (int64_t)blockIdx.x * tiles;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < tiles; i += blockDim.x)
        s += base[i];
    const double2 tot = block_sum2(s, 0.0, red);
    if (threadIdx.x == 0)
        out[blockIdx.x] = tot.x;
}

// dts[L] = 2 sum_g sums[L * G + g] (g ascending); dgammas[i] = 2 sums[p G + i], i < p E
__global__ void grad_finalize_kernel(const double* sums, int p, int G, int E, double* dgammas, double* dts)
{
    for (int L = threadIdx.x; L < p; L += blockDim.x) {
        double s = 0.0;
        for (int g = 0; g < G; ++g)
            s += sums[L * G + g];
        dts[L] = 2.0 * s;
    }
    for (int i = threadIdx.x; i < p * E; i += blockDim.x)
        dgammas[i] = 2.0 * sums[p * G + i];
}

template <int C>
hipError_t launch_gradx_c(const GradPassParams& P, unsigned grid, hipStream_t s)
{
    switch (P.flags) {
    case GMODE_TURN:
        hipLaunchKernelGGL((gradx_kernel<C, GMODE_TURN>), dim3(grid), dim3(kThreads), 0, s, P);
        break;
    case GMODE_MID:
        hipLaunchKernelGGL((gradx_kernel<C, GMODE_MID>), dim3(grid), dim3(kThreads), 0, s, P);
        break;
    case GMODE_BOUND:
        hipLaunchKernelGGL((gradx_kernel<C, GMODE_BOUND>), dim3(grid), dim3(kThreads), 0, s, P);
        break;
    case GMODE_FINAL:
        hipLaunchKernelGGL((gradx_kernel<C, GMODE_FINAL>), dim3(grid), dim3(kThreads), 0, s, P);
        break;
    case GMODE_TURN | GM_QTILE:
        hipLaunchKernelGGL((gradx_kernel<C, GMODE_TURN | GM_QTILE>), dim3(grid), dim3(kThreads), 0, s, P);
        break;
    case GMODE_BOUND | GM_QTILE:
        hipLaunchKernelGGL((gradx_kernel<C, GMODE_BOUND | GM_QTILE>), dim3(grid), dim3(kThreads), 0, s, P);
        break;
    case GMODE_FINAL | GM_QTILE:
        hipLaunchKernelGGL((gradx_kernel<C, GMODE_FINAL | GM_QTILE>), dim3(grid), dim3(kThreads), 0, s, P);
        break;
    case GMODE_BOUND_Z:
        hipLaunchKernelGGL((gradxz_kernel<C, GMODE_BOUND_Z>), dim3(grid), dim3(kThreads), 0, s, P);
        break;
    case GMODE_FINAL_Z:
        hipLaunchKernelGGL((gradxz_kernel<C, GMODE_FINAL_Z>), dim3(grid), dim3(kThreads), 0, s, P);
        break;
    case GMODE_ZSLOT:
        hipLaunchKernelGGL((zslot_kernel<C>), dim3(grid), dim3(kThreads), 0, s, P);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int C>
hipError_t launch_gradf_c(const GradPassParams& P, unsigned grid, hipStream_t s)
{
    switch (P.flags) {
    case GMODE_B_TURN:
        hipLaunchKernelGGL((gradb_kernel<C, GMODE_B_TURN>), dim3(grid), dim3(kThreads), 0, s, P);
        break;
    case GMODE_B_LAM:
        hipLaunchKernelGGL((gradb_kernel<C, GMODE_B_LAM>), dim3(grid), dim3(kThreads), 0, s, P);
        break;
    case GMODE_B_Q:
        hipLaunchKernelGGL((gradb_kernel<C, GMODE_B_Q>), dim3(grid), dim3(kThreads), 0, s, P);
        break;
    case GMODE_B_FINAL:
        hipLaunchKernelGGL((gradb_kernel<C, GMODE_B_FINAL>), dim3(grid), dim3(kThreads), 0, s, P);
        break;
    case GMODE_TURN:
        hipLaunchKernelGGL((gradf_kernel<C, GMODE_TURN>), dim3(grid), dim3(kThreads), 0, s, P);
        break;
    case GMODE_BOUND:
        hipLaunchKernelGGL((gradf_kernel<C, GMODE_BOUND>), dim3(grid), dim3(kThreads), 0, s, P);
        break;
    case GMODE_FINAL:
        hipLaunchKernelGGL((gradf_kernel<C, GMODE_FINAL>), dim3(grid), dim3(kThreads), 0, s, P);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gradpass(const GradPassParams& P, bool circulant, hipStream_t s)
{
    const unsigned grid = (unsigned)(int64_t(1) << (P.n - kTileBits));
    if (circulant) {
        if (P.col_bits == 0) {
            if (P.flags != GMODE_LOWDIAG)
                return hipErrorInvalidValue;
            hipLaunchKernelGGL((gradf_kernel<0, GMODE_LOWDIAG>), dim3(grid), dim3(kThreads), 0, s, P);
            return hipGetLastError();
        }
        switch (P.col_bits) {
        case 3:
            return launch_gradf_c<3>(P, grid, s);
        case 4:
            return launch_gradf_c<4>(P, grid, s);
        case 5:
            return launch_gradf_c<5>(P, grid, s);
        case 6:
            return launch_gradf_c<6>(P, grid, s);
        case 7:
            return launch_gradf_c<7>(P, grid, s);
        case 8:
            return launch_gradf_c<8>(P, grid, s);
        case 9:
            return launch_gradf_c<9>(P, grid, s);
        case 10:
            return launch_gradf_c<10>(P, grid, s);
        case 11:
            return launch_gradf_c<11>(P, grid, s);
        default:
            return hipErrorInvalidValue;
        }
    }
    switch (P.col_bits) {
    case 0:
        return launch_gradx_c<0>(P, grid, s);
    case 3:
        return launch_gradx_c<3>(P, grid, s);
    case 4:
        return launch_gradx_c<4>(P, grid, s);
    case 5:
        return launch_gradx_c<5>(P, grid, s);
    case 6:
        return launch_gradx_c<6>(P, grid, s);
    case 7:
        return launch_gradx_c<7>(P, grid, s);
    case 8:
        return launch_gradx_c<8>(P, grid, s);
    case 9:
        return launch_gradx_c<9>(P, grid, s);
    case 10:
        return launch_gradx_c<10>(P, grid, s);
    case 11:
        return launch_gradx_c<11>(P, grid, s);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_small_grad(const SmallGradParams& P, hipStream_t s)
{
    hipLaunchKernelGGL(small_grad_kernel, dim3(1), dim3(kThreads), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_grad_reduce(const double* slots, int nslots, int64_t tiles, double* sums, int p, int G,
                              int E, double* dgammas, double* dts, hipStream_t s)
{
    if (nslots > 0) {
        hipLaunchKernelGGL(slot_reduce_kernel, dim3(nslots), dim3(256), 0, s, slots, tiles, sums);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(grad_finalize_kernel, dim3(1), dim3(64), 0, s, sums, p, G, E, dgammas, dts);
    return hipGetLastError();
}

}  // namespace qva
