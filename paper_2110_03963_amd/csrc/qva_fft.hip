// qva_fft.hip -- circulant-mixer (QWOA) passes: F^-1 diag(exp(-i t lambda)) F.
//
// The eigensystem of a circulant W is the discrete Fourier transform (paper
// Sec. 3), so exp(-i t W) = F^-1 diag(exp(-i t lambda_m)) F with F the
// unnormalised DFT, F_mj = exp(-2 pi i j m / N).
//
// F is computed in place as a mixed-radix decimation-in-frequency transform
// over the same 4096-amplitude tiles as the hypercube mixer.  The index bits
// of a tile that lie in one register layout form a "digit" (up to 4 bits,
// radix up to 16).  One DIF step over the digit at global bits [gb, gb+w) is
//   y[j_lo + 2^gb m + ...] = W_{2^(gb+w)}^(j_lo m) sum_d x[j_lo + 2^gb d + ...] W_{2^w}^(d m)
// with j_lo the index bits below gb: a 2^w-point DFT in registers (radix-2
// stages with constant twiddles) followed by one exact twiddle per element
// (sincospi of a dyadic rational).  Digits are taken from the top bit down.
// The register DFT leaves each digit bit-reversed and the digit order is
// reversed, so position p ends up holding X[bitrev_n(p)]: the diagonal is
// applied with lambda at the bit-reversed index, and the inverse transform
// (the same steps undone in reverse order, conjugate twiddles, 1/N at the
// end) restores natural order.  No permutation pass is needed.
#include "qva_tile.h"

namespace qva {
namespace {

using namespace tile;

// psi <- scale * exp(-i gamma q) psi in layout A
__device__ __forceinline__ void phase_a(double2 (&v)[kRegs], const double* q, const TileMap& g, int t,
                                        double gamma, double scale)
{
    double qq[kRegs];
#pragma unroll
    for (int r = 0; r < kRegs; ++r)
        qq[r] = ld_nt(q + g(elem<LA>(t, r)));
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
        const double2 ph = expmi(gamma * qq[r]);
        v[r] = cmul(v[r], make_double2(scale * ph.x, scale * ph.y));
        QVA_SCHED_FENCE();
    }
}

// exp(-i t lambda_m) at bit-reversed positions, in layout C of a low-group tile.
__device__ __forceinline__ void diag_c(double2 (&v)[kRegs], const FftPassParams& P, int64_t tile, int t,
                                       double tt)
{
    const int n = P.n;
    if (P.lambda_kind == FFT_LAMBDA_COMPLETE) {
        // position (tile, elem) holds m = 0 only at tile 0, element 0
#pragma unroll
        for (int r = 0; r < kRegs; ++r)
            v[r] = cmul(v[r], complete_diag(tile == 0 && elem<LC>(t, r) == 0, tt, n));
        return;
    }
    if (P.lambda_kind == FFT_LAMBDA_RING) {
        // registers r and r + 1 (r even) hold digits k and k + 8, whose ring
        // eigenvalues are exact negatives: one exponential serves both
        const double2 u = ring_lambda_base(tile, t, n);
#pragma unroll
        for (int r = 0; r < kRegs; r += 2) {
            const double2 e = expmi(tt * ring_lambda(u, r));
            v[r] = cmul(v[r], e);
            v[r + 1] = cmul(v[r + 1], make_double2(e.x, -e.y));
            QVA_SCHED_FENCE();
        }
        return;
    }
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
        double lam;
        if (P.lambda_kind == FFT_LAMBDA_TILED) {
            lam = ld_nt(P.lam + (tile << kTileBits) + r * kThreads + t);
        } else {
            const int64_t pos = (tile << kTileBits) | elem<LC>(t, r);
            const uint64_t m = __brevll((uint64_t)pos) >> (64 - n);
            lam = P.lam[m];
        }
        v[r] = cmul(v[r], expmi(tt * lam));
        QVA_SCHED_FENCE();
    }
}

template <int FLAGS>
__device__ __forceinline__ void expect_store_a(double2 (&v)[kRegs], const FftPassParams& P,
                                               const TileMap& g, int t, double scale, double* red)
{
    if constexpr (FLAGS & FP_EXPECT) {
        double qq[kRegs];
#pragma unroll
        for (int r = 0; r < kRegs; ++r)
            qq[r] = ld_nt(P.q + g(elem<LA>(t, r)));
        double f = 0.0, nr = 0.0;
#pragma unroll
        for (int r = 0; r < kRegs; ++r) {
            const double a = v[r].x * v[r].x + v[r].y * v[r].y;
            f = fma(a, qq[r], f);
            nr += a;
        }
        const double s2 = scale * scale;
        const double2 tot = block_sum2(f * s2, nr * s2, red);
        if (t == 0)
            P.partials[blockIdx.x] = tot;
    }
    if constexpr (FLAGS & FP_STORE)
        store_tile<LA>(v, P.psi, g, t, scale);
}

// ---------------------------------------------------------------- Bluestein
// For N not a power of two the transform is the chirp-z form: with
// w_k = exp(i pi k^2 / N) and jm = (j^2 + m^2 - (m - j)^2) / 2,
//   DFT_N(x)_m = conj(w_m) sum_j (x_j conj(w_j)) w_{m-j},
//   DFT_N^-1(X)_j = (1/N) w_j sum_m (X_m w_m) conj(w_{j-m}),
// each a linear convolution done cyclically over M = 2^n >= 2N - 1 (the
// filter w_k, |k| < N, sits at k and M - k).  Inside one mixer the chirps
// between the two convolutions cancel (conj(w_m) w_m = 1), and so do those
// between the inverse of layer k and the forward of layer k + 1, so the
// evolution stays in the padded buffer: convolve with w, multiply by
// exp(-i t lambda_m) (m < N, zero above), convolve with conj(w), multiply by
// exp(-i gamma q_j) / N (j < N, zero above), ...  The filters' spectra
// (times 1/M, the inverse transform's factor) are computed once per call.

// w_k = exp(i pi k^2 / N), k < N < 2^31, with k^2 reduced mod 2N exactly.
__device__ __forceinline__ double2 chirp(int64_t k, int64_t N)
{
    const uint64_t r = ((uint64_t)k * (uint64_t)k) % (uint64_t)(2 * N);
    double s, c;
    sincospi_red((double)r / (double)N, &s, &c);
    return make_double2(c, s);
}

// Element-wise factor of a Bluestein boundary pass at natural index j.
template <int FLAGS>
__device__ __forceinline__ double2 bluestein_factor(const FftPassParams& P, int64_t j, double ang,
                                                    double invN)
{
    if (j >= P.nb)
        return make_double2(0.0, 0.0);
    if constexpr (FLAGS == FMODE_B_BOUND_LAM) {
        double lam;
        if (P.lambda_kind == FFT_LAMBDA_RING) {
            double s, c;
            sincospi_red((double)(2 * j) / (double)P.nb, &s, &c);  // lambda_j = 2 cos(2 pi j / N)
            lam = 2.0 * c;
        } else {
            lam = P.lam[j];
        }
        return expmi(ang * lam);
    } else {
        const double2 e = expmi(ang * ld_nt(P.q + j));
        return make_double2(e.x * invN, e.y * invN);
    }
}

template <int C, int FLAGS>
__global__ __launch_bounds__(kThreads, 2) void fftpass_kernel(FftPassParams P)
{
    __shared__ double2 lds[1 << kTileBits];
    __shared__ double red[2 * (kThreads / 64)];
    const int t = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const TileMap g = tile_map(tile, P.k, C);
    const double invN = ldexp(1.0, -P.n);
    double2 v[kRegs];

    if constexpr (FLAGS == FMODE_FIRST) {
        const double a0 = 1.0 / sqrt((double)(int64_t(1) << P.n));
#pragma unroll
        for (int r = 0; r < kRegs; ++r)
            v[r] = make_double2(a0, 0.0);
        phase_a(v, P.q, g, t, angle_value(P.phase), 1.0);
        dif_tile<C>(v, lds, g, t);
        store_tile<dif_last<C>()>(v, P.psi, g, t, 1.0);
    } else if constexpr (FLAGS == FMODE_DIF) {
        load_tile<LA>(v, P.psi, g, t);
        dif_tile<C>(v, lds, g, t);
        store_tile<dif_last<C>()>(v, P.psi, g, t, 1.0);
    } else if constexpr (FLAGS == FMODE_DIT || FLAGS == FMODE_DIT_SCALE) {
        load_tile<dif_last<C>()>(v, P.psi, g, t);
        dit_tile<C>(v, lds, g, t);
        store_tile<LA>(v, P.psi, g, t, FLAGS == FMODE_DIT_SCALE ? invN : 1.0);
    } else if constexpr (FLAGS == FMODE_LOWDIAG) {
        load_tile<LA>(v, P.psi, g, t);
        dif_tile<C, true>(v, lds, g, t, P.tw);
        diag_c(v, P, tile, t, angle_value(P.mix1));
        dit_tile<C, true>(v, lds, g, t, P.tw);
        store_tile<LA>(v, P.psi, g, t, 1.0);
    } else if constexpr (FLAGS == FMODE_BOUNDARY) {
        // the angle first, each register's psi and q requested together, the
        // phase factors computed after the whole tile is in flight
        double gam = angle_value(P.phase);
        double qq[kRegs];
#pragma unroll
        for (int r = 0; r < kRegs; ++r) {
            v[r] = ld_nt(P.psi + g(elem<dif_last<C>()>(t, r)));
            qq[r] = ld_nt(P.q + g(elem<LA>(t, r)));
            QVA_ISSUE_FENCE();
        }
        asm volatile("" : "+v"(gam)::"memory");
        dit_tile<C>(v, lds, g, t);
#pragma unroll
        for (int r = 0; r < kRegs; ++r) {
            const double2 ph = expmi(gam * qq[r]);
            v[r] = cmul(v[r], make_double2(invN * ph.x, invN * ph.y));
            QVA_SCHED_FENCE();
        }
        dif_tile<C>(v, lds, g, t);
        store_tile<dif_last<C>()>(v, P.psi, g, t, 1.0);
    } else if constexpr (FLAGS == FMODE_LAST || FLAGS == FMODE_LAST_STORE) {
        load_tile<dif_last<C>()>(v, P.psi, g, t);
        dit_tile<C>(v, lds, g, t);
        expect_store_a<FLAGS>(v, P, g, t, invN, red);
    } else if constexpr (FLAGS == FMODE_B_CHIRP) {
        const int64_t M = int64_t(1) << P.n;
#pragma unroll
        for (int r = 0; r < kRegs; ++r) {
            const int64_t i = g(elem<LA>(t, r));
            const int64_t k = i < P.nb ? i : (i > M - P.nb ? M - i : -1);
            double2 w = k >= 0 ? chirp(k, P.nb) : make_double2(0.0, 0.0);
            v[r] = P.conj ? make_double2(w.x, -w.y) : w;
        }
        dif_tile<C>(v, lds, g, t);
        store_tile<dif_last<C>()>(v, P.psi, g, t, 1.0);
    } else if constexpr (FLAGS == FMODE_B_FIRST) {
        const double a0 = 1.0 / sqrt((double)P.nb);
        const double gam = angle_value(P.phase);
#pragma unroll
        for (int r = 0; r < kRegs; ++r) {
            const int64_t j = g(elem<LA>(t, r));
            if (j < P.nb) {
                const double2 w = chirp(j, P.nb);
                const double2 ph = cmul(expmi(gam * ld_nt(P.q + j)), make_double2(w.x, -w.y));
                v[r] = make_double2(a0 * ph.x, a0 * ph.y);
            } else {
                v[r] = make_double2(0.0, 0.0);
            }
        }
        dif_tile<C>(v, lds, g, t);
        store_tile<dif_last<C>()>(v, P.psi, g, t, 1.0);
    } else if constexpr (FLAGS == FMODE_B_BOUND_LAM || FLAGS == FMODE_B_BOUND_Q) {
        const double ang = FLAGS == FMODE_B_BOUND_LAM ? angle_value(P.mix1) : angle_value(P.phase);
        const double invNb = 1.0 / (double)P.nb;
        load_tile<dif_last<C>()>(v, P.psi, g, t);
        dit_tile<C>(v, lds, g, t);
#pragma unroll
        for (int r = 0; r < kRegs; ++r) {
            v[r] = cmul(v[r], bluestein_factor<FLAGS>(P, g(elem<LA>(t, r)), ang, invNb));
            QVA_SCHED_FENCE();
        }
        dif_tile<C>(v, lds, g, t);
        store_tile<dif_last<C>()>(v, P.psi, g, t, 1.0);
    } else if constexpr (FLAGS == FMODE_B_LOAD) {
        // a_j = psi_j conj(w_j) for j < N, zero above: the input of the
        // forward transform's convolution
#pragma unroll
        for (int r = 0; r < kRegs; ++r) {
            const int64_t j = g(elem<LA>(t, r));
            if (j < P.nb) {
                const double2 w = chirp(j, P.nb);
                v[r] = cmul(ld_nt(P.in + j), make_double2(w.x, -w.y));
            } else {
                v[r] = make_double2(0.0, 0.0);
            }
        }
        dif_tile<C>(v, lds, g, t);
        store_tile<dif_last<C>()>(v, P.psi, g, t, 1.0);
    } else if constexpr (FLAGS == FMODE_B_LAST || FLAGS == FMODE_B_LAST_STORE || FLAGS == FMODE_B_STORE) {
        // x_j after the second convolution; psi_j = w_j x_j / N for j < N
        const double invNb = 1.0 / (double)P.nb;
        load_tile<dif_last<C>()>(v, P.psi, g, t);
        dit_tile<C>(v, lds, g, t);
        double f = 0.0, nr = 0.0;
#pragma unroll
        for (int r = 0; r < kRegs; ++r) {
            const int64_t j = g(elem<LA>(t, r));
            if (j < P.nb) {
                const double2 x = make_double2(v[r].x * invNb, v[r].y * invNb);
                if constexpr (FLAGS & FP_EXPECT) {
                    const double a = x.x * x.x + x.y * x.y;
                    f = fma(a, ld_nt(P.q + j), f);
                    nr += a;
                }
                if constexpr (FLAGS & FP_STORE)
                    st_nt(P.out + j, cmul(chirp(j, P.nb), x));
            }
        }
        if constexpr (FLAGS & FP_EXPECT) {
            const double2 tot = block_sum2(f, nr, red);
            if (t == 0)
                P.partials[blockIdx.x] = tot;
        }
    } else if constexpr (FLAGS == FMODE_LOWMUL) {
        load_tile<LA>(v, P.psi, g, t);
        dif_tile<C, true>(v, lds, g, t, P.tw);
#pragma unroll
        for (int r = 0; r < kRegs; ++r)
            v[r] = cmul(v[r], ld_nt(P.bt + (tile << kTileBits) + r * kThreads + t));
        dit_tile<C, true>(v, lds, g, t, P.tw);
        store_tile<LA>(v, P.psi, g, t, 1.0);
    } else if constexpr (FLAGS == FMODE_LOWDIF_TILED) {
        // the filter's spectrum in the order FMODE_LOWMUL reads it, times 1/M
        const double invM = ldexp(1.0, -P.n);
        load_tile<LA>(v, P.psi, g, t);
        dif_tile<C, true>(v, lds, g, t, P.tw);
#pragma unroll
        for (int r = 0; r < kRegs; ++r)
            st_nt(P.out + (tile << kTileBits) + r * kThreads + t, make_double2(v[r].x * invM, v[r].y * invM));
    }
}

// ---------------------------------------------------------------------------
// Whole state in one workgroup (n <= 12): radix-2 DIF / DIT in LDS.
// ---------------------------------------------------------------------------
__device__ void small_fft(double2* s, int n, bool inverse)
{
    const int N = 1 << n;
    for (int it = 0; it < n; ++it) {
        const int st = inverse ? it : n - 1 - it;  // DIF: top bit first; DIT: bottom first
        const int h = 1 << st;
        for (int m = threadIdx.x; m < N / 2; m += blockDim.x) {
            const int j = ((m >> st) << (st + 1)) | (m & (h - 1));
            const int u = j & (h - 1);
            double sn, cs;
            sincospi_red(ldexp((double)u, -st), &sn, &cs);  // angle pi u / h = 2 pi u / (2h)
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

__device__ void small_circulant(double2* s, const SmallFftParams& P, double tt)
{
    const int n = P.n, N = 1 << n;
    small_fft(s, n, false);
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
        const unsigned m = __brev((unsigned)j) >> (32 - n);
        if (P.lambda_kind == FFT_LAMBDA_COMPLETE) {
            s[j] = cmul(s[j], complete_diag(m == 0, tt, n));
            continue;
        }
        const double lam = P.lambda_kind == FFT_LAMBDA_NATURAL ? P.lam[m] : ring_lambda_m(m, n);
        s[j] = cmul(s[j], expmi(tt * lam));
    }
    __syncthreads();
    small_fft(s, n, true);
    const double invN = ldexp(1.0, -n);
    for (int j = threadIdx.x; j < N; j += blockDim.x)
        s[j] = make_double2(s[j].x * invN, s[j].y * invN);
    __syncthreads();
}

__global__ __launch_bounds__(kThreads) void small_fft_kernel(SmallFftParams P)
{
    __shared__ double2 s[1 << kTileBits];
    __shared__ double red[2 * (kThreads / 64)];
    const int N = 1 << P.n;
    const int t = threadIdx.x;
    const double a0 = 1.0 / sqrt((double)N);
    for (int j = t; j < N; j += blockDim.x)
        s[j] = (P.flags & SM_INIT) ? make_double2(a0, 0.0) : P.psi[j];
    __syncthreads();
    if (P.flags & SM_MIX_ONCE)
        small_circulant(s, P, P.t_val);
    if (P.flags & SM_EVOLVE) {
        for (int layer = 0; layer < P.p; ++layer) {
            const double gam = P.gammas[layer];
            for (int j = t; j < N; j += blockDim.x)
                s[j] = cmul(s[j], expmi(gam * P.q[j]));
            __syncthreads();
            small_circulant(s, P, P.ts[layer]);
        }
    }
    if (P.flags & SM_EXPECT) {
        double f = 0.0, nr = 0.0;
        for (int j = t; j < N; j += blockDim.x) {
            const double a = s[j].x * s[j].x + s[j].y * s[j].y;
            f = fma(a, P.q[j], f);
            nr += a;
        }
        const double2 tot = block_sum2(f, nr, red);
        if (t == 0) {
            P.out_f[0] = tot.x;
            if (P.out_norm)
                P.out_norm[0] = tot.y;
        }
    }
    if (P.flags & SM_STORE)
        for (int j = t; j < N; j += blockDim.x)
            P.psi[j] = s[j];
}

// lam_tiled[tile][r][t] = lambda[bitrev_n(tile * 4096 + r + 16 t)]: the
// eigenvalue each low-group tile needs in layout C, laid out for coalesced reads.
__global__ __launch_bounds__(256) void lambda_tile_kernel(const double* lam, double* out, int n)
{
    const int64_t N = int64_t(1) << n;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        const int64_t tile = i >> kTileBits;
        const int w = (int)(i & ((1 << kTileBits) - 1));
        const int r = w / kThreads, t = w % kThreads;
        const int64_t pos = (tile << kTileBits) | elem<LC>(t, r);
        const uint64_t m = __brevll((uint64_t)pos) >> (64 - n);
        out[i] = lam[m];
    }
}

__global__ __launch_bounds__(kThreads) void twiddle_table_kernel(double2* tab)
{
    twiddle_table_fill(tab, threadIdx.x);
}

template <int C>
hipError_t launch_fft_c(const FftPassParams& P, unsigned grid, hipStream_t s)
{
    switch (P.flags) {
#define QVA_FFT_MODE(F)                                                                 \
    case F:                                                                             \
        hipLaunchKernelGGL((fftpass_kernel<C, F>), dim3(grid), dim3(kThreads), 0, s, P); \
        break;
        QVA_FFT_MODE(FMODE_FIRST)
        QVA_FFT_MODE(FMODE_DIF)
        QVA_FFT_MODE(FMODE_DIT)
        QVA_FFT_MODE(FMODE_DIT_SCALE)
        QVA_FFT_MODE(FMODE_BOUNDARY)
        QVA_FFT_MODE(FMODE_LAST)
        QVA_FFT_MODE(FMODE_LAST_STORE)
        QVA_FFT_MODE(FMODE_B_CHIRP)
        QVA_FFT_MODE(FMODE_B_FIRST)
        QVA_FFT_MODE(FMODE_B_BOUND_LAM)
        QVA_FFT_MODE(FMODE_B_BOUND_Q)
        QVA_FFT_MODE(FMODE_B_LAST)
        QVA_FFT_MODE(FMODE_B_LAST_STORE)
        QVA_FFT_MODE(FMODE_B_LOAD)
        QVA_FFT_MODE(FMODE_B_STORE)
#undef QVA_FFT_MODE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fftpass(const FftPassParams& P, hipStream_t s)
{
    const unsigned grid = (unsigned)(int64_t(1) << (P.n - kTileBits));
    if (P.col_bits == 0) {
        switch (P.flags) {
        case FMODE_LOWDIAG:
            hipLaunchKernelGGL((fftpass_kernel<0, FMODE_LOWDIAG>), dim3(grid), dim3(kThreads), 0, s, P);
            break;
        case FMODE_LOWMUL:
            hipLaunchKernelGGL((fftpass_kernel<0, FMODE_LOWMUL>), dim3(grid), dim3(kThreads), 0, s, P);
            break;
        case FMODE_LOWDIF_TILED:
            hipLaunchKernelGGL((fftpass_kernel<0, FMODE_LOWDIF_TILED>), dim3(grid), dim3(kThreads), 0, s, P);
            break;
        default:
            return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (P.col_bits) {
    case 3:
        return launch_fft_c<3>(P, grid, s);
    case 4:
        return launch_fft_c<4>(P, grid, s);
    case 5:
        return launch_fft_c<5>(P, grid, s);
    case 6:
        return launch_fft_c<6>(P, grid, s);
    case 7:
        return launch_fft_c<7>(P, grid, s);
    case 8:
        return launch_fft_c<8>(P, grid, s);
    case 9:
        return launch_fft_c<9>(P, grid, s);
    case 10:
        return launch_fft_c<10>(P, grid, s);
    case 11:
        return launch_fft_c<11>(P, grid, s);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_small_fft(const SmallFftParams& P, hipStream_t s)
{
    hipLaunchKernelGGL(small_fft_kernel, dim3(1), dim3(kThreads), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_twiddle_table(double2* tab, hipStream_t s)
{
    hipLaunchKernelGGL(twiddle_table_kernel, dim3(1), dim3(kThreads), 0, s, tab);
    return hipGetLastError();
}

hipError_t launch_lambda_tiles(const double* lam, double* out, int n, hipStream_t s)
{
    const int64_t N = int64_t(1) << n;
    int64_t g = (N + 255) / 256;
    if (g > 65536)
        g = 65536;
    hipLaunchKernelGGL(lambda_tile_kernel, dim3((unsigned)g), dim3(256), 0, s, lam, out, n);
    return hipGetLastError();
}

}  // namespace qva
