// qva_mixed.hip -- circulant mixer over N solutions with small prime factors:
// exp(-i t W) = F^-1 diag(exp(-i t lambda_m)) F (paper Sec. 3) with the DFT of
// length N computed in place by mixed-radix tile passes, no padding.
//
// N = A_0 A_1 ... A_{G-1} (qva_mrplan.h), j = j_0 + A_0 (j_1 + A_1 (j_2 + ...)),
// S_g = A_0 ... A_{g-1}.  Decimation in frequency, top group first: the pass of
// group g takes, for each lower index jl < S_g (and each value of the higher
// digits), the A_g-point DFT over j_g and multiplies output m_g by the twiddle
// W_{S_{g+1}}^(jl m_g), W_M = exp(-2 pi i / M).  After all groups, position
// p = sum_g p_g S_g holds X[m] with m = p_{G-1} + A_{G-1} (p_{G-2} + ... +
// A_1 p_0): the diagonal takes lambda at that m, and the inverse passes
// (conjugate twiddle first, then the inverse group DFT, low group first, 1/N
// at the end) restore natural order.
//
// A tile is one group's A_g-point DFT for up to cols_g columns (lower
// indices, contiguous in memory for strided groups; whole contiguous runs of
// A_0 for the low group).  Element e of the tile (e < ncol A_g) is also its
// LDS slot: low group col = e / A_0, j = e mod A_0; strided groups
// j = e / ncol, col = e mod ncol, so consecutive threads touch consecutive
// addresses in HBM.  The group DFT runs in LDS as in-place Cooley-Tukey DIF
// stages over the group's radices (each stage an R-point DFT in registers,
// paired outputs for odd R, then the twiddle W_L^(i m) by recurrence from two
// table roots); the output, digit reversed, is gathered back in natural order
// through a permutation table.  The twiddle between groups is a per-tile root
// (LDS) times a per-group table entry.  Roots W_{A_g}^k, the inter-group
// twiddles and the permutations are computed once per call into the
// workspace.
#include "qva_ctroots.h"
#include "qva_internal.h"

namespace qva {
namespace {

constexpr int kMrThreads = 256;
constexpr int kMrRegs = kMrTileElems / kMrThreads;

// LDS slot of tile element e.  When the low group's radices put a
// power-of-two radix after the odd ones (3496 = 23 19 8), the last stages
// read at strides of 8 or 16 elements (128 or 256 B), which land the lanes
// of a quarter-wave on the same banks; the planner then sets lds_pad and the
// low group's passes are built with PAD: one pad element after every 16
// spreads them.  Other passes keep slot e.
constexpr int kMrLdsElems = kMrTileElems + kMrTileElems / 16;
template <bool PAD>
__device__ __forceinline__ int mr_slot(int e) { return PAD ? e + (e >> 4) : e; }

// A tile's thread index: the workgroup's in the single-vector kernels, the
// half's in the two-vector kernels (two halves of 256 threads).
__device__ __forceinline__ int mr_tid() { return threadIdx.x & (kMrThreads - 1); }

// q = floor(e / d) for 0 <= e < 2^31, 1 <= d <= 4096 via the reciprocal
// rd = 1/d in double: (e + 1/2) / d lies at least 1/(2d) >= 2^-13 inside
// (q, q + 1), far beyond the rounding error of rd and of the product
// (below 2^31 * 2^-52 = 2^-21).
__device__ __forceinline__ int divq(int e, double rd) { return (int)(((double)e + 0.5) * rd); }

struct MrTile {
    int A;         // transform length of the group
    int ncol;      // columns of this tile
    bool low;      // group 0: contiguous columns of A_0
    int64_t base;  // global index of element (col 0, j 0)
    int64_t S;     // global stride of j (strided groups)
    int64_t first; // first column's index: upper index (low group) or lower index jl
    double rA, rncol;
    __device__ __forceinline__ int col_of(int e) const { return low ? divq(e, rA) : e - ncol * divq(e, rncol); }
    __device__ __forceinline__ int j_of(int e) const { return low ? e - A * divq(e, rA) : divq(e, rncol); }
    __device__ __forceinline__ int lidx(int col, int j) const { return low ? col * A + j : j * ncol + col; }
    __device__ __forceinline__ int64_t gidx(int e) const
    {
        if (low)
            return base + e;
        const int j = divq(e, rncol);
        return base + (e - ncol * j) + S * (int64_t)j;
    }
};

__device__ __forceinline__ MrTile mr_tile(const MrGeom* __restrict__ m, int g, int64_t tile)
{
    MrTile T;
    T.A = m->A[g];
    T.low = g == 0;
    const int c = m->cols[g];
    if (g == 0) {
        const int64_t U = m->S[m->G] / T.A;
        const int64_t u0 = tile * c;
        T.ncol = (int)(U - u0 < c ? U - u0 : c);
        T.base = u0 * T.A;
        T.S = 1;
        T.first = u0;
    } else {
        const int64_t Sg = m->S[g];
        const int64_t chunks = (Sg + c - 1) / c;
        const int64_t w = tile / chunks, ch = tile - w * chunks;
        const int64_t jl0 = ch * c;
        T.ncol = (int)(Sg - jl0 < c ? Sg - jl0 : c);
        T.base = jl0 + m->S[g + 1] * w;
        T.S = Sg;
        T.first = jl0;
    }
    T.rA = 1.0 / (double)T.A;
    T.rncol = 1.0 / (double)T.ncol;
    return T;
}

__device__ __forceinline__ double2 conj_if(double2 a, bool c) { return make_double2(a.x, c ? -a.y : a.y); }

// W_R^j = exp(-2 pi i j / R) as compile-time constants (qva_ctroots.h), for
// the radix-29 and -31 stages: held as literals instead of loaded table
// roots, they keep those stages within the registers of two waves per SIMD.
template <int R>
__device__ __forceinline__ double2 ct_w(int j)
{
    constexpr CtRoots<R> t{};
    return make_double2(t.v[j].c, -t.v[j].s);
}

// R-point DFT of x in registers, y_m = sum_k x_k W_R^(k m) (inverse: W^-1),
// with each output handed to out(m, y_m) in pair order: m = 0, then m, R - m
// for m = 1, 2, ..., then m = R/2 for even R.  root(j) = W_R^j (forward sign).
// Odd R = 2h + 1: with a_k = x_k + x_{R-k}, b_k = x_k - x_{R-k} (k <= h, formed
// in place in x),
//   y_m = x_0 + sum_k a_k cos(2 pi k m / R) - i sum_k b_k sin(2 pi k m / R),
// and y_{R-m} the same with +i, so each pair of outputs costs 4h FMAs.
// R = 2^w: radix-2 DIF stages in registers, outputs read bit-reversed.
template <int R, typename Root, typename Out>
__device__ __forceinline__ void dft_regs(double2 (&x)[R], bool inv, Root&& root, Out&& out)
{
    if constexpr ((R & (R - 1)) == 0) {
        constexpr int W = R == 2 ? 1 : (R == 4 ? 2 : (R == 8 ? 3 : 4));
        double2 w[R / 2];
#pragma unroll
        for (int j = 0; j < R / 2; ++j)
            w[j] = conj_if(root(j), inv);
#pragma unroll
        for (int bb = W - 1; bb >= 0; --bb) {
            const int half = 1 << bb;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (r & half)
                    continue;
                const int l = r & (half - 1);
                const double2 a = x[r], c = x[r | half];
                x[r] = make_double2(a.x + c.x, a.y + c.y);
                const double2 d = make_double2(a.x - c.x, a.y - c.y);
                x[r | half] = l == 0 ? d : cmul(d, w[l * (R / (2 * half))]);
            }
        }
        auto rev = [](int m) {
            int rv = 0;
#pragma unroll
            for (int i = 0; i < W; ++i)
                rv |= ((m >> i) & 1) << (W - 1 - i);
            return rv;
        };
        out(0, x[0]);
#pragma unroll
        for (int m = 1; m < R / 2; ++m) {
            out(m, x[rev(m)]);
            out(R - m, x[rev(R - m)]);
        }
        out(R / 2, x[rev(R / 2)]);
    } else {
        constexpr int H = R / 2;
        double2 y0 = x[0];
#pragma unroll
        for (int k = 1; k <= H; ++k) {
            const double2 u = x[k], v = x[R - k];
            x[k] = make_double2(u.x + v.x, u.y + v.y);      // a_k
            x[R - k] = make_double2(u.x - v.x, u.y - v.y);  // b_k
            y0.x += x[k].x;
            y0.y += x[k].y;
        }
        out(0, y0);
#pragma unroll
        for (int m = 1; m <= H; ++m) {
            double2 P = x[0], Q = make_double2(0.0, 0.0);
#pragma unroll
            for (int k = 1; k <= H; ++k) {
                const int j = (k * m) % R;  // 1 .. R - 1
                const double2 r = root(j <= H ? j : R - j);  // (cos, -sin) of 2 pi j' / R
                const double c = r.x;
                const double sv = (j <= H) != inv ? -r.y : r.y;  // sin(2 pi j / R), inverse flipped
                P.x = fma(x[k].x, c, P.x);
                P.y = fma(x[k].y, c, P.y);
                Q.x = fma(x[R - k].x, sv, Q.x);
                Q.y = fma(x[R - k].y, sv, Q.y);
            }
            // y_m = P - i Q, y_{R-m} = P + i Q
            out(m, make_double2(P.x + Q.y, P.y - Q.x));
            out(R - m, make_double2(P.x - Q.y, P.y + Q.x));
            QVA_SCHED_FENCE();
        }
    }
}

// One DIF stage of radix R over sub-length L of every column's A-point DFT
// in LDS: butterfly (b, i), i < L/R, takes elements b L + i + k L/R, forms
// y_m = sum_k x_k W_R^(k m), multiplies y_m by the twiddle W_L^(i m) and
// writes it back in place.  Roots from the group table tab[k] = W_A^k
// (conjugated: inverse).  The twiddles follow from two table roots per
// butterfly, w = W_L^i and W_L^(i R): W_L^(i m) = W_L^(i (m-1)) w for
// m <= R/2 and W_L^(i R) conj(W_L^(i (R-m))) above, at most R/2 + 1 rounded
// products (about 2e-15 for R = 31), read before the butterfly's inputs so
// that no load waits inside the DFT.  The last stage (L = R) has none.
// LDS slot of (col, j): col A + j (low group) or j ncol + col.
template <int R, bool TW, bool PAD>
__device__ __forceinline__ void mr_stage_tw(double2* lds, int A, int ncol, bool low, int L,
                                            const double2* __restrict__ tab, bool inv)
{
    // rstep = A / R, formed from L so that it varies with the stage: the
    // root loads of the different radices are then not hoisted out of the
    // stage loop (held at once, they would exhaust the registers)
    const int mstride = L / R, per_col = A / R, tstep = A / L, rstep = mstride * tstep, wstep = R * tstep;
    const int items = ncol * per_col;
    const double rpc = 1.0 / (double)per_col, rms = 1.0 / (double)mstride, rnc = 1.0 / (double)ncol;
    const int cs = low ? A : 1, js = low ? 1 : ncol;  // element strides of col and j
    constexpr int H = R / 2;
    for (int it = mr_tid(); it < items; it += kMrThreads) {
        int col, bi;
        if (low) {  // i fastest: consecutive threads take consecutive j
            col = divq(it, rpc);
            bi = it - col * per_col;
        } else {    // col fastest: consecutive LDS slots
            bi = divq(it, rnc);
            col = it - bi * ncol;
        }
        const int b = divq(bi, rms), i = bi - b * mstride;
        const int base = col * cs + (b * L + i) * js, step = mstride * js;
        double2 w1 = make_double2(1.0, 0.0), wr = w1;
        if constexpr (TW) {
            w1 = conj_if(tab[i * tstep], inv);
            wr = conj_if(tab[i * wstep], inv);
        }
        double2 x[R];
#pragma unroll
        for (int k = 0; k < R; ++k)
            x[k] = lds[mr_slot<PAD>(base + k * step)];
        double2 wm = w1;  // W_L^(i m) of the last m <= H
        dft_regs<R>(
            x, inv,
            [&](int j) {
                if constexpr (R >= 29)
                    return ct_w<R>(j);
                else
                    return tab[j * rstep];
            },
            [&](int m, double2 y) {
            if constexpr (TW) {
                if (m > H) {
                    y = cmul(y, cmul(wr, make_double2(wm.x, -wm.y)));
                } else if (m > 0) {
                    if (m > 1)
                        wm = cmul(wm, w1);
                    y = cmul(y, wm);
                }
            }
            lds[mr_slot<PAD>(base + m * step)] = y;
        });
    }
}

template <int R, bool PAD>
__device__ __forceinline__ void mr_stage(double2* lds, int A, int ncol, bool low, int L,
                                         const double2* __restrict__ tab, bool inv)
{
    if (L > R)
        mr_stage_tw<R, true, PAD>(lds, A, ncol, low, L, tab, inv);
    else
        mr_stage_tw<R, false, PAD>(lds, A, ncol, low, L, tab, inv);
}

// Every DIF stage of one group's DFT on the tile in LDS.  MAXR: the largest
// radix the kernel is built for (16, 23 or 31); every class runs two waves
// per SIMD (the radix-29 and -31 stages with compile-time roots, and with a
// few dozen bytes of spill per lane, which cost less than one wave).
template <int MAXR, bool PAD>
__device__ __forceinline__ void mr_stages(double2* lds, int A, int ncol, bool low, const double2* __restrict__ gt,
                                          const int* __restrict__ rad, int nrad, bool inv)
{
    int L = A;
    for (int s = 0; s < nrad; ++s) {
        const int r = rad[s];
        switch (r) {
        case 2: mr_stage<2, PAD>(lds, A, ncol, low, L, gt, inv); break;
        case 3: mr_stage<3, PAD>(lds, A, ncol, low, L, gt, inv); break;
        case 4: mr_stage<4, PAD>(lds, A, ncol, low, L, gt, inv); break;
        case 5: mr_stage<5, PAD>(lds, A, ncol, low, L, gt, inv); break;
        case 7: mr_stage<7, PAD>(lds, A, ncol, low, L, gt, inv); break;
        case 8: mr_stage<8, PAD>(lds, A, ncol, low, L, gt, inv); break;
        case 11: mr_stage<11, PAD>(lds, A, ncol, low, L, gt, inv); break;
        case 13: mr_stage<13, PAD>(lds, A, ncol, low, L, gt, inv); break;
        case 16: mr_stage<16, PAD>(lds, A, ncol, low, L, gt, inv); break;
        default:
            if constexpr (MAXR >= 23) {
                switch (r) {
                case 17: mr_stage<17, PAD>(lds, A, ncol, low, L, gt, inv); break;
                case 19: mr_stage<19, PAD>(lds, A, ncol, low, L, gt, inv); break;
                case 23: mr_stage<23, PAD>(lds, A, ncol, low, L, gt, inv); break;
                default:
                    if constexpr (MAXR >= 31) {
                        if (r == 29)
                            mr_stage<29, PAD>(lds, A, ncol, low, L, gt, inv);
                        else
                            mr_stage<31, PAD>(lds, A, ncol, low, L, gt, inv);
                    }
                    break;
                }
            }
            break;
        }
        L /= r;
        __syncthreads();
    }
}

// The group DFT of every column of the tile, through LDS: v holds elements
// e = t + 256 k in natural j order on entry and natural frequency order on
// return (forward: exponent sign -, inv: +; no 1/A).
template <int MAXR, bool PAD>
__device__ __forceinline__ void mr_dft(double2 (&v)[kMrRegs], double2* lds, const MrTile& T,
                                       const MrGeom* __restrict__ m, int g, const double2* tab, const int* perm,
                                       bool inv)
{
    const int t = mr_tid(), ne = T.ncol * T.A;
    const int* gp = perm + m->tab_off[g];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kMrRegs; ++k) {
        const int e = t + k * kMrThreads;
        if (e < ne)
            lds[mr_slot<PAD>(e)] = v[k];
    }
    __syncthreads();
    mr_stages<MAXR, PAD>(lds, T.A, T.ncol, T.low, tab + m->tab_off[g], m->rad[g], m->nrad[g], inv);
#pragma unroll
    for (int k = 0; k < kMrRegs; ++k) {
        const int e = t + k * kMrThreads;
        v[k] = e < ne ? lds[mr_slot<PAD>(T.lidx(T.col_of(e), gp[T.j_of(e)]))] : make_double2(0.0, 0.0);
    }
}

// The twiddle between groups: element (col, m_g) of a strided group's tile
// times W_{S_{g+1}}^(jl m_g) (conjugated: inverse), jl = first + col, as the
// product of the tile's root troot[m_g] = W_{S_{g+1}}^(first m_g) (mr_troot)
// and the group's table entry W_{S_{g+1}}^(col m_g) (col m_g < 4096), each
// rounded once.
__device__ __forceinline__ void mr_twiddle(double2 (&v)[kMrRegs], const MrTile& T, const MrGeom* __restrict__ m, int g,
                                           const double2* __restrict__ tab, const double2* troot, bool inv)
{
    if (T.low)
        return;  // S_0 = 1: no lower index
    const int t = mr_tid(), ne = T.ncol * T.A, cols = m->cols[g];
    const double2* __restrict__ tw = tab + m->tab_len + m->tw_off[g];
#pragma unroll
    for (int k = 0; k < kMrRegs; ++k) {
        const int e = t + k * kMrThreads;
        if (e < ne) {
            const int j = divq(e, T.rncol), col = e - j * T.ncol;
            const double2 w = cmul(tw[j * cols + col], troot[j]);
            v[k] = cmul(v[k], conj_if(w, inv));
        }
    }
}

// troot[m] = W_{S_{g+1}}^(first m) for m < A_g (first m < S_{g+1} < 2^31,
// so 2 first m / S_{g+1} is rounded once).  Followed by a barrier.
__device__ __forceinline__ void mr_troot(double2* troot, const MrGeom* __restrict__ m, const MrTile& T, int g)
{
    if (!T.low) {
        const double Sn = (double)m->S[g + 1];
        for (int j = threadIdx.x; j < T.A; j += blockDim.x) {
            double s, c;
            sincospi_red((double)(2 * T.first * j) / Sn, &s, &c);
            troot[j] = make_double2(c, -s);
        }
    }
    __syncthreads();
}

template <int MAXR, bool PAD>
__device__ __forceinline__ void mr_forward(double2 (&v)[kMrRegs], double2* lds, const MrTile& T, const MrGeom* m,
                                           int g, const double2* tab, const int* perm, const double2* troot)
{
    mr_dft<MAXR, PAD>(v, lds, T, m, g, tab, perm, false);
    mr_twiddle(v, T, m, g, tab, troot, false);
}

template <int MAXR, bool PAD>
__device__ __forceinline__ void mr_inverse(double2 (&v)[kMrRegs], double2* lds, const MrTile& T, const MrGeom* m,
                                           int g, const double2* tab, const int* perm, const double2* troot)
{
    mr_twiddle(v, T, m, g, tab, troot, true);
    mr_dft<MAXR, PAD>(v, lds, T, m, g, tab, perm, true);
}

__device__ __forceinline__ void mr_load(double2 (&v)[kMrRegs], const double2* psi, const MrTile& T)
{
    const int t = mr_tid(), ne = T.ncol * T.A;
#pragma unroll
    for (int k = 0; k < kMrRegs; ++k) {
        const int e = t + k * kMrThreads;
        v[k] = e < ne ? ld_nt(psi + T.gidx(e)) : make_double2(0.0, 0.0);
    }
}

__device__ __forceinline__ void mr_store(const double2 (&v)[kMrRegs], double2* psi, const MrTile& T, double scale)
{
    const int t = mr_tid(), ne = T.ncol * T.A;
#pragma unroll
    for (int k = 0; k < kMrRegs; ++k) {
        const int e = t + k * kMrThreads;
        if (e < ne)
            st_nt(psi + T.gidx(e), make_double2(v[k].x * scale, v[k].y * scale));
    }
}

// The global frequency m held by element (col, f) of a low-group tile after
// its forward DFT: m = rev(u) + (N / A_0) f, u = first + col the upper index
// and rev(u) = p_{G-1} + A_{G-1} (p_{G-2} + ... + A_2 p_1) for
// u = p_1 + A_1 (p_2 + ...)  (u < N / A_0 < 2^31).
__device__ __forceinline__ int64_t mr_rev(const MrGeom* __restrict__ m, int64_t u64)
{
    int u = (int)u64;
    int64_t rev = 0;
    const int G = m->G;
    for (int g = 1; g < G; ++g) {
        const int A = m->A[g];
        const int q = divq(u, m->rA[g]);
        rev = rev * A + (u - q * A);
        u = q;
    }
    return rev;
}

// Columns of a low-group tile whose ring rotation exp(2 pi i rev(u) / N) is
// kept in LDS (tiles with more columns compute lambda per element).
constexpr int kMrColRot = 256;

// colrot[c] = (cos, sin)(2 pi rev(first + c) / N) for the ring, so that
// lambda at (col, f) is 2 cos(2 pi rev / N + 2 pi f / A_0), one product with
// the group's root W_{A_0}^f.  Read after the next __syncthreads.
__device__ __forceinline__ void mr_colrot(double2* colrot, const MrPassParams& P, const MrTile& T)
{
    if (P.lambda_kind != FFT_LAMBDA_RING || T.ncol > kMrColRot)
        return;
    for (int c = threadIdx.x; c < T.ncol; c += blockDim.x) {
        double s, co;
        sincospi_red((double)(2 * mr_rev(P.geom, T.first + c)) / (double)P.N, &s, &co);
        colrot[c] = make_double2(co, s);
    }
}

// lambda at element e of a low-group tile after the forward DFT.
__device__ __forceinline__ double mr_lambda_at(const MrPassParams& P, const MrTile& T, const double2* colrot, int e)
{
    const int col = T.col_of(e), f = T.j_of(e);
    if (P.lambda_kind == FFT_LAMBDA_RING) {
        if (T.ncol <= kMrColRot) {
            const double2 a = colrot[col], w = P.tab[f];  // w = (cos, -sin)(2 pi f / A_0)
            return 2.0 * fma(a.x, w.x, a.y * w.y);
        }
        double s, c;
        const int64_t mf = mr_rev(P.geom, T.first + col) + P.geom->U * (int64_t)f;
        sincospi_red((double)(2 * mf) / (double)P.N, &s, &c);  // 2 cos(2 pi m / N)
        return 2.0 * c;
    }
    return P.lam[mr_rev(P.geom, T.first + col) + P.geom->U * (int64_t)f];
}

// psi <- exp(-i tt lambda_m) psi at the frequencies of a low-group tile
// (natural order after mr_forward).
__device__ __forceinline__ void mr_diag(double2 (&v)[kMrRegs], const MrPassParams& P, const MrTile& T,
                                        const double2* colrot, double tt)
{
    const int t = mr_tid(), ne = T.ncol * T.A;
#pragma unroll
    for (int k = 0; k < kMrRegs; ++k) {
        const int e = t + k * kMrThreads;
        if (e < ne)
            v[k] = cmul(v[k], expmi(tt * mr_lambda_at(P, T, colrot, e)));
        QVA_SCHED_FENCE();
    }
}

// psi <- scale exp(-i gamma q) psi in natural order.
__device__ __forceinline__ void mr_phase(double2 (&v)[kMrRegs], const double* q, const MrTile& T, double gamma, double scale)
{
    const int t = mr_tid(), ne = T.ncol * T.A;
#pragma unroll
    for (int k = 0; k < kMrRegs; ++k) {
        const int e = t + k * kMrThreads;
        if (e < ne) {
            const double2 ph = expmi(gamma * ld_nt(q + T.gidx(e)));
            v[k] = cmul(v[k], make_double2(scale * ph.x, scale * ph.y));
        }
        QVA_SCHED_FENCE();
    }
}

__device__ __forceinline__ void mr_expect(const double2 (&v)[kMrRegs], const double* q, const MrTile& T, double* red,
                          double2* out)
{
    const int t = mr_tid(), ne = T.ncol * T.A;
    double f = 0.0, nr = 0.0;
#pragma unroll
    for (int k = 0; k < kMrRegs; ++k) {
        const int e = t + k * kMrThreads;
        if (e < ne) {
            const double a = v[k].x * v[k].x + v[k].y * v[k].y;
            f = fma(a, ld_nt(q + T.gidx(e)), f);
            nr += a;
        }
    }
    const double2 tot = block_sum2(f, nr, red);
    if (t == 0)
        *out = tot;
}

template <int MODE, int MAXR, bool PAD>
__global__ __launch_bounds__(kMrThreads, 2) void mrpass_kernel(MrPassParams P)
{
    __shared__ double2 lds[PAD ? kMrLdsElems : kMrTileElems];
    __shared__ double red[2 * (kMrThreads / 64)];
    const MrGeom* __restrict__ m = P.geom;
    const int g = P.g;
    // the low group (the diagonal's pass) has no inter-group twiddle: its
    // LDS stays within two workgroups per CU
    __shared__ double2 troot[MODE == MR_LOWDIAG ? 1 : kMrMaxStrided];
    const MrTile T = mr_tile(m, g, blockIdx.x);
    const int* perm = reinterpret_cast<const int*>(P.tab + m->tab_len + m->tw_len);
    const double invN = 1.0 / (double)P.N;
    mr_troot(troot, m, T, g);
    double2 v[kMrRegs];
    if constexpr (MODE == MR_FIRST) {
        const double a0 = 1.0 / sqrt((double)P.N);
#pragma unroll
        for (int k = 0; k < kMrRegs; ++k)
            v[k] = make_double2(a0, 0.0);
        mr_phase(v, P.q, T, angle_value(P.gamma), 1.0);
        mr_forward<MAXR, PAD>(v, lds, T, m, g, P.tab, perm, troot);
        mr_store(v, P.psi, T, 1.0);
    } else if constexpr (MODE == MR_DIF) {
        mr_load(v, P.psi, T);
        mr_forward<MAXR, PAD>(v, lds, T, m, g, P.tab, perm, troot);
        mr_store(v, P.psi, T, 1.0);
    } else if constexpr (MODE == MR_DIT) {
        mr_load(v, P.psi, T);
        mr_inverse<MAXR, PAD>(v, lds, T, m, g, P.tab, perm, troot);
        mr_store(v, P.psi, T, P.scale_inv_n ? invN : 1.0);
    } else if constexpr (MODE == MR_LOWDIAG) {
        __shared__ double2 colrot[kMrColRot];
        mr_colrot(colrot, P, T);
        mr_load(v, P.psi, T);
        mr_forward<MAXR, PAD>(v, lds, T, m, g, P.tab, perm, troot);  // its first barrier publishes colrot
        mr_diag(v, P, T, colrot, angle_value(P.t));
        mr_inverse<MAXR, PAD>(v, lds, T, m, g, P.tab, perm, troot);
        mr_store(v, P.psi, T, 1.0);
    } else if constexpr (MODE == MR_BOUNDARY) {
        const double gam = angle_value(P.gamma);
        mr_load(v, P.psi, T);
        mr_inverse<MAXR, PAD>(v, lds, T, m, g, P.tab, perm, troot);
        mr_phase(v, P.q, T, gam, invN);
        mr_forward<MAXR, PAD>(v, lds, T, m, g, P.tab, perm, troot);
        mr_store(v, P.psi, T, 1.0);
    } else {  // MR_LAST, MR_LAST_STORE
        mr_load(v, P.psi, T);
        mr_inverse<MAXR, PAD>(v, lds, T, m, g, P.tab, perm, troot);
#pragma unroll
        for (int k = 0; k < kMrRegs; ++k)
            v[k] = make_double2(v[k].x * invN, v[k].y * invN);
        mr_expect(v, P.q, T, red, P.partials + blockIdx.x);
        if constexpr (MODE == MR_LAST_STORE)
            mr_store(v, P.psi, T, 1.0);
    }
}

// Sum over the tile of h_j Im(conj(x_j) p_j) (h = q or lambda).
__device__ __forceinline__ double im_term(double2 x, double2 p) { return x.x * p.y - x.y * p.x; }

// Two-vector passes of the adjoint walk (phi = psi, chi), one half of a
// 512-thread workgroup per vector: threads 0-255 hold phi (psi), 256-511 chi,
// and each half runs the group transforms on its own LDS tile at the same
// time (the stages' barriers are common to both).  The inner products and
// the factors both vectors take (the inverse diagonal, the inverse phase)
// pass from the phi half to the chi half through LDS.  The two tiles
// (128 KiB) and 512 threads give two waves per SIMD.  Passes with per-tile
// slots run on max_tiles workgroups: those beyond the group's tiles write a
// zero.
template <int MODE, int MAXR, bool PAD>
__global__ __launch_bounds__(2 * kMrThreads, 1) void mrgrad2_kernel(MrPassParams P)
{
    __shared__ double2 lds[2][PAD ? kMrLdsElems : kMrTileElems];
    __shared__ double red[2 * (2 * kMrThreads / 64)];
    __shared__ double2 troot[kMrMaxStrided];
    const MrGeom* __restrict__ m = P.geom;
    const int g = P.g;
    if (blockIdx.x >= m->tiles[g]) {
        if (P.slot && threadIdx.x == 0)
            P.slot[blockIdx.x] = 0.0;
        return;
    }
    const int half = threadIdx.x >= kMrThreads ? 1 : 0, t = mr_tid();
    const MrTile T = mr_tile(m, g, blockIdx.x);
    const int* perm = reinterpret_cast<const int*>(P.tab + m->tab_len + m->tw_len);
    const double invN = 1.0 / (double)P.N;
    const int ne = T.ncol * T.A;
    double2* own = lds[half];
    double2* vec = half ? P.chi : P.psi;
    mr_troot(troot, m, T, g);
    double2 v[kMrRegs];
    if constexpr (MODE == MRG_TURN) {
        // phi: inverse top group, 1/N, (<Q>, norm); chi = Q phi (phi handed to
        // the chi half, which transforms zeros meanwhile); forward top group
        if (half == 0) {
            mr_load(v, P.psi, T);
        } else {
#pragma unroll
            for (int k = 0; k < kMrRegs; ++k)
                v[k] = make_double2(0.0, 0.0);
        }
        mr_inverse<MAXR, PAD>(v, own, T, m, g, P.tab, perm, troot);
        __syncthreads();
        if (half == 0) {
#pragma unroll
            for (int k = 0; k < kMrRegs; ++k) {
                const int e = t + k * kMrThreads;
                v[k] = make_double2(v[k].x * invN, v[k].y * invN);
                if (e < ne)
                    lds[1][e] = v[k];
            }
        }
        __syncthreads();
        double f = 0.0, nr = 0.0;
#pragma unroll
        for (int k = 0; k < kMrRegs; ++k) {
            const int e = t + k * kMrThreads;
            const double qq = e < ne ? ld_nt(P.q + T.gidx(e)) : 0.0;
            if (half == 0) {
                const double a = v[k].x * v[k].x + v[k].y * v[k].y;
                f = fma(a, qq, f);
                nr += a;
            } else {
                const double2 pv = e < ne ? lds[1][e] : make_double2(0.0, 0.0);
                v[k] = make_double2(qq * pv.x, qq * pv.y);
            }
        }
        const double2 tot = block_sum2(f, nr, red);
        if (threadIdx.x == 0)
            P.partials[blockIdx.x] = tot;
        mr_forward<MAXR, PAD>(v, own, T, m, g, P.tab, perm, troot);
        mr_store(v, vec, T, 1.0);
    } else if constexpr (MODE == MRG_LOWDIAG) {
        __shared__ double2 colrot[kMrColRot];
        mr_colrot(colrot, P, T);
        const double tt = angle_value(P.t);
        mr_load(v, vec, T);
        mr_forward<MAXR, PAD>(v, own, T, m, g, P.tab, perm, troot);
        __syncthreads();
        if (half == 1) {
#pragma unroll
            for (int k = 0; k < kMrRegs; ++k) {
                const int e = t + k * kMrThreads;
                if (e < ne)
                    lds[1][e] = v[k];
            }
        }
        __syncthreads();
        double acc = 0.0;
        if (half == 0) {
#pragma unroll
            for (int k = 0; k < kMrRegs; ++k) {
                const int e = t + k * kMrThreads;
                if (e < ne) {
                    const double lam = mr_lambda_at(P, T, colrot, e);
                    acc = fma(lam, im_term(lds[1][e], v[k]), acc);
                    const double2 d = expmi(-tt * lam);  // exp(+i t lambda): the inverse diagonal
                    v[k] = cmul(v[k], d);
                    lds[0][e] = d;
                }
                QVA_SCHED_FENCE();
            }
        }
        __syncthreads();
        if (half == 1) {
#pragma unroll
            for (int k = 0; k < kMrRegs; ++k) {
                const int e = t + k * kMrThreads;
                if (e < ne)
                    v[k] = cmul(v[k], lds[0][e]);
            }
        }
        const double2 tot = block_sum2(acc * invN, 0.0, red);  // its barriers end the reads of lds[0]
        if (threadIdx.x == 0)
            P.slot[blockIdx.x] = tot.x;
        mr_inverse<MAXR, PAD>(v, own, T, m, g, P.tab, perm, troot);
        mr_store(v, vec, T, 1.0);
    } else {  // MRG_BOUND, MRG_FINAL
        mr_load(v, vec, T);
        mr_inverse<MAXR, PAD>(v, own, T, m, g, P.tab, perm, troot);
#pragma unroll
        for (int k = 0; k < kMrRegs; ++k)
            v[k] = make_double2(v[k].x * invN, v[k].y * invN);
        __syncthreads();
        if (half == 1) {
#pragma unroll
            for (int k = 0; k < kMrRegs; ++k) {
                const int e = t + k * kMrThreads;
                if (e < ne)
                    lds[1][e] = v[k];
            }
        }
        __syncthreads();
        const double gam = angle_value(P.gamma);
        double acc = 0.0;
        if (half == 0) {
#pragma unroll
            for (int k = 0; k < kMrRegs; ++k) {
                const int e = t + k * kMrThreads;
                if (e < ne) {
                    const double qq = ld_nt(P.q + T.gidx(e));
                    acc = fma(qq, im_term(lds[1][e], v[k]), acc);
                    if constexpr (MODE == MRG_BOUND) {
                        const double2 u = expmi(-gam * qq);  // exp(+i gamma q): the inverse phase
                        v[k] = cmul(v[k], u);
                        lds[0][e] = u;
                    }
                }
                QVA_SCHED_FENCE();
            }
        }
        if constexpr (MODE == MRG_BOUND) {
            __syncthreads();
            if (half == 1) {
#pragma unroll
                for (int k = 0; k < kMrRegs; ++k) {
                    const int e = t + k * kMrThreads;
                    if (e < ne)
                        v[k] = cmul(v[k], lds[0][e]);
                }
            }
        }
        const double2 tot = block_sum2(acc, 0.0, red);
        if (threadIdx.x == 0)
            P.slot[blockIdx.x] = tot.x;
        if constexpr (MODE == MRG_BOUND) {
            mr_forward<MAXR, PAD>(v, own, T, m, g, P.tab, perm, troot);
            mr_store(v, vec, T, 1.0);
        }
    }
}

// N <= 4096 (one group): the whole evolution, and with MRG_SMALL the adjoint
// walk, in one workgroup.
template <int MODE, int MAXR, bool PAD>
__global__ __launch_bounds__(kMrThreads, 1) void mrsmall_kernel(MrPassParams P)
{
    __shared__ double2 lds[PAD ? kMrLdsElems : kMrTileElems];
    __shared__ double red[2 * (kMrThreads / 64)];
    const MrGeom* __restrict__ m = P.geom;
    __shared__ double2 colrot[kMrColRot];
    const MrTile T = mr_tile(m, 0, 0);
    const int* perm = reinterpret_cast<const int*>(P.tab + m->tab_len + m->tw_len);
    const int t = mr_tid(), ne = T.ncol * T.A;
    const double invN = 1.0 / (double)P.N;
    mr_colrot(colrot, P, T);  // published by the first transform's barrier
    double2 p[kMrRegs];
    if constexpr (MODE == MR_SMALL_MIX) {
        // the mixer alone: F^-1 diag(exp(-i t lambda)) F on the caller's state
        mr_load(p, P.psi, T);
        mr_dft<MAXR, PAD>(p, lds, T, m, 0, P.tab, perm, false);
        mr_diag(p, P, T, colrot, angle_value(P.t));
        mr_dft<MAXR, PAD>(p, lds, T, m, 0, P.tab, perm, true);
        mr_store(p, P.psi, T, invN);
        return;
    }
    const double a0 = 1.0 / sqrt((double)P.N);
#pragma unroll
    for (int k = 0; k < kMrRegs; ++k)
        p[k] = make_double2(t + k * kMrThreads < ne ? a0 : 0.0, 0.0);
    for (int L = 0; L < P.p; ++L) {
        mr_phase(p, P.q, T, P.gammas[L], 1.0);
        mr_dft<MAXR, PAD>(p, lds, T, m, 0, P.tab, perm, false);
        mr_diag(p, P, T, colrot, P.ts[L]);
        mr_dft<MAXR, PAD>(p, lds, T, m, 0, P.tab, perm, true);
#pragma unroll
        for (int k = 0; k < kMrRegs; ++k)
            p[k] = make_double2(p[k].x * invN, p[k].y * invN);
    }
    double2 fv;
    {
        double f = 0.0, nr = 0.0;
#pragma unroll
        for (int k = 0; k < kMrRegs; ++k) {
            const int e = t + k * kMrThreads;
            if (e < ne) {
                const double a = p[k].x * p[k].x + p[k].y * p[k].y;
                f = fma(a, P.q[e], f);
                nr += a;
            }
        }
        fv = block_sum2(f, nr, red);
    }
    if (t == 0) {
        P.out_f[0] = fv.x;
        if (P.out_norm)
            P.out_norm[0] = fv.y;
    }
    if constexpr (MODE == MR_SMALL_STORE)
        mr_store(p, P.psi, T, 1.0);
    if constexpr (MODE == MRG_SMALL) {
        double2 x[kMrRegs];
#pragma unroll
        for (int k = 0; k < kMrRegs; ++k) {
            const int e = t + k * kMrThreads;
            const double qq = e < ne ? P.q[e] : 0.0;
            x[k] = make_double2(qq * p[k].x, qq * p[k].y);
        }
        for (int L = P.p - 1; L >= 0; --L) {
            // the mixer of layer L: Im <chi|W|phi> at the spectrum, then undone
            mr_dft<MAXR, PAD>(p, lds, T, m, 0, P.tab, perm, false);
            mr_dft<MAXR, PAD>(x, lds, T, m, 0, P.tab, perm, false);
            double acc = 0.0;
            const double tt = P.ts[L];
#pragma unroll
            for (int k = 0; k < kMrRegs; ++k) {
                const int e = t + k * kMrThreads;
                if (e < ne) {
                    const double lam = mr_lambda_at(P, T, colrot, e);
                    acc = fma(lam, im_term(x[k], p[k]), acc);
                    const double2 d = expmi(-tt * lam);
                    p[k] = cmul(p[k], d);
                    x[k] = cmul(x[k], d);
                }
            }
            const double2 st = block_sum2(acc * invN, 0.0, red);
            if (t == 0)
                P.dts[L] = 2.0 * st.x;
            mr_dft<MAXR, PAD>(p, lds, T, m, 0, P.tab, perm, true);
            mr_dft<MAXR, PAD>(x, lds, T, m, 0, P.tab, perm, true);
            // the phase of layer L
            const double gam = P.gammas[L];
            acc = 0.0;
#pragma unroll
            for (int k = 0; k < kMrRegs; ++k) {
                const int e = t + k * kMrThreads;
                p[k] = make_double2(p[k].x * invN, p[k].y * invN);
                x[k] = make_double2(x[k].x * invN, x[k].y * invN);
                if (e < ne) {
                    const double qq = P.q[e];
                    acc = fma(qq, im_term(x[k], p[k]), acc);
                    const double2 u = expmi(-gam * qq);
                    p[k] = cmul(p[k], u);
                    x[k] = cmul(x[k], u);
                }
            }
            const double2 sg = block_sum2(acc, 0.0, red);
            if (t == 0)
                P.dgammas[L] = 2.0 * sg.x;
        }
    }
}

// The geometry's device copy (the passes read it from there: indexing a
// by-value kernel argument with runtime indices would copy it to scratch).
__global__ __launch_bounds__(64) void mr_geom_kernel(MrGeom m, MrGeom* out)
{
    if (threadIdx.x == 0)
        *out = m;
}

// Group g's roots W_{A_g}^k and the digit-reversal permutation of its DIF
// stages: frequency f = d_0 + r_0 (d_1 + r_1 (...)) sits at position
// sum_s d_s L_s / r_s (L_s the sub-length of stage s).  Reads the device
// copy of the geometry.
__global__ __launch_bounds__(256) void mr_table_kernel(const MrGeom* __restrict__ m, double2* tab)
{
    const int g = blockIdx.x;
    const int A = m->A[g];
    int* perm = reinterpret_cast<int*>(tab + m->tab_len + m->tw_len) + m->tab_off[g];
    for (int k = threadIdx.x; k < A; k += blockDim.x) {
        // exp(-2 pi i k / A), with 2k / A rounded once (exact for A a power of two)
        double s, c;
        sincospi_red((double)(2 * k) / (double)A, &s, &c);
        tab[m->tab_off[g] + k] = make_double2(c, -s);
        int f = k, L = A, pos = 0;
        for (int st = 0; st < m->nrad[g]; ++st) {
            const int r = m->rad[g][st];
            const int d = f % r;
            f /= r;
            L /= r;
            pos += d * L;
        }
        perm[k] = pos;
    }
    if (g == 0)
        return;
    // W_{S_{g+1}}^(c j) at m j cols + c (c j < cols A_g <= 4096, rounded once)
    const int cols = m->cols[g];
    const double Sn = (double)m->S[g + 1];
    double2* tw = tab + m->tab_len + m->tw_off[g];
    for (int k = threadIdx.x; k < cols * A; k += blockDim.x) {
        const int j = k / cols, c = k - j * cols;
        double s, co;
        sincospi_red((double)(2 * c * j) / Sn, &s, &co);
        tw[k] = make_double2(co, -s);
    }
}

}  // namespace

size_t mr_table_bytes(const MrGeom& m)
{
    return (size_t)(m.tab_len + m.tw_len) * sizeof(double2) + (size_t)m.tab_len * sizeof(int);
}

hipError_t launch_mr_tables(const MrGeom& m, MrGeom* geom_dev, double2* tab, hipStream_t s)
{
    hipLaunchKernelGGL(mr_geom_kernel, dim3(1), dim3(64), 0, s, m, geom_dev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(mr_table_kernel, dim3(m.G), dim3(256), 0, s, geom_dev, tab);
    return hipGetLastError();
}

template <int MAXR>
hipError_t launch_mr_modes(const MrPassParams& P, int mode, dim3 grid, hipStream_t s)
{
    switch (mode) {
#define QVA_MR_MODE(K, M) \
    case M:               \
        hipLaunchKernelGGL((K<M, MAXR, false>), grid, dim3(kMrThreads), 0, s, P); \
        break;
        QVA_MR_MODE(mrpass_kernel, MR_FIRST)
        QVA_MR_MODE(mrpass_kernel, MR_DIF)
        QVA_MR_MODE(mrpass_kernel, MR_DIT)
        QVA_MR_MODE(mrpass_kernel, MR_LOWDIAG)
        QVA_MR_MODE(mrpass_kernel, MR_BOUNDARY)
        QVA_MR_MODE(mrpass_kernel, MR_LAST)
        QVA_MR_MODE(mrpass_kernel, MR_LAST_STORE)
        QVA_MR_MODE(mrsmall_kernel, MR_SMALL)
        QVA_MR_MODE(mrsmall_kernel, MR_SMALL_STORE)
        QVA_MR_MODE(mrsmall_kernel, MR_SMALL_MIX)
        QVA_MR_MODE(mrsmall_kernel, MRG_SMALL)
#undef QVA_MR_MODE
#define QVA_MR_MODE2(M)                                                                      \
    case M:                                                                                  \
        hipLaunchKernelGGL((mrgrad2_kernel<M, MAXR, false>), grid, dim3(2 * kMrThreads), 0, s, P); \
        break;
        QVA_MR_MODE2(MRG_TURN)
        QVA_MR_MODE2(MRG_LOWDIAG)
        QVA_MR_MODE2(MRG_BOUND)
        QVA_MR_MODE2(MRG_FINAL)
#undef QVA_MR_MODE2
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// The low group's passes with padded LDS slots (MrGeom::lds_pad).
template <int MAXR>
hipError_t launch_mr_low_padded(const MrPassParams& P, int mode, dim3 grid, hipStream_t s)
{
    if (mode == MR_LOWDIAG) {
        hipLaunchKernelGGL((mrpass_kernel<MR_LOWDIAG, MAXR, true>), grid, dim3(kMrThreads), 0, s, P);
    } else if (mode == MRG_LOWDIAG) {
        hipLaunchKernelGGL((mrgrad2_kernel<MRG_LOWDIAG, MAXR, true>), grid, dim3(2 * kMrThreads), 0, s, P);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_mrpass(const MrPassParams& P0, const MrGeom& m, int mode, hipStream_t s)
{
    int64_t maxt = 0;
    for (int g = 0; g < m.G; ++g)
        maxt = m.tiles[g] > maxt ? m.tiles[g] : maxt;
    MrPassParams P = P0;
    const bool wide = mode == MRG_LOWDIAG || mode == MRG_BOUND || mode == MRG_FINAL;
    const bool small = mode == MR_SMALL || mode == MR_SMALL_STORE || mode == MR_SMALL_MIX || mode == MRG_SMALL;
    P.grid = small ? 1 : (wide ? maxt : m.tiles[P.g]);
    int maxr = 0;
    for (int g = 0; g < m.G; ++g)
        for (int i = 0; i < m.nrad[g]; ++i)
            maxr = m.rad[g][i] > maxr ? m.rad[g][i] : maxr;
    const dim3 grid((unsigned)P.grid);
    if (m.lds_pad && (mode == MR_LOWDIAG || mode == MRG_LOWDIAG)) {
        if (maxr > 23)
            return launch_mr_low_padded<31>(P, mode, grid, s);
        if (maxr > 16)
            return launch_mr_low_padded<23>(P, mode, grid, s);
        return launch_mr_low_padded<16>(P, mode, grid, s);
    }
    if (maxr > 23)
        return launch_mr_modes<31>(P, mode, grid, s);
    if (maxr > 16)
        return launch_mr_modes<23>(P, mode, grid, s);
    return launch_mr_modes<16>(P, mode, grid, s);
}

}  // namespace qva
