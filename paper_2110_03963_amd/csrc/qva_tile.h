// qva_tile.h -- register/LDS machinery of the 4096-amplitude tile passes.
//
// A pass loads a tile of 2^12 amplitudes whose index bits cover one group of
// qubits (see qva_plan.h), keeps 16 amplitudes in each of 256 threads, and
// moves between register layouts through LDS so that every bit of the group
// is, in turn, a register bit.  Element index e (12 bits) of a tile maps to
// the global index base + (e mod 2^C) + (e >> C) 2^k: C contiguous column bits
// (coalescing) and the group's bits [k, k + 12 - C).
#pragma once

#include "qva_internal.h"

namespace qva {
namespace tile {

// Register layouts of a 4096-amplitude tile (256 threads x 16 registers).
// A: registers = element bits [8,12); B: [4,8); C: [0,4);
// A3: registers = element bits {3, 9, 10, 11} (for tiles with 3 column bits).
enum { LA = 0, LB = 1, LC = 2, LA3 = 3 };

template <int L>
__device__ __forceinline__ int elem(int t, int r)
{
    if constexpr (L == LA)
        return t | (r << 8);
    else if constexpr (L == LB)
        return (t & 15) | (r << 4) | ((t >> 4) << 8);
    else if constexpr (L == LC)
        return r | (t << 4);
    else
        return (t & 7) | ((r & 1) << 3) | ((t >> 3) << 4) | ((r >> 1) << 9);
}

// Element bit held by register bit j of layout L.
template <int L>
constexpr int reg_elem_bit(int j)
{
    if (L == LA)
        return 8 + j;
    if (L == LB)
        return 4 + j;
    if (L == LC)
        return j;
    return j == 0 ? 3 : 8 + j;
}

// Digit of layout L for a tile whose first C element bits are columns: the
// register bits holding target (transform) bits, [dlo, dlo + dw).
template <int C, int L>
constexpr int digit_lo()
{
    int j = 0;
    while (j < 4 && reg_elem_bit<L>(j) < C)
        ++j;
    return j;
}

template <int C, int L>
constexpr int digit_w()
{
    if (L == LA3)
        return C == 3 ? 1 : 0;
    return 4 - digit_lo<C, L>();
}

__device__ __forceinline__ int swz(int e) { return e ^ (((e >> 3) ^ (e >> 6) ^ (e >> 9)) & 7); }

template <int FROM, int TO>
__device__ __forceinline__ void exchange(double2 (&v)[kRegs], double2* lds, int t)
{
    if constexpr (FROM != TO) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kRegs; ++r)
            lds[swz(elem<FROM>(t, r))] = v[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kRegs; ++r)
            v[r] = lds[swz(elem<TO>(t, r))];
    }
}

// exp(-2 pi i k / 16), k = 0..7
__device__ __forceinline__ double2 w16(int k)
{
    constexpr double c1 = 0.92387953251128675613;  // cos(pi/8)
    constexpr double s1 = 0.38268343236508977173;  // sin(pi/8)
    constexpr double h = 0.70710678118654752440;   // sqrt(1/2)
    switch (k & 7) {
    case 0:
        return make_double2(1.0, 0.0);
    case 1:
        return make_double2(c1, -s1);
    case 2:
        return make_double2(h, -h);
    case 3:
        return make_double2(s1, -c1);
    case 4:
        return make_double2(0.0, -1.0);
    case 5:
        return make_double2(-s1, -c1);
    case 6:
        return make_double2(-h, -h);
    default:
        return make_double2(-c1, -s1);
    }
}

__device__ __forceinline__ double2 cmul_conj(double2 a, double2 w)  // a * conj(w)
{
    return make_double2(a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y);
}

// 2^W-point DFT (DIF radix-2 stages) over register bits [LO, LO+W); output
// bit-reversed within the digit.
template <int LO, int W>
__device__ __forceinline__ void local_dif(double2 (&v)[kRegs])
{
#pragma unroll
    for (int bb = W - 1; bb >= 0; --bb) {
        const int b = LO + bb;
#pragma unroll
        for (int r = 0; r < kRegs; ++r) {
            if (r & (1 << b))
                continue;
            const int l = (r >> LO) & ((1 << bb) - 1);
            const int k = l << (3 - bb);  // W_{2^(bb+1)}^l = W_16^(l 2^(3-bb))
            const double2 a = v[r], c = v[r | (1 << b)];
            v[r] = make_double2(a.x + c.x, a.y + c.y);
            const double2 d = make_double2(a.x - c.x, a.y - c.y);
            v[r | (1 << b)] = k == 0 ? d : (k == 4 ? make_double2(d.y, -d.x) : cmul(d, w16(k)));
        }
    }
}

// Inverse of local_dif up to the factor 2^W (conjugate twiddles, ascending).
template <int LO, int W>
__device__ __forceinline__ void local_dit(double2 (&v)[kRegs])
{
#pragma unroll
    for (int bb = 0; bb < W; ++bb) {
        const int b = LO + bb;
#pragma unroll
        for (int r = 0; r < kRegs; ++r) {
            if (r & (1 << b))
                continue;
            const int l = (r >> LO) & ((1 << bb) - 1);
            const int k = l << (3 - bb);
            const double2 a = v[r];
            double2 c = v[r | (1 << b)];
            c = k == 0 ? c : (k == 4 ? make_double2(-c.y, c.x) : cmul_conj(c, w16(k)));
            v[r] = make_double2(a.x + c.x, a.y + c.y);
            v[r | (1 << b)] = make_double2(a.x - c.x, a.y - c.y);
        }
    }
}

struct TileMap {
    int64_t base;
    int k;
    int C;
    __device__ __forceinline__ int64_t operator()(int e) const
    {
        return base + (e & ((1 << C) - 1)) + ((int64_t)(e >> C) << k);
    }
};

__device__ __forceinline__ int rev_bits(int x, int w) { return (int)(__brev((unsigned)x) >> (32 - w)); }

// w-bit reversal of a compile-time register digit.
constexpr int rev_c(int x, int w)
{
    int y = 0;
    for (int i = 0; i < w; ++i)
        y |= ((x >> i) & 1) << (w - 1 - i);
    return y;
}

// Twiddles of one digit: W_{2^(gb+w)}^(j_lo * m) for the register holding
// digit value m (bit-reversed digit bits) and index bits j_lo below the
// digit (global bit gb).  j_lo does not depend on the digit bits, only on the
// thread and on the column register bits below the digit, so for each such
// column value b the twiddles are the powers w^m of one root
// w = exp(-i pi j_lo / 2^(gb+w-1)).  The w roots w^(2^i) are computed exactly
// (sincospi_red of a dyadic rational) and w^m is their product over the set
// bits of m: at most w - 1 complex products, about 1 ulp each.
// apply(r, tw) is called for every register r with m != 0 (forward sign).
//
// TAB (contiguous low-group tiles only, k = 0): every root is a power of
// W_4096 and does not depend on the tile, so it is read from `tab`, the
// table tab[k] = W_4096^k = exp(-2 pi i k / 4096) that twiddle_table_kernel
// writes once per call with the same sincospi_red arguments: the roots, and
// so the twiddles, are bit-identical to the computed ones.
template <int C, int L, bool TAB = false, typename F>
__device__ __forceinline__ void digit_twiddles(const TileMap& g, int t, F&& apply,
                                               const double2* __restrict__ tab = nullptr)
{
    constexpr int LO = digit_lo<C, L>(), W = digit_w<C, L>();
    static_assert(!TAB || C == 0, "table twiddles are for contiguous low-group tiles");
    if constexpr (W > 0) {
        const int gb = g.k + (reg_elem_bit<L>(LO) - C);  // global bit of the digit's lowest bit
        if (gb == 0)
            return;  // no index bits below the digit: all twiddles are 1
        const int64_t lomask = (int64_t(1) << gb) - 1;
        constexpr int NB = 1 << LO;  // values of the column register bits below the digit
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int64_t jlo = g(elem<L>(t, b)) & lomask;
            double2 pw[W];  // w^(2^i)
#pragma unroll
            for (int i = 0; i < W; ++i) {
                if constexpr (TAB) {
                    // w^(2^i) = W_4096^(j_lo 2^(i + 12 - gb - W)), gb + W <= 12
                    pw[i] = tab[((int)jlo << (i + kTileBits - gb - W)) & ((1 << kTileBits) - 1)];
                } else {
                    double s, c;
                    sincospi_red(ldexp((double)jlo, i - (gb + W - 1)), &s, &c);
                    pw[i] = make_double2(c, -s);
                }
            }
#pragma unroll
            for (int m = 1; m < (1 << W); ++m) {
                double2 tw = make_double2(1.0, 0.0);
                bool first = true;
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    if ((m >> i) & 1) {
                        tw = first ? pw[i] : cmul(tw, pw[i]);
                        first = false;
                    }
                }
#pragma unroll
                for (int r = 0; r < kRegs; ++r) {
                    if ((r & (NB - 1)) == b && rev_c((r >> LO) & ((1 << W) - 1), W) == m)
                        apply(r, tw);
                }
                QVA_SCHED_FENCE();
            }
        }
    }
}

// Twiddles after (forward) or before (inverse, conjugated) the digit's
// register DFT.
template <int C, int L, bool INV, bool TAB = false>
__device__ __forceinline__ void digit_twiddle(double2 (&v)[kRegs], const TileMap& g, int t,
                                              const double2* tab = nullptr)
{
    digit_twiddles<C, L, TAB>(g, t, [&](int r, double2 tw) {
        v[r] = INV ? cmul_conj(v[r], tw) : cmul(v[r], tw);
    }, tab);
}

// W_4096^k = exp(-2 pi i k / 4096), k < 4096: the root table of the
// low-group digits (one workgroup of 256 threads, 16 entries each).
__device__ __forceinline__ void twiddle_table_fill(double2* tab, int t)
{
#pragma unroll 4
    for (int r = 0; r < kRegs; ++r) {
        const int k = r * kThreads + t;
        double s, c;
        sincospi_red(ldexp((double)k, 1 - kTileBits), &s, &c);
        tab[k] = make_double2(c, -s);
    }
}

// Ring eigenvalues lambda_m = 2 cos(2 pi m / N) at the bit-reversed
// positions of a low-group tile in layout C.  Position (tile, elem<LC>(t, r))
// holds m = rev4(r) 2^(n-4) + rev8(t) 2^(n-12) + rev_{n-12}(tile), so with
// u = exp(2 pi i (rev8(t) 2^(n-12) + rev_{n-12}(tile)) / N), computed once per
// thread, lambda = 2 Re(u exp(2 pi i rev4(r) / 16)) = 2 Re(u conj(W_16^rev4(r))).
__device__ __forceinline__ double2 ring_lambda_base(int64_t tile, int t, int n)
{
    const int hb = n - kTileBits;
    const int64_t rt = hb > 0 ? (int64_t)(__brevll((uint64_t)tile) >> (64 - hb)) : 0;
    const int64_t a = ((int64_t)rev_bits(t, 8) << hb) | rt;
    double s, c;
    sincospi_red(ldexp((double)a, 1 - n), &s, &c);
    return make_double2(c, s);
}

// exp(-i t lambda_m) for the complete graph's eigenvalues (N - 1 at m = 0,
// -1 elsewhere; N = 2^n), with t N formed exactly:
// exp(-i t (N - 1)) = exp(-i t N) e^{i t}.
__device__ __forceinline__ double2 complete_diag(bool m0, double t, int n)
{
    const double2 e1 = expmi(-t);
    return m0 ? cmul(expmi(t * ldexp(1.0, n)), e1) : e1;
}

// lambda_m = 2 cos(2 pi m / N) for a single index m (whole-state paths).
__device__ __forceinline__ double ring_lambda_m(uint64_t m, int n)
{
    double s, c;
    sincospi_red(ldexp((double)m, 1 - n), &s, &c);
    return 2.0 * c;
}

__device__ __forceinline__ double ring_lambda(double2 u, int r)
{
    const int k = rev_c(r, 4);
    const double2 w = w16(k & 7);  // W_16^k = -W_16^(k-8) for k >= 8
    const double l = 2.0 * fma(u.x, w.x, u.y * w.y);
    return (k & 8) ? -l : l;
}

template <int C, int L, bool TAB = false>
__device__ __forceinline__ void dif_digit(double2 (&v)[kRegs], const TileMap& g, int t, const double2* tab)
{
    constexpr int LO = digit_lo<C, L>(), W = digit_w<C, L>();
    if constexpr (W > 0) {
        local_dif<LO, W>(v);
        digit_twiddle<C, L, false, TAB>(v, g, t, tab);
    }
}

template <int C, int L, bool TAB = false>
__device__ __forceinline__ void dit_digit(double2 (&v)[kRegs], const TileMap& g, int t, const double2* tab)
{
    constexpr int LO = digit_lo<C, L>(), W = digit_w<C, L>();
    if constexpr (W > 0) {
        digit_twiddle<C, L, true, TAB>(v, g, t, tab);
        local_dit<LO, W>(v);
    }
}

// Layout sequences of the forward transform of one tile (digits top-down).
template <int C>
constexpr int dif_last()
{
    return C == 0 ? LC : (C == 3 ? LA3 : (C < 8 ? LB : LA));
}

// Forward (DIF) over every target bit of the tile: enters in A, leaves in
// dif_last<C>().  TAB: low-group root table (C = 0 only, see digit_twiddles).
template <int C, bool TAB = false>
__device__ __forceinline__ void dif_tile(double2 (&v)[kRegs], double2* lds, const TileMap& g, int t,
                                         const double2* tab = nullptr)
{
    dif_digit<C, LA, TAB>(v, g, t, tab);
    if constexpr (C < 8) {
        exchange<LA, LB>(v, lds, t);
        dif_digit<C, LB, TAB>(v, g, t, tab);
        if constexpr (C == 0) {
            exchange<LB, LC>(v, lds, t);
            dif_digit<C, LC, TAB>(v, g, t, tab);
        } else if constexpr (C == 3) {
            exchange<LB, LA3>(v, lds, t);
            dif_digit<C, LA3>(v, g, t, tab);
        }
    }
}

// Inverse (DIT): enters in dif_last<C>(), leaves in A.
template <int C, bool TAB = false>
__device__ __forceinline__ void dit_tile(double2 (&v)[kRegs], double2* lds, const TileMap& g, int t,
                                         const double2* tab = nullptr)
{
    if constexpr (C < 8) {
        if constexpr (C == 0) {
            dit_digit<C, LC, TAB>(v, g, t, tab);
            exchange<LC, LB>(v, lds, t);
        } else if constexpr (C == 3) {
            dit_digit<C, LA3>(v, g, t, tab);
            exchange<LA3, LB>(v, lds, t);
        }
        dit_digit<C, LB, TAB>(v, g, t, tab);
        exchange<LB, LA>(v, lds, t);
    }
    dit_digit<C, LA, TAB>(v, g, t, tab);
}

template <int L>
__device__ __forceinline__ void load_tile(double2 (&v)[kRegs], const double2* psi, const TileMap& g, int t)
{
#pragma unroll
    for (int r = 0; r < kRegs; ++r)
        v[r] = ld_nt(psi + g(elem<L>(t, r)));
}

template <int L>
__device__ __forceinline__ void store_tile(const double2 (&v)[kRegs], double2* psi, const TileMap& g,
                                           int t, double scale)
{
#pragma unroll
    for (int r = 0; r < kRegs; ++r)
        st_nt(psi + g(elem<L>(t, r)), make_double2(v[r].x * scale, v[r].y * scale));
}


// ------------------------------------------------------- hypercube mixer
template <int L>
constexpr int reg_base()
{
    return L == LA ? 8 : (L == LB ? 4 : 0);
}

// Register bits of layout L that are target qubits when the tile's first C
// element bits are plain columns.
template <int C, int L>
constexpr int target_mask()
{
    int m = 0;
    for (int j = 0; j < 4; ++j)
        if (reg_base<L>() + j >= C)
            m |= 1 << j;
    return m;
}

template <int MASK, bool TAN>
__device__ __forceinline__ void rotate_regs(double2 (&v)[kRegs], double k)
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (!((MASK >> j) & 1))
            continue;
#pragma unroll
        for (int r = 0; r < kRegs; ++r) {
            if (r & (1 << j))
                continue;
            if constexpr (TAN)
                bfly_tan(v[r], v[r | (1 << j)], k);
            else
                bfly_cot(v[r], v[r | (1 << j)], k);
        }
    }
}

// The same register of lane (lane ^ 8): DPP row_mirror (lane ^ 15 within each
// row of 16 lanes) followed by row_half_mirror (lane ^ 7 within each half
// row).  Every lane of the wave must be active.
__device__ __forceinline__ double lane_xor8(double v)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(0, lo, 0x140, 0xF, 0xF, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, 0x140, 0xF, 0xF, false);
    lo = __builtin_amdgcn_update_dpp(0, lo, 0x141, 0xF, 0xF, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, 0x141, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double2 lane_xor8(double2 v) { return make_double2(lane_xor8(v.x), lane_xor8(v.y)); }

// The rotation of element bit 3 in layouts A and B, where it is thread bit 3:
// the other member of each pair is the same register of lane ^ 8.  B is
// symmetric in the pair, so each lane forms its own half of the butterfly
// with the same operations as bfly_tan / bfly_cot.  Used for tiles with 3
// column bits, whose only target bit below 4 is bit 3: it saves the round
// trip through layout C.
template <bool TAN>
__device__ __forceinline__ void rotate_lane8(double2 (&v)[kRegs], double k)
{
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
        const double2 u = lane_xor8(v[r]);
        if constexpr (TAN)
            v[r] = make_double2(fma(k, u.y, v[r].x), fma(-k, u.x, v[r].y));
        else
            v[r] = make_double2(fma(-k, v[r].y, u.x), fma(k, v[r].x, u.y));
    }
}

// Layout in which the first mixer application ends: B when the tile has
// target bits in [4,8), else A.
template <int C>
constexpr int last_layout()
{
    return C < 8 ? LB : LA;
}

// Rotations of every target qubit of the tile; enters in A, leaves in
// last_layout<C>().  Order A, C, B (A with bit 3 across lanes, B for C = 3).
template <int C, bool TAN>
__device__ __forceinline__ void mix_forward(double2 (&v)[kRegs], double2* lds, int t, double k)
{
    rotate_regs<target_mask<C, LA>(), TAN>(v, k);
    if constexpr (C == 3) {
        rotate_lane8<TAN>(v, k);
        exchange<LA, LB>(v, lds, t);
        rotate_regs<target_mask<C, LB>(), TAN>(v, k);
    } else if constexpr (C < 4) {
        exchange<LA, LC>(v, lds, t);
        rotate_regs<target_mask<C, LC>(), TAN>(v, k);
        exchange<LC, LB>(v, lds, t);
        rotate_regs<target_mask<C, LB>(), TAN>(v, k);
    } else if constexpr (C < 8) {
        exchange<LA, LB>(v, lds, t);
        rotate_regs<target_mask<C, LB>(), TAN>(v, k);
    }
}

// Same rotations in reverse layout order; enters in last_layout<C>(), leaves in A.
template <int C, bool TAN>
__device__ __forceinline__ void mix_reverse(double2 (&v)[kRegs], double2* lds, int t, double k)
{
    if constexpr (C == 3) {
        rotate_regs<target_mask<C, LB>(), TAN>(v, k);
        exchange<LB, LA>(v, lds, t);
        rotate_lane8<TAN>(v, k);
    } else if constexpr (C < 4) {
        rotate_regs<target_mask<C, LB>(), TAN>(v, k);
        exchange<LB, LC>(v, lds, t);
        rotate_regs<target_mask<C, LC>(), TAN>(v, k);
        exchange<LC, LA>(v, lds, t);
    } else if constexpr (C < 8) {
        rotate_regs<target_mask<C, LB>(), TAN>(v, k);
        exchange<LB, LA>(v, lds, t);
    }
    rotate_regs<target_mask<C, LA>(), TAN>(v, k);
}

// Tile of workgroup b when two neighbouring tiles share cache lines of q (3
// column bits: a tile's q row is 64 bytes, half of a 128-byte line, the other
// half in the tile with the next column chunk).  Workgroups go to the eight
// XCDs round-robin, so workgroups b and b + 8 run back to back on the same
// XCD: b = 16 m + 8 h + x gets tile 16 m + 2 x + h, and both halves of each
// line are read through the same L2.  A bijection of [0, 16 M).
__device__ __forceinline__ int64_t paired_tile(int64_t b)
{
    return (b & ~int64_t(15)) | ((b & 7) << 1) | ((b >> 3) & 1);
}

__device__ __forceinline__ TileMap tile_map(int64_t tile, int k, int C)
{
    TileMap g;
    g.k = k;
    g.C = C;
    const int lobits = k - C;
    g.base = ((tile & ((int64_t(1) << lobits) - 1)) << C) | ((tile >> lobits) << (k + kTileBits - C));
    return g;
}

}  // namespace tile
}  // namespace qva
