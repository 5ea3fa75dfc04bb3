// qva_passes.h -- tile bodies of the hypercube-mixer passes, forward and
// backward, as device functions: the per-pass kernels and the batched
// (multi-instance) kernel call the same code.
#pragma once

#include <type_traits>

#include "qva_tile.h"

namespace qva {
namespace passes {

using namespace tile;

// ------------------------------------------------------------ forward
// q at the tile's elements in layout L.
template <int L>
__device__ __forceinline__ void load_q(double (&qq)[kRegs], const double* q, const TileMap& g, int t)
{
#pragma unroll
    for (int r = 0; r < kRegs; ++r)
        qq[r] = ld_nt(q + g(elem<L>(t, r)));
}

// psi <- scale * exp(-i gamma q) psi with q already in registers.
__device__ __forceinline__ void phase_vals(double2 (&v)[kRegs], const double (&qq)[kRegs], double gamma,
                                           double2 scale)
{
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
        v[r] = cmul(v[r], cmul(scale, expmi(gamma * qq[r])));
        QVA_SCHED_FENCE();
    }
}

// In-register Walsh-Hadamard transform over the 4 register bits:
// a[r] <- sum_m (-1)^popcount(m & r) a[m].
__device__ __forceinline__ void wht16(double (&a)[kRegs])
{
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int r = 0; r < kRegs; ++r)
            if (!(r & (1 << b))) {
                const double u = a[r], w = a[r | (1 << b)];
                a[r] = u + w;
                a[r | (1 << b)] = u - w;
            }
}

// psi <- scale * exp(-i gamma q) psi in layout L
template <int L>
__device__ __forceinline__ void phase_regs(double2 (&v)[kRegs], const double* q, const TileMap& g,
                                           int t, double gamma, double2 scale)
{
    double qq[kRegs];
    load_q<L>(qq, q, g, t);
    phase_vals(v, qq, gamma, scale);
}

// sum_e gam[e] c_e (-1)^popcount(j & S_e), e ascending (one basis state)
__device__ __forceinline__ double zterm_angle(int64_t j, const ZTerm* terms, int n_terms, const double* gam)
{
    double a = 0.0;
    for (int e = 0; e < n_terms; ++e) {
        const double v = gam[e] * terms[e].coef;
        a += (__popcll((uint64_t)j & terms[e].support) & 1) ? -v : v;
    }
    return a;
}

// Global index bit of register bit b of layout L in a tile with C column bits.
template <int L, int C>
__device__ __forceinline__ int reg_global_bit(const TileMap& g, int b)
{
    const int eb = reg_elem_bit<L>(b);
    return eb < C ? eb : g.k + eb - C;
}

// Extended-QAOA phase angles of the registers of layout L (eq.
// phase_shift_qaoa_ex with Z-string terms):
//   ph[r] = sum_e gam[e] c_e (-1)^popcount(j_r & S_e).
// The register bits of j_r are global bits that no other part of j_r sets, so
// (-1)^popcount(j_r & S_e) = (-1)^popcount(j_0 & S_e) (-1)^popcount(r & m_e),
// where m_e (the register bits S_e covers) is the same for every thread.  Each
// term adds its signed value to the coefficient cf[m_e], and ph is the
// 16-point Walsh-Hadamard transform of cf.  cf is a register vector indexed
// by the wave-uniform m_e (relative register addressing, no branches).
template <int L, int C>
__device__ __forceinline__ void zterm_angles(double (&ph)[kRegs], const ZTerm* terms, int n_terms,
                                             const double* gam, const TileMap& g, int t)
{
    typedef double dvec16 __attribute__((ext_vector_type(16)));
    int gb[4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
        gb[b] = reg_global_bit<L, C>(g, b);
    const uint64_t j0 = (uint64_t)g(elem<L>(t, 0));
    dvec16 cf = 0.0;
    for (int e = 0; e < n_terms; ++e) {
        const uint64_t S = terms[e].support;
        const double v0 = gam[e] * terms[e].coef;
        const double v = (__popcll(j0 & S) & 1) ? -v0 : v0;
        int m = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b)
            m |= (int)((S >> gb[b]) & 1) << b;
        cf[__builtin_amdgcn_readfirstlane(m)] += v;
    }
#pragma unroll
    for (int r = 0; r < kRegs; ++r)
        ph[r] = cf[r];
    wht16(ph);
}

// qq: q in layout L (read only with XP_EXPECT).
template <int L, int FLAGS>
__device__ __forceinline__ void tail(double2 (&v)[kRegs], const XPassParams& P, const TileMap& g,
                                     int t, double2 fs, double* red, int64_t tile,
                                     const double (&qq)[kRegs])
{
    if constexpr (FLAGS & XP_EXPECT) {
        double f = 0.0, nr = 0.0;
#pragma unroll
        for (int r = 0; r < kRegs; ++r) {
            double a = v[r].x * v[r].x + v[r].y * v[r].y;
            f = fma(a, qq[r], f);
            nr += a;
        }
        const double s2 = fs.x * fs.x + fs.y * fs.y;
        double2 tot = block_sum2(f * s2, nr * s2, red);
        if (t == 0)
            P.partials[tile] = tot;
    }
    if constexpr (FLAGS & XP_STORE) {
        constexpr bool sc = FLAGS & XP_FINAL_SCALE;
#pragma unroll
        for (int r = 0; r < kRegs; ++r)
            st_nt(P.psi + g(elem<L>(t, r)), sc ? cmul(v[r], fs) : v[r]);
    }
}

// One tile of a hypercube-mixer pass (see XPassParams and the XP_* flags).
// lds: 4096 amplitudes of shared memory; red: 8 doubles of shared memory.
// Every global read of the tile (psi, and q where the pass needs it) is
// issued before any arithmetic, so the tile's whole input is in flight at once.
template <int C, int FLAGS>
__device__ __forceinline__ void xpass_tile(const XPassParams& P, int64_t tile, double2* lds, double* red)
{
    constexpr int flags = FLAGS;
    static_assert(((flags & XP_PHASE_PRE) ? 1 : 0) + ((flags & XP_PHASE_MID) ? 1 : 0) +
                          ((flags & XP_EXPECT) ? 1 : 0) <= 1,
                  "one use of q per pass");
    constexpr bool zterms = flags & XP_ZTERMS;
    static_assert(!zterms || (flags & (XP_PHASE_PRE | XP_PHASE_MID)), "Z-string terms need a phase");
    // layout of the tail (store / expectation) and of the pass's phase / use of q
    constexpr int LT = ((flags & XP_MIX2) || !(flags & XP_MIX1)) ? LA : last_layout<C>();
    constexpr int LQ = (flags & XP_PHASE_PRE) ? LA : (flags & XP_PHASE_MID) ? last_layout<C>() : LT;
    constexpr bool use_q = zterms ? bool(flags & XP_EXPECT) : bool(flags & (XP_PHASE_PRE | XP_PHASE_MID | XP_EXPECT));

    const int t = threadIdx.x;
    const TileMap g = tile_map(tile, P.k, C);

    // Issue order of the tile's reads (measured per pass kind):
    // * a pass that reads psi and q for its phase reads its angles first,
    //   requests each register's psi and q together (the rows of a tile
    //   then arrive together, which matters most at large row strides), and
    //   computes the angles' sine and cosine while the tile is in flight;
    // * the first pass requests q before anything else;
    // * a pass without q requests psi before anything else;
    // * the last pass and the Z-string passes keep the compiler's order.
    constexpr bool phased = (flags & (XP_PHASE_PRE | XP_PHASE_MID)) && !zterms;
    constexpr bool early_angles = phased && !(flags & XP_INIT);
    double th_phase = 0.0, th_mix1 = 0.0, th_mix2 = 0.0;
    if constexpr (early_angles) {
        th_phase = angle_value(P.phase);
        th_mix1 = (flags & XP_MIX1) ? angle_value(P.mix1) : 0.0;
        th_mix2 = (flags & XP_MIX2) ? angle_value(P.mix2) : 0.0;
    }
    double2 v[kRegs];
    double qq[kRegs];
    if constexpr (flags & XP_INIT) {
        const double a0 = 1.0 / sqrt((double)(int64_t(1) << P.n));
#pragma unroll
        for (int r = 0; r < kRegs; ++r)
            v[r] = make_double2(a0, 0.0);
        if constexpr (use_q) {
            load_q<LQ>(qq, P.q, g, t);
            if constexpr (phased)
                QVA_ISSUE_FENCE();
        }
    } else if constexpr (early_angles && use_q) {
        // with the tile-ordered copy of q (phase between the rotations only),
        // register r's q is entry r * 256 + t of the tile's contiguous run
        const bool qtile = (flags & XP_PHASE_MID) && P.qt != nullptr;
        const double* qb = qtile ? P.qt + (tile << kTileBits) : P.q;
#pragma unroll
        for (int r = 0; r < kRegs; ++r) {
            v[r] = ld_nt(P.psi + g(elem<LA>(t, r)));
            qq[r] = ld_nt(qb + (qtile ? (int64_t)(r * kThreads + t) : g(elem<LQ>(t, r))));
            QVA_ISSUE_FENCE();
        }
    } else {
        if constexpr (!use_q && !zterms)
            QVA_ISSUE_FENCE();
#pragma unroll
        for (int r = 0; r < kRegs; ++r)
            v[r] = ld_nt(P.psi + g(elem<LA>(t, r)));
        if constexpr (use_q)
            load_q<LQ>(qq, P.q, g, t);
    }
    if constexpr (early_angles) {
        // the angles are used from here on: their sine and cosine follow the reads
        asm volatile("" : "+v"(th_phase), "+v"(th_mix1), "+v"(th_mix2)::"memory");
    } else {
        th_phase = phased ? angle_value(P.phase) : 0.0;
        th_mix1 = (flags & XP_MIX1) ? angle_value(P.mix1) : 0.0;
        th_mix2 = (flags & XP_MIX2) ? angle_value(P.mix2) : 0.0;
    }
    // Z-string terms: the phase angles themselves stand in for q (gamma = 1)
    if constexpr (zterms)
        zterm_angles<LQ, C>(qq, P.terms, P.n_terms, P.phase.ptr + P.phase.idx, g, t);
    const double gam = zterms ? 1.0 : th_phase;

    if constexpr (flags & XP_PHASE_PRE)
        phase_vals(v, qq, gam, make_double2(1.0, 0.0));

    double2 S1 = make_double2(1.0, 0.0);
    if constexpr (flags & XP_MIX1) {
        const MixCoef m = mix_coef(th_mix1);
        if (m.tanform)
            mix_forward<C, true>(v, lds, t, m.k);
        else
            mix_forward<C, false>(v, lds, t, m.k);
        S1 = cpow_int(m.sigma, P.n);
    }
    if constexpr (flags & XP_PHASE_MID)
        phase_vals(v, qq, gam, S1);
    if constexpr (flags & XP_MIX2) {
        const MixCoef m = mix_coef(th_mix2);
        if (m.tanform)
            mix_reverse<C, true>(v, lds, t, m.k);
        else
            mix_reverse<C, false>(v, lds, t, m.k);
    }
    const double2 fs = (flags & XP_FINAL_SCALE) ? S1 : make_double2(1.0, 0.0);
    tail<LT, flags>(v, P, g, t, fs, red, tile, qq);
}


// ------------------------------------------------------------ backward
// Deterministic block sum of K doubles (every thread gets the sums).
// `red` holds K * (blockDim.x / 64) doubles.
template <int K>
__device__ __forceinline__ void block_sum_k(double (&v)[K], double* red)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < K; ++i)
        v[i] = wave_sum(v[i]);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < K; ++i)
            red[K * wid + i] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < K; ++i) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w)
            s += red[K * w + i];
        v[i] = s;
    }
}

// Im(conj(chi_a) phi_b + conj(chi_b) phi_a)
__device__ __forceinline__ double im_pair(double2 a, double2 b, double2 ca, double2 cb)
{
    double s = ca.x * b.y;
    s = fma(-ca.y, b.x, s);
    s = fma(cb.x, a.y, s);
    s = fma(-cb.y, a.x, s);
    return s;
}

// exp(-i th X) with (c, s) = (cos th, sin th) applied to the pair (a, b).
__device__ __forceinline__ void rot_pair(double2& a, double2& b, double c, double s)
{
    const double2 a0 = a, b0 = b;
    a = make_double2(fma(c, a0.x, s * b0.y), fma(c, a0.y, -s * b0.x));
    b = make_double2(fma(c, b0.x, s * a0.y), fma(c, b0.y, -s * a0.x));
}

// Rotate both vectors on the target register bits of MASK, accumulating
// Im <chi|X_i|phi> over those qubits first.
template <int MASK>
__device__ __forceinline__ void rot2_regs(double2 (&p)[kRegs], double2 (&x)[kRegs], double c, double s,
                                          double& acc)
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (!((MASK >> j) & 1))
            continue;
#pragma unroll
        for (int r = 0; r < kRegs; ++r) {
            if (r & (1 << j))
                continue;
            const int r1 = r | (1 << j);
            acc += im_pair(p[r], p[r1], x[r], x[r1]);
            rot_pair(p[r], p[r1], c, s);
            rot_pair(x[r], x[r1], c, s);
        }
    }
}

// rot2_regs for element bit 3 held as thread bit 3 (layouts A and B): the pair
// partner is lane ^ 8; the lane with bit 3 clear adds the pair's term.
__device__ __forceinline__ void rot2_lane8(double2 (&p)[kRegs], double2 (&x)[kRegs], double c, double s,
                                           double& acc, int t)
{
    const bool low = !(t & 8);
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
        const double2 pu = lane_xor8(p[r]), xu = lane_xor8(x[r]);
        const double d = im_pair(p[r], pu, x[r], xu);
        acc += low ? d : 0.0;
        p[r] = make_double2(fma(c, p[r].x, s * pu.y), fma(c, p[r].y, -s * pu.x));
        x[r] = make_double2(fma(c, x[r].x, s * xu.y), fma(c, x[r].y, -s * xu.x));
    }
}

template <int FROM, int TO>
__device__ __forceinline__ void exchange2(double2 (&p)[kRegs], double2 (&x)[kRegs], double2* lds, int t)
{
    exchange<FROM, TO>(p, lds, t);
    exchange<FROM, TO>(x, lds, t);
}

// Rotations of every target qubit on both vectors; A -> last_layout<C>().
template <int C>
__device__ __forceinline__ void mix2_forward(double2 (&p)[kRegs], double2 (&x)[kRegs], double2* lds, int t,
                                             double c, double s, double& acc)
{
    rot2_regs<target_mask<C, LA>()>(p, x, c, s, acc);
    if constexpr (C == 3) {
        rot2_lane8(p, x, c, s, acc, t);
        exchange2<LA, LB>(p, x, lds, t);
        rot2_regs<target_mask<C, LB>()>(p, x, c, s, acc);
    } else if constexpr (C < 4) {
        exchange2<LA, LC>(p, x, lds, t);
        rot2_regs<target_mask<C, LC>()>(p, x, c, s, acc);
        exchange2<LC, LB>(p, x, lds, t);
        rot2_regs<target_mask<C, LB>()>(p, x, c, s, acc);
    } else if constexpr (C < 8) {
        exchange2<LA, LB>(p, x, lds, t);
        rot2_regs<target_mask<C, LB>()>(p, x, c, s, acc);
    }
}

// Same, last_layout<C>() -> A.
template <int C>
__device__ __forceinline__ void mix2_reverse(double2 (&p)[kRegs], double2 (&x)[kRegs], double2* lds, int t,
                                             double c, double s, double& acc)
{
    if constexpr (C == 3) {
        rot2_regs<target_mask<C, LB>()>(p, x, c, s, acc);
        exchange2<LB, LA>(p, x, lds, t);
        rot2_lane8(p, x, c, s, acc, t);
    } else if constexpr (C < 4) {
        rot2_regs<target_mask<C, LB>()>(p, x, c, s, acc);
        exchange2<LB, LC>(p, x, lds, t);
        rot2_regs<target_mask<C, LC>()>(p, x, c, s, acc);
        exchange2<LC, LA>(p, x, lds, t);
    } else if constexpr (C < 8) {
        rot2_regs<target_mask<C, LB>()>(p, x, c, s, acc);
        exchange2<LB, LA>(p, x, lds, t);
    }
    rot2_regs<target_mask<C, LA>()>(p, x, c, s, acc);
}

// (cos, sin) of the inverse rotation exp(+i t X) = exp(-i (-t) X)
__device__ __forceinline__ void inv_cs(double t, double& c, double& s)
{
    double sn, cs;
    sincos_red(t, &sn, &cs);
    c = cs;
    s = -sn;
}

// q at the registers of layout L of a tile: from q itself, or (QT) from the
// tile's contiguous run qtile of the tile-ordered copy, which holds register
// r's entry at r * 256 + t.  A compile-time choice: the two-vector passes sit
// at their register limit, and a run-time choice between the two address
// forms spills.
template <int L, bool QT>
__device__ __forceinline__ void load_q_regs(double (&qq)[kRegs], const double* q, const double* qtile,
                                            const TileMap& g, int t)
{
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
        if constexpr (QT)
            qq[r] = ld_nt(qtile + r * kThreads + t);
        else
            qq[r] = ld_nt(q + g(elem<L>(t, r)));
    }
}

// sum_j q_j Im(conj(chi_j) phi_j) over the registers of layout L, and the
// inverse phase exp(+i gamma q) applied to both vectors (q as load_q_regs).
template <int L, bool SCALE, bool QT = false>
__device__ __forceinline__ double unphase2(double2 (&p)[kRegs], double2 (&x)[kRegs], const double* q,
                                           const TileMap& g, int t, double gamma, double scale,
                                           const double* qtile = nullptr)
{
    double qq[kRegs];
    load_q_regs<L, QT>(qq, q, qtile, g, t);
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
        if constexpr (SCALE) {
            p[r] = make_double2(p[r].x * scale, p[r].y * scale);
            x[r] = make_double2(x[r].x * scale, x[r].y * scale);
        }
        acc = fma(qq[r], x[r].x * p[r].y - x[r].y * p[r].x, acc);
        const double2 ph = expmi(-gamma * qq[r]);
        p[r] = cmul(p[r], ph);
        x[r] = cmul(x[r], ph);
        QVA_SCHED_FENCE();
    }
    return acc;
}

template <int L>
__device__ __forceinline__ void store2(const double2 (&p)[kRegs], const double2 (&x)[kRegs],
                                       const GradPassParams& P, const TileMap& g, int t)
{
    store_tile<L>(p, P.phi, g, t, 1.0);
    store_tile<L>(x, P.chi, g, t, 1.0);
}

template <int L>
__device__ __forceinline__ void load2(double2 (&p)[kRegs], double2 (&x)[kRegs], const GradPassParams& P,
                                      const TileMap& g, int t)
{
    load_tile<L>(p, P.phi, g, t);
    load_tile<L>(x, P.chi, g, t);
}

// Write the block sums of the accumulators to their per-tile slots.
__device__ __forceinline__ void write_slots(const GradPassParams& P, double a1, double ag, double a2,
                                            double* red, int64_t tile)
{
    double v[3] = {a1, ag, a2};
    block_sum_k<3>(v, red);
    if (threadIdx.x == 0) {
        if (P.slot_t1)
            P.slot_t1[tile] = v[0];
        if (P.slot_g)
            P.slot_g[tile] = v[1];
        if (P.slot_t2)
            P.slot_t2[tile] = v[2];
    }
}

// Walsh-Hadamard transform of a tile of reals over its 12 element bits.  d
// holds the tile in layout L; afterwards lds[swz(m)].x = sum_e (-1)^popcount(e & m) d_e
// for every element mask m (visible to the whole block).  lds: the tile
// exchange buffer (the first write waits for the block); the reals sit in
// the amplitude slots, so the addresses are the exchanges' own.  The register
// bits of LC, LB and LA are element bits [0,4), [4,8) and [8,12); L's own
// register bits are transformed in place first when L is one of them.
template <int L>
__device__ __forceinline__ void wht_tile(double (&d)[kRegs], double2* lds, int t)
{
    constexpr bool own = L != LA3;
    if constexpr (own)
        wht16(d);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRegs; ++r)
        lds[swz(elem<L>(t, r))].x = d[r];
    auto stage = [&](auto lw) {
        constexpr int W = decltype(lw)::value;
        if constexpr (!(own && W == L)) {
            __syncthreads();
#pragma unroll
            for (int r = 0; r < kRegs; ++r)
                d[r] = lds[swz(elem<W>(t, r))].x;
            wht16(d);
#pragma unroll
            for (int r = 0; r < kRegs; ++r)
                lds[swz(elem<W>(t, r))].x = d[r];
        }
    };
    stage(std::integral_constant<int, LC>());
    stage(std::integral_constant<int, LB>());
    stage(std::integral_constant<int, LA>());
    __syncthreads();
}

// Per-term slots of the extended-QAOA gradient: for every term e,
//   slot_terms[e * tiles + tile] = sum over the tile of c_e (-1)^popcount(j & S_e) d_j,
// d_j = Im(conj(chi_j) phi_j) held in layout L.  Within the tile j = base + j(e)
// with j(e) the global bits of element index e, so the sign splits into a
// constant (-1)^popcount(base & S_e) and (-1)^popcount(e & m_e), m_e the
// element bits whose global bits S_e covers: the sum is one value of the
// tile's Walsh-Hadamard transform.  Every term is read off the same
// transform, with no per-term reduction.
template <int C, int L>
__device__ __forceinline__ void zterm_slots(double (&d)[kRegs], const GradPassParams& P, const TileMap& g,
                                            int t, int64_t tile, double2* lds)
{
    wht_tile<L>(d, lds, t);
    const int64_t tiles = int64_t(1) << (P.n - kTileBits);
    for (int e = t; e < P.n_terms; e += kThreads) {
        const uint64_t S = P.terms[e].support;
        int m = 0;
#pragma unroll
        for (int eb = 0; eb < kTileBits; ++eb) {
            const int gb = eb < C ? eb : g.k + eb - C;
            m |= (int)((S >> gb) & 1) << eb;
        }
        const double v = P.terms[e].coef * lds[swz(m)].x;
        P.slot_terms[(int64_t)e * tiles + tile] = (__popcll((uint64_t)g.base & S) & 1) ? -v : v;
    }
}

// The per-term slots of an extended-QAOA phase (see zterm_slots) from the
// values d_j = Im(conj(chi_j) phi_j) that its backward pass stored to zd, read
// in the layout in which that pass held them.
template <int C>
__device__ __forceinline__ void zslot_tile(const GradPassParams& P, int64_t tile, double2* lds)
{
    constexpr int L = last_layout<C>();
    const int t = threadIdx.x;
    const TileMap g = tile_map(tile, P.k, C);
    double d[kRegs];
#pragma unroll
    for (int r = 0; r < kRegs; ++r)
        d[r] = __builtin_nontemporal_load(P.zd + g(elem<L>(t, r)));
    zterm_slots<C, L>(d, P, g, t, tile, lds);
}

// Block sum of one accumulator to its per-tile slot (skipped when null).
__device__ __forceinline__ void write_slot(double* slot, double a, double* red, int64_t tile)
{
    double v[1] = {a};
    block_sum_k<1>(v, red);
    if (slot && threadIdx.x == 0)
        slot[tile] = v[0];
}

// ------------------------------------------------ hypercube-mixer passes
// One tile of a backward hypercube-mixer pass (see GradPassParams and GMODE_*).
// lds: 4096 amplitudes of shared memory; red: 16 doubles of shared memory.
template <int C, int MODE>
__device__ __forceinline__ void gradx_tile(const GradPassParams& P, int64_t tile, double2* lds, double* red)
{
    const int t = threadIdx.x;
    const TileMap g = tile_map(tile, P.k, C);
    double2 p[kRegs], x[kRegs];
    double a1 = 0.0, ag = 0.0, a2 = 0.0;
    constexpr bool qtiled = MODE & GM_QTILE;

    if constexpr ((MODE & ~GM_QTILE) == GMODE_TURN) {
        // last forward group of the last layer, <Q>, chi = Q psi_p, then the
        // inverse of the same rotations on both vectors
        const double tt = angle_value(P.t1);
        const MixCoef m = mix_coef(tt);
        double c, s;
        inv_cs(tt, c, s);
        load_tile<LA>(p, P.phi, g, t);
        if (m.tanform)
            mix_forward<C, true>(p, lds, t, m.k);
        else
            mix_forward<C, false>(p, lds, t, m.k);
        const double2 S = cpow_int(m.sigma, P.n);
        constexpr int L = last_layout<C>();
        double qq[kRegs];
        load_q_regs<L, qtiled>(qq, P.q, qtiled ? P.qt + (tile << kTileBits) : nullptr, g, t);
        double f = 0.0, nr = 0.0;
#pragma unroll
        for (int r = 0; r < kRegs; ++r) {
            p[r] = cmul(p[r], S);
            const double a = p[r].x * p[r].x + p[r].y * p[r].y;
            f = fma(a, qq[r], f);
            nr += a;
            x[r] = make_double2(qq[r] * p[r].x, qq[r] * p[r].y);
        }
        double fv[2] = {f, nr};
        block_sum_k<2>(fv, red);
        if (t == 0)
            P.fpart[tile] = make_double2(fv[0], fv[1]);
        mix2_reverse<C>(p, x, lds, t, c, s, a1);
        write_slots(P, a1, 0.0, 0.0, red, tile);
        store2<LA>(p, x, P, g, t);
    } else {
        constexpr int BM = MODE & ~(GM_ZTERMS | GM_QTILE);
        constexpr bool zterms = MODE & GM_ZTERMS;
        static_assert(!qtiled || (!zterms && BM != GMODE_MID), "tiled q where the pass reads q");
        static_assert(!zterms || BM == GMODE_BOUND || BM == GMODE_FINAL, "Z-string terms at a phase only");
        constexpr int L = last_layout<C>();
        // The angles are read before the tile, each register's phi and chi are
        // requested together (issue fences keep that order), and the angles'
        // sine and cosine are computed while the tile is in flight, before any
        // other work, so that their temporaries are dead by the time the
        // rotations need registers.
        double c, s, c2 = 1.0, s2 = 0.0, gam = 0.0;
        double th1 = angle_value(P.t1), th2 = 0.0;
        if constexpr (BM == GMODE_BOUND)
            th2 = angle_value(P.t2);
        if constexpr (BM != GMODE_MID && !zterms)
            gam = angle_value(P.gamma);
        // Z-string phase angles depend only on the tile's position: formed
        // before the tile is loaded, their coefficient registers are free again
        // while both vectors are held
        double dv[kRegs];
        if constexpr (zterms)
            zterm_angles<L, C>(dv, P.terms, P.n_terms, P.gamma.ptr + P.gamma.idx, g, t);
#pragma unroll
        for (int r = 0; r < kRegs; ++r) {
            p[r] = ld_nt(P.phi + g(elem<LA>(t, r)));
            x[r] = ld_nt(P.chi + g(elem<LA>(t, r)));
            QVA_ISSUE_FENCE();
        }
        asm volatile("" : "+v"(th1), "+v"(th2), "+v"(gam)::"memory");
        inv_cs(th1, c, s);
        if constexpr (BM == GMODE_BOUND)
            inv_cs(th2, c2, s2);
        mix2_forward<C>(p, x, lds, t, c, s, a1);
        if constexpr (BM == GMODE_MID) {
            write_slots(P, a1, 0.0, 0.0, red, tile);
            store2<L>(p, x, P, g, t);
        } else {
            // the forward pass applied the layer's scalar factor together with
            // the phase; the direct-form inverse rotations need none
            if constexpr (zterms) {
                // the mixer slot first (its block sum is taken before the
                // phase; the phase's own per-term sums come from zslot_tile)
                write_slot(P.slot_t1, a1, red, tile);
                // register by register the inverse phase on both vectors and
                // Im(conj(chi) phi) in place of the angle (taken after the
                // phase, which it does not change)
#pragma unroll
                for (int r = 0; r < kRegs; ++r) {
                    const double2 u = expmi(-dv[r]);
                    p[r] = cmul(p[r], u);
                    x[r] = cmul(x[r], u);
                    dv[r] = x[r].x * p[r].y - x[r].y * p[r].x;
                    QVA_SCHED_FENCE();
                }
                // the per-term sums follow in a pass of their own (zslot_tile):
                // their transform beside both vectors would cost this pass
                // half its waves
#pragma unroll
                for (int r = 0; r < kRegs; ++r)
                    __builtin_nontemporal_store(dv[r], P.zd + g(elem<L>(t, r)));
            } else {
                ag = unphase2<L, false, qtiled>(p, x, P.q, g, t, gam, 1.0,
                                                qtiled ? P.qt + (tile << kTileBits) : nullptr);
            }
            if constexpr (BM == GMODE_BOUND) {
                mix2_reverse<C>(p, x, lds, t, c2, s2, a2);
                if constexpr (zterms)
                    write_slot(P.slot_t2, a2, red, tile);
                else
                    write_slots(P, a1, ag, a2, red, tile);
                store2<LA>(p, x, P, g, t);
            } else if constexpr (!zterms) {  // GMODE_FINAL
                write_slots(P, a1, ag, 0.0, red, tile);
            }
        }
    }
}

}  // namespace passes
}  // namespace qva
