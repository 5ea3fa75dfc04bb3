// qva_xy.hip -- QAOAz parity-mixer passes (Sec. 2.4.1, eqs. parity_terms,
// qaoaz_mixers, qaoaz).
//
// A factor exp(-i t (X_a X_b + Y_a Y_b)) leaves the basis states whose bits a
// and b agree alone and rotates each pair (bits a, b = 10 ; 01) by
// cos 2t - i sin 2t sigma_x.  A pass holds one tile (4096 amplitudes over the
// index bits [0, C) and [k, k + 12 - C), or the whole register for n <= 12) in
// LDS and applies its list of factors in order; the planner only lists a
// factor in a pass once every earlier factor sharing a qubit with it is done.
// Each thread rotates 4 of the tile's 1024 amplitude pairs per factor.
//
// The first pass of a layer applies the phase exp(-i gamma q) first (each
// thread on its own amplitudes, before they go to LDS); the last pass of the
// evolution takes the (f, norm) partials, and for the gradient also writes
// chi = q psi.  The backward pass undoes a forward pass on both vectors,
// accumulating Im <chi|X_a X_b + Y_a Y_b|phi> before each factor is undone and
// Im <chi|Q|phi> before the phase is.
#include "qva_passes.h"

namespace qva {
namespace {

using namespace tile;

// Index with zero bits inserted at positions lo < hi.
__device__ __forceinline__ int insert_two_zeros(int i, int lo, int hi)
{
    i = ((i >> lo) << (lo + 1)) | (i & ((1 << lo) - 1));
    return ((i >> hi) << (hi + 1)) | (i & ((1 << hi) - 1));
}

// (u, w) <- (c u - i s w, c w - i s u)
__device__ __forceinline__ void xy_rot(double2& u, double2& w, double c, double s)
{
    const double2 u0 = u, w0 = w;
    u = make_double2(fma(c, u0.x, s * w0.y), fma(c, u0.y, -s * w0.x));
    w = make_double2(fma(c, w0.x, s * u0.y), fma(c, w0.y, -s * u0.x));
}

// One tile in LDS (64 KiB): two workgroups per CU, of 1024 threads holding 4
// amplitudes each (eight waves per SIMD: the factor loop is LDS-latency
// bound; 2^26 amplitudes, p = 6: 9.06 ms per evolution with 256 threads,
// 8.72 with 512, 8.58 with 1024).
constexpr int kXyThreads = 1024;
constexpr int kXyRegs = (1 << kTileBits) / kXyThreads;

__global__ __launch_bounds__(kXyThreads, 2) void xypass_kernel(XyPassParams P)
{
    constexpr int kThreads = kXyThreads, kRegs = kXyRegs;
    __shared__ double2 s[1 << kTileBits];
    __shared__ double red[2 * (kThreads / 64)];
    const int t = threadIdx.x;
    const int E = P.elems;
    const TileMap g = tile_map(blockIdx.x, P.k, P.C);
    const bool phase = P.flags & XY_PHASE, expect = P.flags & XY_EXPECT;
    double2 v[kRegs];
    double qq[kRegs];
#pragma unroll
    for (int m = 0; m < kRegs; ++m) {
        const int e = t + kThreads * m;
        if (e < E)
            v[m] = ld_nt(P.psi + g(e));
    }
    if (phase || expect) {
#pragma unroll
        for (int m = 0; m < kRegs; ++m) {
            const int e = t + kThreads * m;
            qq[m] = e < E ? ld_nt(P.q + g(e)) : 0.0;
        }
    }
    if (phase) {
        const double gam = P.gammas[P.layer];
#pragma unroll
        for (int m = 0; m < kRegs; ++m) {
            if (t + kThreads * m < E)
                v[m] = cmul(v[m], expmi(gam * qq[m]));
            QVA_SCHED_FENCE();
        }
    }
    if (P.n_ops > 0) {
        double sn, c;
        sincos_red(2.0 * P.ts[P.layer], &sn, &c);
#pragma unroll
        for (int m = 0; m < kRegs; ++m) {
            const int e = t + kThreads * m;
            if (e < E)
                s[e] = v[m];
        }
        for (int o = 0; o < P.n_ops; ++o) {
            __syncthreads();
            const int a = P.ea[o], b = P.eb[o];
            const int lo = a < b ? a : b, hi = a < b ? b : a;
            if (E == (1 << kTileBits)) {
                // a full tile: 4 pairs per thread, all reads issued before any write
                constexpr int J = (1 << kTileBits) / 4 / kThreads;
                int e1[J], e2[J];
                double2 u[J], w[J];
#pragma unroll
                for (int m = 0; m < J; ++m) {
                    const int x = insert_two_zeros(t + kThreads * m, lo, hi);
                    e1[m] = x | (1 << a);
                    e2[m] = x | (1 << b);
                    u[m] = s[e1[m]];
                    w[m] = s[e2[m]];
                }
#pragma unroll
                for (int m = 0; m < J; ++m) {
                    xy_rot(u[m], w[m], c, sn);
                    s[e1[m]] = u[m];
                    s[e2[m]] = w[m];
                }
            } else {
                for (int i = t; i < E / 4; i += kThreads) {
                    const int x = insert_two_zeros(i, lo, hi);
                    const int e1 = x | (1 << a), e2 = x | (1 << b);
                    double2 u = s[e1], w = s[e2];
                    xy_rot(u, w, c, sn);
                    s[e1] = u;
                    s[e2] = w;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kRegs; ++m) {
            const int e = t + kThreads * m;
            if (e < E)
                v[m] = s[e];
        }
    }
    if (expect) {
        double f = 0.0, nr = 0.0;
#pragma unroll
        for (int m = 0; m < kRegs; ++m) {
            if (t + kThreads * m < E) {
                const double pr = v[m].x * v[m].x + v[m].y * v[m].y;
                f = fma(pr, qq[m], f);
                nr += pr;
            }
        }
        const double2 tot = block_sum2(f, nr, red);
        if (t == 0)
            P.partials[blockIdx.x] = tot;
    }
    if (P.flags & XY_STORE) {
#pragma unroll
        for (int m = 0; m < kRegs; ++m) {
            const int e = t + kThreads * m;
            if (e < E)
                st_nt(P.psi + g(e), v[m]);
        }
    }
    if (P.flags & XY_CHI) {
#pragma unroll
        for (int m = 0; m < kRegs; ++m) {
            const int e = t + kThreads * m;
            if (e < E)
                st_nt(P.chi + g(e), make_double2(qq[m] * v[m].x, qq[m] * v[m].y));
        }
    }
}

// Inverse of one forward pass on (phi, chi); both tiles sit in LDS.  The
// two tiles (128 KiB) leave room for one workgroup per CU, so the pass runs
// 1024 threads (four waves per SIMD), each holding 4 amplitudes of each
// vector (with 256 threads it ran at one wave per SIMD: 1.23 ms per launch
// at 2^26 amplitudes, 1.11 ms with 512 or 1024).
constexpr int kXyGradThreads = 1024;
constexpr int kXyGradRegs = (1 << kTileBits) / kXyGradThreads;

__global__ __launch_bounds__(kXyGradThreads, 1) void xygrad_kernel(XyPassParams P)
{
    constexpr int kThreads = kXyGradThreads, kRegs = kXyGradRegs;
    __shared__ double2 sp[1 << kTileBits];
    __shared__ double2 sx[1 << kTileBits];
    __shared__ double red[2 * (kThreads / 64)];
    const int t = threadIdx.x;
    const int E = P.elems;
    const TileMap g = tile_map(blockIdx.x, P.k, P.C);
    const bool phase = P.flags & XY_PHASE;
    double2 p[kRegs], x[kRegs];
#pragma unroll
    for (int m = 0; m < kRegs; ++m) {
        const int e = t + kThreads * m;
        if (e < E) {
            p[m] = ld_nt(P.psi + g(e));
            x[m] = ld_nt(P.chi + g(e));
        }
    }
    double qq[kRegs];
    if (phase) {
#pragma unroll
        for (int m = 0; m < kRegs; ++m) {
            const int e = t + kThreads * m;
            qq[m] = e < E ? ld_nt(P.q + g(e)) : 0.0;
        }
    }
    double at = 0.0, ag = 0.0;
    if (P.n_ops > 0) {
        // the inverse rotation: exp(+i t (XX + YY)) = rotation by -t
        double sn, c;
        sincos_red(2.0 * P.ts[P.layer], &sn, &c);
        sn = -sn;
#pragma unroll
        for (int m = 0; m < kRegs; ++m) {
            const int e = t + kThreads * m;
            if (e < E) {
                sp[e] = p[m];
                sx[e] = x[m];
            }
        }
        for (int o = P.n_ops - 1; o >= 0; --o) {
            __syncthreads();
            const int a = P.ea[o], b = P.eb[o];
            const int lo = a < b ? a : b, hi = a < b ? b : a;
            if (E == (1 << kTileBits)) {
                constexpr int J = (1 << kTileBits) / 4 / kThreads;
                int e1[J], e2[J];
                double2 p1[J], p2[J], x1[J], x2[J];
#pragma unroll
                for (int m = 0; m < J; ++m) {
                    const int xi = insert_two_zeros(t + kThreads * m, lo, hi);
                    e1[m] = xi | (1 << a);
                    e2[m] = xi | (1 << b);
                    p1[m] = sp[e1[m]];
                    p2[m] = sp[e2[m]];
                    x1[m] = sx[e1[m]];
                    x2[m] = sx[e2[m]];
                }
#pragma unroll
                for (int m = 0; m < J; ++m) {
                    // (XX + YY) maps e1 <-> e2 with weight 2
                    at += 2.0 * passes::im_pair(p1[m], p2[m], x1[m], x2[m]);
                    xy_rot(p1[m], p2[m], c, sn);
                    xy_rot(x1[m], x2[m], c, sn);
                    sp[e1[m]] = p1[m];
                    sp[e2[m]] = p2[m];
                    sx[e1[m]] = x1[m];
                    sx[e2[m]] = x2[m];
                }
            } else {
                for (int i = t; i < E / 4; i += kThreads) {
                    const int xi = insert_two_zeros(i, lo, hi);
                    const int e1 = xi | (1 << a), e2 = xi | (1 << b);
                    double2 p1 = sp[e1], p2 = sp[e2], x1 = sx[e1], x2 = sx[e2];
                    // (XX + YY) maps e1 <-> e2 with weight 2
                    at += 2.0 * passes::im_pair(p1, p2, x1, x2);
                    xy_rot(p1, p2, c, sn);
                    xy_rot(x1, x2, c, sn);
                    sp[e1] = p1;
                    sp[e2] = p2;
                    sx[e1] = x1;
                    sx[e2] = x2;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kRegs; ++m) {
            const int e = t + kThreads * m;
            if (e < E) {
                p[m] = sp[e];
                x[m] = sx[e];
            }
        }
    }
    if (phase) {
        const double gam = P.gammas[P.layer];
#pragma unroll
        for (int m = 0; m < kRegs; ++m) {
            if (t + kThreads * m < E) {
                ag = fma(qq[m], x[m].x * p[m].y - x[m].y * p[m].x, ag);
                const double2 u = expmi(-gam * qq[m]);
                p[m] = cmul(p[m], u);
                x[m] = cmul(x[m], u);
            }
            QVA_SCHED_FENCE();
        }
    }
    const double2 tot = block_sum2(at, ag, red);
    if (t == 0) {
        if (P.slot_t)
            P.slot_t[blockIdx.x] = tot.x;
        if (P.slot_g)
            P.slot_g[blockIdx.x] = tot.y;
    }
#pragma unroll
    for (int m = 0; m < kRegs; ++m) {
        const int e = t + kThreads * m;
        if (e < E) {
            st_nt(P.psi + g(e), p[m]);
            st_nt(P.chi + g(e), x[m]);
        }
    }
}

}  // namespace

hipError_t launch_xypass(const XyPassParams& P, int64_t tiles, hipStream_t s)
{
    if (P.n_ops < 0 || P.n_ops > kMaxXyOps || P.elems < 1 || P.elems > (1 << kTileBits))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(xypass_kernel, dim3((unsigned)tiles), dim3(kXyThreads), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_xygrad(const XyPassParams& P, int64_t tiles, hipStream_t s)
{
    if (P.n_ops < 0 || P.n_ops > kMaxXyOps || P.elems < 1 || P.elems > (1 << kTileBits))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(xygrad_kernel, dim3((unsigned)tiles), dim3(kXyGradThreads), 0, s, P);
    return hipGetLastError();
}

}  // namespace qva
