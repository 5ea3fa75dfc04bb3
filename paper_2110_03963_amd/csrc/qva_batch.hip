// qva_batch.hip -- many independent QAOA instances (hypercube mixer),
// forward + adjoint gradient, one launch per round of passes.
//
// Round r holds pass r of every instance that has one: the passes of one
// instance must run in order (each pass reads the whole state the previous
// pass wrote), while different instances are independent.  Kernel boundaries
// order the rounds; the items of a round (an instance, its pass r, a run of
// its tiles) are grouped by pass kind, mode and tile geometry, and each group
// is one launch of a kernel specialised for it that runs the same tile
// bodies as the single-instance passes.  Instances with n = 12 are one tile: their
// whole forward and backward sweep runs in registers and LDS in a single
// item.
#include "qva_passes.h"

namespace qva {
namespace {

using namespace tile;
using namespace passes;

__device__ __forceinline__ Angle dev_angle(const double* ptr, int idx)
{
    Angle a;
    a.ptr = ptr;
    a.idx = idx < 0 ? 0 : idx;
    a.val = 0.0;
    return a;
}

// exp(-i th X) on the register bits of MASK (direct form, unitary).
template <int MASK>
__device__ __forceinline__ void rot1_regs(double2 (&v)[kRegs], double c, double s)
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (!((MASK >> j) & 1))
            continue;
#pragma unroll
        for (int r = 0; r < kRegs; ++r)
            if (!(r & (1 << j)))
                rot_pair(v[r], v[r | (1 << j)], c, s);
    }
}

// n = 12: the whole state is one tile; every layer forward, <Q>, and every
// layer backward (with the inner products of the adjoint method) without
// leaving the workgroup.  Layers always go A -> C -> B -> A.
__device__ void whole12(const BatchInst& d, double2* lds, double* red)
{
    const int t = threadIdx.x;
    const TileMap g = tile_map(0, 0, 0);
    double2 p[kRegs], x[kRegs];
    const double a0 = 1.0 / 64.0;  // 4096^(-1/2)
#pragma unroll
    for (int r = 0; r < kRegs; ++r)
        p[r] = make_double2(a0, 0.0);
    for (int L = 0; L < d.p; ++L) {
        double sn, cs;
        sincos_red(d.ts[L], &sn, &cs);
        phase_regs<LA>(p, d.q, g, t, d.gammas[L], make_double2(1.0, 0.0));
        rot1_regs<0xF>(p, cs, sn);
        exchange<LA, LC>(p, lds, t);
        rot1_regs<0xF>(p, cs, sn);
        exchange<LC, LB>(p, lds, t);
        rot1_regs<0xF>(p, cs, sn);
        exchange<LB, LA>(p, lds, t);
    }
    double qq[kRegs];
#pragma unroll
    for (int r = 0; r < kRegs; ++r)
        qq[r] = d.q[g(elem<LA>(t, r))];
    double f = 0.0;
#pragma unroll
    for (int r = 0; r < kRegs; ++r) {
        f = fma(p[r].x * p[r].x + p[r].y * p[r].y, qq[r], f);
        x[r] = make_double2(qq[r] * p[r].x, qq[r] * p[r].y);
    }
    double fv[1] = {f};
    block_sum_k<1>(fv, red);
    if (t == 0)
        d.out_f[0] = fv[0];
    for (int L = d.p - 1; L >= 0; --L) {
        double c, s;
        inv_cs(d.ts[L], c, s);
        const double gam = d.gammas[L];
        double at = 0.0;
        rot2_regs<0xF>(p, x, c, s, at);
        exchange2<LA, LC>(p, x, lds, t);
        rot2_regs<0xF>(p, x, c, s, at);
        exchange2<LC, LB>(p, x, lds, t);
        rot2_regs<0xF>(p, x, c, s, at);
        exchange2<LB, LA>(p, x, lds, t);
        const double ag = unphase2<LA, false>(p, x, d.q, g, t, gam, 1.0);
        double v2[2] = {at, ag};
        block_sum_k<2>(v2, red);
        if (t == 0) {
            d.dts[L] = 2.0 * v2[0];
            d.dgammas[L] = 2.0 * v2[1];
        }
    }
}

// f and the gradient of one instance from its per-tile partials, in a fixed
// order: thread i adds partials i, i + 256, ..., then a fixed tree.
__device__ void batch_reduce(const BatchInst& d, double* red, double* sums)
{
    const int t = threadIdx.x;
    double f = 0.0;
    for (int64_t i = t; i < d.tiles; i += blockDim.x)
        f += d.fpart[i].x;
    double fv[1] = {f};
    block_sum_k<1>(fv, red);
    if (t == 0)
        d.out_f[0] = fv[0];
    for (int sl = 0; sl < d.nslots; ++sl) {
        const double* base = d.slots + (int64_t)sl * d.tiles;
        double s = 0.0;
        for (int64_t i = t; i < d.tiles; i += blockDim.x)
            s += base[i];
        double sv[1] = {s};
        block_sum_k<1>(sv, red);
        if (t == 0)
            sums[sl] = sv[0];
    }
    __syncthreads();
    for (int L = t; L < d.p; L += blockDim.x) {
        double s = 0.0;
        for (int gg = 0; gg < d.G; ++gg)
            s += sums[L * d.G + gg];
        d.dts[L] = 2.0 * s;
        d.dgammas[L] = 2.0 * sums[d.p * d.G + L];
    }
}

__device__ __forceinline__ XPassParams fwd_params(const BatchInst& d, const BatchPass& ps)
{
    XPassParams X{};
    X.psi = d.psi;
    X.q = d.q;
    X.mix1 = dev_angle(d.ts, ps.t1);
    X.mix2 = dev_angle(d.ts, ps.t2);
    X.phase = dev_angle(d.gammas, ps.gamma);
    X.n = d.n;
    X.k = ps.k;
    X.col_bits = ps.col_bits;
    X.flags = ps.mode;
    X.partials = d.fpart;
    return X;
}

__device__ __forceinline__ GradPassParams bwd_params(const BatchInst& d, const BatchPass& ps)
{
    GradPassParams G{};
    G.phi = d.psi;
    G.chi = d.chi;
    G.q = d.q;
    G.t1 = dev_angle(d.ts, ps.t1);
    G.t2 = dev_angle(d.ts, ps.t2);
    G.gamma = dev_angle(d.gammas, ps.gamma);
    G.n = d.n;
    G.k = ps.k;
    G.col_bits = ps.col_bits;
    G.flags = ps.mode;
    G.slot_t1 = ps.slot_t1 >= 0 ? d.slots + (int64_t)ps.slot_t1 * d.tiles : nullptr;
    G.slot_g = ps.slot_g >= 0 ? d.slots + (int64_t)ps.slot_g * d.tiles : nullptr;
    G.slot_t2 = ps.slot_t2 >= 0 ? d.slots + (int64_t)ps.slot_t2 * d.tiles : nullptr;
    G.fpart = d.fpart;
    return G;
}

// Items of one round that share (kind, mode, column bits) run in one launch
// of a kernel specialised for them.
template <int C, int MODE>
__global__ __launch_bounds__(kThreads, 2) void batch_fwd_kernel(BatchRoundParams R)
{
    __shared__ double2 lds[1 << kTileBits];
    __shared__ double red[4 * (kThreads / 64)];
    const BatchItem it = R.items[R.first + blockIdx.x];
    const BatchInst d = R.inst[it.inst];
    const XPassParams X = fwd_params(d, R.pass[d.pass_off + it.pass]);
    xpass_tile<C, MODE>(X, it.tile, lds, red);
}

template <int C, int MODE>
__global__ __launch_bounds__(kThreads, 2) void batch_bwd_kernel(BatchRoundParams R)
{
    __shared__ double2 lds[1 << kTileBits];
    __shared__ double red[4 * (kThreads / 64)];
    const BatchItem it = R.items[R.first + blockIdx.x];
    const BatchInst d = R.inst[it.inst];
    const GradPassParams G = bwd_params(d, R.pass[d.pass_off + it.pass]);
    gradx_tile<C, MODE>(G, it.tile, lds, red);
}

__global__ __launch_bounds__(kThreads, 2) void batch_whole_kernel(BatchRoundParams R)
{
    __shared__ double2 lds[1 << kTileBits];
    __shared__ double red[4 * (kThreads / 64)];
    const BatchItem it = R.items[R.first + blockIdx.x];
    whole12(R.inst[it.inst], lds, red);
}

__global__ __launch_bounds__(kThreads) void batch_reduce_kernel(BatchRoundParams R)
{
    __shared__ double sums[1024];
    __shared__ double red[4 * (kThreads / 64)];
    const BatchItem it = R.items[R.first + blockIdx.x];
    batch_reduce(R.inst[it.inst], red, sums);
}

template <int C>
hipError_t launch_fwd_c(const BatchRoundParams& R, int mode, int nitems, hipStream_t s)
{
    if (mode == XMODE_FIRST)
        hipLaunchKernelGGL((batch_fwd_kernel<C, XMODE_FIRST>), dim3(nitems), dim3(kThreads), 0, s, R);
    else if (mode == XMODE_MIDDLE)
        hipLaunchKernelGGL((batch_fwd_kernel<C, XMODE_MIDDLE>), dim3(nitems), dim3(kThreads), 0, s, R);
    else if (mode == XMODE_BOUNDARY)
        hipLaunchKernelGGL((batch_fwd_kernel<C, XMODE_BOUNDARY>), dim3(nitems), dim3(kThreads), 0, s, R);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int C>
hipError_t launch_bwd_c(const BatchRoundParams& R, int mode, int nitems, hipStream_t s)
{
    if (mode == GMODE_TURN)
        hipLaunchKernelGGL((batch_bwd_kernel<C, GMODE_TURN>), dim3(nitems), dim3(kThreads), 0, s, R);
    else if (mode == GMODE_MID)
        hipLaunchKernelGGL((batch_bwd_kernel<C, GMODE_MID>), dim3(nitems), dim3(kThreads), 0, s, R);
    else if (mode == GMODE_BOUND)
        hipLaunchKernelGGL((batch_bwd_kernel<C, GMODE_BOUND>), dim3(nitems), dim3(kThreads), 0, s, R);
    else if (mode == GMODE_FINAL)
        hipLaunchKernelGGL((batch_bwd_kernel<C, GMODE_FINAL>), dim3(nitems), dim3(kThreads), 0, s, R);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// theta <- theta - lr * grad for every instance (one workgroup per instance)
__global__ __launch_bounds__(64) void batch_sgd_kernel(const BatchInst* inst, double lr)
{
    const BatchInst d = inst[blockIdx.x];
    for (int j = threadIdx.x; j < d.p; j += blockDim.x) {
        d.gammas[j] = fma(-lr, d.dgammas[j], d.gammas[j]);
        d.ts[j] = fma(-lr, d.dts[j], d.ts[j]);
    }
}

}  // namespace

hipError_t launch_batch_group(const BatchRoundParams& R, int kind, int mode, int col_bits, int nitems,
                              hipStream_t s)
{
    if (nitems <= 0)
        return hipSuccess;
    switch (kind) {
    case BP_WHOLE:
        hipLaunchKernelGGL(batch_whole_kernel, dim3(nitems), dim3(kThreads), 0, s, R);
        return hipGetLastError();
    case BP_REDUCE:
        hipLaunchKernelGGL(batch_reduce_kernel, dim3(nitems), dim3(kThreads), 0, s, R);
        return hipGetLastError();
    case BP_FWD:
    case BP_BWD: {
#define QVA_BATCH_C(CB)                                                                  \
    case CB:                                                                             \
        return kind == BP_FWD ? launch_fwd_c<CB>(R, mode, nitems, s) : launch_bwd_c<CB>(R, mode, nitems, s);
        switch (col_bits) {
            QVA_BATCH_C(0)
            QVA_BATCH_C(3)
            QVA_BATCH_C(4)
            QVA_BATCH_C(5)
            QVA_BATCH_C(6)
            QVA_BATCH_C(7)
            QVA_BATCH_C(8)
            QVA_BATCH_C(9)
            QVA_BATCH_C(10)
            QVA_BATCH_C(11)
        default:
            return hipErrorInvalidValue;
        }
#undef QVA_BATCH_C
    }
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_sgd(const BatchInst* inst, int count, int max_p, double lr, hipStream_t s)
{
    (void)max_p;
    if (count <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(batch_sgd_kernel, dim3(count), dim3(64), 0, s, inst, lr);
    return hipGetLastError();
}

}  // namespace qva
