// qva_complete.hip -- QWOA mixer of the complete graph in closed form.
//
// The complete graph on N vertices has adjacency W = J - I (J the all-ones
// matrix); its circulant eigenvalues (paper Sec. 3) are N - 1 once and -1
// (N - 1 times).  Because J^2 = N J,
//   exp(-i t W) = e^{i t} exp(-i t J) = e^{i t} (I + c J),  c = (e^{-i t N} - 1) / N,
// so exp(-i t W) psi = e^{i t} (psi + c S 1) with S = sum_j psi_j: one global
// sum and one elementwise update, instead of two Fourier transforms.
//
// An evolution keeps phi_k = U_Q(gamma_k) psi_{k-1} in memory.  One pass per
// layer reads phi_k and q, forms psi_k = e^{i t_k} (phi_k + c_k S_k), applies
// the phase of layer k+1 and writes phi_{k+1} together with per-block sums of
// it; a fixed-order reduction of those sums (final_reduce) gives S_{k+1},
// which stays in device memory for the next pass.  The first pass generates
// psi_0 = N^{-1/2} and the last one reduces <Q> instead of writing.
//
// Any N >= 1 works (the solution count of a constrained problem need not be a
// power of two): blocks hold kCompleteChunk amplitudes and the last block's
// lanes beyond N load zeros, add nothing to the sums and store nothing.  For
// N = 2^n, t N is exact; otherwise it is rounded once.
#include "qva_internal.h"

namespace qva {
namespace {

constexpr int kRegsC = kCompleteChunk / kThreads;

// Amplitude r of a thread is in range (the last block may be partial).
__device__ __forceinline__ bool in_range(int64_t base, int r, int64_t N) { return base + r * kThreads < N; }

template <int FLAGS>
__global__ __launch_bounds__(kThreads) void complete_kernel(CompleteParams P)
{
    __shared__ double red[2 * (kThreads / 64)];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kCompleteChunk + t;
    const double Nd = (double)P.N;

    double2 v[kRegsC];
    double qq[kRegsC];
    if constexpr (FLAGS & CP_INIT) {
        const double a0 = 1.0 / sqrt(Nd);
#pragma unroll
        for (int r = 0; r < kRegsC; ++r)
            v[r] = in_range(base, r, P.N) ? make_double2(a0, 0.0) : make_double2(0.0, 0.0);
    } else {
#pragma unroll
        for (int r = 0; r < kRegsC; ++r)
            v[r] = in_range(base, r, P.N) ? ld_nt(P.psi + base + r * kThreads) : make_double2(0.0, 0.0);
    }
    if constexpr (FLAGS & (CP_PHASE | CP_EXPECT)) {
#pragma unroll
        for (int r = 0; r < kRegsC; ++r)
            qq[r] = in_range(base, r, P.N) ? ld_nt(P.q + base + r * kThreads) : 0.0;
    }
    if constexpr (FLAGS & CP_MIX) {
        const double tm = P.ts ? P.ts[P.mix_layer] : P.t_val;
        const double2 eit = expmi(-tm);   // e^{i t}
        const double2 e = expmi(tm * Nd);  // e^{-i t N}
        const double invN = 1.0 / Nd;
        const double2 c = make_double2((e.x - 1.0) * invN, e.y * invN);
        const double2 d = cmul(eit, cmul(c, *P.sum_in));  // e^{it} c S, the same for every j
#pragma unroll
        for (int r = 0; r < kRegsC; ++r) {
            const double2 w = cmul(eit, v[r]);
            v[r] = in_range(base, r, P.N) ? make_double2(w.x + d.x, w.y + d.y) : make_double2(0.0, 0.0);
        }
    }
    if constexpr (FLAGS & CP_PHASE) {
        const double gamma = P.gammas[P.phase_layer];
#pragma unroll
        for (int r = 0; r < kRegsC; ++r) {
            v[r] = cmul(v[r], expmi(gamma * qq[r]));
            QVA_SCHED_FENCE();
        }
    }
    if constexpr (FLAGS & CP_SUM) {
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int r = 0; r < kRegsC; ++r) {
            sx += v[r].x;
            sy += v[r].y;
        }
        const double2 tot = block_sum2(sx, sy, red);
        if (t == 0)
            P.partials[blockIdx.x] = tot;
    }
    if constexpr (FLAGS & CP_EXPECT) {
        double f = 0.0, nr = 0.0;
#pragma unroll
        for (int r = 0; r < kRegsC; ++r) {
            const double a = v[r].x * v[r].x + v[r].y * v[r].y;
            f = fma(a, qq[r], f);
            nr += a;
        }
        const double2 tot = block_sum2(f, nr, red);
        if (t == 0)
            P.partials[blockIdx.x] = tot;
    }
    if constexpr (FLAGS & CP_STORE) {
#pragma unroll
        for (int r = 0; r < kRegsC; ++r)
            if (in_range(base, r, P.N))
                st_nt(P.psi + base + r * kThreads, v[r]);
    }
}

// ---------------------------------------------------------------- adjoint
// Backward walk (phi, chi) from (psi_p, Q psi_p), layer by layer:
//   dt_k     = 2 Im <chi|W|phi> = 2 (Im(conj(S_chi) S_phi) - Im<chi|phi>) on psi_k,
//   phi, chi <- exp(+i t_k W) (.) = e^{-i t_k} ((.) + conj(c_k) S),
//   dgamma_k = 2 Im <chi|Q|phi> on phi_k,
//   phi, chi <- exp(+i gamma_k q) (.).
// Every pass that writes also leaves per-block parts of the next layer's
// sums; complete_gsum reduces them in a fixed order.
template <int MODE>
__global__ __launch_bounds__(kThreads) void complete_grad_kernel(CompleteGradParams P)
{
    __shared__ double red[kCompleteParts * (kThreads / 64)];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kCompleteChunk + t;
    const double Nd = (double)P.N;
    const double invN = 1.0 / Nd;
    const double tm = P.ts[P.layer];

    // lanes beyond N hold zeros, which every update below keeps at zero
    // (no term is added to them) and which add nothing to any sum
    double2 a[kRegsC], b[kRegsC];
    double qq[kRegsC];
#pragma unroll
    for (int r = 0; r < kRegsC; ++r) {
        const bool in = in_range(base, r, P.N);
        a[r] = in ? ld_nt(P.phi + base + r * kThreads) : make_double2(0.0, 0.0);
        qq[r] = in ? ld_nt(P.q + base + r * kThreads) : 0.0;
    }
    if constexpr (MODE != GCMODE_TURN) {
#pragma unroll
        for (int r = 0; r < kRegsC; ++r)
            b[r] = in_range(base, r, P.N) ? ld_nt(P.chi + base + r * kThreads) : make_double2(0.0, 0.0);
    }
    double parts[kCompleteParts] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if constexpr (MODE == GCMODE_TURN) {
        // psi_p = e^{it} (phi + c S), c = (e^{-itN} - 1)/N; chi = Q psi_p
        const double2 eit = expmi(-tm);
        const double2 e = expmi(tm * Nd);
        const double2 c = make_double2((e.x - 1.0) * invN, e.y * invN);
        const double2 d = cmul(eit, cmul(c, P.sums_in[0]));
        double f = 0.0, nr = 0.0;
#pragma unroll
        for (int r = 0; r < kRegsC; ++r) {
            const double2 w = cmul(eit, a[r]);
            a[r] = in_range(base, r, P.N) ? make_double2(w.x + d.x, w.y + d.y) : make_double2(0.0, 0.0);
            b[r] = make_double2(qq[r] * a[r].x, qq[r] * a[r].y);
            const double pr = a[r].x * a[r].x + a[r].y * a[r].y;
            f = fma(pr, qq[r], f);
            nr += pr;
        }
        const double2 tot = block_sum2(f, nr, red);
        if (t == 0)
            P.fpart[blockIdx.x] = tot;
    } else {
        // inverse mixer: e^{-it} (x + conj(c) S_x)
        const double2 emit = expmi(tm);                                  // e^{-it}
        const double2 e = expmi(-tm * Nd);                               // e^{+itN}
        const double2 cb = make_double2((e.x - 1.0) * invN, e.y * invN);  // conj(c)
        const double2 da = cmul(emit, cmul(cb, P.sums_in[0]));
        const double2 db = cmul(emit, cmul(cb, P.sums_in[1]));
        const double gamma = P.gammas[P.layer];
        double gq = 0.0;
#pragma unroll
        for (int r = 0; r < kRegsC; ++r) {
            const bool in = in_range(base, r, P.N);
            double2 w = cmul(emit, a[r]);
            a[r] = in ? make_double2(w.x + da.x, w.y + da.y) : make_double2(0.0, 0.0);
            w = cmul(emit, b[r]);
            b[r] = in ? make_double2(w.x + db.x, w.y + db.y) : make_double2(0.0, 0.0);
            gq = fma(qq[r], b[r].x * a[r].y - b[r].y * a[r].x, gq);
            const double2 ph = expmi(-gamma * qq[r]);  // exp(+i gamma q)
            a[r] = cmul(a[r], ph);
            b[r] = cmul(b[r], ph);
            QVA_SCHED_FENCE();
        }
        parts[5] = gq;
    }
    if constexpr (MODE != GCMODE_BACK_LAST) {
#pragma unroll
        for (int r = 0; r < kRegsC; ++r) {
            parts[0] += a[r].x;
            parts[1] += a[r].y;
            parts[2] += b[r].x;
            parts[3] += b[r].y;
            parts[4] = fma(b[r].x, a[r].y, fma(-b[r].y, a[r].x, parts[4]));
        }
    }
    // deterministic block sum of the parts (waves, then the block's waves in
    // order); the barrier keeps these writes after every read of `red` above
    const int lane = t & 63, wid = t >> 6;
#pragma unroll
    for (int i = 0; i < kCompleteParts; ++i)
        parts[i] = wave_sum(parts[i]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < kCompleteParts; ++i)
            red[kCompleteParts * wid + i] = parts[i];
    }
    __syncthreads();
    if (t < kCompleteParts) {
        double s = 0.0;
        for (int w = 0; w < kThreads / 64; ++w)
            s += red[kCompleteParts * w + t];
        P.part[(int64_t)blockIdx.x * kCompleteParts + t] = s;
    }
    if constexpr (MODE != GCMODE_BACK_LAST) {
#pragma unroll
        for (int r = 0; r < kRegsC; ++r) {
            if (in_range(base, r, P.N)) {
                st_nt(P.phi + base + r * kThreads, a[r]);
                st_nt(P.chi + base + r * kThreads, b[r]);
            }
        }
    }
}

constexpr int kGsumThreads = 1024;

// One workgroup: component i summed as thread j adds blocks j, j + 1024, ...
// in order, then a fixed tree over the threads.
__global__ __launch_bounds__(kGsumThreads) void complete_gsum_kernel(const double* part, int64_t blocks,
                                                                     double2* state_out, double* sums,
                                                                     int t_slot, int g_slot)
{
    __shared__ double red[kCompleteParts * (kGsumThreads / 64)];
    __shared__ double tot[kCompleteParts];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    double v[kCompleteParts] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t i = t; i < blocks; i += kGsumThreads) {
#pragma unroll
        for (int c = 0; c < kCompleteParts; ++c)
            v[c] += part[i * kCompleteParts + c];
    }
#pragma unroll
    for (int c = 0; c < kCompleteParts; ++c)
        v[c] = wave_sum(v[c]);
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < kCompleteParts; ++c)
            red[kCompleteParts * wid + c] = v[c];
    }
    __syncthreads();
    if (t < kCompleteParts) {
        double s = 0.0;
        for (int w = 0; w < kGsumThreads / 64; ++w)
            s += red[kCompleteParts * w + t];
        tot[t] = s;
    }
    __syncthreads();
    if (t == 0) {
        const double2 sa = make_double2(tot[0], tot[1]), sb = make_double2(tot[2], tot[3]);
        state_out[0] = sa;
        state_out[1] = sb;
        if (t_slot >= 0)
            sums[t_slot] = (sb.x * sa.y - sb.y * sa.x) - tot[4];
        if (g_slot >= 0)
            sums[g_slot] = tot[5];
    }
}

}  // namespace

hipError_t launch_complete_grad(const CompleteGradParams& P, hipStream_t s)
{
    if (P.N < 1)
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)((P.N + kCompleteChunk - 1) / kCompleteChunk));
    switch (P.flags) {
    case GCMODE_TURN:
        hipLaunchKernelGGL(complete_grad_kernel<GCMODE_TURN>, grid, dim3(kThreads), 0, s, P);
        break;
    case GCMODE_BACK:
        hipLaunchKernelGGL(complete_grad_kernel<GCMODE_BACK>, grid, dim3(kThreads), 0, s, P);
        break;
    case GCMODE_BACK_LAST:
        hipLaunchKernelGGL(complete_grad_kernel<GCMODE_BACK_LAST>, grid, dim3(kThreads), 0, s, P);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_complete_gsum(const double* part, int64_t blocks, double2* state_out, double* sums,
                                int t_slot, int g_slot, hipStream_t s)
{
    hipLaunchKernelGGL(complete_gsum_kernel, dim3(1), dim3(kGsumThreads), 0, s, part, blocks, state_out,
                       sums, t_slot, g_slot);
    return hipGetLastError();
}

hipError_t launch_complete(const CompleteParams& P, hipStream_t s)
{
    if (P.N < 1)
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)((P.N + kCompleteChunk - 1) / kCompleteChunk));
    switch (P.flags) {
    case CPMODE_FIRST:
        hipLaunchKernelGGL(complete_kernel<CPMODE_FIRST>, grid, dim3(kThreads), 0, s, P);
        break;
    case CPMODE_LAYER:
        hipLaunchKernelGGL(complete_kernel<CPMODE_LAYER>, grid, dim3(kThreads), 0, s, P);
        break;
    case CPMODE_SUM:
        hipLaunchKernelGGL(complete_kernel<CPMODE_SUM>, grid, dim3(kThreads), 0, s, P);
        break;
    case CPMODE_MIX:
        hipLaunchKernelGGL(complete_kernel<CPMODE_MIX>, grid, dim3(kThreads), 0, s, P);
        break;
    case CPMODE_LAST:
        hipLaunchKernelGGL(complete_kernel<CPMODE_LAST>, grid, dim3(kThreads), 0, s, P);
        break;
    case CPMODE_LAST_STORE:
        hipLaunchKernelGGL(complete_kernel<CPMODE_LAST_STORE>, grid, dim3(kThreads), 0, s, P);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace qva
