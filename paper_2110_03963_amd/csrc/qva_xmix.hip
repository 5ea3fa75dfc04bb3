// qva_xmix.hip -- hypercube-mixer (QAOA) passes over the state vector.
//
// The mixer exp(-i t sum_i X_i) is the product of commuting single-qubit
// rotations exp(-i t X_i) (paper Sec. 2.3.1, eq. mixing_qaoa with the
// hypercube W_X of its coupling figure).  Qubits are processed in groups: one
// pass loads a tile of 2^12 amplitudes whose index bits cover a whole group,
// applies every rotation of the group in registers (with LDS exchanges
// between register layouts), and stores the tile back in place.  A tile of
// the low group is 4096 contiguous amplitudes; a tile of a high group with g
// qubits starting at bit k is 2^g rows (stride 2^k) of 2^(12-g) contiguous
// amplitudes, so every global access is a run of >= 128 bytes.
//
// Elementwise work is fused into the passes: the initial state, the phase
// exp(-i gamma q_j) (eq. phase_shift_qaoa) or its extended form with one angle
// per Z-string term of Q (eq. phase_shift_qaoa_ex), and the expectation sum
// |psi_j|^2 q_j (eq. objective_generic).
#include "qva_passes.h"

namespace qva {
namespace {

using namespace tile;
using namespace passes;

template <int C, int FLAGS>
__global__ __launch_bounds__(kThreads, 2) void xpass_kernel(XPassParams P)
{
    __shared__ double2 lds[1 << kTileBits];
    __shared__ double red[2 * (kThreads / 64)];
    xpass_tile<C, FLAGS>(P, C == 3 ? paired_tile(blockIdx.x) : (int64_t)blockIdx.x, lds, red);
}

// ---------------------------------------------------------------------------
// Whole state in one workgroup (n <= 12): every layer in a single launch.
// ---------------------------------------------------------------------------
__device__ void small_mix(double2* s, int n, double t)
{
    double sn, c;
    sincos_red(t, &sn, &c);
    const int N = 1 << n;
    for (int i = 0; i < n; ++i) {
        const int bit = 1 << i;
        for (int m = threadIdx.x; m < N / 2; m += blockDim.x) {
            const int j = ((m >> i) << (i + 1)) | (m & (bit - 1));
            const double2 a = s[j], b = s[j | bit];
            s[j] = make_double2(c * a.x + sn * b.y, c * a.y - sn * b.x);
            s[j | bit] = make_double2(c * b.x + sn * a.y, c * b.y - sn * a.x);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kThreads) void small_kernel(SmallParams P)
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
        small_mix(s, P.n, P.t_val);
    if (P.flags & SM_EVOLVE) {
        for (int layer = 0; layer < P.p; ++layer) {
            if (P.n_terms > 0) {
                const double* row = P.gammas + (int64_t)layer * P.n_terms;
                for (int j = t; j < N; j += blockDim.x)
                    s[j] = cmul(s[j], expmi(zterm_angle(j, P.terms, P.n_terms, row)));
            } else {
                const double gam = P.gammas[layer];
                for (int j = t; j < N; j += blockDim.x)
                    s[j] = cmul(s[j], expmi(gam * P.q[j]));
            }
            __syncthreads();
            small_mix(s, P.n, P.ts[layer]);
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

}  // namespace

namespace {

// q in the order a pass of this group reads it when it applies the phase
// between two mixer applications (XP_PHASE_MID, layout last_layout<C>()):
// out[(tile << 12) + r * 256 + t] = q at element elem<L>(t, r) of the tile.
template <int C>
__global__ __launch_bounds__(kThreads) void qtile_kernel(const double* __restrict__ q, double* __restrict__ out,
                                                        int k)
{
    constexpr int L = last_layout<C>();
    const int t = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const TileMap g = tile_map(tile, k, C);
    double* o = out + (tile << kTileBits);
#pragma unroll
    for (int r = 0; r < kRegs; ++r)
        o[r * kThreads + t] = ld_nt(q + g(elem<L>(t, r)));
}

template <int C>
hipError_t launch_qtile_c(const double* q, double* out, int n, int k, hipStream_t s)
{
    const unsigned grid = (unsigned)(int64_t(1) << (n - kTileBits));
    hipLaunchKernelGGL((qtile_kernel<C>), dim3(grid), dim3(kThreads), 0, s, q, out, k);
    return hipGetLastError();
}

template <int C>
hipError_t launch_xpass_c(const XPassParams& P, unsigned grid, hipStream_t s)
{
    switch (P.flags) {
#define QVA_XPASS_MODE(F)                                                            \
    case F:                                                                          \
        hipLaunchKernelGGL((xpass_kernel<C, F>), dim3(grid), dim3(kThreads), 0, s, P); \
        break;
        QVA_XPASS_MODE(XMODE_FIRST)
        QVA_XPASS_MODE(XMODE_MIDDLE)
        QVA_XPASS_MODE(XMODE_BOUNDARY)
        QVA_XPASS_MODE(XMODE_LAST)
        QVA_XPASS_MODE(XMODE_LAST_STORE)
        QVA_XPASS_MODE(XMODE_MIX_SCALE)
        QVA_XPASS_MODE(XMODE_FIRST_Z)
        QVA_XPASS_MODE(XMODE_BOUNDARY_Z)
#undef QVA_XPASS_MODE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_xpass(const XPassParams& P, hipStream_t s)
{
    const unsigned grid = (unsigned)(int64_t(1) << (P.n - kTileBits));
    switch (P.col_bits) {
    case 0:
        return launch_xpass_c<0>(P, grid, s);
    case 3:
        return launch_xpass_c<3>(P, grid, s);
    case 4:
        return launch_xpass_c<4>(P, grid, s);
    case 5:
        return launch_xpass_c<5>(P, grid, s);
    case 6:
        return launch_xpass_c<6>(P, grid, s);
    case 7:
        return launch_xpass_c<7>(P, grid, s);
    case 8:
        return launch_xpass_c<8>(P, grid, s);
    case 9:
        return launch_xpass_c<9>(P, grid, s);
    case 10:
        return launch_xpass_c<10>(P, grid, s);
    case 11:
        return launch_xpass_c<11>(P, grid, s);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_qtile(const double* q, double* out, int n, int k, int col_bits, hipStream_t s)
{
    switch (col_bits) {
    case 0:
        return launch_qtile_c<0>(q, out, n, k, s);
    case 3:
        return launch_qtile_c<3>(q, out, n, k, s);
    case 4:
        return launch_qtile_c<4>(q, out, n, k, s);
    case 5:
        return launch_qtile_c<5>(q, out, n, k, s);
    case 6:
        return launch_qtile_c<6>(q, out, n, k, s);
    case 7:
        return launch_qtile_c<7>(q, out, n, k, s);
    case 8:
        return launch_qtile_c<8>(q, out, n, k, s);
    case 9:
        return launch_qtile_c<9>(q, out, n, k, s);
    case 10:
        return launch_qtile_c<10>(q, out, n, k, s);
    case 11:
        return launch_qtile_c<11>(q, out, n, k, s);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_small(const SmallParams& P, hipStream_t s)
{
    hipLaunchKernelGGL(small_kernel, dim3(1), dim3(kThreads), 0, s, P);
    return hipGetLastError();
}

}  // namespace qva
