// qva_elementwise.hip -- initial state, standalone phase, expectation partials
// and the fixed-order final reduction.
#include "qva_internal.h"

namespace qva {
namespace {

constexpr int kEwThreads = 256;
constexpr int64_t kExpectChunk = 4096;   // amplitudes per partial (minimum)
constexpr int64_t kMaxPartials = 4096;   // partials of the standalone expectation

__global__ __launch_bounds__(kEwThreads) void init_uniform_kernel(double2* psi, int64_t N)
{
    const double a0 = 1.0 / sqrt((double)N);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < N; j += stride)
        st_nt(psi + j, make_double2(a0, 0.0));
}

// psi_j <- exp(-i gamma q_j) psi_j (paper Sec. 3, diagonal action)
__global__ __launch_bounds__(kEwThreads) void phase_kernel(double2* psi, const double* q, int64_t N,
                                                          double gamma)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < N; j += stride)
        st_nt(psi + j, cmul(ld_nt(psi + j), expmi(gamma * ld_nt(q + j))));
}

// Block b sums |psi_j|^2 q_j and |psi_j|^2 over its contiguous chunk.
__global__ __launch_bounds__(kEwThreads) void expect_partial_kernel(const double2* psi,
                                                                   const double* q, int64_t N,
                                                                   int64_t chunk, double2* partials)
{
    __shared__ double red[2 * (kEwThreads / 64)];
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < N ? lo + chunk : N;
    double f = 0.0, nr = 0.0;
    for (int64_t j = lo + threadIdx.x; j < hi; j += blockDim.x) {
        const double2 v = ld_nt(psi + j);
        const double a = v.x * v.x + v.y * v.y;
        f = fma(a, ld_nt(q + j), f);
        nr += a;
    }
    const double2 tot = block_sum2(f, nr, red);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = tot;
}

constexpr int kReduceThreads = 1024;

// One workgroup: thread i adds partials i, i + 1024, ... in order, then a
// fixed tree over the threads.  Same result for the same inputs every time.
__global__ __launch_bounds__(kReduceThreads) void final_reduce_kernel(const double2* partials,
                                                                     int64_t count, double* out_f,
                                                                     double* out_norm)
{
    __shared__ double red[2 * (kReduceThreads / 64)];
    double f = 0.0, nr = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += blockDim.x) {
        const double2 p = partials[i];
        f += p.x;
        nr += p.y;
    }
    const double2 tot = block_sum2(f, nr, red);
    if (threadIdx.x == 0) {
        out_f[0] = tot.x;
        if (out_norm)
            out_norm[0] = tot.y;
    }
}

unsigned ew_grid(int64_t N)
{
    int64_t g = (N + kEwThreads - 1) / kEwThreads;
    return (unsigned)(g < 65536 ? g : 65536);
}

}  // namespace

hipError_t launch_init_uniform(double2* psi, int64_t N, hipStream_t s)
{
    hipLaunchKernelGGL(init_uniform_kernel, dim3(ew_grid(N)), dim3(kEwThreads), 0, s, psi, N);
    return hipGetLastError();
}

hipError_t launch_phase(double2* psi, const double* q, int64_t N, double gamma, hipStream_t s)
{
    hipLaunchKernelGGL(phase_kernel, dim3(ew_grid(N)), dim3(kEwThreads), 0, s, psi, q, N, gamma);
    return hipGetLastError();
}

int64_t expect_partial_count(int64_t N)
{
    int64_t c = (N + kExpectChunk - 1) / kExpectChunk;
    return c < kMaxPartials ? c : kMaxPartials;
}

hipError_t launch_expect_partials(const double2* psi, const double* q, int64_t N,
                                  double2* partials, hipStream_t s)
{
    const int64_t count = expect_partial_count(N);
    const int64_t chunk = (N + count - 1) / count;
    hipLaunchKernelGGL(expect_partial_kernel, dim3((unsigned)count), dim3(kEwThreads), 0, s, psi,
                       q, N, chunk, partials);
    return hipGetLastError();
}

hipError_t launch_final_reduce(const double2* partials, int64_t count, double* out_f,
                               double* out_norm, hipStream_t s)
{
    hipLaunchKernelGGL(final_reduce_kernel, dim3(1), dim3(kReduceThreads), 0, s, partials, count,
                       out_f, out_norm);
    return hipGetLastError();
}

}  // namespace qva
