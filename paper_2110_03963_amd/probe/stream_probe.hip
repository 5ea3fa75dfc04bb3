// stream_probe.hip -- the attainable HBM rate of the tile passes' access
// pattern, without their arithmetic.
//
// Each block streams one tile in place over 2^n amplitudes: 4096 elements =
// 2^C contiguous amplitudes (16 << C bytes) in each of 2^(12-C) rows at a
// stride of 2^k amplitudes, exactly the element -> index map of the tile
// passes; it reads psi and q (24 bytes per amplitude) and writes psi back
// (16), the traffic of a hypercube boundary pass.  With -2 it streams two
// vectors, reading psi, chi and q and writing psi and chi: 72 bytes per
// amplitude, the traffic of a backward boundary pass.  Prints one JSON object
// per (C, k): the time of one pass over the register and its rate.
//
// usage: stream_probe [-2] [n] [C k]...   (default n = 28 and a row-length sweep)
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#define CHECK(x)                                                                    \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess) {                                                     \
            std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 1;                                                               \
        }                                                                           \
    } while (0)

// Workgroup -> tile as in the passes: with 3 column bits neighbouring tiles
// share the 128-byte lines of q, so workgroups b and b + 8 (back to back on
// one XCD) take the two tiles of a pair (grids of at least 16 workgroups).
__device__ __forceinline__ long tile_of(long b, int C)
{
    if (C != 3 || (gridDim.x & 15))
        return b;
    return (b & ~15L) | ((b & 7) << 1) | ((b >> 3) & 1);
}

// Two vectors: each register's psi, chi and q are requested together.
__global__ __launch_bounds__(256) void tile_stream2(double2* psi, double2* chi, const double* q, int C, int k)
{
    constexpr int R = 16;
    const long tile = tile_of(blockIdx.x, C);
    const int lobits = k - C;
    const long base = ((tile & ((1L << lobits) - 1)) << C) | ((tile >> lobits) << (k + 12 - C));
    const int t = threadIdx.x;
    double2 v[R], w[R];
    double qq[R];
    long at[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = t | (r << 8);
        at[r] = base + (e & ((1 << C) - 1)) + ((long)(e >> C) << k);
        v[r].x = __builtin_nontemporal_load(&psi[at[r]].x);
        v[r].y = __builtin_nontemporal_load(&psi[at[r]].y);
        w[r].x = __builtin_nontemporal_load(&chi[at[r]].x);
        w[r].y = __builtin_nontemporal_load(&chi[at[r]].y);
        qq[r] = __builtin_nontemporal_load(q + at[r]);
        asm volatile("" ::: "memory");
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        __builtin_nontemporal_store(v[r].x * qq[r], &psi[at[r]].x);
        __builtin_nontemporal_store(v[r].y * qq[r], &psi[at[r]].y);
        __builtin_nontemporal_store(w[r].x * qq[r], &chi[at[r]].x);
        __builtin_nontemporal_store(w[r].y * qq[r], &chi[at[r]].y);
    }
}

__global__ __launch_bounds__(256) void tile_stream(double2* psi, const double* q, int C, int k)
{
    constexpr int R = 16;
    const long tile = tile_of(blockIdx.x, C);
    const int lobits = k - C;
    const long base = ((tile & ((1L << lobits) - 1)) << C) | ((tile >> lobits) << (k + 12 - C));
    const int t = threadIdx.x;
    double2 v[R];
    double qq[R];
    long at[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = t | (r << 8);
        at[r] = base + (e & ((1 << C) - 1)) + ((long)(e >> C) << k);
        v[r].x = __builtin_nontemporal_load(&psi[at[r]].x);
        v[r].y = __builtin_nontemporal_load(&psi[at[r]].y);
        qq[r] = __builtin_nontemporal_load(q + at[r]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        __builtin_nontemporal_store(v[r].x * qq[r], &psi[at[r]].x);
        __builtin_nontemporal_store(v[r].y * qq[r], &psi[at[r]].y);
    }
}

int main(int argc, char** argv)
{
    int a0 = 1;
    const bool two = argc > 1 && std::string(argv[1]) == "-2";
    if (two)
        ++a0;
    const int n = argc > a0 ? std::atoi(argv[a0]) : 28;
    if (n < 13 || n > (two ? 30 : 31)) {
        std::fprintf(stderr, "n must be in 13..%d\n", two ? 30 : 31);
        return 2;
    }
    std::vector<std::pair<int, int>> cases;
    for (int i = a0 + 1; i + 1 < argc; i += 2)
        cases.push_back({std::atoi(argv[i]), std::atoi(argv[i + 1])});
    if (cases.empty())
        for (int C = 3; C <= 9; ++C) {
            cases.push_back({C, 12});
            cases.push_back({C, n - (12 - C)});
        }
    for (const auto& c : cases)
        if (c.first < 3 || c.first > 11 || c.second < c.first || c.second + 12 - c.first > n) {
            std::fprintf(stderr, "bad tile: C=%d k=%d\n", c.first, c.second);
            return 2;
        }
    const size_t N = (size_t)1 << n;
    double2* psi;
    double2* chi = nullptr;
    double* q;
    CHECK(hipMalloc(&psi, N * sizeof(double2)));
    CHECK(hipMalloc(&q, N * sizeof(double)));
    CHECK(hipMemset(psi, 0, N * sizeof(double2)));
    CHECK(hipMemset(q, 0, N * sizeof(double)));
    if (two) {
        CHECK(hipMalloc(&chi, N * sizeof(double2)));
        CHECK(hipMemset(chi, 0, N * sizeof(double2)));
    }
    const double bytes_per_amp = two ? 72.0 : 40.0;
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const unsigned grid = (unsigned)(N >> 12);
    auto launch = [&](int C, int k) {
        if (two)
            tile_stream2<<<grid, 256>>>(psi, chi, q, C, k);
        else
            tile_stream<<<grid, 256>>>(psi, q, C, k);
    };
    for (const auto& c : cases) {
        for (int w = 0; w < 2; ++w)
            launch(c.first, c.second);
        CHECK(hipGetLastError());
        CHECK(hipDeviceSynchronize());
        const int reps = 10;
        CHECK(hipEventRecord(e0));
        for (int r = 0; r < reps; ++r)
            launch(c.first, c.second);
        CHECK(hipEventRecord(e1));
        CHECK(hipEventSynchronize(e1));
        float ms = 0.0f;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        ms /= reps;
        std::printf("{\"n\": %d, \"C\": %d, \"k\": %d, \"row_bytes\": %d, \"bytes_per_amp\": %.0f, \"ms\": %.4f, "
                    "\"GBps\": %.1f}\n",
                    n, c.first, c.second, 16 << c.first, bytes_per_amp, ms,
                    bytes_per_amp * (double)N / (ms * 1e-3) / 1e9);
        std::fflush(stdout);
    }
    CHECK(hipFree(psi));
    CHECK(hipFree(q));
    if (chi)
        CHECK(hipFree(chi));
    return 0;
}
