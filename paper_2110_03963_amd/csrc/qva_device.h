// qva_device.h -- device helpers shared by the libqva kernels (gfx950, wave64).
//
// Amplitudes are double2 (x = re, y = im).  All arithmetic is IEEE double.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qva {

// Scheduling fence: the unrolled iterations of a register-heavy loop body
// (an inlined sincos, say) are not interleaved across it, which keeps their
// temporaries from being live all at once.
#define QVA_SCHED_FENCE() __builtin_amdgcn_sched_barrier(0)

// Issue fence: an empty asm statement with a memory clobber.  The compiler
// moves no memory access across it, so it fixes the order in which a tile's
// global reads are issued (left alone, the compiler regroups them and may
// place a pass's angle reads and their sine / cosine ahead of the tile's).
#define QVA_ISSUE_FENCE() asm volatile("" ::: "memory")

typedef double dvec2 __attribute__((ext_vector_type(2)));

// Streaming (non-temporal) 16-byte load/store of one amplitude: every
// amplitude is touched once per pass, so there is nothing to keep in cache.
__device__ __forceinline__ double2 ld_nt(const double2* p)
{
    dvec2 v = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(p));
    return make_double2(v.x, v.y);
}

__device__ __forceinline__ void st_nt(double2* p, double2 a)
{
    dvec2 v;
    v.x = a.x;
    v.y = a.y;
    __builtin_nontemporal_store(v, reinterpret_cast<dvec2*>(p));
}

__device__ __forceinline__ double ld_nt(const double* p) { return __builtin_nontemporal_load(p); }

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// sin and cos of x = j pi/2 + z, |z| <= pi/4 (j an integer-valued double,
// |j| < 2^51).  The Maclaurin series are summed through z^17 (sin) and z^16
// (cos); the first omitted terms are below 2.1e-18 on |z| <= pi/4.  The
// quadrant j mod 4 swaps the two and sets their signs.
__host__ __device__ __forceinline__ void sincos_quadrant(double z, double j, double* sn, double* cs)
{
    constexpr double kRound = 6755399441055744.0;  // 1.5 * 2^52
    const double z2 = z * z;
    // sin z = z + z^3 (-1/3! + z^2 (1/5! - ...)), coefficients (-1)^k / (2k+1)!
    double s = 1.0 / 355687428096000.0;
    s = fma(s, z2, -1.0 / 1307674368000.0);
    s = fma(s, z2, 1.0 / 6227020800.0);
    s = fma(s, z2, -1.0 / 39916800.0);
    s = fma(s, z2, 1.0 / 362880.0);
    s = fma(s, z2, -1.0 / 5040.0);
    s = fma(s, z2, 1.0 / 120.0);
    s = fma(s, z2, -1.0 / 6.0);
    const double sz = fma(z * z2, s, z);
    // cos z = 1 + z^2 (-1/2! + z^2 (1/4! - ...)), coefficients (-1)^k / (2k)!
    double c = 1.0 / 20922789888000.0;
    c = fma(c, z2, -1.0 / 87178291200.0);
    c = fma(c, z2, 1.0 / 479001600.0);
    c = fma(c, z2, -1.0 / 3628800.0);
    c = fma(c, z2, 1.0 / 40320.0);
    c = fma(c, z2, -1.0 / 720.0);
    c = fma(c, z2, 1.0 / 24.0);
    c = fma(c, z2, -0.5);
    const double cz = fma(c, z2, 1.0);
    // j + 1.5 * 2^52 holds j in its low mantissa bits; the low two are the
    // quadrant: (sin x, cos x) = (sz, cz), (cz, -sz), (-sz, -cz), (-cz, sz).
    const uint32_t q = (uint32_t)__builtin_bit_cast(uint64_t, j + kRound);
    const bool swap = q & 1u;
    const uint64_t s_neg = (uint64_t)((q >> 1) & 1u) << 63;
    const uint64_t c_neg = (uint64_t)(((q + 1u) >> 1) & 1u) << 63;
    *sn = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, swap ? cz : sz) ^ s_neg);
    *cs = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, swap ? sz : cz) ^ c_neg);
}

// sin x and cos x, with no library call.
//
// Reduction by quarter turns: 1/pi = kInvPiHi + kInvPiLo to about 2^-109
// relative, y = fl(x kInvPiHi), and e = x/pi - y from the exact product
// error (one fma) plus x kInvPiLo, so x = pi (y + e).  With j = rint(2y),
// t = y - j/2 is exact (|t| <= 1/4) and z = pi (t + e), evaluated with pi
// split in two doubles, lies in [-pi/4, pi/4] up to rounding; x = j pi/2 + z.
// The result is within about 1.5e-16 absolute of sin x, cos x for
// |x| < 2^41 (rounding of z and of the sums), checked on the host against
// long double.
__host__ __device__ __forceinline__ void sincos_red(double x, double* sn, double* cs)
{
    constexpr double kInvPiHi = 0.3183098861837907;      // 1/pi rounded to double
    constexpr double kInvPiLo = -1.9678676675182486e-17;  // 1/pi - kInvPiHi
    constexpr double kPiHi = 3.141592653589793;           // pi rounded to double
    constexpr double kPiLo = 1.2246467991473532e-16;      // pi - kPiHi
    const double y = x * kInvPiHi;
    const double e = fma(x, kInvPiLo, fma(x, kInvPiHi, -y));
    const double j = rint(y + y);
    const double t = fma(-0.5, j, y);
    const double z = fma(kPiHi, t, fma(kPiLo, t, kPiHi * e));
    sincos_quadrant(z, j, sn, cs);
}

// sin(pi y) and cos(pi y) (twiddle factors: y is a dyadic rational, so the
// reduction t = y - j/2 is exact and only z = pi t is rounded).
__host__ __device__ __forceinline__ void sincospi_red(double y, double* sn, double* cs)
{
    constexpr double kPiHi = 3.141592653589793;
    constexpr double kPiLo = 1.2246467991473532e-16;
    const double j = rint(y + y);
    const double t = fma(-0.5, j, y);
    const double z = fma(kPiHi, t, kPiLo * t);
    sincos_quadrant(z, j, sn, cs);
}

// exp(-i x) = (cos x, -sin x)
__host__ __device__ __forceinline__ double2 expmi(double x)
{
    double s, c;
    sincos_red(x, &s, &c);
    return make_double2(c, -s);
}

// A scalar parameter that is read from a device array when `ptr` is set,
// otherwise taken by value (host scalars of the primitive entry points).
struct Angle {
    const double* ptr;
    int idx;
    double val;
};

__device__ __forceinline__ double angle_value(const Angle& a) { return a.ptr ? a.ptr[a.idx] : a.val; }

// exp(-i t X) on one qubit pair, factored as sigma * B where B has a unit
// entry on the larger of |cos t|, |sin t|:
//   |cos t| >= |sin t|:  sigma = cos t,     B = [[1, -i tan t], [-i tan t, 1]]
//   otherwise:           sigma = -i sin t,  B = [[i cot t, 1], [1, i cot t]]
// B costs four FMAs per pair; the sigma of every qubit of a layer is collected
// into one complex factor sigma^n applied once (B / |sigma| is unitary up to a
// real factor, so the factoring does not change the conditioning).
struct MixCoef {
    double k;       // tan t or cot t
    bool tanform;
    double2 sigma;  // per-qubit scalar factor
};

__device__ __forceinline__ MixCoef mix_coef(double t)
{
    double s, c;
    sincos_red(t, &s, &c);
    MixCoef m;
    if (fabs(c) >= fabs(s)) {
        m.k = s / c;
        m.tanform = true;
        m.sigma = make_double2(c, 0.0);
    } else {
        m.k = c / s;
        m.tanform = false;
        m.sigma = make_double2(0.0, -s);
    }
    return m;
}

// sigma^n by repeated multiplication (n <= 34; identical in every thread).
__device__ __forceinline__ double2 cpow_int(double2 s, int n)
{
    double2 r = make_double2(1.0, 0.0);
    for (int i = 0; i < n; ++i)
        r = cmul(r, s);
    return r;
}

// B applied to the pair (a, b), tan form: a' = a - i k b, b' = b - i k a.
__device__ __forceinline__ void bfly_tan(double2& a, double2& b, double k)
{
    double2 a2, b2;
    a2.x = fma(k, b.y, a.x);
    a2.y = fma(-k, b.x, a.y);
    b2.x = fma(k, a.y, b.x);
    b2.y = fma(-k, a.x, b.y);
    a = a2;
    b = b2;
}

// B applied to the pair (a, b), cot form: a' = i k a + b, b' = a + i k b.
__device__ __forceinline__ void bfly_cot(double2& a, double2& b, double k)
{
    double2 a2, b2;
    a2.x = fma(-k, a.y, b.x);
    a2.y = fma(k, a.x, b.y);
    b2.x = fma(-k, b.y, a.x);
    b2.y = fma(k, b.x, a.y);
    a = a2;
    b = b2;
}

// Sum over the 64 lanes of a wave (butterfly shuffles; same order in every
// wave, so the result is deterministic).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic block sum of two doubles; every thread gets the result.
// `red` must hold 2 * (blockDim.x / 64) doubles of shared memory.
__device__ __forceinline__ double2 block_sum2(double a, double b, double* red)
{
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) {
        red[2 * wid] = a;
        red[2 * wid + 1] = b;
    }
    __syncthreads();
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < nw; ++w) {
        sa += red[2 * w];
        sb += red[2 * w + 1];
    }
    return make_double2(sa, sb);
}

}  // namespace qva
