// qva_ctroots.h -- the roots of unity W_R^j = exp(-2 pi i j / R) as
// compile-time constants (constexpr: usable on the host and in kernels).
//
// The angle 2 pi j / R is folded into [0, pi/4] with integer arithmetic on
// j / R: the quadrant k = floor(4 j / R) and the rest r = 4 j - k R, in units
// of pi / (2 R); above pi/4 the complement (R - r) swaps cos and sin.  cos and
// sin of x <= pi/4 are then summed from their Taylor series to x^27 (the
// truncation is below 1e-25).  x itself is rounded twice (r / R, then the
// product with pi/2), so the roots are within 3 ulp (2.4 measured over the
// radices 2..31), against about 1 for the table roots of the other radices.
#pragma once

namespace qva {

struct CtRoot {
    double c, s;  // cos and sin of 2 pi j / R
};

constexpr double ct_sin(double x)
{
    double t = x, s = x;
    for (int k = 1; k < 14; ++k) {
        t *= -x * x / ((double)(2 * k) * (double)(2 * k + 1));
        s += t;
    }
    return s;
}

constexpr double ct_cos(double x)
{
    double t = 1.0, s = 1.0;
    for (int k = 1; k < 14; ++k) {
        t *= -x * x / ((double)(2 * k - 1) * (double)(2 * k));
        s += t;
    }
    return s;
}

// cos and sin of 2 pi j / R, 0 <= j < R.
constexpr CtRoot ct_root(int j, int R)
{
    const int k = (4 * j) / R, r = 4 * j - k * R;
    constexpr double half_pi = 1.57079632679489661923132169163975;
    double c = 0.0, s = 0.0;
    if (2 * r <= R) {
        const double x = half_pi * ((double)r / (double)R);
        c = ct_cos(x);
        s = ct_sin(x);
    } else {
        const double x = half_pi * ((double)(R - r) / (double)R);
        c = ct_sin(x);
        s = ct_cos(x);
    }
    switch (k & 3) {
    case 0:
        return {c, s};
    case 1:
        return {-s, c};
    case 2:
        return {-c, -s};
    default:
        return {s, -c};
    }
}

// The R roots of one radix, built at compile time.
template <int R>
struct CtRoots {
    CtRoot v[R];
    constexpr CtRoots() : v()
    {
        for (int j = 0; j < R; ++j)
            v[j] = ct_root(j, R);
    }
};

}  // namespace qva
