// Host build of the kernels' sincos_red / expmi, compared with long double
// sinl / cosl.  Prints one line per argument range: name, count, max |error|
// of sin, of cos, and of exp(-i x) (complex modulus).
#include "qva_device.h"

#include <cmath>
#include <cstdio>
#include <random>

static void check(const char* name, const double* xs, int n)
{
    double es = 0.0, ec = 0.0, ee = 0.0;
    for (int i = 0; i < n; ++i) {
        const double x = xs[i];
        double s, c;
        qva::sincos_red(x, &s, &c);
        const long double rs = sinl((long double)x), rc = cosl((long double)x);
        es = fmax(es, (double)fabsl((long double)s - rs));
        ec = fmax(ec, (double)fabsl((long double)c - rc));
        const double2 e = qva::expmi(x);
        const long double dr = (long double)e.x - rc, di = (long double)e.y + rs;
        ee = fmax(ee, (double)sqrtl(dr * dr + di * di));
    }
    std::printf("%s %d %.3e %.3e %.3e\n", name, n, es, ec, ee);
}

int main()
{
    std::mt19937_64 rng(20211007);
    const int n = 400000;
    static double xs[400000];
    const double spans[] = {1.0, 4.0, 100.0, 1e4, 1e7, 1e10, 1e12};
    for (double span : spans) {
        std::uniform_real_distribution<double> u(-span, span);
        for (int i = 0; i < n; ++i)
            xs[i] = u(rng);
        char name[64];
        std::snprintf(name, sizeof name, "uniform_%g", span);
        check(name, xs, n);
    }
    // next to multiples of pi/2 (where the reduced angle is smallest)
    std::uniform_int_distribution<long long> k(-1000000, 1000000);
    std::uniform_int_distribution<int> d(-4, 4);
    for (int i = 0; i < n; ++i) {
        double x = (double)((long double)k(rng) * 1.5707963267948966192313216916397514L);
        for (int s = d(rng); s != 0; s += (s > 0 ? -1 : 1))
            x = std::nextafter(x, s > 0 ? INFINITY : -INFINITY);
        xs[i] = x;
    }
    check("near_half_pi_multiples", xs, n);
    // tiny and exact cases
    const double special[] = {0.0, -0.0, 1e-300, -1e-300, 1e-8, 0.5, 1.5707963267948966,
                              3.141592653589793, -3.141592653589793, 6.283185307179586};
    check("special", special, (int)(sizeof special / sizeof special[0]));
    return 0;
}
