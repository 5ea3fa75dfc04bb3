// Host check of the compile-time roots of unity (qva_ctroots.h): prints the
// largest error, in ulps of the exact value, against long-double cos and sin
// over the radices the mixed-radix passes use, then the table's deviation.
#include <cmath>
#include <cstdio>

#include "qva_ctroots.h"

// evaluated at compile time
static_assert(qva::ct_root(0, 31).c == 1.0 && qva::ct_root(0, 31).s == 0.0, "W^0 = 1");
static_assert(qva::ct_root(2, 4).c == -1.0 && qva::ct_root(2, 4).s == 0.0, "W_4^2 = -1");
constexpr qva::CtRoots<29> kRoots29{};

int main()
{
    const int radices[] = {2, 3, 4, 5, 7, 8, 11, 13, 16, 17, 19, 23, 29, 31};
    const long double pi = 3.141592653589793238462643383279502884L;
    // largest error in units of the last place of the exact value
    auto ulps = [](double got, long double exact) {
        const long double m = std::fabs(exact);
        if (m < 1e-15L)  // an exact zero (cos of a right angle): long double pi leaves ~1e-20
            return std::fabs((long double)got - exact) < 1e-18L ? 0.0 : 1e9;
        const long double ulp = std::ldexp(1.0L, std::ilogb((double)m) - 52);
        return (double)(std::fabs((long double)got - exact) / ulp);
    };
    double worst = 0.0;
    for (int R : radices)
        for (int j = 0; j < R; ++j) {
            const qva::CtRoot w = qva::ct_root(j, R);
            const long double a = 2.0L * pi * (long double)j / (long double)R;
            worst = std::fmax(worst, std::fmax(ulps(w.c, std::cos(a)), ulps(w.s, std::sin(a))));
        }
    double table = 0.0;
    for (int j = 0; j < 29; ++j)
        table = std::fmax(table, std::fabs(kRoots29.v[j].c - qva::ct_root(j, 29).c));
    std::printf("%.3e %.3e\n", worst, table);
    return 0;
}
