// Host check of the mixed-radix planner's LDS padding choice: for each N on
// the command line prints "N pad cost_unpadded cost_padded".
#include <cstdio>
#include <cstdlib>

#include "qva_mrplan.h"

int main(int argc, char** argv)
{
    for (int i = 1; i < argc; ++i) {
        const long long N = std::atoll(argv[i]);
        qva::MrGeom m{};
        if (!qva::mr_plan(N, m)) {
            std::printf("%lld none 0 0\n", N);
            continue;
        }
        std::printf("%lld %d %lld %lld\n", N, m.lds_pad, (long long)qva::mr_low_lds_cost(m, false),
                    (long long)qva::mr_low_lds_cost(m, true));
    }
    return 0;
}
