// Host build of the parity-mixer planner (xy_layer_plan): for rings and random
// pair lists it checks that every pair is applied exactly once, inside its
// pass's tile, at most kMaxXyOps per pass, and never before an earlier pair
// that shares a qubit with it.  Prints "ok <cases> <passes>" or the first
// failure.
#include "qva_plan.h"

#include <cstdio>
#include <random>
#include <utility>
#include <vector>

using Pairs = std::vector<std::pair<int, int>>;

static int qubit_of(const qva::XyGroup& g, int n, int eb)
{
    if (n <= qva::kTileBits || (g.C == 0 && g.k == 0) || eb < g.C)
        return eb;
    return g.k + eb - g.C;
}

static bool check(int n, const Pairs& pairs, int* passes, const char* what)
{
    const std::vector<qva::XyLayerPass> plan = qva::xy_layer_plan(n, pairs);
    if (plan.empty()) {
        std::printf("FAIL %s n=%d: empty plan\n", what, n);
        return false;
    }
    *passes += (int)plan.size();
    // execution order of the original indices (repeated pairs matched in order)
    std::vector<int> used(pairs.size(), 0), order;
    for (const auto& ps : plan) {
        if ((int)ps.ops.size() > qva::kMaxXyOps) {
            std::printf("FAIL %s n=%d: %zu ops in a pass\n", what, n, ps.ops.size());
            return false;
        }
        for (const auto& op : ps.ops) {
            const int a = qubit_of(ps.g, n, op.first), b = qubit_of(ps.g, n, op.second);
            if (!ps.g.holds(a) || !ps.g.holds(b) || ps.g.elem_bit(a) != op.first || ps.g.elem_bit(b) != op.second) {
                std::printf("FAIL %s n=%d: pair (%d,%d) outside its tile\n", what, n, a, b);
                return false;
            }
            int idx = -1;
            for (int i = 0; i < (int)pairs.size(); ++i)
                if (!used[i] && pairs[i].first == a && pairs[i].second == b) {
                    idx = i;
                    break;
                }
            if (idx < 0) {
                std::printf("FAIL %s n=%d: pair (%d,%d) not in the list or applied twice\n", what, n, a, b);
                return false;
            }
            used[idx] = 1;
            order.push_back(idx);
        }
    }
    if (order.size() != pairs.size()) {
        std::printf("FAIL %s n=%d: %zu of %zu pairs applied\n", what, n, order.size(), pairs.size());
        return false;
    }
    std::vector<int> pos(pairs.size());
    for (int i = 0; i < (int)order.size(); ++i)
        pos[order[i]] = i;
    for (int i = 0; i < (int)pairs.size(); ++i)
        for (int j = i + 1; j < (int)pairs.size(); ++j) {
            const bool share = pairs[i].first == pairs[j].first || pairs[i].first == pairs[j].second ||
                               pairs[i].second == pairs[j].first || pairs[i].second == pairs[j].second;
            if (share && pos[i] > pos[j]) {
                std::printf("FAIL %s n=%d: pair %d applied after later pair %d\n", what, n, i, j);
                return false;
            }
        }
    return true;
}

static Pairs ring(const std::vector<int>& r)
{
    const int m = (int)r.size();
    Pairs p;
    for (int a = 1; a <= m - 1; a += 2)
        p.push_back({r[a - 1], r[a]});
    for (int a = 2; a <= m; a += 2)
        p.push_back({r[a - 1], r[a % m]});
    if (m % 2 == 1 && m >= 3)
        p.push_back({r[m - 1], r[0]});
    return p;
}

int main()
{
    int cases = 0, passes = 0;
    std::mt19937 rng(7);
    for (int n = 2; n <= 33; ++n) {
        std::vector<int> all, even, odd;
        for (int i = 0; i < n; ++i) {
            all.push_back(i);
            (i % 2 ? odd : even).push_back(i);
        }
        if (!check(n, ring(all), &passes, "ring"))
            return 1;
        Pairs two = ring(even);
        for (const auto& pr : ring(odd))
            two.push_back(pr);
        if (!check(n, two, &passes, "two interleaved rings"))
            return 1;
        cases += 2;
        for (int rep = 0; rep < 20; ++rep) {
            Pairs r;
            const int cnt = 1 + (int)(rng() % 120);
            while ((int)r.size() < cnt) {
                const int a = (int)(rng() % n), b = (int)(rng() % n);
                if (a != b && qva::xy_pair_fits(n, a, b))
                    r.push_back({a, b});
            }
            if (!check(n, r, &passes, "random"))
                return 1;
            ++cases;
        }
    }
    std::printf("ok %d %d\n", cases, passes);
    return 0;
}
