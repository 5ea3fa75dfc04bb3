// qva_plan.h -- host-side pass planning for the fused evolution.
//
// The hypercube mixer factorises over qubits and its factors commute, so a
// layer may process its qubit groups in any order.  Layers alternate the
// order (0..P-1, then P-1..0, ...): the last group of layer k is then the
// first group of layer k+1, and one pass applies [group of layer k] ->
// [phase of layer k+1] -> [same group of layer k+1].  With P groups and p
// layers this gives p(P-1)+1 passes instead of pP passes plus p phase sweeps.
#pragma once

#include <vector>

#include "qva_internal.h"

namespace qva {

struct XGroup {
    int k;        // first qubit of the group
    int bits;     // number of qubits in the group
    int col_bits; // contiguous low index bits per tile row (0 for the low group)
};

// Group 0 is qubits [0, 12) (contiguous tiles); the remaining qubits are split
// into the fewest groups of at most kMaxHighBits, sizes as equal as possible.
inline std::vector<XGroup> x_groups(int n)
{
    std::vector<XGroup> g;
    if (n <= kTileBits) {
        g.push_back({0, n, 0});
        return g;
    }
    g.push_back({0, kTileBits, 0});
    const int rem = n - kTileBits;
    const int nh = (rem + kMaxHighBits - 1) / kMaxHighBits;
    const int base = rem / nh, extra = rem % nh;
    int k = kTileBits;
    for (int i = 0; i < nh; ++i) {
        const int b = base + (i < extra ? 1 : 0);
        g.push_back({k, b, kTileBits - b});
        k += b;
    }
    return g;
}

struct XPass {
    int group;
    int flags;        // XP_* flags
    int layer1;       // layer of the first mixer application
    int layer2;       // layer of the second mixer application, or -1
    int phase_layer;  // layer whose phase is applied, or -1
};

// Pass list of a p-layer evolution (p >= 1) over P >= 2 groups.  The first
// pass generates psi_0 and applies the first phase; the last pass reduces
// <Q> and applies the last layer's scalar factor.
inline std::vector<XPass> x_evolve_plan(int P, int p, bool store)
{
    std::vector<std::pair<int, int>> seq;  // (group, layer) in application order
    for (int L = 0; L < p; ++L)
        for (int i = 0; i < P; ++i)
            seq.push_back({(L % 2 == 0) ? i : P - 1 - i, L});
    std::vector<XPass> plan;
    plan.push_back({seq[0].first, XP_INIT | XP_PHASE_PRE | XP_MIX1, 0, -1, 0});
    size_t i = 1;
    while (i < seq.size()) {
        const int g = seq[i].first, L = seq[i].second;
        if (i + 1 < seq.size() && seq[i + 1].first == g) {
            plan.push_back({g, XP_MIX1 | XP_PHASE_MID | XP_MIX2, L, L + 1, L + 1});
            i += 2;
        } else {
            plan.push_back({g, XP_MIX1, L, -1, -1});
            i += 1;
        }
    }
    for (size_t j = 0; j + 1 < plan.size(); ++j)
        plan[j].flags |= XP_STORE;
    plan.back().flags |= XP_EXPECT | XP_FINAL_SCALE | (store ? XP_STORE : 0);
    return plan;
}

}  // namespace qva
