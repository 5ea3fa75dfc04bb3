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

// Group 0 is qubits [0, 12) (contiguous tiles); the qubits above are split
// into strided groups of the given sizes (each 1..kMaxHighBits, from qubit
// 12 upward).
inline std::vector<XGroup> x_groups_split(int n, const std::vector<int>& high)
{
    std::vector<XGroup> g;
    if (n <= kTileBits) {
        g.push_back({0, n, 0});
        return g;
    }
    g.push_back({0, kTileBits, 0});
    int k = kTileBits;
    for (int b : high) {
        g.push_back({k, b, kTileBits - b});
        k += b;
    }
    return g;
}

// The default split: the fewest groups of at most kMaxHighBits, sizes as
// equal as possible.
inline std::vector<int> x_split_default(int n)
{
    std::vector<int> hi;
    if (n <= kTileBits)
        return hi;
    const int rem = n - kTileBits;
    const int nh = (rem + kMaxHighBits - 1) / kMaxHighBits;
    const int base = rem / nh, extra = rem % nh;
    for (int i = 0; i < nh; ++i)
        hi.push_back(base + (i < extra ? 1 : 0));
    return hi;
}

inline std::vector<XGroup> x_groups_default(int n) { return x_groups_split(n, x_split_default(n)); }

struct XPass {
    int group;
    int flags;        // XP_* flags
    int layer1;       // layer of the first mixer application
    int layer2;       // layer of the second mixer application, or -1
    int phase_layer;  // layer whose phase is applied, or -1
};

// Order in which even layers visit the groups (odd layers reverse it).  The
// two ends of the order are the boundary groups, whose passes also carry the
// phase; the low (contiguous, 12-qubit) group is placed in the middle when
// there are three or more groups, so the phase rides on the smaller strided
// groups and per-pass arithmetic stays balanced.
inline std::vector<int> x_layer_order(int P)
{
    std::vector<int> order;
    if (P < 3) {
        for (int i = 0; i < P; ++i)
            order.push_back(i);
        return order;
    }
    const int mid = P / 2;
    for (int i = 1; i <= mid; ++i)
        order.push_back(i);
    order.push_back(0);
    for (int i = mid + 1; i < P; ++i)
        order.push_back(i);
    return order;
}

// Pass list of a p-layer evolution (p >= 1) over P >= 2 groups.  The first
// pass generates psi_0 and applies the first phase; the last pass reduces
// <Q> and applies the last layer's scalar factor.
inline std::vector<XPass> x_evolve_plan(int P, int p, bool store)
{
    const std::vector<int> order = x_layer_order(P);
    std::vector<std::pair<int, int>> seq;  // (group, layer) in application order
    for (int L = 0; L < p; ++L)
        for (int i = 0; i < P; ++i)
            seq.push_back({order[(L % 2 == 0) ? i : P - 1 - i], L});
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

// ------------------------------------------------------------- circulant
// A circulant mixer is F^-1 diag F.  Layer k: forward transform top group
// down to the low group, the low group's pass applies the diagonal between
// its forward and inverse halves, then the inverse transform back up.  The
// top group's inverse of layer k, the phase of layer k+1 and the top group's
// forward transform of layer k+1 share one pass: 2(P-1) passes per layer + 1.
struct FPass {
    int group;
    int mode;         // FMODE_*
    int layer;        // layer whose t the pass's diagonal uses, or -1
    int phase_layer;  // layer whose gamma the pass applies, or -1
};

inline std::vector<FPass> fft_evolve_plan(int P, int p, bool store)
{
    std::vector<FPass> plan;
    const int c = P - 1;
    plan.push_back({c, FMODE_FIRST, -1, 0});
    for (int L = 0; L < p; ++L) {
        for (int g = P - 2; g >= 1; --g)
            plan.push_back({g, FMODE_DIF, -1, -1});
        plan.push_back({0, FMODE_LOWDIAG, L, -1});
        for (int g = 1; g <= P - 2; ++g)
            plan.push_back({g, FMODE_DIT, -1, -1});
        if (L + 1 < p)
            plan.push_back({c, FMODE_BOUNDARY, -1, L + 1});
        else
            plan.push_back({c, store ? FMODE_LAST_STORE : FMODE_LAST, -1, -1});
    }
    return plan;
}

// One circulant mixer application (P >= 2 groups).
inline std::vector<FPass> fft_mix_plan(int P)
{
    std::vector<FPass> plan;
    for (int g = P - 1; g >= 1; --g)
        plan.push_back({g, FMODE_DIF, -1, -1});
    plan.push_back({0, FMODE_LOWDIAG, 0, -1});
    for (int g = 1; g <= P - 1; ++g)
        plan.push_back({g, g == P - 1 ? FMODE_DIT_SCALE : FMODE_DIT, -1, -1});
    return plan;
}

// ------------------------------------------------------------ QAOAz XY
// The parity mixer is a product of two-qubit factors that do not all commute:
// a factor must act after every earlier factor sharing one of its qubits, and
// only those.  A pass loads tiles over the bits [0, C) and [k, k + 12 - C)
// (C = 0: the contiguous bits [0, 12); n <= 12: the whole register) and
// applies, in list order, the pending factors whose two qubits lie in the
// tile and whose earlier neighbours are done.  The planner picks passes
// greedily (the tile that takes the most factors; ties to contiguous tiles,
// then to longer rows) until the layer's factors are used up.  Every layer
// has the same factors, so one layer's pass list serves all layers.
struct XyGroup {
    int C, k;
    bool holds(int bit) const { return bit < (C == 0 && k == 0 ? kTileBits : C) || (C > 0 && bit >= k && bit < k + kTileBits - C); }
    int elem_bit(int bit) const { return bit < C || (C == 0 && k == 0) ? bit : bit - k + C; }
};

struct XyLayerPass {
    XyGroup g;
    std::vector<std::pair<int, int>> ops;  // element bits of the tile
};

// Whether some tile holds both qubits of a pair.
inline bool xy_pair_fits(int n, int a, int b)
{
    if (n <= kTileBits)
        return true;
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return hi < kTileBits || lo <= kTileBits - 2 || hi - lo <= kMaxHighBits - 1;
}

inline std::vector<XyLayerPass> xy_layer_plan(int n, const std::vector<std::pair<int, int>>& pairs)
{
    std::vector<XyLayerPass> plan;
    if (n <= kTileBits) {
        // one tile is the whole register (C = k = n: element bit = qubit)
        XyLayerPass ps{{n, n}, {}};
        for (const auto& pr : pairs) {
            if ((int)ps.ops.size() == kMaxXyOps) {
                plan.push_back(ps);
                ps.ops.clear();
            }
            ps.ops.push_back(pr);
        }
        plan.push_back(ps);
        return plan;
    }
    std::vector<XyGroup> cand;
    cand.push_back({0, 0});
    for (int C = kTileBits - 1; C >= kMinColBits; --C)
        for (int k = C; k + kTileBits - C <= n; ++k)
            cand.push_back({C, k});
    std::vector<std::pair<int, int>> pending = pairs;
    if (pending.empty()) {
        plan.push_back({{0, 0}, {}});
        return plan;
    }
    while (!pending.empty()) {
        int best = -1;
        std::vector<int> best_take;
        for (int c = 0; c < (int)cand.size(); ++c) {
            const XyGroup& g = cand[c];
            std::vector<int> take;
            uint64_t blocked = 0;
            for (int i = 0; i < (int)pending.size() && (int)take.size() < kMaxXyOps; ++i) {
                const int a = pending[i].first, b = pending[i].second;
                const uint64_t m = (uint64_t(1) << a) | (uint64_t(1) << b);
                if (!(blocked & m) && g.holds(a) && g.holds(b))
                    take.push_back(i);
                else
                    blocked |= m;
            }
            if (take.size() > best_take.size()) {
                best = c;
                best_take = take;
            }
        }
        if (best < 0)
            return {};  // a pair no tile holds (rejected earlier by xy_pair_fits)
        XyLayerPass ps{cand[best], {}};
        for (int i : best_take)
            ps.ops.push_back({ps.g.elem_bit(pending[i].first), ps.g.elem_bit(pending[i].second)});
        for (int j = (int)best_take.size() - 1; j >= 0; --j)
            pending.erase(pending.begin() + best_take[j]);
        plan.push_back(ps);
    }
    return plan;
}

}  // namespace qva
