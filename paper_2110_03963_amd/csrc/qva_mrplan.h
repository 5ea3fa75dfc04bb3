// qva_mrplan.h -- host planning of the mixed-radix circulant passes.
//
// A circulant mixer over N solutions (N not a power of two, e.g. the C(m, k)
// feasible subsets of a constrained QWOA, paper Sec. 2.4.2) is diagonal in
// the DFT of length N (Sec. 3).  When every prime factor of N is at most
// kMrMaxPrime, the DFT is done in place by tile passes over a factorisation
// N = A_0 A_1 ... A_{G-1}: the index j = j_0 + A_0 (j_1 + A_1 (j_2 + ...)),
// group 0 contiguous (A_0 <= 4096 amplitudes, a tile holds whole columns of
// it), groups g >= 1 strided by S_g = A_0 ... A_{g-1} (A_g <= 512, so a tile
// keeps at least 8 contiguous amplitudes per row).  Each group's A_g-point
// DFT runs in LDS as Cooley-Tukey stages over the group's radices; N with a
// larger prime factor takes Bluestein's transform instead.
#pragma once

#include <algorithm>
#include <cstdint>
#include <functional>
#include <vector>

#include "qva_internal.h"

namespace qva {

// Prime factors of N in ascending order (N >= 2).
inline std::vector<int> prime_factors(int64_t N)
{
    std::vector<int> f;
    for (int64_t p = 2; p * p <= N; ++p)
        while (N % p == 0) {
            f.push_back((int)p);
            N /= p;
        }
    if (N > 1)
        f.push_back(N > INT32_MAX ? -1 : (int)N);
    return f;
}

// Radices of one group's DFT: its odd primes, and its factors of 2 merged
// into radix 16, 8, 4 or 2 stages.
inline std::vector<int> mr_radices(std::vector<int> primes)
{
    std::vector<int> r;
    int twos = 0;
    for (int p : primes) {
        if (p == 2)
            ++twos;
        else
            r.push_back(p);
    }
    while (twos >= 4) {
        r.push_back(16);
        twos -= 4;
    }
    if (twos > 0)
        r.push_back(1 << twos);
    std::sort(r.begin(), r.end(), [](int a, int b) { return a > b; });
    return r;
}

// LDS cost of the low group's DFT stages, in the lane pattern of the stage
// code: stage s of radix R over sub-length L has its items (one butterfly
// each; item it is column it / (A/R), butterfly b = bi / (L/R), offset
// i = bi mod (L/R), bi = it mod (A/R)) read element col A + b L + i + k L/R.
// A 16-byte LDS read serves a quarter-wave (16 lanes) from 16 granules of
// 16 bytes, so a quarter costs the largest number of its lanes on one
// granule (slot mod 16).  Summed over each stage's first four waves, times R
// (reads per butterfly).  pad: slot e + floor(e / 16) instead of e.
inline int64_t mr_low_lds_cost(const MrGeom& m, bool pad)
{
    const int A = m.A[0], ncol = m.cols[0];
    int L = A;
    int64_t cost = 0;
    for (int s = 0; s < m.nrad[0]; ++s) {
        const int R = m.rad[0][s], ms = L / R, per_col = A / R, items = ncol * per_col;
        for (int q0 = 0; q0 < 256 && q0 < items; q0 += 16) {
            int cnt[16] = {0}, mx = 0;
            for (int it = q0; it < q0 + 16 && it < items; ++it) {
                const int col = it / per_col, bi = it % per_col, b = bi / ms, i = bi % ms;
                const int e = col * A + b * L + i;
                const int slot = pad ? e + (e >> 4) : e;
                mx = std::max(mx, ++cnt[slot & 15]);
            }
            cost += (int64_t)mx * R;
        }
        L /= R;
    }
    return cost;
}

// Columns per tile: as many as fit 4096 elements, at most the number there
// are.  A strided group whose stride S_g is a multiple of 8 amplitudes takes a
// multiple of 8 columns, so that every row starts and ends on a 128-byte line.
inline int mr_cols(int A, int64_t lower_or_upper, bool strided)
{
    int64_t c = kMrTileElems / A;
    if (c > lower_or_upper)
        c = lower_or_upper;
    if (strided && lower_or_upper % 8 == 0 && c >= 8)
        c -= c % 8;
    return (int)(c < 1 ? 1 : c);
}

// Relative HBM cost of streaming a strided group's rows of c amplitudes
// (16 c bytes; q rows of 8 c bytes): rows that do not start on a 128-byte
// line fetch about 112 bytes more on average, and short rows stream below
// the rate of long ones (measured: 128-byte rows near 0.73 and 256-byte rows
// near 0.9 of the rate of rows of 512 bytes and more), modelled as
// 1 + 48 / row bytes.
inline double mr_row_cost(int c, bool aligned)
{
    const double bytes = 16.0 * c;
    const double waste = aligned ? 1.0 : (bytes + 112.0) / bytes;
    return waste * (1.0 + 48.0 / bytes);
}

// The factorisation: the fewest groups for which the prime factors fit the
// caps (A_0 <= 4096, A_g <= 512), then the assignment with the lowest
// modelled HBM cost per layer: each pass's bytes (low group 32 B per
// amplitude, middle groups 2 x 32 B, the top group 40 B) times mr_row_cost of
// its rows (the contiguous low group costs 1); ties to fuller tiles, then to
// the larger contiguous group.  Identical primes are assigned by count, so
// the search is over compositions.  Returns false when some prime factor
// exceeds kMrMaxPrime or no assignment into kMrMaxGroups groups fits.
inline bool mr_plan(int64_t N, MrGeom& out)
{
    if (N < 2 || N >= (int64_t(1) << 31))
        return false;
    const std::vector<int> pf = prime_factors(N);
    std::vector<std::pair<int, int>> pe;  // (prime, multiplicity)
    for (int p : pf) {
        if (p < 0 || p > kMrMaxPrime)
            return false;
        if (!pe.empty() && pe.back().first == p)
            ++pe.back().second;
        else
            pe.push_back({p, 1});
    }
    for (int G = 1; G <= kMrMaxGroups; ++G) {
        if (G == 1 && N > kMrTileElems)
            continue;
        std::vector<int64_t> prod(G, 1);
        std::vector<std::vector<int>> cnt(pe.size(), std::vector<int>(G, 0)), best_cnt;
        double best = -1e300;
        std::function<void(size_t, int, int)> rec = [&](size_t i, int g, int left) {
            if (i == pe.size()) {
                double cost = 0.0, fill = 0.0;
                int64_t S = 1;
                for (int h = 0; h < G; ++h) {
                    if (prod[h] == 1)
                        return;  // every group takes a factor
                    const int A = (int)prod[h];
                    const int c = mr_cols(A, h == 0 ? N / A : S, h > 0);
                    fill += (double)(A * (int64_t)c) / kMrTileElems;
                    if (h == 0)
                        cost += 32.0;
                    else
                        cost += (h == G - 1 ? 40.0 : 64.0) * mr_row_cost(c, S % 8 == 0 && c % 8 == 0);
                    S *= A;
                }
                // lower cost first; fuller tiles and a larger contiguous group break ties
                const double score = -cost + 1e-6 * fill + 1e-12 * (double)prod[0];
                if (score > best) {
                    best = score;
                    best_cnt = cnt;
                }
                return;
            }
            if (g == G - 1) {  // the rest of prime i goes to the last group
                const int p = pe[i].first;
                int64_t f = 1;
                for (int k = 0; k < left; ++k)
                    f *= p;
                const int64_t cap = g == 0 ? kMrTileElems : kMrMaxStrided;
                if (prod[g] * f > cap)
                    return;
                prod[g] *= f;
                cnt[i][g] = left;
                rec(i + 1, 0, i + 1 < pe.size() ? pe[i + 1].second : 0);
                prod[g] /= f;
                cnt[i][g] = 0;
                return;
            }
            const int p = pe[i].first;
            const int64_t cap = g == 0 ? kMrTileElems : kMrMaxStrided;
            int64_t f = 1;
            for (int k = 0; k <= left; ++k) {
                if (prod[g] * f > cap)
                    break;
                prod[g] *= f;
                cnt[i][g] = k;
                rec(i, g + 1, left - k);
                prod[g] /= f;
                cnt[i][g] = 0;
                f *= p;
            }
        };
        rec(0, 0, pe[0].second);
        if (best_cnt.empty())
            continue;
        MrGeom m{};
        m.G = G;
        int64_t S = 1;
        int tab = 0;
        for (int g = 0; g < G; ++g) {
            std::vector<int> primes;
            int A = 1;
            for (size_t i = 0; i < pe.size(); ++i)
                for (int k = 0; k < best_cnt[i][g]; ++k) {
                    primes.push_back(pe[i].first);
                    A *= pe[i].first;
                }
            m.A[g] = A;
            m.S[g] = S;
            const std::vector<int> r = mr_radices(primes);
            m.nrad[g] = (int)r.size();
            for (size_t i = 0; i < r.size(); ++i)
                m.rad[g][i] = r[i];
            m.cols[g] = g == 0 ? mr_cols(A, N / A, false) : mr_cols(A, S, true);
            m.tab_off[g] = tab;
            tab += A;
            S *= A;
        }
        m.S[G] = S;
        m.tab_len = tab;
        int tw = 0;
        for (int g = 1; g < G; ++g) {
            m.tw_off[g] = tw;
            tw += m.cols[g] * m.A[g];
        }
        m.tw_len = tw;
        for (int g = 0; g < G; ++g)
            m.rA[g] = 1.0 / (double)m.A[g];
        m.U = N / m.A[0];
        // pad when it saves at least a third of the low group's LDS cost
        // (the padded slot costs two more instructions per access)
        m.lds_pad = 3 * mr_low_lds_cost(m, true) <= 2 * mr_low_lds_cost(m, false) ? 1 : 0;
        for (int g = 0; g < G; ++g) {
            const int64_t cols_total = g == 0 ? N / m.A[0] : m.S[g];
            const int64_t chunks = (cols_total + m.cols[g] - 1) / m.cols[g];
            m.tiles[g] = g == 0 ? chunks : chunks * (N / m.S[g + 1]);
        }
        out = m;
        return true;
    }
    return false;
}

// Tiles of the widest pass (per-tile partial sums and gradient slots).
inline int64_t mr_max_tiles(const MrGeom& m)
{
    int64_t t = 0;
    for (int g = 0; g < m.G; ++g)
        t = std::max(t, m.tiles[g]);
    return t;
}

// Pass list of a p-layer evolution over G >= 2 groups (as fft_evolve_plan
// for the power-of-two transform): the top group's inverse of layer k, the
// phase of k+1 and its forward share one pass; the low group's pass applies
// the diagonal between its forward and inverse halves.  (One group, N <= 4096:
// the whole evolution is one workgroup's launch, MR_SMALL.)
struct MrPass {
    int group;
    int mode;         // MR_*
    int layer;        // layer of the diagonal's t, or -1
    int phase_layer;  // layer whose gamma the pass applies, or -1
};

inline std::vector<MrPass> mr_evolve_plan(int G, int p, bool store)
{
    std::vector<MrPass> plan;
    const int c = G - 1;
    plan.push_back({c, MR_FIRST, -1, 0});
    for (int L = 0; L < p; ++L) {
        for (int g = G - 2; g >= 1; --g)
            plan.push_back({g, MR_DIF, -1, -1});
        plan.push_back({0, MR_LOWDIAG, L, -1});
        for (int g = 1; g <= G - 2; ++g)
            plan.push_back({g, MR_DIT, -1, -1});
        if (L + 1 < p)
            plan.push_back({c, MR_BOUNDARY, -1, L + 1});
        else
            plan.push_back({c, store ? MR_LAST_STORE : MR_LAST, -1, -1});
    }
    return plan;
}

}  // namespace qva
