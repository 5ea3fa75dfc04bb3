// qva_api.cpp -- the C ABI of libqva: argument validation, pass planning and
// kernel enqueueing.  Declared in include/qva.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <map>
#include <mutex>
#include <stdint.h>
#include <tuple>
#include <vector>

#include "qva.h"
#include "qva_internal.h"
#include "qva_mrplan.h"
#include "qva_plan.h"

using namespace qva;

namespace {

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int hip_status(hipError_t e) { return e == hipSuccess ? QVA_OK : QVA_ERR_HIP; }

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// N of a problem: n_states when given, else 2^n_qubits.
int64_t problem_N(const qva_problem* P)
{
    return P->n_states > 0 ? P->n_states : (int64_t(1) << P->n_qubits);
}

static_assert(sizeof(ZTerm) == sizeof(qva_zterm) && offsetof(qva_zterm, coef) == offsetof(ZTerm, coef),
              "ZTerm mirrors qva_zterm");

// Z-string terms of an extended-QAOA phase (0: the plain phase exp(-i gamma q)).
int problem_terms(const qva_problem* P) { return P->n_terms > 0 ? P->n_terms : 0; }

uint64_t q_tiles_key(int n);

// Whether P's passes read qva_problem.q_tiles: the hypercube mixer without
// Z-string terms, over more qubits than one tile holds.
bool reads_q_tiles(const qva_problem* P)
{
    return P->mixer == QVA_MIX_X && problem_terms(P) == 0 && P->n_qubits > kTileBits;
}

int check_problem(const qva_problem* P, int p)
{
    if (!P || p < 0)
        return QVA_ERR_ARG;
    if (P->n_terms < 0 || P->n_terms > QVA_MAX_TERMS)
        return QVA_ERR_ARG;
    if (P->n_terms > 0) {
        if (P->mixer != QVA_MIX_X)
            return QVA_ERR_UNSUPPORTED;
        if (!P->terms)
            return QVA_ERR_ARG;
        if (!aligned(P->terms, 8))
            return QVA_ERR_ALIGN;
    }
    if (P->mixer != QVA_MIX_X && P->mixer != QVA_MIX_CIRCULANT && P->mixer != QVA_MIX_XY)
        return QVA_ERR_ARG;
    if (P->n_qubits < 1 || P->n_qubits > QVA_MAX_QUBITS)
        return QVA_ERR_SIZE;
    if (P->n_states < 0)
        return QVA_ERR_SIZE;
    if (P->n_states > 0 && P->n_states != (int64_t(1) << P->n_qubits)) {
        // 2^(n-1) < N < 2^n; a circulant mixer (the ring and arrays through
        // Bluestein's transform, N < 2^31)
        if (P->n_states <= (int64_t(1) << (P->n_qubits - 1)) || P->n_states > (int64_t(1) << P->n_qubits))
            return QVA_ERR_SIZE;
        if (P->mixer != QVA_MIX_CIRCULANT)
            return QVA_ERR_UNSUPPORTED;
        if (P->lambda_kind != QVA_LAMBDA_COMPLETE && P->n_states >= (int64_t(1) << 31))
            return QVA_ERR_UNSUPPORTED;
    }
    if (!P->q)
        return QVA_ERR_ARG;
    if (!aligned(P->q, 8))
        return QVA_ERR_ALIGN;
    if (P->mixer == QVA_MIX_XY) {
        if (P->n_xy_pairs < 0 || P->n_xy_pairs > QVA_MAX_XY_PAIRS || (P->n_xy_pairs > 0 && !P->xy_pairs))
            return QVA_ERR_ARG;
        for (int i = 0; i < P->n_xy_pairs; ++i) {
            const int a = P->xy_pairs[2 * i], b = P->xy_pairs[2 * i + 1];
            if (a < 0 || b < 0 || a >= P->n_qubits || b >= P->n_qubits || a == b)
                return QVA_ERR_ARG;
        }
        for (int i = 0; i < P->n_xy_pairs; ++i)
            if (!xy_pair_fits(P->n_qubits, P->xy_pairs[2 * i], P->xy_pairs[2 * i + 1]))
                return QVA_ERR_UNSUPPORTED;
    }
    if (P->mixer == QVA_MIX_CIRCULANT) {
        if (P->lambda_kind != QVA_LAMBDA_ARRAY && P->lambda_kind != QVA_LAMBDA_RING &&
            P->lambda_kind != QVA_LAMBDA_COMPLETE)
            return QVA_ERR_ARG;
        if (P->lambda_kind == QVA_LAMBDA_ARRAY) {
            if (!P->lambda)
                return QVA_ERR_ARG;
            if (!aligned(P->lambda, 8))
                return QVA_ERR_ALIGN;
        }
    }
    if (P->q_tiles && reads_q_tiles(P)) {
        if (!aligned(P->q_tiles, 8))
            return QVA_ERR_ALIGN;
        if (P->q_tiles_key != q_tiles_key(P->n_qubits))
            return QVA_ERR_ARG;  // written for another group split
    }
    return QVA_OK;
}

// --------------------------------------------------- group split (tuning)
// Sizes of the strided qubit groups above the contiguous 12-qubit group, per
// register size n: set by qva_set_group_split (an autotuner's choice), else
// x_split_default.  Read by every planner through x_groups.
std::mutex g_split_mu;
std::vector<int> g_split[QVA_MAX_QUBITS + 1];

std::vector<int> x_split(int n)
{
    if (n > kTileBits && n <= QVA_MAX_QUBITS) {
        std::lock_guard<std::mutex> lock(g_split_mu);
        if (!g_split[n].empty())
            return g_split[n];
    }
    return x_split_default(n);
}

std::vector<XGroup> x_groups(int n) { return x_groups_split(n, x_split(n)); }

// Key of a tile-ordered copy of q: FNV-1a over the register size and the
// strided group sizes it was laid out for.
uint64_t q_tiles_key(int n)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](uint64_t v) {
        h ^= v;
        h *= 1099511628211ull;
    };
    mix(0x7154u);
    mix((uint64_t)n);
    for (int b : x_split(n))
        mix((uint64_t)b);
    return h;
}

// This launch's block of the tile-ordered copy of q, or null: only passes that
// apply the plain phase between two mixer applications read it.
const double* q_tiles_block(const qva_problem* P, int group, int xflags)
{
    if (!P->q_tiles || !reads_q_tiles(P) || !(xflags & XP_PHASE_MID) || (xflags & XP_ZTERMS) || group < 0)
        return nullptr;
    return P->q_tiles + ((int64_t)group << P->n_qubits);
}

// ----------------------------------------------------- hypercube evolution
Angle dev_angle(const double* ptr, int idx)
{
    Angle a;
    a.ptr = ptr;
    a.idx = idx;
    a.val = 0.0;
    return a;
}

Angle host_angle(double v)
{
    Angle a;
    a.ptr = nullptr;
    a.idx = 0;
    a.val = v;
    return a;
}

XPassParams xpass_base(double2* psi, const double* q, int n, const XGroup& g)
{
    XPassParams x{};
    x.psi = psi;
    x.q = q;
    x.n = n;
    x.k = g.k;
    x.col_bits = g.col_bits;
    x.mix1 = x.mix2 = x.phase = host_angle(0.0);
    x.partials = nullptr;
    return x;
}

// One launch of a plan (see qva_pass_info).
struct Launch {
    int kind;
    int group;        // index into x_groups(n), or -1
    int xmode;        // XMODE_* for tile passes
    int layer1, layer2, phase_layer;
};

// zterms: the phases are extended-QAOA Z-string products (XP_ZTERMS).
std::vector<Launch> x_launches(int n, int p, bool store, bool zterms = false)
{
    std::vector<Launch> L;
    if (n <= kTileBits) {
        L.push_back({QVA_PASS_WHOLE, 0, 0, -1, -1, -1});
        return L;
    }
    if (p == 0) {
        L.push_back({QVA_PASS_INIT, -1, 0, -1, -1, -1});
        L.push_back({QVA_PASS_EXPECT, -1, 0, -1, -1, -1});
        L.push_back({QVA_PASS_REDUCE, -1, 0, -1, -1, -1});
        return L;
    }
    const int P = (int)x_groups(n).size();
    for (const XPass& ps : x_evolve_plan(P, p, store)) {
        int kind = QVA_PASS_MIDDLE;
        if (ps.flags == XMODE_FIRST)
            kind = QVA_PASS_FIRST;
        else if (ps.flags == XMODE_BOUNDARY)
            kind = QVA_PASS_BOUNDARY;
        else if (ps.flags == XMODE_LAST)
            kind = QVA_PASS_LAST;
        else if (ps.flags == XMODE_LAST_STORE)
            kind = QVA_PASS_LAST_STORE;
        const int zf = (zterms && ps.phase_layer >= 0) ? XP_ZTERMS : 0;
        L.push_back({kind, ps.group, ps.flags | zf, ps.layer1, ps.layer2, ps.phase_layer});
    }
    L.push_back({QVA_PASS_REDUCE, -1, 0, -1, -1, -1});
    return L;
}

// Algorithmic HBM bytes of a launch (each element read or written once).
double launch_bytes(const Launch& l, int n, bool store)
{
    const double N = std::ldexp(1.0, n);
    const double amp = 16.0, real = 8.0;
    switch (l.kind) {
    case QVA_PASS_WHOLE:
        return real * N + (store ? amp * N : 0.0);
    case QVA_PASS_FIRST:  // the Z-string phase reads no q
        return ((l.xmode & XP_ZTERMS) ? 0.0 : real) * N + amp * N;
    case QVA_PASS_MIDDLE:
        return 2 * amp * N;
    case QVA_PASS_BOUNDARY:
        return ((l.xmode & XP_ZTERMS) ? 0.0 : real) * N + 2 * amp * N;
    case QVA_PASS_LAST:
        return (amp + real) * N;
    case QVA_PASS_LAST_STORE:
        return (2 * amp + real) * N;
    case QVA_PASS_INIT:
        return amp * N;
    case QVA_PASS_EXPECT:
        return (amp + real) * N;
    case QVA_PASS_REDUCE:
        return n > kTileBits ? 16.0 * std::ldexp(1.0, n - kTileBits) : 16.0;
    default:
        return 0.0;
    }
}

// ---------------------------------------------------------- circulant plan
int fft_pass_kind(int mode)
{
    switch (mode) {
    case FMODE_FIRST:
        return QVA_PASS_FFT_FIRST;
    case FMODE_DIF:
        return QVA_PASS_FFT_DIF;
    case FMODE_LOWDIAG:
        return QVA_PASS_FFT_LOWDIAG;
    case FMODE_DIT:
    case FMODE_DIT_SCALE:
        return QVA_PASS_FFT_DIT;
    case FMODE_BOUNDARY:
        return QVA_PASS_FFT_BOUNDARY;
    case FMODE_LAST:
        return QVA_PASS_FFT_LAST;
    default:
        return QVA_PASS_FFT_LAST_STORE;
    }
}

bool lambda_tiled(const qva_problem* P)
{
    return P->lambda_kind == QVA_LAMBDA_ARRAY && P->n_qubits > kTileBits;
}

// The complete graph's mixer in closed form (no transform): n > 12, or any
// N that is not a power of two.
bool complete_closed_form(const qva_problem* P)
{
    return P->mixer == QVA_MIX_CIRCULANT && P->lambda_kind == QVA_LAMBDA_COMPLETE &&
           (P->n_qubits > kTileBits || problem_N(P) != (int64_t(1) << P->n_qubits));
}

// A ring or eigenvalue-array circulant over N solutions, N not a power of
// two: Bluestein's chirp-z transform over a padded power of two M.
// The mixed-radix factorisation of N (cached: the planner searches the
// assignments of N's prime factors to groups).
bool mixed_geom(int64_t N, MrGeom* out)
{
    static std::mutex mu;
    static std::map<int64_t, std::pair<bool, MrGeom>> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(N);
    if (it == cache.end()) {
        MrGeom m{};
        const bool ok = mr_plan(N, m);
        if (cache.size() > 256)
            cache.clear();
        it = cache.emplace(N, std::make_pair(ok, m)).first;
    }
    if (out)
        *out = it->second.second;
    return it->second.first;
}

// A ring or eigenvalue-array circulant over N solutions, N not a power of
// two but with every prime factor <= 31: the in-place mixed-radix transform.
constexpr bool kMixedRadix = true;

bool mixed_path(const qva_problem* P)
{
    return kMixedRadix && P->mixer == QVA_MIX_CIRCULANT && P->lambda_kind != QVA_LAMBDA_COMPLETE &&
           problem_N(P) != (int64_t(1) << P->n_qubits) && mixed_geom(problem_N(P), nullptr);
}

bool bluestein_path(const qva_problem* P)
{
    return P->mixer == QVA_MIX_CIRCULANT && P->lambda_kind != QVA_LAMBDA_COMPLETE &&
           problem_N(P) != (int64_t(1) << P->n_qubits) && !mixed_path(P);
}

// log2 M: the smallest power of two >= 2N - 1, and at least 2^13 (tile passes).
int blu_bits_n(int64_t N)
{
    int b = kTileBits + 1;
    while ((int64_t(1) << b) < 2 * N - 1)
        ++b;
    return b;
}

int blu_bits(const qva_problem* P) { return blu_bits_n(problem_N(P)); }

// Workspace of a Bluestein evolution: partials, then the padded buffer and the
// two filter spectra (M amplitudes each).  The lone mixer (with_partials
// false) needs no partials.
struct BluLayout {
    size_t parts = 0, pad = 0, b0 = 0, b1 = 0, tw = 0, total = 0;
};

BluLayout blu_layout_n(int64_t N, bool with_partials)
{
    BluLayout L;
    const int64_t M = int64_t(1) << blu_bits_n(N);
    const int64_t e = expect_partial_count(N), tiles = M >> kTileBits;
    size_t off = with_partials ? align256((size_t)(e > tiles ? e : tiles) * sizeof(double2)) : 0;
    L.pad = off;
    off += (size_t)M * sizeof(double2);
    L.b0 = off;
    off += (size_t)M * sizeof(double2);
    L.b1 = off;
    off += (size_t)M * sizeof(double2);
    L.tw = off;
    off += kTwiddleTableBytes;
    L.total = off;
    return L;
}

BluLayout blu_layout(const qva_problem* P) { return blu_layout_n(problem_N(P), true); }

// Blocks of the closed-form passes (kCompleteChunk amplitudes each, the last
// one possibly partial).
int64_t cpl_blocks(const qva_problem* P)
{
    return (problem_N(P) + kCompleteChunk - 1) / kCompleteChunk;
}

// Bytes of the closed-form evolution's partial sums (also the p = 0 path).
size_t cpl_partials_bytes(const qva_problem* P)
{
    const int64_t b = cpl_blocks(P), e = expect_partial_count(problem_N(P));
    return (size_t)(b > e ? b : e) * sizeof(double2);
}

std::vector<Launch> fft_launches(const qva_problem* P, int p, bool store)
{
    const int n = P->n_qubits;
    std::vector<Launch> L;
    if (n <= kTileBits && !complete_closed_form(P) && !bluestein_path(P) && !mixed_path(P)) {
        L.push_back({QVA_PASS_WHOLE, 0, 0, -1, -1, -1});
        return L;
    }
    if (p == 0) {
        L.push_back({QVA_PASS_INIT, -1, 0, -1, -1, -1});
        L.push_back({QVA_PASS_EXPECT, -1, 0, -1, -1, -1});
        L.push_back({QVA_PASS_REDUCE, -1, 0, -1, -1, -1});
        return L;
    }
    if (complete_closed_form(P)) {
        L.push_back({QVA_PASS_CPL_FIRST, -1, CPMODE_FIRST, -1, -1, 0});
        L.push_back({QVA_PASS_CPL_SUM, -1, 0, -1, -1, -1});
        for (int k = 0; k + 1 < p; ++k) {
            L.push_back({QVA_PASS_CPL_LAYER, -1, CPMODE_LAYER, k, -1, k + 1});
            L.push_back({QVA_PASS_CPL_SUM, -1, 0, -1, -1, -1});
        }
        L.push_back({store ? QVA_PASS_CPL_LAST_STORE : QVA_PASS_CPL_LAST, -1,
                     store ? CPMODE_LAST_STORE : CPMODE_LAST, p - 1, -1, -1});
        L.push_back({QVA_PASS_REDUCE, -1, 0, -1, -1, -1});
        return L;
    }
    if (bluestein_path(P)) {
        // groups of the padded transform: top c, middles 1..c-1, low 0
        const int c = (int)x_groups(blu_bits(P)).size() - 1;
        auto conv_front = [&](std::vector<Launch>& V) {
            for (int g = c - 1; g >= 1; --g)
                V.push_back({QVA_PASS_FFT_DIF, g, FMODE_DIF, -1, -1, -1});
        };
        auto conv_back = [&](std::vector<Launch>& V) {
            for (int g = 1; g <= c - 1; ++g)
                V.push_back({QVA_PASS_FFT_DIT, g, FMODE_DIT, -1, -1, -1});
        };
        L.push_back({QVA_PASS_TWIDDLE_PREP, -1, 0, -1, -1, -1});
        for (int which = 0; which < 2; ++which) {  // the filters w and conj(w)
            L.push_back({QVA_PASS_BLU_CHIRP, c, FMODE_B_CHIRP, -1, which, -1});
            conv_front(L);
            L.push_back({QVA_PASS_BLU_TILE, 0, FMODE_LOWDIF_TILED, -1, which, -1});
        }
        L.push_back({QVA_PASS_BLU_FIRST, c, FMODE_B_FIRST, -1, -1, 0});
        for (int k = 0; k < p; ++k) {
            conv_front(L);
            L.push_back({QVA_PASS_BLU_MUL, 0, FMODE_LOWMUL, -1, 0, -1});
            conv_back(L);
            L.push_back({QVA_PASS_BLU_LAMBDA, c, FMODE_B_BOUND_LAM, k, -1, -1});
            conv_front(L);
            L.push_back({QVA_PASS_BLU_MUL, 0, FMODE_LOWMUL, -1, 1, -1});
            conv_back(L);
            if (k + 1 < p)
                L.push_back({QVA_PASS_BLU_PHASE, c, FMODE_B_BOUND_Q, -1, -1, k + 1});
            else
                L.push_back({store ? QVA_PASS_BLU_LAST_STORE : QVA_PASS_BLU_LAST, c,
                             store ? FMODE_B_LAST_STORE : FMODE_B_LAST, -1, -1, -1});
        }
        L.push_back({QVA_PASS_REDUCE, -1, 0, -1, -1, -1});
        return L;
    }
    L.push_back({QVA_PASS_TWIDDLE_PREP, -1, 0, -1, -1, -1});
    if (lambda_tiled(P))
        L.push_back({QVA_PASS_LAMBDA_PREP, -1, 0, -1, -1, -1});
    const int G = (int)x_groups(n).size();
    for (const FPass& f : fft_evolve_plan(G, p, store))
        L.push_back({fft_pass_kind(f.mode), f.group, f.mode, f.layer, -1, f.phase_layer});
    L.push_back({QVA_PASS_REDUCE, -1, 0, -1, -1, -1});
    return L;
}

double fft_launch_bytes(const Launch& l, int n, bool store, bool tiled)
{
    const double N = std::ldexp(1.0, n);
    const double amp = 16.0, real = 8.0;
    switch (l.kind) {
    case QVA_PASS_WHOLE:
        return real * N + (tiled ? real * N : 0.0) + (store ? amp * N : 0.0);
    case QVA_PASS_FFT_FIRST:
        return (real + amp) * N;
    case QVA_PASS_FFT_DIF:
    case QVA_PASS_FFT_DIT:
        return 2 * amp * N;
    case QVA_PASS_FFT_LOWDIAG:
        return 2 * amp * N + (tiled ? real * N : 0.0);
    case QVA_PASS_FFT_BOUNDARY:
        return (2 * amp + real) * N;
    case QVA_PASS_FFT_LAST:
        return (amp + real) * N;
    case QVA_PASS_FFT_LAST_STORE:
        return (2 * amp + real) * N;
    case QVA_PASS_LAMBDA_PREP:
        return 2 * real * N;
    case QVA_PASS_TWIDDLE_PREP:
        return (double)kTwiddleTableBytes;
    default: {
        Launch x = l;
        return launch_bytes(x, n, store);
    }
    }
}

// Algorithmic bytes of the closed-form complete-graph launches (any N).
double cpl_launch_bytes(const Launch& l, const qva_problem* P, int p)
{
    const double N = (double)problem_N(P), parts = 16.0 * (double)cpl_blocks(P);
    const double amp = 16.0, real = 8.0;
    switch (l.kind) {
    case QVA_PASS_CPL_FIRST:
        return (real + amp) * N + parts;
    case QVA_PASS_CPL_LAYER:
        return (2 * amp + real) * N + parts;
    case QVA_PASS_CPL_LAST:
        return (amp + real) * N + parts;
    case QVA_PASS_CPL_LAST_STORE:
        return (2 * amp + real) * N + parts;
    case QVA_PASS_CPL_SUM:
        return parts;
    case QVA_PASS_INIT:
        return amp * N;
    case QVA_PASS_EXPECT:
        return (amp + real) * N;
    case QVA_PASS_REDUCE:
        return 16.0 * (double)(p == 0 ? expect_partial_count(problem_N(P)) : cpl_blocks(P));
    default:
        return 0.0;
    }
}

// Algorithmic bytes of the Bluestein launches (M-amplitude passes; q and
// lambda over the N solutions).
double blu_launch_bytes(const Launch& l, const qva_problem* P, int p)
{
    const double N = (double)problem_N(P), M = std::ldexp(1.0, blu_bits(P));
    const double amp = 16.0, real = 8.0;
    const double lam = P->lambda_kind == QVA_LAMBDA_ARRAY ? real * N : 0.0;
    switch (l.kind) {
    case QVA_PASS_FFT_DIF:
    case QVA_PASS_FFT_DIT:
        return 2 * amp * M;
    case QVA_PASS_BLU_CHIRP:
        return amp * M;
    case QVA_PASS_TWIDDLE_PREP:
        return (double)kTwiddleTableBytes;
    case QVA_PASS_BLU_TILE:
        return 2 * amp * M;
    case QVA_PASS_BLU_FIRST:
        return amp * M + real * N;
    case QVA_PASS_BLU_MUL:
        return 3 * amp * M;
    case QVA_PASS_BLU_LAMBDA:
        return 2 * amp * M + lam;
    case QVA_PASS_BLU_PHASE:
        return 2 * amp * M + real * N;
    case QVA_PASS_BLU_LAST:
        return amp * M + real * N;
    case QVA_PASS_BLU_LAST_STORE:
        return amp * M + (real + amp) * N;
    case QVA_PASS_INIT:
        return amp * N;
    case QVA_PASS_EXPECT:
        return (amp + real) * N;
    case QVA_PASS_REDUCE:
        return 16.0 * (double)(p == 0 ? expect_partial_count(problem_N(P)) : (int64_t(M) >> kTileBits));
    default:
        return 0.0;
    }
}

// Records an event pair around every launch when the caller asked for it.
struct EventHook {
    void* const* ev = nullptr;
    int n = 0;
    int i = 0;
    void before(hipStream_t s)
    {
        if (ev && 2 * i + 1 < n)
            (void)hipEventRecord(reinterpret_cast<hipEvent_t>(ev[2 * i]), s);
    }
    void after(hipStream_t s)
    {
        if (ev && 2 * i + 1 < n)
            (void)hipEventRecord(reinterpret_cast<hipEvent_t>(ev[2 * i + 1]), s);
        ++i;
    }
};

int evolve_x(const qva_problem* P, const double* gammas, const double* ts, int p, double2* psi,
             double* out_f, double* out_norm, bool store, double2* partials, hipStream_t s,
             EventHook& hook)
{
    const int n = P->n_qubits;
    const int64_t N = int64_t(1) << n;
    const int E = problem_terms(P);
    const std::vector<XGroup> groups = x_groups(n);
    for (const Launch& l : x_launches(n, p, store, E > 0)) {
        hipError_t e = hipSuccess;
        hook.before(s);
        switch (l.kind) {
        case QVA_PASS_WHOLE: {
            SmallParams sp{};
            sp.psi = psi;
            sp.q = P->q;
            sp.terms = reinterpret_cast<const ZTerm*>(P->terms);
            sp.n_terms = E;
            sp.gammas = gammas;
            sp.ts = ts;
            sp.n = n;
            sp.p = p;
            sp.flags = SM_INIT | SM_EVOLVE | SM_EXPECT | (store ? SM_STORE : 0);
            sp.out_f = out_f;
            sp.out_norm = out_norm;
            e = launch_small(sp, s);
            break;
        }
        case QVA_PASS_INIT:
            e = launch_init_uniform(psi, N, s);
            break;
        case QVA_PASS_EXPECT:
            e = launch_expect_partials(psi, P->q, N, partials, s);
            break;
        case QVA_PASS_REDUCE: {
            const int64_t count = p == 0 ? expect_partial_count(N) : (int64_t(1) << (n - kTileBits));
            e = launch_final_reduce(partials, count, out_f, out_norm, s);
            break;
        }
        default: {
            XPassParams x = xpass_base(psi, P->q, n, groups[l.group]);
            x.flags = l.xmode;
            x.mix1 = dev_angle(ts, l.layer1);
            x.mix2 = dev_angle(ts, l.layer2 >= 0 ? l.layer2 : 0);
            x.phase = dev_angle(gammas, l.phase_layer >= 0 ? l.phase_layer * (E > 0 ? E : 1) : 0);
            x.terms = reinterpret_cast<const ZTerm*>(P->terms);
            x.n_terms = E;
            x.partials = partials;
            x.qt = q_tiles_block(P, l.group, l.xmode);
            e = launch_xpass(x, s);
            break;
        }
        }
        hook.after(s);
        if (e != hipSuccess)
            return QVA_ERR_HIP;
    }
    return QVA_OK;
}

int small_lambda_kind(int kind)
{
    return kind == QVA_LAMBDA_RING ? FFT_LAMBDA_RING
                                   : (kind == QVA_LAMBDA_COMPLETE ? FFT_LAMBDA_COMPLETE : FFT_LAMBDA_NATURAL);
}

// Workspace of the circulant evolution: partial sums, then (array lambda)
// the per-tile copy of lambda.
size_t circ_partials_bytes(int n) { return (size_t)(int64_t(1) << (n - kTileBits)) * sizeof(double2); }

// Offset of the low-group root table in the workspace of the power-of-two
// circulant evolution (after the partials and the per-tile lambda copy).
size_t circ_twiddle_offset(const qva_problem* P)
{
    const int n = P->n_qubits;
    size_t off = circ_partials_bytes(n);
    if (lambda_tiled(P))
        off += (size_t)(int64_t(1) << n) * sizeof(double);
    return align256(off);
}

// Bluestein evolution (N not a power of two, ring or eigenvalue array).
int evolve_bluestein(const qva_problem* P, const double* gammas, const double* ts, int p, double2* psi,
                     double* out_f, double* out_norm, bool store, char* work, hipStream_t s,
                     EventHook& hook)
{
    const int nb = blu_bits(P);
    const std::vector<XGroup> groups = x_groups(nb);
    const BluLayout W = blu_layout(P);
    double2* partials = reinterpret_cast<double2*>(work);
    double2* pad = reinterpret_cast<double2*>(work + W.pad);
    double2* spec[2] = {reinterpret_cast<double2*>(work + W.b0), reinterpret_cast<double2*>(work + W.b1)};
    double2* tw = reinterpret_cast<double2*>(work + W.tw);
    for (const Launch& l : fft_launches(P, p, store)) {
        hipError_t e = hipSuccess;
        hook.before(s);
        if (l.kind == QVA_PASS_REDUCE) {
            e = launch_final_reduce(partials, int64_t(1) << (nb - kTileBits), out_f, out_norm, s);
        } else if (l.kind == QVA_PASS_TWIDDLE_PREP) {
            e = launch_twiddle_table(tw, s);
        } else {
            const XGroup& g = groups[l.group];
            FftPassParams f{};
            f.psi = pad;
            f.q = P->q;
            f.lam = P->lambda;
            f.lambda_kind = P->lambda_kind == QVA_LAMBDA_RING ? FFT_LAMBDA_RING : FFT_LAMBDA_NATURAL;
            f.mix1 = dev_angle(ts, l.layer1 >= 0 ? l.layer1 : 0);
            f.phase = dev_angle(gammas, l.phase_layer >= 0 ? l.phase_layer : 0);
            f.n = nb;
            f.k = g.k;
            f.col_bits = g.col_bits;
            f.flags = l.xmode;
            f.partials = partials;
            f.nb = problem_N(P);
            f.bt = spec[l.layer2 > 0 ? 1 : 0];
            f.out = l.kind == QVA_PASS_BLU_TILE ? spec[l.layer2 > 0 ? 1 : 0] : psi;
            f.conj = l.layer2 > 0 ? 1 : 0;
            f.tw = tw;
            e = launch_fftpass(f, s);
        }
        hook.after(s);
        if (e != hipSuccess)
            return QVA_ERR_HIP;
    }
    return QVA_OK;
}

// The mixer alone, exp(-i t W) = F^-1 diag(exp(-i t lambda)) F, for N that
// is neither a power of two nor a product of primes <= 31 (ring or
// eigenvalue array), through Bluestein's transform on the padded buffer:
// a_j = psi_j conj(w_j) (zero for j >= N), the convolution with w,
// exp(-i t lambda_m) (zero for m >= N), the convolution with conj(w), and
// psi_j = w_j x_j / N (j < N).  The chirps between the two convolutions
// cancel as in the evolution.  work: blu_layout_n(N, false).
int bluestein_mix(double2* psi, const double* lambda, int lambda_kind, int64_t N, double t, char* work,
                  hipStream_t s)
{
    const int nb = blu_bits_n(N);
    const std::vector<XGroup> groups = x_groups(nb);
    const int c = (int)groups.size() - 1;  // top group; middles 1..c-1, low 0
    const BluLayout W = blu_layout_n(N, false);
    double2* pad = reinterpret_cast<double2*>(work + W.pad);
    double2* spec[2] = {reinterpret_cast<double2*>(work + W.b0), reinterpret_cast<double2*>(work + W.b1)};
    double2* tw = reinterpret_cast<double2*>(work + W.tw);
    if (launch_twiddle_table(tw, s) != hipSuccess)
        return QVA_ERR_HIP;
    auto pass = [&](int group, int mode, int which) {
        const XGroup& g = groups[group];
        FftPassParams f{};
        f.psi = pad;
        f.lam = lambda;
        f.lambda_kind = lambda_kind == QVA_LAMBDA_RING ? FFT_LAMBDA_RING : FFT_LAMBDA_NATURAL;
        f.mix1 = host_angle(t);
        f.phase = host_angle(0.0);
        f.n = nb;
        f.k = g.k;
        f.col_bits = g.col_bits;
        f.flags = mode;
        f.nb = N;
        f.bt = spec[which];
        f.out = mode == FMODE_LOWDIF_TILED ? spec[which] : psi;
        f.in = psi;
        f.conj = which;
        f.tw = tw;
        return launch_fftpass(f, s) == hipSuccess;
    };
    auto front = [&](int which) {
        for (int g = c - 1; g >= 1; --g)
            if (!pass(g, FMODE_DIF, which))
                return false;
        return true;
    };
    auto back = [&](int which) {
        for (int g = 1; g <= c - 1; ++g)
            if (!pass(g, FMODE_DIT, which))
                return false;
        return true;
    };
    // the filters' spectra (times 1/M): w, then conj(w)
    for (int which = 0; which < 2; ++which)
        if (!pass(c, FMODE_B_CHIRP, which) || !front(which) || !pass(0, FMODE_LOWDIF_TILED, which))
            return QVA_ERR_HIP;
    const bool ok = pass(c, FMODE_B_LOAD, 0) && front(0) && pass(0, FMODE_LOWMUL, 0) && back(0) &&
                    pass(c, FMODE_B_BOUND_LAM, 0) && front(1) && pass(0, FMODE_LOWMUL, 1) && back(1) &&
                    pass(c, FMODE_B_STORE, 0);
    return ok ? QVA_OK : QVA_ERR_HIP;
}

// Workspace of the complete graph's lone mixer: per-block partial sums, then S.
size_t complete_mix_bytes(int64_t N)
{
    const int64_t blocks = (N + kCompleteChunk - 1) / kCompleteChunk;
    return align256((size_t)blocks * sizeof(double2)) + 256;
}

// The complete graph's mixer alone over any N, in closed form:
// psi <- e^{i t} (psi + c S 1), S = sum_j psi_j, c = (e^{-i t N} - 1) / N
// (one summing pass, the fixed-order reduction of its block sums, one update
// pass).  work: complete_mix_bytes(N).
int complete_mix(double2* psi, int64_t N, double t, char* work, hipStream_t s)
{
    const int64_t blocks = (N + kCompleteChunk - 1) / kCompleteChunk;
    double2* partials = reinterpret_cast<double2*>(work);
    double2* sum = reinterpret_cast<double2*>(work + align256((size_t)blocks * sizeof(double2)));
    CompleteParams c{};
    c.psi = psi;
    c.partials = partials;
    c.N = N;
    c.flags = CPMODE_SUM;
    if (launch_complete(c, s) != hipSuccess)
        return QVA_ERR_HIP;
    if (launch_final_reduce(partials, blocks, &sum->x, &sum->y, s) != hipSuccess)
        return QVA_ERR_HIP;
    c.flags = CPMODE_MIX;
    c.sum_in = sum;
    c.ts = nullptr;
    c.t_val = t;
    return hip_status(launch_complete(c, s));
}

// ----------------------------------------------- mixed-radix circulant
// One launch of a mixed-radix plan.
struct MrLaunch {
    int kind;    // qva_pass_kind
    int mode;    // MR_* / MRG_*
    int group;
    int layer;   // layer of the diagonal's t, or -1
    int gamma;   // layer whose phase the launch applies (or walks back), or -1
    int slot;    // gradient slot, or -1
};

int mr_kind(int mode)
{
    switch (mode) {
    case MR_FIRST:
        return QVA_PASS_MR_FIRST;
    case MR_DIF:
        return QVA_PASS_MR_DIF;
    case MR_DIT:
        return QVA_PASS_MR_DIT;
    case MR_LOWDIAG:
        return QVA_PASS_MR_LOWDIAG;
    case MR_BOUNDARY:
        return QVA_PASS_MR_BOUNDARY;
    case MR_LAST:
        return QVA_PASS_MR_LAST;
    default:
        return QVA_PASS_MR_LAST_STORE;
    }
}

// p >= 1.  Evolution: tables, the pass list, the partial-sum reduction.
// Gradient: tables, the forward without its last pass, the turn, then every
// forward pass undone in reverse (inner products where they are fused), the
// reductions.  Slots: t of layer L at L, gamma of layer L at p + L.
std::vector<MrLaunch> mr_launches(const MrGeom& m, int p, bool store, bool grad)
{
    std::vector<MrLaunch> L;
    L.push_back({QVA_PASS_MR_TABLES, 0, -1, -1, -1, -1});
    if (m.G == 1) {
        if (grad)
            L.push_back({QVA_PASS_GRAD_MR_SMALL, MRG_SMALL, 0, -1, -1, -1});
        else
            L.push_back({QVA_PASS_MR_SMALL, store ? MR_SMALL_STORE : MR_SMALL, 0, -1, -1, -1});
        return L;
    }
    const std::vector<MrPass> fw = mr_evolve_plan(m.G, p, grad ? false : store);
    const int nf = (int)fw.size();
    for (int i = 0; i < (grad ? nf - 1 : nf); ++i)
        L.push_back({mr_kind(fw[i].mode), fw[i].mode, fw[i].group, fw[i].layer, fw[i].phase_layer, -1});
    if (!grad) {
        L.push_back({QVA_PASS_REDUCE, 0, -1, -1, -1, -1});
        return L;
    }
    L.push_back({QVA_PASS_GRAD_MR_TURN, MRG_TURN, fw[nf - 1].group, -1, -1, -1});
    for (int i = nf - 2; i >= 0; --i) {
        const MrPass& f = fw[i];
        if (f.mode == MR_DIF)
            L.push_back({QVA_PASS_GRAD_MR_DIT, MR_DIT, f.group, -1, -1, -1});
        else if (f.mode == MR_DIT)
            L.push_back({QVA_PASS_GRAD_MR_DIF, MR_DIF, f.group, -1, -1, -1});
        else if (f.mode == MR_LOWDIAG)
            L.push_back({QVA_PASS_GRAD_MR_LOWDIAG, MRG_LOWDIAG, f.group, f.layer, -1, f.layer});
        else if (f.mode == MR_BOUNDARY)
            L.push_back({QVA_PASS_GRAD_MR_BOUND, MRG_BOUND, f.group, -1, f.phase_layer, p + f.phase_layer});
        else  // MR_FIRST
            L.push_back({QVA_PASS_GRAD_MR_FINAL, MRG_FINAL, f.group, -1, 0, p});
    }
    L.push_back({QVA_PASS_REDUCE, 0, -1, -1, -1, -1});
    L.push_back({QVA_PASS_GRAD_REDUCE, 0, -1, -1, -1, -1});
    return L;
}

// Workspace of the mixed-radix path: tables, per-tile (f, norm) partials,
// and for the gradient 2p per-tile slot arrays and their sums.
struct MrLayout {
    int64_t tiles = 0;
    size_t geom = 0, tab = 0, part = 0, slots = 0, sums = 0, total = 0;
};

MrLayout mr_layout(const MrGeom& m, int p, bool grad)
{
    MrLayout w;
    w.tiles = mr_max_tiles(m);
    size_t off = 0;
    w.geom = off;
    off = align256(off + sizeof(MrGeom));
    w.tab = off;
    off = align256(off + mr_table_bytes(m));
    w.part = off;
    off = align256(off + (size_t)w.tiles * sizeof(double2));
    if (grad) {
        w.slots = off;
        off = align256(off + (size_t)(2 * p) * (size_t)w.tiles * sizeof(double));
        w.sums = off;
        off = align256(off + (size_t)(2 * p) * sizeof(double));
    }
    w.total = off;
    return w;
}

double mr_launch_bytes(const MrLaunch& l, const qva_problem* P, const MrGeom& m, int p)
{
    const double N = (double)problem_N(P), amp = 16.0, real = 8.0;
    const double lam = P->lambda_kind == QVA_LAMBDA_ARRAY ? real * N : 0.0;
    switch (l.kind) {
    case QVA_PASS_MR_TABLES:
        return (double)(mr_table_bytes(m) + sizeof(MrGeom));
    case QVA_PASS_MR_FIRST:
        return (amp + real) * N;
    case QVA_PASS_MR_DIF:
    case QVA_PASS_MR_DIT:
        return 2 * amp * N;
    case QVA_PASS_MR_LOWDIAG:
        return 2 * amp * N + lam;
    case QVA_PASS_MR_BOUNDARY:
        return (2 * amp + real) * N;
    case QVA_PASS_MR_LAST:
        return (amp + real) * N;
    case QVA_PASS_MR_LAST_STORE:
        return (2 * amp + real) * N;
    case QVA_PASS_MR_SMALL:
        return real * N + lam + (l.mode == MR_SMALL_STORE ? amp * N : 0.0);
    case QVA_PASS_GRAD_MR_SMALL:
        return real * N + lam;
    case QVA_PASS_GRAD_MR_TURN:
        return (3 * amp + real) * N;
    case QVA_PASS_GRAD_MR_DIF:
    case QVA_PASS_GRAD_MR_DIT:
        return 4 * amp * N;
    case QVA_PASS_GRAD_MR_LOWDIAG:
        return 4 * amp * N + lam;
    case QVA_PASS_GRAD_MR_BOUND:
        return (4 * amp + real) * N;
    case QVA_PASS_GRAD_MR_FINAL:
        return (2 * amp + real) * N;
    case QVA_PASS_REDUCE:
        return 16.0 * (double)m.tiles[m.G - 1];
    case QVA_PASS_GRAD_REDUCE:
        return 8.0 * (double)(2 * p) * (double)mr_max_tiles(m);
    default:
        return 0.0;
    }
}

// Evolution (grad = false) or adjoint gradient over the mixed-radix passes.
int mixed_run(const qva_problem* P, const double* gammas, const double* ts, int p, double2* psi, double2* chi,
              double* out_f, double* out_norm, double* dgammas, double* dts, bool store, bool grad, char* work,
              hipStream_t s, EventHook& hook)
{
    MrGeom m{};
    if (!mixed_geom(problem_N(P), &m))
        return QVA_ERR_UNSUPPORTED;
    const MrLayout W = mr_layout(m, p, grad);
    MrGeom* geom = reinterpret_cast<MrGeom*>(work + W.geom);
    double2* tab = reinterpret_cast<double2*>(work + W.tab);
    double2* part = reinterpret_cast<double2*>(work + W.part);
    double* slots = reinterpret_cast<double*>(work + W.slots);
    double* sums = reinterpret_cast<double*>(work + W.sums);
    for (const MrLaunch& l : mr_launches(m, p, store, grad)) {
        hipError_t e = hipSuccess;
        hook.before(s);
        if (l.kind == QVA_PASS_MR_TABLES) {
            e = launch_mr_tables(m, geom, tab, s);
        } else if (l.kind == QVA_PASS_REDUCE) {
            e = launch_final_reduce(part, m.tiles[m.G - 1], out_f, out_norm, s);
        } else if (l.kind == QVA_PASS_GRAD_REDUCE) {
            e = launch_grad_reduce(slots, 2 * p, W.tiles, sums, p, 1, 1, dgammas, dts, s);
        } else {
            MrPassParams mp{};
            mp.psi = psi;
            mp.chi = chi;
            mp.q = P->q;
            mp.lam = P->lambda;
            mp.lambda_kind = P->lambda_kind == QVA_LAMBDA_RING ? FFT_LAMBDA_RING : FFT_LAMBDA_NATURAL;
            mp.t = dev_angle(ts, l.layer >= 0 ? l.layer : 0);
            mp.gamma = dev_angle(gammas, l.gamma >= 0 ? l.gamma : 0);
            mp.gammas = gammas;
            mp.ts = ts;
            mp.p = p;
            mp.N = problem_N(P);
            mp.geom = geom;
            mp.g = l.group;
            mp.tab = tab;
            mp.partials = part;
            mp.slot = l.slot >= 0 ? slots + (int64_t)l.slot * W.tiles : nullptr;
            mp.out_f = out_f;
            mp.out_norm = out_norm;
            mp.dgammas = dgammas;
            mp.dts = dts;
            if (l.kind == QVA_PASS_GRAD_MR_DIF || l.kind == QVA_PASS_GRAD_MR_DIT) {
                // no inner product: the single-vector transform, once per vector
                e = launch_mrpass(mp, m, l.mode, s);
                if (e == hipSuccess) {
                    mp.psi = chi;
                    e = launch_mrpass(mp, m, l.mode, s);
                }
            } else {
                e = launch_mrpass(mp, m, l.mode, s);
            }
        }
        hook.after(s);
        if (e != hipSuccess)
            return QVA_ERR_HIP;
    }
    return QVA_OK;
}

// The mixer alone, exp(-i t W) = F^-1 diag(exp(-i t lambda)) F, on the
// caller's state over the mixed-radix passes: the forward groups top-down,
// the low group with the diagonal, the inverse groups bottom-up, the last
// one scaled by 1/N (N <= 4096: one workgroup).  work: the geometry, then the
// tables.
int mixed_mix(double2* psi, const double* lambda, int lambda_kind, const MrGeom& m, double t, char* work,
              hipStream_t s)
{
    MrGeom* geom = reinterpret_cast<MrGeom*>(work);
    double2* tab = reinterpret_cast<double2*>(work + align256(sizeof(MrGeom)));
    if (launch_mr_tables(m, geom, tab, s) != hipSuccess)
        return QVA_ERR_HIP;
    MrPassParams mp{};
    mp.psi = psi;
    mp.lam = lambda;
    mp.lambda_kind = lambda_kind == QVA_LAMBDA_RING ? FFT_LAMBDA_RING : FFT_LAMBDA_NATURAL;
    mp.t = host_angle(t);
    mp.gamma = host_angle(0.0);
    mp.N = m.S[m.G];
    mp.geom = geom;
    mp.tab = tab;
    if (m.G == 1)
        return hip_status(launch_mrpass(mp, m, MR_SMALL_MIX, s));
    for (int g = m.G - 1; g >= 1; --g) {
        mp.g = g;
        if (launch_mrpass(mp, m, MR_DIF, s) != hipSuccess)
            return QVA_ERR_HIP;
    }
    mp.g = 0;
    if (launch_mrpass(mp, m, MR_LOWDIAG, s) != hipSuccess)
        return QVA_ERR_HIP;
    for (int g = 1; g < m.G; ++g) {
        mp.g = g;
        mp.scale_inv_n = g == m.G - 1;
        if (launch_mrpass(mp, m, MR_DIT, s) != hipSuccess)
            return QVA_ERR_HIP;
    }
    return QVA_OK;
}

int evolve_circ(const qva_problem* P, const double* gammas, const double* ts, int p, double2* psi,
                double* out_f, double* out_norm, bool store, char* work, hipStream_t s,
                EventHook& hook)
{
    const int n = P->n_qubits;
    const int64_t N = problem_N(P);
    const bool closed = complete_closed_form(P);
    const bool blu = bluestein_path(P);
    if (blu && p > 0)
        return evolve_bluestein(P, gammas, ts, p, psi, out_f, out_norm, store, work, s, hook);
    if (mixed_path(P) && p > 0)
        return mixed_run(P, gammas, ts, p, psi, nullptr, out_f, out_norm, nullptr, nullptr, store, false, work, s,
                         hook);
    const std::vector<XGroup> groups = x_groups(n);
    double2* partials = reinterpret_cast<double2*>(work);
    double* lam_tiles = n > kTileBits ? reinterpret_cast<double*>(work + circ_partials_bytes(n)) : nullptr;
    double2* tw = n > kTileBits ? reinterpret_cast<double2*>(work + circ_twiddle_offset(P)) : nullptr;
    // complete graph in closed form: the running state sum follows the partials
    double2* state_sum = closed ? reinterpret_cast<double2*>(work + align256(cpl_partials_bytes(P))) : nullptr;
    const bool tiled = lambda_tiled(P);
    for (const Launch& l : fft_launches(P, p, store)) {
        hipError_t e = hipSuccess;
        hook.before(s);
        switch (l.kind) {
        case QVA_PASS_WHOLE: {
            SmallFftParams sp{};
            sp.psi = psi;
            sp.q = P->q;
            sp.gammas = gammas;
            sp.ts = ts;
            sp.lam = P->lambda;
            sp.lambda_kind = small_lambda_kind(P->lambda_kind);
            sp.n = n;
            sp.p = p;
            sp.flags = SM_INIT | SM_EVOLVE | SM_EXPECT | (store ? SM_STORE : 0);
            sp.out_f = out_f;
            sp.out_norm = out_norm;
            e = launch_small_fft(sp, s);
            break;
        }
        case QVA_PASS_INIT:
            e = launch_init_uniform(psi, N, s);
            break;
        case QVA_PASS_EXPECT:
            e = launch_expect_partials(psi, P->q, N, partials, s);
            break;
        case QVA_PASS_REDUCE: {
            const int64_t count = p == 0 ? expect_partial_count(N)
                                         : (closed ? cpl_blocks(P) : (int64_t(1) << (n - kTileBits)));
            e = launch_final_reduce(partials, count, out_f, out_norm, s);
            break;
        }
        case QVA_PASS_LAMBDA_PREP:
            e = launch_lambda_tiles(P->lambda, lam_tiles, n, s);
            break;
        case QVA_PASS_TWIDDLE_PREP:
            e = launch_twiddle_table(tw, s);
            break;
        case QVA_PASS_CPL_SUM:
            e = launch_final_reduce(partials, cpl_blocks(P), &state_sum->x, &state_sum->y, s);
            break;
        case QVA_PASS_CPL_FIRST:
        case QVA_PASS_CPL_LAYER:
        case QVA_PASS_CPL_LAST:
        case QVA_PASS_CPL_LAST_STORE: {
            CompleteParams c{};
            c.psi = psi;
            c.q = P->q;
            c.gammas = gammas;
            c.ts = ts;
            c.sum_in = state_sum;
            c.partials = partials;
            c.N = N;
            c.mix_layer = l.layer1;
            c.phase_layer = l.phase_layer;
            c.flags = l.xmode;
            e = launch_complete(c, s);
            break;
        }
        default: {
            const XGroup& g = groups[l.group];
            FftPassParams f{};
            f.psi = psi;
            f.q = P->q;
            f.lam = tiled ? lam_tiles : P->lambda;
            f.lambda_kind = tiled ? FFT_LAMBDA_TILED : small_lambda_kind(P->lambda_kind);
            f.mix1 = dev_angle(ts, l.layer1 >= 0 ? l.layer1 : 0);
            f.phase = dev_angle(gammas, l.phase_layer >= 0 ? l.phase_layer : 0);
            f.n = n;
            f.k = g.k;
            f.col_bits = g.col_bits;
            f.flags = l.xmode;
            f.partials = partials;
            f.tw = tw;
            e = launch_fftpass(f, s);
            break;
        }
        }
        hook.after(s);
        if (e != hipSuccess)
            return QVA_ERR_HIP;
    }
    return QVA_OK;
}

// ------------------------------------------------------------- gradient
// Workspace of qva_grad (n > 12): per-tile (f, norm) partials, per-tile
// partials of every (parameter, group) slot, the slot sums, and for an array
// lambda the per-tile copy of lambda.
struct GradLayout {
    int64_t tiles = 0;
    int G = 1;       // t-slots per layer: qubit groups (hypercube) or 1 (circulant)
    int E = 1;       // gamma slots per layer: 1, or the number of Z-string terms
    int nslots = 0;  // p * (G + E) per-tile slot arrays (none for the closed-form mixer)
    size_t fpart = 0, slots = 0, sums = 0, lam = 0, part = 0, state = 0, total = 0;
    size_t pad_phi = 0, pad_chi = 0, b0 = 0, b1 = 0;  // Bluestein: padded vectors, filter spectra
    size_t tw = 0;   // circulant transform passes: the low-group root table
    size_t zd = 0;   // extended QAOA: Im(conj(chi_j) phi_j) at a phase, 2^n doubles
};


GradLayout grad_layout(const qva_problem* P, int p)
{
    GradLayout g;
    const int n = P->n_qubits;
    if (bluestein_path(P)) {
        // (f, norm) partials, both padded vectors, the two filter spectra, 2p
        // per-tile slots and their sums
        const int64_t M = int64_t(1) << blu_bits(P);
        g.tiles = M >> kTileBits;
        g.G = 1;
        g.nslots = 2 * p;
        size_t off = 0;
        const int64_t e = expect_partial_count(problem_N(P));
        g.fpart = off;
        off = align256(off + (size_t)(e > g.tiles ? e : g.tiles) * sizeof(double2));
        g.pad_phi = off;
        off += (size_t)M * sizeof(double2);
        g.pad_chi = off;
        off += (size_t)M * sizeof(double2);
        g.b0 = off;
        off += (size_t)M * sizeof(double2);
        g.b1 = off;
        off += (size_t)M * sizeof(double2);
        g.slots = off;
        off = align256(off + (size_t)g.nslots * (size_t)g.tiles * sizeof(double));
        g.sums = off;
        off = align256(off + (size_t)(g.nslots > 0 ? g.nslots : 1) * sizeof(double));
        g.tw = off;
        off += kTwiddleTableBytes;
        g.total = off;
        return g;
    }
    if (complete_closed_form(P)) {
        // (f, norm) partials, per-block parts, running sums, then 2p slot sums
        g.tiles = cpl_blocks(P);
        g.G = 1;
        size_t off = 0;
        g.fpart = off;
        off = align256(off + cpl_partials_bytes(P));
        g.part = off;
        off = align256(off + (size_t)g.tiles * kCompleteParts * sizeof(double));
        g.state = off;
        off = align256(off + 4 * sizeof(double2));
        g.sums = off;
        off = align256(off + (size_t)(2 * (p > 0 ? p : 1)) * sizeof(double));
        g.lam = g.slots = off;
        g.total = off;
        return g;
    }
    if (n <= kTileBits)
        return g;
    g.tiles = int64_t(1) << (n - kTileBits);
    g.G = P->mixer == QVA_MIX_X ? (int)x_groups(n).size() : 1;
    g.E = problem_terms(P) > 0 ? problem_terms(P) : 1;
    g.nslots = p * (g.G + g.E);
    size_t off = 0;
    g.fpart = off;
    off = align256(off + (size_t)g.tiles * sizeof(double2));
    g.slots = off;
    off = align256(off + (size_t)g.nslots * (size_t)g.tiles * sizeof(double));
    g.sums = off;
    off = align256(off + (size_t)(g.nslots > 0 ? g.nslots : 1) * sizeof(double));
    g.lam = off;
    if (P->mixer == QVA_MIX_CIRCULANT && lambda_tiled(P))
        off = align256(off + (size_t)(int64_t(1) << n) * sizeof(double));
    g.zd = off;
    if (P->mixer == QVA_MIX_X && problem_terms(P) > 0)
        off = align256(off + (size_t)(int64_t(1) << n) * sizeof(double));
    g.tw = off;
    if (P->mixer == QVA_MIX_CIRCULANT)
        off += kTwiddleTableBytes;
    g.total = off;
    return g;
}

// One launch of the gradient plan.
struct GLaunch {
    int kind;               // qva_pass_kind
    int group;              // qubit group, or -1
    int mode;               // XMODE_* / FMODE_* (forward) or GMODE_* (backward)
    int t1, t2, gamma;      // layers of the angles (-1: none)
    int slot_t1, slot_g, slot_t2;  // slot indices (-1: none)
    int vec = 0;            // Bluestein single-vector passes: 0 phi, 1 chi
};

std::vector<GLaunch> grad_launches(const qva_problem* P, int p)
{
    std::vector<GLaunch> L;
    const int n = P->n_qubits;
    const bool circ = P->mixer == QVA_MIX_CIRCULANT;
    if (n <= kTileBits && !complete_closed_form(P) && !bluestein_path(P) && !mixed_path(P)) {
        L.push_back({QVA_PASS_GRAD_WHOLE, -1, 0, -1, -1, -1, -1, -1, -1});
        return L;
    }
    if (p == 0) {
        L.push_back({QVA_PASS_INIT, -1, 0, -1, -1, -1, -1, -1, -1});
        L.push_back({QVA_PASS_EXPECT, -1, 0, -1, -1, -1, -1, -1, -1});
        L.push_back({QVA_PASS_REDUCE, -1, 0, -1, -1, -1, -1, -1, -1});
        return L;
    }
    if (bluestein_path(P)) {
        // the forward up to the last convolution (the filters first), the turn,
        // then per layer backwards: the inverse mixer (its two convolutions,
        // once per vector, with Im<chi|W|phi> between them) and the inverse phase
        const int c = (int)x_groups(blu_bits(P)).size() - 1;
        std::vector<Launch> fw = fft_launches(P, p, false);
        fw.pop_back();  // REDUCE
        fw.pop_back();  // the last pass (B_LAST): the turn replaces it
        for (const Launch& l : fw)
            L.push_back({l.kind, l.group, l.xmode, l.layer1, l.layer2, l.phase_layer, -1, -1, -1});
        L.push_back({QVA_PASS_GRAD_BLU_TURN, c, GMODE_B_TURN, -1, -1, -1, -1, -1, -1});
        auto conv = [&](int filt) {
            for (int v = 0; v < 2; ++v) {
                for (int gi = c - 1; gi >= 1; --gi)
                    L.push_back({QVA_PASS_FFT_DIF, gi, FMODE_DIF, -1, -1, -1, -1, -1, -1, v});
                L.push_back({QVA_PASS_BLU_MUL, 0, FMODE_LOWMUL, -1, filt, -1, -1, -1, -1, v});
                for (int gi = 1; gi <= c - 1; ++gi)
                    L.push_back({QVA_PASS_FFT_DIT, gi, FMODE_DIT, -1, -1, -1, -1, -1, -1, v});
            }
        };
        for (int k = p - 1; k >= 0; --k) {
            conv(0);
            L.push_back({QVA_PASS_GRAD_BLU_LAMBDA, c, GMODE_B_LAM, k, -1, -1, k, -1, -1});
            conv(1);
            L.push_back({k > 0 ? QVA_PASS_GRAD_BLU_PHASE : QVA_PASS_GRAD_BLU_FINAL, c,
                         k > 0 ? GMODE_B_Q : GMODE_B_FINAL, -1, -1, k, -1, p + k, -1});
        }
        L.push_back({QVA_PASS_REDUCE, -1, 0, -1, -1, -1, -1, -1, -1});
        L.push_back({QVA_PASS_GRAD_REDUCE, -1, 0, -1, -1, -1, -1, -1, -1});
        return L;
    }
    if (complete_closed_form(P)) {
        // forward without the last mixer, then the walk back (slots index the sums)
        L.push_back({QVA_PASS_CPL_FIRST, -1, CPMODE_FIRST, -1, -1, 0, -1, -1, -1});
        L.push_back({QVA_PASS_CPL_SUM, -1, 0, -1, -1, -1, -1, -1, -1});
        for (int k = 0; k + 1 < p; ++k) {
            L.push_back({QVA_PASS_CPL_LAYER, -1, CPMODE_LAYER, k, -1, k + 1, -1, -1, -1});
            L.push_back({QVA_PASS_CPL_SUM, -1, 0, -1, -1, -1, -1, -1, -1});
        }
        L.push_back({QVA_PASS_GRAD_CPL_TURN, -1, GCMODE_TURN, p - 1, -1, -1, -1, -1, -1});
        L.push_back({QVA_PASS_GRAD_CPL_SUM, -1, 0, -1, -1, -1, p - 1, -1, -1});
        for (int k = p - 1; k >= 0; --k) {
            L.push_back({QVA_PASS_GRAD_CPL_BACK, -1, k > 0 ? GCMODE_BACK : GCMODE_BACK_LAST, k, -1, k, -1, -1, -1});
            L.push_back({QVA_PASS_GRAD_CPL_SUM, -1, 0, -1, -1, -1, k > 0 ? k - 1 : -1, p + k, -1});
        }
        L.push_back({QVA_PASS_REDUCE, -1, 0, -1, -1, -1, -1, -1, -1});
        L.push_back({QVA_PASS_GRAD_REDUCE, -1, 0, -1, -1, -1, -1, -1, -1});
        return L;
    }
    const int PG = (int)x_groups(n).size();
    const int G = circ ? 1 : PG;
    const int E = problem_terms(P);
    const int zf = E > 0 ? XP_ZTERMS : 0, gz = E > 0 ? GM_ZTERMS : 0;
    auto tslot = [&](int layer, int g) { return layer * G + (circ ? 0 : g); };
    // gamma slot of a layer (with Z-string terms, the first of its E slots)
    auto gslot = [&](int layer) { return p * G + layer * (E > 0 ? E : 1); };
    if (!circ) {
        const std::vector<XPass> fw = x_evolve_plan(PG, p, false);
        const int m = (int)fw.size();
        for (int i = 0; i + 1 < m; ++i) {
            const XPass& f = fw[i];
            const int kind = f.flags == XMODE_FIRST ? QVA_PASS_FIRST
                                                    : (f.flags == XMODE_BOUNDARY ? QVA_PASS_BOUNDARY : QVA_PASS_MIDDLE);
            L.push_back({kind, f.group, f.flags | (f.phase_layer >= 0 ? zf : 0), f.layer1, f.layer2, f.phase_layer,
                         -1, -1, -1});
        }
        const XPass& last = fw[m - 1];
        L.push_back({QVA_PASS_GRAD_TURN, last.group, GMODE_TURN, last.layer1, -1, -1,
                     tslot(last.layer1, last.group), -1, -1});
        for (int i = m - 2; i >= 1; --i) {
            const XPass& f = fw[i];
            if (f.flags == XMODE_MIDDLE)
                L.push_back({QVA_PASS_GRAD_MID, f.group, GMODE_MID, f.layer1, -1, -1,
                             tslot(f.layer1, f.group), -1, -1});
            else {
                L.push_back({QVA_PASS_GRAD_BOUND, f.group, GMODE_BOUND | gz, f.layer2, f.layer1, f.phase_layer,
                             tslot(f.layer2, f.group), gz ? -1 : gslot(f.phase_layer), tslot(f.layer1, f.group)});
                if (gz)
                    L.push_back({QVA_PASS_GRAD_ZSLOT, f.group, GMODE_ZSLOT, -1, -1, f.phase_layer, -1,
                                 gslot(f.phase_layer), -1});
            }
        }
        const XPass& first = fw[0];
        L.push_back({QVA_PASS_GRAD_FINAL, first.group, GMODE_FINAL | gz, 0, -1, 0, tslot(0, first.group),
                     gz ? -1 : gslot(0), -1});
        if (gz)
            L.push_back({QVA_PASS_GRAD_ZSLOT, first.group, GMODE_ZSLOT, -1, -1, 0, -1, gslot(0), -1});
    } else {
        L.push_back({QVA_PASS_TWIDDLE_PREP, -1, 0, -1, -1, -1, -1, -1, -1});
        if (lambda_tiled(P))
            L.push_back({QVA_PASS_LAMBDA_PREP, -1, 0, -1, -1, -1, -1, -1, -1});
        const std::vector<FPass> fw = fft_evolve_plan(PG, p, false);
        const int m = (int)fw.size();
        for (int i = 0; i + 1 < m; ++i) {
            const FPass& f = fw[i];
            L.push_back({fft_pass_kind(f.mode), f.group, f.mode, f.layer, -1, f.phase_layer, -1, -1, -1});
        }
        const FPass& last = fw[m - 1];
        L.push_back({QVA_PASS_GRAD_TURN, last.group, GMODE_TURN, -1, -1, -1, -1, -1, -1});
        for (int i = m - 2; i >= 1; --i) {
            const FPass& f = fw[i];
            if (f.mode == FMODE_DIF)
                L.push_back({QVA_PASS_GRAD_DIT, f.group, GMODE_DIT, -1, -1, -1, -1, -1, -1});
            else if (f.mode == FMODE_DIT)
                L.push_back({QVA_PASS_GRAD_DIF, f.group, GMODE_DIF, -1, -1, -1, -1, -1, -1});
            else if (f.mode == FMODE_LOWDIAG)
                L.push_back({QVA_PASS_GRAD_LOWDIAG, f.group, GMODE_LOWDIAG, f.layer, -1, -1,
                             tslot(f.layer, 0), -1, -1});
            else  // FMODE_BOUNDARY
                L.push_back({QVA_PASS_GRAD_BOUND, f.group, GMODE_BOUND, -1, -1, f.phase_layer, -1,
                             gslot(f.phase_layer), -1});
        }
        const FPass& first = fw[0];
        L.push_back({QVA_PASS_GRAD_FINAL, first.group, GMODE_FINAL, -1, -1, 0, -1, gslot(0), -1});
    }
    L.push_back({QVA_PASS_REDUCE, -1, 0, -1, -1, -1, -1, -1, -1});
    L.push_back({QVA_PASS_GRAD_REDUCE, -1, 0, -1, -1, -1, -1, -1, -1});
    return L;
}

double grad_launch_bytes(const GLaunch& l, const qva_problem* P, int p)
{
    const int n = P->n_qubits;
    const double N = (double)problem_N(P);
    const bool tiled = P->mixer == QVA_MIX_CIRCULANT && lambda_tiled(P);
    const double blocks = (double)cpl_blocks(P);
    switch (l.kind) {
    case QVA_PASS_GRAD_WHOLE:
        return 8.0 * N * (tiled ? 2 : 1);
    case QVA_PASS_GRAD_TURN:
        return 56.0 * N;
    case QVA_PASS_GRAD_MID:
    case QVA_PASS_GRAD_DIF:
    case QVA_PASS_GRAD_DIT:
        return 64.0 * N;
    case QVA_PASS_GRAD_LOWDIAG:
        return 64.0 * N + (tiled ? 8.0 * N : 0.0);
    case QVA_PASS_GRAD_BOUND:  // (a Z-string phase writes Im(conj(chi) phi) instead of reading q)
        return 72.0 * N;
    case QVA_PASS_GRAD_FINAL:
        return 40.0 * N;
    case QVA_PASS_GRAD_ZSLOT:  // the stored values in, one slot per term and tile out
        return 8.0 * N + 8.0 * problem_terms(P) * (N / 4096.0);
    case QVA_PASS_GRAD_REDUCE: {
        const GradLayout g = grad_layout(P, p);
        return 8.0 * (double)g.nslots * (double)g.tiles;
    }
    case QVA_PASS_GRAD_CPL_TURN:
        return 56.0 * N + 16.0 * (1 + kCompleteParts / 2) * blocks;
    case QVA_PASS_GRAD_CPL_BACK:
        return (l.mode == GCMODE_BACK ? 72.0 : 40.0) * N + 8.0 * kCompleteParts * blocks;
    case QVA_PASS_GRAD_CPL_SUM:
        return 8.0 * kCompleteParts * blocks;
    case QVA_PASS_GRAD_BLU_TURN:  // psi in, both out, q at j < N
    case QVA_PASS_GRAD_BLU_LAMBDA:
    case QVA_PASS_GRAD_BLU_PHASE:
    case QVA_PASS_GRAD_BLU_FINAL: {
        const double M = std::ldexp(1.0, blu_bits(P));
        const double lamb = P->lambda_kind == QVA_LAMBDA_ARRAY ? 8.0 * N : 0.0;
        if (l.kind == QVA_PASS_GRAD_BLU_TURN)
            return 48.0 * M + 8.0 * N;
        if (l.kind == QVA_PASS_GRAD_BLU_LAMBDA)
            return 64.0 * M + lamb;
        return (l.kind == QVA_PASS_GRAD_BLU_PHASE ? 64.0 : 32.0) * M + 8.0 * N;
    }
    default: {
        Launch x{l.kind, l.group, l.mode, l.t1, l.t2, l.gamma};
        if (complete_closed_form(P))
            return cpl_launch_bytes(x, P, p);
        if (bluestein_path(P))
            return blu_launch_bytes(x, P, p);
        return P->mixer == QVA_MIX_CIRCULANT ? fft_launch_bytes(x, n, false, tiled) : launch_bytes(x, n, false);
    }
    }
}

int grad_run(const qva_problem* P, const double* gammas, const double* ts, int p, double2* psi, double2* chi,
             double* out_f, double* dgammas, double* dts, char* work, hipStream_t s, EventHook& hook)
{
    if (mixed_path(P) && p > 0)
        return mixed_run(P, gammas, ts, p, psi, chi, out_f, nullptr, dgammas, dts, false, true, work, s, hook);
    const int n = P->n_qubits;
    const int64_t N = problem_N(P);
    const bool circ = P->mixer == QVA_MIX_CIRCULANT;
    const std::vector<XGroup> groups = x_groups(n);
    const GradLayout W = grad_layout(P, p);
    double2* fpart = reinterpret_cast<double2*>(work + W.fpart);
    double* slots = reinterpret_cast<double*>(work + W.slots);
    double* sums = reinterpret_cast<double*>(work + W.sums);
    double* lam_tiles = reinterpret_cast<double*>(work + W.lam);
    double* cpart = reinterpret_cast<double*>(work + W.part);
    double2* cstate = reinterpret_cast<double2*>(work + W.state);  // [0]: forward sum, [1..2]: backward
    double2* tw = reinterpret_cast<double2*>(work + W.tw);
    const bool blu = bluestein_path(P);
    const bool tiled = circ && lambda_tiled(P) && !blu;
    const std::vector<XGroup> bgroups = blu ? x_groups(blu_bits(P)) : std::vector<XGroup>();
    double2* pads[2] = {reinterpret_cast<double2*>(work + W.pad_phi), reinterpret_cast<double2*>(work + W.pad_chi)};
    double2* spec[2] = {reinterpret_cast<double2*>(work + W.b0), reinterpret_cast<double2*>(work + W.b1)};
    const int blu_kind = P->lambda_kind == QVA_LAMBDA_RING ? FFT_LAMBDA_RING : FFT_LAMBDA_NATURAL;
    auto slot_ptr = [&](int idx) -> double* { return idx >= 0 ? slots + (int64_t)idx * W.tiles : nullptr; };
    for (const GLaunch& l : grad_launches(P, p)) {
        hipError_t e = hipSuccess;
        hook.before(s);
        const bool blu_fft = blu && l.group >= 0 &&
                             (l.kind == QVA_PASS_BLU_CHIRP || l.kind == QVA_PASS_BLU_TILE || l.kind == QVA_PASS_BLU_FIRST ||
                              l.kind == QVA_PASS_BLU_MUL || l.kind == QVA_PASS_BLU_LAMBDA || l.kind == QVA_PASS_BLU_PHASE ||
                              l.kind == QVA_PASS_FFT_DIF || l.kind == QVA_PASS_FFT_DIT);
        if (blu_fft) {
            // the forward's single-vector passes over a padded buffer (as in evolve_bluestein)
            const XGroup& g = bgroups[l.group];
            FftPassParams f{};
            f.psi = pads[l.vec];
            f.q = P->q;
            f.lam = P->lambda;
            f.lambda_kind = blu_kind;
            f.mix1 = dev_angle(ts, l.t1 >= 0 ? l.t1 : 0);
            f.phase = dev_angle(gammas, l.gamma >= 0 ? l.gamma : 0);
            f.n = blu_bits(P);
            f.k = g.k;
            f.col_bits = g.col_bits;
            f.flags = l.mode;
            f.partials = fpart;
            f.nb = N;
            f.bt = spec[l.t2 > 0 ? 1 : 0];
            f.out = l.kind == QVA_PASS_BLU_TILE ? spec[l.t2 > 0 ? 1 : 0] : nullptr;
            f.conj = l.t2 > 0 ? 1 : 0;
            f.tw = tw;
            e = launch_fftpass(f, s);
            hook.after(s);
            if (e != hipSuccess)
                return QVA_ERR_HIP;
            continue;
        }
        switch (l.kind) {
        case QVA_PASS_GRAD_WHOLE: {
            SmallGradParams sp{};
            sp.q = P->q;
            sp.terms = reinterpret_cast<const ZTerm*>(P->terms);
            sp.n_terms = problem_terms(P);
            sp.gammas = gammas;
            sp.ts = ts;
            sp.lam = P->lambda;
            sp.lambda_kind = small_lambda_kind(P->lambda_kind);
            sp.circulant = circ ? 1 : 0;
            sp.n = n;
            sp.p = p;
            sp.out_f = out_f;
            sp.dgammas = dgammas;
            sp.dts = dts;
            e = launch_small_grad(sp, s);
            break;
        }
        case QVA_PASS_INIT:
            e = launch_init_uniform(psi, N, s);
            break;
        case QVA_PASS_EXPECT:
            e = launch_expect_partials(psi, P->q, N, fpart, s);
            break;
        case QVA_PASS_REDUCE: {
            const int64_t count = p == 0 ? expect_partial_count(N) : W.tiles;
            e = launch_final_reduce(fpart, count, out_f, nullptr, s);
            break;
        }
        case QVA_PASS_GRAD_REDUCE:
            e = launch_grad_reduce(slots, W.nslots, W.tiles, sums, p, W.G, W.E, dgammas, dts, s);
            break;
        case QVA_PASS_CPL_FIRST:
        case QVA_PASS_CPL_LAYER: {
            CompleteParams c{};
            c.psi = psi;
            c.q = P->q;
            c.gammas = gammas;
            c.ts = ts;
            c.sum_in = cstate;
            c.partials = fpart;
            c.N = N;
            c.mix_layer = l.t1;
            c.phase_layer = l.gamma;
            c.flags = l.mode;
            e = launch_complete(c, s);
            break;
        }
        case QVA_PASS_CPL_SUM:
            e = launch_final_reduce(fpart, W.tiles, &cstate->x, &cstate->y, s);
            break;
        case QVA_PASS_GRAD_CPL_TURN:
        case QVA_PASS_GRAD_CPL_BACK: {
            CompleteGradParams c{};
            c.phi = psi;
            c.chi = chi;
            c.q = P->q;
            c.gammas = gammas;
            c.ts = ts;
            c.sums_in = l.kind == QVA_PASS_GRAD_CPL_TURN ? cstate : cstate + 1;
            c.part = cpart;
            c.fpart = fpart;
            c.N = N;
            c.layer = l.t1;
            c.flags = l.mode;
            e = launch_complete_grad(c, s);
            break;
        }
        case QVA_PASS_GRAD_CPL_SUM:
            e = launch_complete_gsum(cpart, W.tiles, cstate + 1, sums, l.slot_t1, l.slot_g, s);
            break;
        case QVA_PASS_LAMBDA_PREP:
            e = launch_lambda_tiles(P->lambda, lam_tiles, n, s);
            break;
        case QVA_PASS_TWIDDLE_PREP:
            e = launch_twiddle_table(tw, s);
            break;
        case QVA_PASS_FIRST:
        case QVA_PASS_MIDDLE:
        case QVA_PASS_BOUNDARY: {
            XPassParams x = xpass_base(psi, P->q, n, groups[l.group]);
            x.flags = l.mode;
            x.mix1 = dev_angle(ts, l.t1);
            x.mix2 = dev_angle(ts, l.t2 >= 0 ? l.t2 : 0);
            x.phase = dev_angle(gammas, l.gamma >= 0 ? l.gamma * W.E : 0);
            x.terms = reinterpret_cast<const ZTerm*>(P->terms);
            x.n_terms = problem_terms(P);
            x.qt = q_tiles_block(P, l.group, l.mode);
            e = launch_xpass(x, s);
            break;
        }
        case QVA_PASS_FFT_FIRST:
        case QVA_PASS_FFT_DIF:
        case QVA_PASS_FFT_LOWDIAG:
        case QVA_PASS_FFT_DIT:
        case QVA_PASS_FFT_BOUNDARY: {
            const XGroup& g = groups[l.group];
            FftPassParams f{};
            f.psi = psi;
            f.q = P->q;
            f.lam = tiled ? lam_tiles : P->lambda;
            f.lambda_kind = tiled ? FFT_LAMBDA_TILED : small_lambda_kind(P->lambda_kind);
            f.mix1 = dev_angle(ts, l.t1 >= 0 ? l.t1 : 0);
            f.phase = dev_angle(gammas, l.gamma >= 0 ? l.gamma : 0);
            f.n = n;
            f.k = g.k;
            f.col_bits = g.col_bits;
            f.flags = l.mode;
            f.tw = tw;
            e = launch_fftpass(f, s);
            break;
        }
        case QVA_PASS_GRAD_DIF:
        case QVA_PASS_GRAD_DIT: {
            // no inner product here: the single-vector transform, once per vector
            const XGroup& g = groups[l.group];
            FftPassParams f{};
            f.n = n;
            f.k = g.k;
            f.col_bits = g.col_bits;
            f.flags = l.kind == QVA_PASS_GRAD_DIF ? FMODE_DIF : FMODE_DIT;
            f.psi = psi;
            e = launch_fftpass(f, s);
            if (e == hipSuccess) {
                f.psi = chi;
                e = launch_fftpass(f, s);
            }
            break;
        }
        default: {  // backward passes
            const XGroup& g = blu ? bgroups[l.group] : groups[l.group];
            GradPassParams gp{};
            gp.phi = blu ? pads[0] : psi;
            gp.chi = blu ? pads[1] : chi;
            gp.q = P->q;
            gp.lam = tiled ? lam_tiles : P->lambda;
            gp.lambda_kind = blu ? blu_kind : tiled ? FFT_LAMBDA_TILED : small_lambda_kind(P->lambda_kind);
            gp.nb = N;
            gp.t1 = dev_angle(ts, l.t1 >= 0 ? l.t1 : 0);
            gp.t2 = dev_angle(ts, l.t2 >= 0 ? l.t2 : 0);
            gp.gamma = dev_angle(gammas, l.gamma >= 0 ? l.gamma * W.E : 0);
            gp.n = blu ? blu_bits(P) : n;
            gp.k = g.k;
            gp.col_bits = g.col_bits;
            gp.flags = l.mode;
            gp.slot_t1 = slot_ptr(l.slot_t1);
            gp.slot_g = l.kind == QVA_PASS_GRAD_ZSLOT ? nullptr : slot_ptr(l.slot_g);
            gp.slot_t2 = slot_ptr(l.slot_t2);
            gp.fpart = fpart;
            gp.terms = reinterpret_cast<const ZTerm*>(P->terms);
            gp.n_terms = problem_terms(P);
            gp.slot_terms = l.kind == QVA_PASS_GRAD_ZSLOT ? slot_ptr(l.slot_g) : nullptr;
            gp.zd = reinterpret_cast<double*>(work + W.zd);
            gp.tw = tw;
            // the hypercube's backward passes that read q take it from the
            // tile-ordered copy when the problem has one (same layout as the
            // forward boundary passes, last_layout<C>())
            if (!circ && !blu && (l.mode == GMODE_TURN || l.mode == GMODE_BOUND || l.mode == GMODE_FINAL)) {
                gp.qt = q_tiles_block(P, l.group, XP_PHASE_MID);
                if (gp.qt)
                    gp.flags |= GM_QTILE;
            }
            e = launch_gradpass(gp, circ, s);
            break;
        }
        }
        hook.after(s);
        if (e != hipSuccess)
            return QVA_ERR_HIP;
    }
    return QVA_OK;
}

int evolve_common(const qva_problem* P, const double* gammas_dev, const double* ts_dev, int p,
                  qva_c128* psi, double* out_f_dev, double* out_norm_dev, int flags, void* work,
                  size_t work_bytes, void* stream, EventHook& hook);

int grad_common(const qva_problem* P, const double* gammas_dev, const double* ts_dev, int p,
                qva_c128* psi, qva_c128* chi, double* out_f_dev, double* dgammas_dev, double* dts_dev,
                void* work, size_t work_bytes, void* stream, EventHook& hook);

}  // namespace

namespace {

// ------------------------------------------------------------ QAOAz XY
std::vector<std::pair<int, int>> xy_pairs_of(const qva_problem* P)
{
    std::vector<std::pair<int, int>> v;
    for (int i = 0; i < P->n_xy_pairs; ++i)
        v.push_back({P->xy_pairs[2 * i], P->xy_pairs[2 * i + 1]});
    return v;
}

int64_t xy_tiles(int n) { return n <= kTileBits ? 1 : int64_t(1) << (n - kTileBits); }

// One launch of the parity-mixer plan: pass = index into the layer plan.
struct XyLaunch {
    int kind, pass, layer, flags, slot_t, slot_g;
};

// Forward: each layer's passes in order, the phase in the first; the last pass
// takes <Q> (the turn of the gradient also writes psi_p and Q psi_p).  Backward:
// every forward pass inverted, in reverse order; t slot (layer, pass), gamma
// slot of the layer with its first pass.
std::vector<XyLaunch> xy_launches(const qva_problem* P, int p, bool store, bool grad)
{
    const int G = (int)xy_layer_plan(P->n_qubits, xy_pairs_of(P)).size();
    std::vector<XyLaunch> L;
    if (p == 0) {
        L.push_back({QVA_PASS_EXPECT, -1, -1, 0, -1, -1});
        L.push_back({QVA_PASS_REDUCE, -1, -1, 0, -1, -1});
        return L;
    }
    for (int k = 0; k < p; ++k)
        for (int i = 0; i < G; ++i) {
            int fl = (i == 0 ? XY_PHASE : 0) | XY_STORE, kind = QVA_PASS_XY;
            if (k == p - 1 && i == G - 1) {
                if (grad) {
                    fl |= XY_EXPECT | XY_CHI;
                    kind = QVA_PASS_XY_TURN;
                } else {
                    fl = (fl & ~XY_STORE) | XY_EXPECT | (store ? XY_STORE : 0);
                    kind = QVA_PASS_XY_LAST;
                }
            }
            L.push_back({kind, i, k, fl, -1, -1});
        }
    if (grad)
        for (int k = p - 1; k >= 0; --k)
            for (int i = G - 1; i >= 0; --i)
                L.push_back({QVA_PASS_GRAD_XY, i, k, i == 0 ? XY_PHASE : 0, k * G + i, i == 0 ? p * G + k : -1});
    L.push_back({QVA_PASS_REDUCE, -1, -1, 0, -1, -1});
    if (grad)
        L.push_back({QVA_PASS_GRAD_REDUCE, -1, -1, 0, -1, -1});
    return L;
}

// Workspace: (f, norm) partials per tile, then for the gradient p (G + 1)
// per-tile slot arrays and their sums.
struct XyLayout {
    int64_t tiles = 1;
    int G = 1, nslots = 0;
    size_t fpart = 0, slots = 0, sums = 0, total = 0;
};

XyLayout xy_layout(const qva_problem* P, int p, bool grad)
{
    XyLayout w;
    const int n = P->n_qubits;
    w.tiles = xy_tiles(n);
    w.G = (int)xy_layer_plan(n, xy_pairs_of(P)).size();
    const int64_t parts = std::max<int64_t>(w.tiles, expect_partial_count(int64_t(1) << n));
    size_t off = align256((size_t)parts * sizeof(double2));
    if (grad && p > 0) {
        w.nslots = p * (w.G + 1);
        w.slots = off;
        off = align256(off + (size_t)w.nslots * (size_t)w.tiles * sizeof(double));
        w.sums = off;
        off = align256(off + (size_t)w.nslots * sizeof(double));
    }
    w.total = off;
    return w;
}

double xy_launch_bytes(const XyLaunch& l, const qva_problem* P, int p, bool grad)
{
    const int n = P->n_qubits;
    const double N = std::ldexp(1.0, n);
    switch (l.kind) {
    case QVA_PASS_EXPECT:
        return 24.0 * N;
    case QVA_PASS_REDUCE:
        return 16.0 * (double)(p == 0 ? expect_partial_count(int64_t(1) << n) : xy_tiles(n));
    case QVA_PASS_GRAD_REDUCE: {
        const XyLayout w = xy_layout(P, p, grad);
        return 8.0 * (double)w.nslots * (double)w.tiles;
    }
    case QVA_PASS_GRAD_XY:
        return (64.0 + ((l.flags & XY_PHASE) ? 8.0 : 0.0)) * N;
    default:
        return (16.0 + ((l.flags & (XY_PHASE | XY_EXPECT)) ? 8.0 : 0.0) + ((l.flags & XY_STORE) ? 16.0 : 0.0) +
                ((l.flags & XY_CHI) ? 16.0 : 0.0)) *
               N;
    }
}

int xy_run(const qva_problem* P, const double* gammas, const double* ts, int p, double2* psi, double2* chi,
           double* out_f, double* out_norm, double* dgammas, double* dts, bool store, bool grad, char* work,
           hipStream_t s, EventHook& hook)
{
    const int n = P->n_qubits;
    const int64_t N = int64_t(1) << n;
    const std::vector<XyLayerPass> lp = xy_layer_plan(n, xy_pairs_of(P));
    if (lp.empty())
        return QVA_ERR_UNSUPPORTED;
    const XyLayout W = xy_layout(P, p, grad);
    double2* fpart = reinterpret_cast<double2*>(work + W.fpart);
    double* slots = reinterpret_cast<double*>(work + W.slots);
    double* sums = reinterpret_cast<double*>(work + W.sums);
    for (const XyLaunch& l : xy_launches(P, p, store, grad)) {
        hipError_t e = hipSuccess;
        hook.before(s);
        switch (l.kind) {
        case QVA_PASS_EXPECT:
            e = launch_expect_partials(psi, P->q, N, fpart, s);
            break;
        case QVA_PASS_REDUCE:
            e = launch_final_reduce(fpart, p == 0 ? expect_partial_count(N) : W.tiles, out_f, out_norm, s);
            break;
        case QVA_PASS_GRAD_REDUCE:
            e = launch_grad_reduce(slots, W.nslots, W.tiles, sums, p, W.G, 1, dgammas, dts, s);
            break;
        default: {
            const XyLayerPass& ps = lp[l.pass];
            XyPassParams x{};
            x.psi = psi;
            x.chi = chi;
            x.q = P->q;
            x.gammas = gammas;
            x.ts = ts;
            x.n = n;
            x.k = ps.g.k;
            x.C = ps.g.C;
            x.elems = n <= kTileBits ? (int)N : (1 << kTileBits);
            x.flags = l.flags;
            x.layer = l.layer;
            x.n_ops = (int)ps.ops.size();
            for (int o = 0; o < x.n_ops; ++o) {
                x.ea[o] = (uint8_t)ps.ops[o].first;
                x.eb[o] = (uint8_t)ps.ops[o].second;
            }
            x.partials = fpart;
            x.slot_t = l.slot_t >= 0 ? slots + (int64_t)l.slot_t * W.tiles : nullptr;
            x.slot_g = l.slot_g >= 0 ? slots + (int64_t)l.slot_g * W.tiles : nullptr;
            e = l.kind == QVA_PASS_GRAD_XY ? launch_xygrad(x, W.tiles, s) : launch_xypass(x, W.tiles, s);
            break;
        }
        }
        hook.after(s);
        if (e != hipSuccess)
            return QVA_ERR_HIP;
    }
    return QVA_OK;
}

}  // namespace

// ------------------------------------------------- static per-device scratch
// The workspace of qva_evolve_noalloc.  In host code `scratch` is only a
// host-side stand-in for the symbol, never a device address: host code uses
// the address hipGetSymbolAddress returns for each device (static_scratch).
static __device__ __align__(256) unsigned char scratch[QVA_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices];

// Device address of the scratch array of the GPU that `s` belongs to (the
// current device for the NULL stream), looked up once per device with that
// device current.
int static_scratch(hipStream_t s, void** out)
{
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess)
        return QVA_ERR_HIP;
    int dev = cur;
    if (s) {
        hipDevice_t d = 0;
        if (hipStreamGetDevice(s, &d) != hipSuccess)
            return QVA_ERR_HIP;
        dev = d;
    }
    if (dev < 0 || dev >= kMaxScratchDevices)
        return QVA_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        if (dev != cur && hipSetDevice(dev) != hipSuccess)
            return QVA_ERR_HIP;
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (dev != cur)
            (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr)
            return QVA_ERR_HIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return QVA_OK;
}

}  // namespace

extern "C" {

const char* qva_status_string(int status)
{
    switch (status) {
    case QVA_OK:
        return "ok";
    case QVA_ERR_ARG:
        return "invalid argument";
    case QVA_ERR_SIZE:
        return "size out of the supported range";
    case QVA_ERR_ALIGN:
        return "misaligned device pointer";
    case QVA_ERR_WORKSPACE:
        return "workspace missing or too small";
    case QVA_ERR_HIP:
        return "HIP launch or runtime error";
    case QVA_ERR_UNSUPPORTED:
        return "unsupported request";
    case QVA_ERR_SCRATCH:
        return "request needs more workspace than the static scratch holds";
    default:
        return "unknown status";
    }
}

const char* qva_version(void) { return "libqva 0.1 (gfx950)"; }

int qva_set_group_split(int n_qubits, const int* bits, int count)
{
    if (n_qubits <= kTileBits || n_qubits > QVA_MAX_QUBITS)
        return QVA_ERR_SIZE;
    if (count < 0 || count > n_qubits - kTileBits || (count > 0 && !bits))
        return QVA_ERR_ARG;
    std::vector<int> hi;
    int sum = 0;
    for (int i = 0; i < count; ++i) {
        if (bits[i] < 1 || bits[i] > kMaxHighBits)
            return QVA_ERR_ARG;
        hi.push_back(bits[i]);
        sum += bits[i];
    }
    if (count > 0 && sum != n_qubits - kTileBits)
        return QVA_ERR_ARG;
    std::lock_guard<std::mutex> lock(g_split_mu);
    g_split[n_qubits] = hi;
    return QVA_OK;
}

int qva_get_group_split(int n_qubits, int* bits, int max)
{
    if (n_qubits < 1 || n_qubits > QVA_MAX_QUBITS)
        return QVA_ERR_SIZE;
    if (max < 0 || (max > 0 && !bits))
        return QVA_ERR_ARG;
    const std::vector<int> hi = x_split(n_qubits);
    for (int i = 0; i < (int)hi.size() && i < max; ++i)
        bits[i] = hi[i];
    return (int)hi.size();
}

int qva_parity_ring_pairs(const int* ring, int m, int* pairs, int max_pairs)
{
    if (m < 0 || (m > 0 && !ring) || max_pairs < 0 || (max_pairs > 0 && !pairs))
        return QVA_ERR_ARG;
    if (m < 2)
        return 0;
    int count = 0;
    auto put = [&](int a, int b) {
        if (count < max_pairs) {
            pairs[2 * count] = a;
            pairs[2 * count + 1] = b;
        }
        ++count;
    };
    // ring positions a = 1..m are ring[a - 1]; position m + 1 wraps to 1
    for (int a = 1; a < m; a += 2)  // B_odd
        put(ring[a - 1], ring[a]);
    for (int a = 2; a <= m; a += 2)  // B_even
        put(ring[a - 1], ring[a % m]);
    if (m % 2 == 1 && m >= 3)  // B_last
        put(ring[m - 1], ring[0]);
    return count;
}

int qva_init_uniform(qva_c128* psi, int64_t N, void* stream)
{
    if (!psi || N < 1)
        return psi ? QVA_ERR_SIZE : QVA_ERR_ARG;
    if (!aligned(psi, 16))
        return QVA_ERR_ALIGN;
    return hip_status(launch_init_uniform(reinterpret_cast<double2*>(psi), N, as_stream(stream)));
}

int qva_phase(qva_c128* psi, const double* q, int64_t N, double gamma, void* stream)
{
    if (!psi || !q)
        return QVA_ERR_ARG;
    if (N < 1)
        return QVA_ERR_SIZE;
    if (!aligned(psi, 16) || !aligned(q, 8))
        return QVA_ERR_ALIGN;
    return hip_status(launch_phase(reinterpret_cast<double2*>(psi), q, N, gamma, as_stream(stream)));
}

int qva_mix_x(qva_c128* psi, int n_qubits, double t, void* stream)
{
    if (!psi)
        return QVA_ERR_ARG;
    if (n_qubits < 1 || n_qubits > QVA_MAX_QUBITS)
        return QVA_ERR_SIZE;
    if (!aligned(psi, 16))
        return QVA_ERR_ALIGN;
    double2* d = reinterpret_cast<double2*>(psi);
    hipStream_t s = as_stream(stream);
    if (n_qubits <= kTileBits) {
        SmallParams sp{};
        sp.psi = d;
        sp.n = n_qubits;
        sp.t_val = t;
        sp.flags = SM_MIX_ONCE | SM_STORE;
        return hip_status(launch_small(sp, s));
    }
    const std::vector<XGroup> groups = x_groups(n_qubits);
    for (size_t i = 0; i < groups.size(); ++i) {
        XPassParams x = xpass_base(d, nullptr, n_qubits, groups[i]);
        x.flags = XP_MIX1 | XP_STORE | (i + 1 == groups.size() ? XP_FINAL_SCALE : 0);
        x.mix1 = host_angle(t);
        if (launch_xpass(x, s) != hipSuccess)
            return QVA_ERR_HIP;
    }
    return QVA_OK;
}

size_t qva_mix_circulant_workspace_bytes(int64_t N)
{
    if (N >= 2 && (N & (N - 1)) != 0) {
        // enough for every eigenvalue kind: the complete graph's sums, and for
        // the ring and arrays the mixed-radix tables or Bluestein's buffers
        if (N > (int64_t(1) << QVA_MAX_QUBITS))
            return 0;
        const size_t cpl = complete_mix_bytes(N);
        MrGeom m{};
        if (mixed_geom(N, &m))
            return std::max(cpl, align256(sizeof(MrGeom)) + align256(mr_table_bytes(m)));
        if (N < (int64_t(1) << 31))
            return std::max(cpl, blu_layout_n(N, false).total);
        return cpl;
    }
    return N > (int64_t(1) << kTileBits) ? kTwiddleTableBytes : 0;
}

int qva_mix_circulant(qva_c128* psi, const double* lambda, int lambda_kind, int64_t N, double t, void* work,
                      size_t work_bytes, void* stream)
{
    if (!psi)
        return QVA_ERR_ARG;
    if (lambda_kind != QVA_LAMBDA_ARRAY && lambda_kind != QVA_LAMBDA_RING &&
        lambda_kind != QVA_LAMBDA_COMPLETE)
        return QVA_ERR_ARG;
    if (lambda_kind == QVA_LAMBDA_ARRAY && !lambda)
        return QVA_ERR_ARG;
    if (N < 2)
        return QVA_ERR_SIZE;
    if ((N & (N - 1)) != 0) {
        // N solutions, not a power of two: the complete graph in closed form
        // (N <= 2^QVA_MAX_QUBITS); the ring and arrays through the
        // mixed-radix passes (prime factors <= 31), else Bluestein's
        // transform (N < 2^31)
        if (N > (int64_t(1) << QVA_MAX_QUBITS))
            return QVA_ERR_SIZE;
        MrGeom m{};
        const bool mixed = lambda_kind != QVA_LAMBDA_COMPLETE && mixed_geom(N, &m);
        if (lambda_kind != QVA_LAMBDA_COMPLETE && !mixed && N >= (int64_t(1) << 31))
            return QVA_ERR_UNSUPPORTED;
        if (!aligned(psi, 16) || (lambda_kind == QVA_LAMBDA_ARRAY && !aligned(lambda, 8)))
            return QVA_ERR_ALIGN;
        if (!work || work_bytes < qva_mix_circulant_workspace_bytes(N))
            return QVA_ERR_WORKSPACE;
        if (!aligned(work, 16))
            return QVA_ERR_ALIGN;
        double2* d = reinterpret_cast<double2*>(psi);
        char* w = static_cast<char*>(work);
        if (lambda_kind == QVA_LAMBDA_COMPLETE)
            return complete_mix(d, N, t, w, as_stream(stream));
        if (mixed)
            return mixed_mix(d, lambda, lambda_kind, m, t, w, as_stream(stream));
        return bluestein_mix(d, lambda, lambda_kind, N, t, w, as_stream(stream));
    }
    int n = 0;
    while (n <= QVA_MAX_QUBITS && (int64_t(1) << n) < N)
        ++n;
    if (n > QVA_MAX_QUBITS)
        return QVA_ERR_SIZE;
    if (!aligned(psi, 16) || (lambda_kind == QVA_LAMBDA_ARRAY && !aligned(lambda, 8)))
        return QVA_ERR_ALIGN;
    const size_t need = qva_mix_circulant_workspace_bytes(N);
    if (need && (!work || work_bytes < need))
        return QVA_ERR_WORKSPACE;
    if (work && !aligned(work, 16))
        return QVA_ERR_ALIGN;
    double2* d = reinterpret_cast<double2*>(psi);
    hipStream_t s = as_stream(stream);
    const int lk = small_lambda_kind(lambda_kind);
    if (n <= kTileBits) {
        SmallFftParams sp{};
        sp.psi = d;
        sp.lam = lambda;
        sp.lambda_kind = lk;
        sp.n = n;
        sp.t_val = t;
        sp.flags = SM_MIX_ONCE | SM_STORE;
        return hip_status(launch_small_fft(sp, s));
    }
    double2* tw = reinterpret_cast<double2*>(work);
    if (launch_twiddle_table(tw, s) != hipSuccess)
        return QVA_ERR_HIP;
    const std::vector<XGroup> groups = x_groups(n);
    for (const FPass& fp : fft_mix_plan((int)groups.size())) {
        FftPassParams f{};
        f.psi = d;
        f.lam = lambda;
        f.lambda_kind = lk;
        f.mix1 = host_angle(t);
        f.phase = host_angle(0.0);
        f.n = n;
        f.k = groups[fp.group].k;
        f.col_bits = groups[fp.group].col_bits;
        f.flags = fp.mode;
        f.tw = tw;
        if (launch_fftpass(f, s) != hipSuccess)
            return QVA_ERR_HIP;
    }
    return QVA_OK;
}

size_t qva_q_tiles_bytes(const qva_problem* P)
{
    if (!P)
        return 0;
    qva_problem Q = *P;  // a copy the descriptor already carries is not an input here
    Q.q_tiles = nullptr;
    if (check_problem(&Q, 0) != QVA_OK || !reads_q_tiles(&Q))
        return 0;
    return x_groups(Q.n_qubits).size() * (size_t(1) << Q.n_qubits) * sizeof(double);
}

int qva_q_tiles(const qva_problem* P, double* out, size_t out_bytes, uint64_t* key, void* stream)
{
    if (!P)
        return QVA_ERR_ARG;
    qva_problem Q = *P;  // the copy being written is not an input here
    Q.q_tiles = nullptr;
    int st = check_problem(&Q, 0);
    if (st != QVA_OK)
        return st;
    if (!out || !key)
        return QVA_ERR_ARG;
    if (!aligned(out, 8))
        return QVA_ERR_ALIGN;
    const size_t need = qva_q_tiles_bytes(&Q);
    if (need == 0)
        return QVA_ERR_UNSUPPORTED;
    if (out_bytes < need)
        return QVA_ERR_WORKSPACE;
    const int n = Q.n_qubits;
    const std::vector<XGroup> groups = x_groups(n);
    for (size_t i = 0; i < groups.size(); ++i)
        if (launch_qtile(Q.q, out + ((int64_t)i << n), n, groups[i].k, groups[i].col_bits,
                         as_stream(stream)) != hipSuccess)
            return QVA_ERR_HIP;
    *key = q_tiles_key(n);
    return QVA_OK;
}

size_t qva_expectation_workspace_bytes(int64_t N)
{
    if (N < 1)
        return 0;
    return (size_t)expect_partial_count(N) * sizeof(double2);
}

size_t qva_workspace_bytes(const qva_problem* P, int p, int for_grad)
{
    if (check_problem(P, p) != QVA_OK)
        return 0;
    const int n = P->n_qubits;
    if (P->mixer == QVA_MIX_XY)
        return xy_layout(P, p, for_grad != 0).total;
    if (complete_closed_form(P)) {
        if (for_grad && p > 0)
            return grad_layout(P, p).total;
        return align256(cpl_partials_bytes(P)) + 256;  // partials, then the running state sum
    }
    if (mixed_path(P)) {
        if (p == 0)
            return (size_t)expect_partial_count(problem_N(P)) * sizeof(double2);
        MrGeom m{};
        mixed_geom(problem_N(P), &m);
        return mr_layout(m, p, for_grad != 0).total;
    }
    if (bluestein_path(P)) {
        if (p == 0)
            return (size_t)expect_partial_count(problem_N(P)) * sizeof(double2);
        return for_grad ? grad_layout(P, p).total : blu_layout(P).total;
    }
    if (n <= kTileBits)
        return 0;
    if (for_grad && p > 0)
        return grad_layout(P, p).total;
    if (P->mixer == QVA_MIX_CIRCULANT && p > 0)
        return circ_twiddle_offset(P) + kTwiddleTableBytes;
    size_t bytes = circ_partials_bytes(n);
    if (P->mixer == QVA_MIX_CIRCULANT && lambda_tiled(P))
        bytes += (size_t)(int64_t(1) << n) * sizeof(double);
    return bytes;
}

int qva_expectation(const qva_c128* psi, const double* q, int64_t N, double* out_f_dev,
                    double* out_norm_dev, void* work, size_t work_bytes, void* stream)
{
    if (!psi || !q || !out_f_dev)
        return QVA_ERR_ARG;
    if (N < 1)
        return QVA_ERR_SIZE;
    if (!aligned(psi, 16) || !aligned(q, 8) || !aligned(out_f_dev, 8) ||
        (out_norm_dev && !aligned(out_norm_dev, 8)))
        return QVA_ERR_ALIGN;
    const size_t need = qva_expectation_workspace_bytes(N);
    if (!work || work_bytes < need)
        return QVA_ERR_WORKSPACE;
    if (!aligned(work, 16))
        return QVA_ERR_ALIGN;
    hipStream_t s = as_stream(stream);
    double2* partials = reinterpret_cast<double2*>(work);
    hipError_t e = launch_expect_partials(reinterpret_cast<const double2*>(psi), q, N, partials, s);
    if (e == hipSuccess)
        e = launch_final_reduce(partials, expect_partial_count(N), out_f_dev, out_norm_dev, s);
    return hip_status(e);
}

int qva_evolve(const qva_problem* P, const double* gammas_dev, const double* ts_dev, int p,
               qva_c128* psi, double* out_f_dev, double* out_norm_dev, int flags, void* work,
               size_t work_bytes, void* stream)
{
    EventHook hook;
    return evolve_common(P, gammas_dev, ts_dev, p, psi, out_f_dev, out_norm_dev, flags, work,
                         work_bytes, stream, hook);
}

int qva_evolve_timed(const qva_problem* P, const double* gammas_dev, const double* ts_dev, int p,
                     qva_c128* psi, double* out_f_dev, double* out_norm_dev, int flags, void* work,
                     size_t work_bytes, void* const* events, int n_events, void* stream)
{
    if (!events || n_events < 0)
        return QVA_ERR_ARG;
    EventHook hook;
    hook.ev = events;
    hook.n = n_events;
    return evolve_common(P, gammas_dev, ts_dev, p, psi, out_f_dev, out_norm_dev, flags, work,
                         work_bytes, stream, hook);
}

int qva_evolve_noalloc(const qva_problem* P, const double* gammas_dev, const double* ts_dev, int p,
                       qva_c128* psi, double* out_f_dev, double* out_norm_dev, int flags, void* stream)
{
    // argument errors first (as qva_evolve reports them), then the size limit,
    // all before the device is touched
    int st = check_problem(P, p);
    if (st != QVA_OK)
        return st;
    if (!psi || !out_f_dev || (p > 0 && (!gammas_dev || !ts_dev)) || (flags & ~QVA_EVOLVE_SKIP_FINAL_STATE))
        return QVA_ERR_ARG;
    const size_t need = qva_workspace_bytes(P, p, 0);
    if (need > QVA_STATIC_SCRATCH_BYTES)
        return QVA_ERR_SCRATCH;
    void* work = nullptr;
    if (need) {
        st = static_scratch(as_stream(stream), &work);
        if (st != QVA_OK)
            return st;
    }
    EventHook hook;
    return evolve_common(P, gammas_dev, ts_dev, p, psi, out_f_dev, out_norm_dev, flags, work,
                         need ? QVA_STATIC_SCRATCH_BYTES : 0, stream, hook);
}

int qva_plan(const qva_problem* P, int p, int for_grad, int flags, qva_pass_info* out, int max_out)
{
    int st = check_problem(P, p);
    if (st != QVA_OK)
        return st;
    if (max_out < 0 || (max_out > 0 && !out) || (flags & ~QVA_EVOLVE_SKIP_FINAL_STATE))
        return QVA_ERR_ARG;
    if (P->mixer == QVA_MIX_XY) {
        const bool store = !(flags & QVA_EVOLVE_SKIP_FINAL_STATE);
        const std::vector<XyLayerPass> lp = xy_layer_plan(P->n_qubits, xy_pairs_of(P));
        const std::vector<XyLaunch> L = xy_launches(P, p, store, for_grad != 0);
        for (int i = 0; i < (int)L.size() && i < max_out; ++i) {
            const XyLaunch& l = L[i];
            const bool tile = l.pass >= 0;
            out[i].kind = l.kind;
            out[i].group_first = tile ? lp[l.pass].g.k : -1;
            out[i].group_bits = tile ? (P->n_qubits <= kTileBits ? P->n_qubits : kTileBits - lp[l.pass].g.C) : 0;
            out[i].col_bits = tile && P->n_qubits > kTileBits ? lp[l.pass].g.C : 0;
            out[i].mix_layer = tile && !lp[l.pass].ops.empty() ? l.layer : -1;
            out[i].mix_layer2 = (int)(tile ? lp[l.pass].ops.size() : 0);
            out[i].phase_layer = (l.flags & XY_PHASE) ? l.layer : -1;
            out[i].bytes = xy_launch_bytes(l, P, p, for_grad != 0);
        }
        return (int)L.size();
    }
    if (mixed_path(P) && p > 0) {
        MrGeom m{};
        mixed_geom(problem_N(P), &m);
        const std::vector<MrLaunch> L = mr_launches(m, p, !(flags & QVA_EVOLVE_SKIP_FINAL_STATE), for_grad != 0);
        for (int i = 0; i < (int)L.size() && i < max_out; ++i) {
            const MrLaunch& l = L[i];
            const bool tiles = l.group >= 0 && l.kind != QVA_PASS_MR_TABLES;
            out[i].kind = l.kind;
            out[i].group_first = tiles ? l.group : -1;
            out[i].group_bits = tiles ? m.A[l.group] : 0;
            out[i].col_bits = tiles ? m.cols[l.group] : 0;
            out[i].mix_layer = l.layer;
            out[i].mix_layer2 = -1;
            out[i].phase_layer = l.gamma;
            out[i].bytes = mr_launch_bytes(l, P, m, p);
        }
        return (int)L.size();
    }
    if (for_grad) {
        const std::vector<XGroup> groups = x_groups(bluestein_path(P) ? blu_bits(P) : P->n_qubits);
        const std::vector<GLaunch> L = grad_launches(P, p);
        for (int i = 0; i < (int)L.size() && i < max_out; ++i) {
            const GLaunch& l = L[i];
            out[i].kind = l.kind;
            out[i].group_first = l.group >= 0 ? groups[l.group].k : -1;
            out[i].group_bits = l.group >= 0 ? groups[l.group].bits : 0;
            out[i].col_bits = l.group >= 0 ? groups[l.group].col_bits : 0;
            out[i].mix_layer = l.t1;
            out[i].mix_layer2 = l.t2;
            out[i].phase_layer = l.gamma;
            out[i].bytes = grad_launch_bytes(l, P, p);
        }
        return (int)L.size();
    }
    const bool store = !(flags & QVA_EVOLVE_SKIP_FINAL_STATE);
    const int n = P->n_qubits;
    const bool circ = P->mixer == QVA_MIX_CIRCULANT;
    const std::vector<XGroup> groups = x_groups(bluestein_path(P) ? blu_bits(P) : n);
    const std::vector<Launch> L = circ ? fft_launches(P, p, store) : x_launches(n, p, store, problem_terms(P) > 0);
    for (int i = 0; i < (int)L.size() && i < max_out; ++i) {
        const Launch& l = L[i];
        out[i].kind = l.kind;
        out[i].group_first = l.group >= 0 ? groups[l.group].k : -1;
        out[i].group_bits = l.group >= 0 ? groups[l.group].bits : 0;
        out[i].col_bits = l.group >= 0 ? groups[l.group].col_bits : 0;
        out[i].mix_layer = l.layer1;
        out[i].mix_layer2 = l.layer2;
        out[i].phase_layer = l.phase_layer;
        out[i].bytes = complete_closed_form(P) ? cpl_launch_bytes(l, P, p)
                       : bluestein_path(P) ? blu_launch_bytes(l, P, p)
                       : circ ? fft_launch_bytes(l, n, store, lambda_tiled(P)) : launch_bytes(l, n, store);
    }
    return (int)L.size();
}

int qva_grad(const qva_problem* P, const double* gammas_dev, const double* ts_dev, int p,
             qva_c128* psi, qva_c128* chi, double* out_f_dev, double* dgammas_dev,
             double* dts_dev, void* work, size_t work_bytes, void* stream)
{
    EventHook hook;
    return grad_common(P, gammas_dev, ts_dev, p, psi, chi, out_f_dev, dgammas_dev, dts_dev, work,
                       work_bytes, stream, hook);
}

int qva_grad_timed(const qva_problem* P, const double* gammas_dev, const double* ts_dev, int p,
                   qva_c128* psi, qva_c128* chi, double* out_f_dev, double* dgammas_dev,
                   double* dts_dev, void* work, size_t work_bytes, void* const* events, int n_events,
                   void* stream)
{
    if (!events || n_events < 0)
        return QVA_ERR_ARG;
    EventHook hook;
    hook.ev = events;
    hook.n = n_events;
    return grad_common(P, gammas_dev, ts_dev, p, psi, chi, out_f_dev, dgammas_dev, dts_dev, work,
                       work_bytes, stream, hook);
}

}  // extern "C"

namespace {

int evolve_common(const qva_problem* P, const double* gammas_dev, const double* ts_dev, int p,
                  qva_c128* psi, double* out_f_dev, double* out_norm_dev, int flags, void* work,
                  size_t work_bytes, void* stream, EventHook& hook)
{
    int st = check_problem(P, p);
    if (st != QVA_OK)
        return st;
    if (!psi || !out_f_dev || (p > 0 && (!gammas_dev || !ts_dev)))
        return QVA_ERR_ARG;
    if (flags & ~QVA_EVOLVE_SKIP_FINAL_STATE)
        return QVA_ERR_ARG;
    if (!aligned(psi, 16) || !aligned(out_f_dev, 8) || (out_norm_dev && !aligned(out_norm_dev, 8)) ||
        (gammas_dev && !aligned(gammas_dev, 8)) || (ts_dev && !aligned(ts_dev, 8)))
        return QVA_ERR_ALIGN;
    const size_t need = qva_workspace_bytes(P, p, 0);
    if (need && (!work || work_bytes < need))
        return QVA_ERR_WORKSPACE;
    if (work && !aligned(work, 16))
        return QVA_ERR_ALIGN;
    const bool store = !(flags & QVA_EVOLVE_SKIP_FINAL_STATE);
    if (P->mixer == QVA_MIX_XY)
        return xy_run(P, gammas_dev, ts_dev, p, reinterpret_cast<double2*>(psi), nullptr, out_f_dev, out_norm_dev,
                      nullptr, nullptr, store, false, reinterpret_cast<char*>(work), as_stream(stream), hook);
    if (P->mixer == QVA_MIX_X)
        return evolve_x(P, gammas_dev, ts_dev, p, reinterpret_cast<double2*>(psi), out_f_dev,
                        out_norm_dev, store, reinterpret_cast<double2*>(work), as_stream(stream),
                        hook);
    return evolve_circ(P, gammas_dev, ts_dev, p, reinterpret_cast<double2*>(psi), out_f_dev,
                       out_norm_dev, store, reinterpret_cast<char*>(work), as_stream(stream), hook);
}

}  // namespace

namespace {

int grad_common(const qva_problem* P, const double* gammas_dev, const double* ts_dev, int p,
                qva_c128* psi, qva_c128* chi, double* out_f_dev, double* dgammas_dev, double* dts_dev,
                void* work, size_t work_bytes, void* stream, EventHook& hook)
{
    int st = check_problem(P, p);
    if (st != QVA_OK)
        return st;
    if (!psi || !chi || !out_f_dev || (p > 0 && (!gammas_dev || !ts_dev || !dgammas_dev || !dts_dev)))
        return QVA_ERR_ARG;
    if (psi == chi)
        return QVA_ERR_ARG;
    if (!aligned(psi, 16) || !aligned(chi, 16) || !aligned(out_f_dev, 8) ||
        (gammas_dev && !aligned(gammas_dev, 8)) || (ts_dev && !aligned(ts_dev, 8)) ||
        (dgammas_dev && !aligned(dgammas_dev, 8)) || (dts_dev && !aligned(dts_dev, 8)))
        return QVA_ERR_ALIGN;
    const size_t need = qva_workspace_bytes(P, p, 1);
    if (need && (!work || work_bytes < need))
        return QVA_ERR_WORKSPACE;
    if (work && !aligned(work, 256))
        return QVA_ERR_ALIGN;
    if (P->mixer == QVA_MIX_XY)
        return xy_run(P, gammas_dev, ts_dev, p, reinterpret_cast<double2*>(psi), reinterpret_cast<double2*>(chi),
                      out_f_dev, nullptr, dgammas_dev, dts_dev, true, true, reinterpret_cast<char*>(work),
                      as_stream(stream), hook);
    return grad_run(P, gammas_dev, ts_dev, p, reinterpret_cast<double2*>(psi), reinterpret_cast<double2*>(chi),
                    out_f_dev, dgammas_dev, dts_dev, reinterpret_cast<char*>(work), as_stream(stream), hook);
}

}  // namespace

// ----------------------------------------------------------------- batched
struct qva_batch_plan_s {
    struct Group {
        int first, count, kind, mode, col_bits, round, lane;
    };
    std::vector<BatchInst> inst;
    std::vector<BatchPass> pass;
    std::vector<BatchItem> items;
    std::vector<Group> groups;
    std::vector<size_t> fpart_off, slots_off;  // per instance, from the scratch start
    size_t off_inst = 0, off_pass = 0, off_items = 0, off_scratch = 0, total = 0;
    int rounds = 0;
    int64_t tiles_total = 0;
    void* uploaded = nullptr;
    // lanes > 1: lane k >= 1 runs on lane_streams[k - 1] (made by qva_batch_upload),
    // forked from and joined back into the caller's stream
    int lanes = 1;
    std::vector<hipStream_t> lane_streams;
    std::vector<hipEvent_t> lane_events;  // [0]: fork, [k]: join of lane k
    ~qva_batch_plan_s()
    {
        for (hipStream_t x : lane_streams)
            (void)hipStreamDestroy(x);
        for (hipEvent_t e : lane_events)
            (void)hipEventDestroy(e);
    }
};

namespace {

int batch_check_item(const qva_batch_item& it)
{
    if (it.n_qubits < 12 || it.n_qubits > 30)
        return QVA_ERR_SIZE;
    if (it.p < 1 || it.p > QVA_BATCH_MAX_DEPTH)
        return QVA_ERR_SIZE;
    if (!it.q || !it.gammas || !it.ts || !it.psi || !it.chi || !it.out_f || !it.dgammas || !it.dts)
        return QVA_ERR_ARG;
    if (!aligned(it.q, 8) || !aligned(it.gammas, 8) || !aligned(it.ts, 8) || !aligned(it.psi, 16) ||
        !aligned(it.chi, 16) || !aligned(it.out_f, 8) || !aligned(it.dgammas, 8) || !aligned(it.dts, 8))
        return QVA_ERR_ALIGN;
    if (it.psi == it.chi)
        return QVA_ERR_ARG;
    return QVA_OK;
}

// Passes of one instance in execution order (forward, turn, backward, reduce).
std::vector<BatchPass> batch_passes(const qva_batch_item& it)
{
    std::vector<BatchPass> out;
    if (it.n_qubits == kTileBits) {
        out.push_back({BP_WHOLE, 0, 0, 0, -1, -1, -1, -1, -1, -1});
        return out;
    }
    qva_problem P{QVA_MIX_X, it.n_qubits, it.q, nullptr, 0};
    const std::vector<XGroup> groups = x_groups(it.n_qubits);
    for (const GLaunch& l : grad_launches(&P, it.p)) {
        BatchPass b{};
        b.t1 = l.t1;
        b.t2 = l.t2;
        b.gamma = l.gamma;
        b.slot_t1 = l.slot_t1;
        b.slot_g = l.slot_g;
        b.slot_t2 = l.slot_t2;
        b.mode = l.mode;
        if (l.group >= 0) {
            b.k = groups[l.group].k;
            b.col_bits = groups[l.group].col_bits;
        }
        switch (l.kind) {
        case QVA_PASS_FIRST:
        case QVA_PASS_MIDDLE:
        case QVA_PASS_BOUNDARY:
            b.kind = BP_FWD;
            break;
        case QVA_PASS_GRAD_TURN:
        case QVA_PASS_GRAD_MID:
        case QVA_PASS_GRAD_BOUND:
        case QVA_PASS_GRAD_FINAL:
            b.kind = BP_BWD;
            break;
        case QVA_PASS_GRAD_REDUCE:
            b.kind = BP_REDUCE;
            break;
        default:  // the f reduction is part of the per-instance reduce
            continue;
        }
        out.push_back(b);
    }
    return out;
}

int64_t pass_tiles(const BatchPass& b, int n)
{
    return (b.kind == BP_FWD || b.kind == BP_BWD) ? (int64_t(1) << (n - kTileBits)) : 1;
}

}  // namespace

extern "C" {

int qva_batch_create(const qva_batch_item* items, int count, int align, qva_batch_plan* out)
{
    return qva_batch_create_lanes(items, count, align, 1, out);
}

int qva_batch_create_lanes(const qva_batch_item* items, int count, int align, int lanes, qva_batch_plan* out)
{
    if (!out || !items || count < 1)
        return QVA_ERR_ARG;
    if (align != QVA_BATCH_ALIGN_START && align != QVA_BATCH_ALIGN_END && align != QVA_BATCH_ALIGN_SPREAD)
        return QVA_ERR_ARG;
    if (lanes < 1 || lanes > QVA_BATCH_MAX_LANES)
        return QVA_ERR_ARG;
    for (int i = 0; i < count; ++i) {
        int st = batch_check_item(items[i]);
        if (st != QVA_OK)
            return st;
    }
    qva_batch_plan_s* B = new qva_batch_plan_s();
    std::vector<std::vector<BatchPass>> per(count);
    std::vector<int64_t> load_of(count);
    int maxpass = 0;
    for (int i = 0; i < count; ++i) {
        per[i] = batch_passes(items[i]);
        maxpass = std::max(maxpass, (int)per[i].size());
        int64_t l = 0;
        for (const BatchPass& b : per[i])
            l += pass_tiles(b, items[i].n_qubits);
        load_of[i] = l;
    }
    // lanes: largest instances first, each to the lane with the fewest tiles
    // so far (ties: the lowest lane)
    std::vector<int> order(count), lane_of(count, 0);
    for (int i = 0; i < count; ++i)
        order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return load_of[a] > load_of[b]; });
    {
        std::vector<int64_t> lane_load(lanes, 0);
        for (int i : order) {
            int best = 0;
            for (int l = 1; l < lanes; ++l)
                if (lane_load[l] < lane_load[best])
                    best = l;
            lane_of[i] = best;
            lane_load[best] += load_of[i];
        }
    }
    // start round of every instance, per lane (each lane is its own sequence
    // of rounds)
    std::vector<int> start(count, 0);
    std::vector<int> lane_rounds(lanes, 0);
    for (int i = 0; i < count; ++i)
        lane_rounds[lane_of[i]] = std::max(lane_rounds[lane_of[i]], (int)per[i].size());
    if (align == QVA_BATCH_ALIGN_END) {
        for (int i = 0; i < count; ++i)
            start[i] = lane_rounds[lane_of[i]] - (int)per[i].size();
    } else if (align == QVA_BATCH_ALIGN_SPREAD) {
        // largest instances first; each takes the offset that keeps the
        // busiest round of its lane least loaded (ties: earliest)
        std::vector<std::vector<int64_t>> round_load(lanes);
        for (int l = 0; l < lanes; ++l)
            round_load[l].assign(lane_rounds[l], 0);
        for (int i : order) {
            std::vector<int64_t>& rl = round_load[lane_of[i]];
            const int np = (int)per[i].size();
            int best = 0;
            int64_t best_peak = -1;
            for (int s0 = 0; s0 + np <= (int)rl.size(); ++s0) {
                int64_t peak = 0;
                for (int j = 0; j < np; ++j)
                    peak = std::max(peak, rl[s0 + j] + pass_tiles(per[i][j], items[i].n_qubits));
                if (best_peak < 0 || peak < best_peak) {
                    best_peak = peak;
                    best = s0;
                }
            }
            start[i] = best;
            for (int j = 0; j < np; ++j)
                rl[best + j] += pass_tiles(per[i][j], items[i].n_qubits);
        }
    }
    B->rounds = *std::max_element(lane_rounds.begin(), lane_rounds.end());
    B->lanes = lanes;
    (void)maxpass;
    // instance and pass tables, per-instance scratch layout
    size_t scratch = 0;
    for (int i = 0; i < count; ++i) {
        const qva_batch_item& it = items[i];
        BatchInst d{};
        d.psi = reinterpret_cast<double2*>(it.psi);
        d.chi = reinterpret_cast<double2*>(it.chi);
        d.q = it.q;
        d.gammas = it.gammas;
        d.ts = it.ts;
        d.out_f = it.out_f;
        d.dgammas = it.dgammas;
        d.dts = it.dts;
        d.n = it.n_qubits;
        d.p = it.p;
        d.tiles = it.n_qubits > kTileBits ? (int64_t(1) << (it.n_qubits - kTileBits)) : 1;
        d.G = (int)x_groups(it.n_qubits).size();
        d.nslots = it.n_qubits > kTileBits ? it.p * (d.G + 1) : 0;
        d.pass_off = (int)B->pass.size();
        d.npass = (int)per[i].size();
        B->pass.insert(B->pass.end(), per[i].begin(), per[i].end());
        B->fpart_off.push_back(scratch);
        scratch = align256(scratch + (size_t)d.tiles * sizeof(double2));
        B->slots_off.push_back(scratch);
        scratch = align256(scratch + (size_t)d.nslots * (size_t)d.tiles * sizeof(double));
        B->inst.push_back(d);
    }
    // work items, ordered by (round, lane, kind, mode, tile geometry, instance,
    // tile): one launch per (round, lane, kind, mode, geometry)
    using Key = std::tuple<int, int, int, int, int, int, int>;
    std::vector<std::pair<Key, BatchItem>> all;
    for (int i = 0; i < count; ++i) {
        for (int j = 0; j < (int)per[i].size(); ++j) {
            const BatchPass& b = per[i][j];
            const int64_t nt = pass_tiles(b, items[i].n_qubits);
            for (int64_t tl = 0; tl < nt; ++tl)
                all.push_back({Key(start[i] + j, lane_of[i], b.kind, b.mode, b.col_bits, i, (int)tl),
                               BatchItem{i, j, (int)tl, 0}});
        }
    }
    std::sort(all.begin(), all.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    for (size_t x = 0; x < all.size(); ++x) {
        const Key& k = all[x].first;
        B->items.push_back(all[x].second);
        const bool same = !B->groups.empty() && x > 0 && std::get<0>(all[x - 1].first) == std::get<0>(k) &&
                          std::get<1>(all[x - 1].first) == std::get<1>(k) &&
                          std::get<2>(all[x - 1].first) == std::get<2>(k) &&
                          std::get<3>(all[x - 1].first) == std::get<3>(k) &&
                          std::get<4>(all[x - 1].first) == std::get<4>(k);
        if (same)
            B->groups.back().count += 1;
        else
            B->groups.push_back({(int)x, 1, std::get<2>(k), std::get<3>(k), std::get<4>(k), std::get<0>(k),
                                 std::get<1>(k)});
    }
    B->tiles_total = (int64_t)B->items.size();
    size_t off = 0;
    B->off_inst = off;
    off = align256(off + B->inst.size() * sizeof(BatchInst));
    B->off_pass = off;
    off = align256(off + B->pass.size() * sizeof(BatchPass));
    B->off_items = off;
    off = align256(off + B->items.size() * sizeof(BatchItem));
    B->off_scratch = off;
    B->total = off + scratch;
    *out = B;
    return QVA_OK;
}

size_t qva_batch_workspace_bytes(qva_batch_plan plan) { return plan ? plan->total : 0; }

int qva_batch_rounds(qva_batch_plan plan) { return plan ? plan->rounds : QVA_ERR_ARG; }

int qva_batch_launches(qva_batch_plan plan) { return plan ? (int)plan->groups.size() : QVA_ERR_ARG; }

int64_t qva_batch_tiles(qva_batch_plan plan) { return plan ? plan->tiles_total : QVA_ERR_ARG; }

int qva_batch_upload(qva_batch_plan plan, void* work, size_t work_bytes, void* stream)
{
    if (!plan || !work)
        return QVA_ERR_ARG;
    if (work_bytes < plan->total)
        return QVA_ERR_WORKSPACE;
    if (!aligned(work, 256))
        return QVA_ERR_ALIGN;
    char* base = reinterpret_cast<char*>(work);
    std::vector<BatchInst> inst = plan->inst;
    for (size_t i = 0; i < inst.size(); ++i) {
        inst[i].fpart = reinterpret_cast<double2*>(base + plan->off_scratch + plan->fpart_off[i]);
        inst[i].slots = reinterpret_cast<double*>(base + plan->off_scratch + plan->slots_off[i]);
    }
    std::vector<char> host(plan->off_scratch, 0);
    std::memcpy(host.data() + plan->off_inst, inst.data(), inst.size() * sizeof(BatchInst));
    std::memcpy(host.data() + plan->off_pass, plan->pass.data(), plan->pass.size() * sizeof(BatchPass));
    std::memcpy(host.data() + plan->off_items, plan->items.data(), plan->items.size() * sizeof(BatchItem));
    hipStream_t s = as_stream(stream);
    if (hipMemcpyAsync(work, host.data(), host.size(), hipMemcpyHostToDevice, s) != hipSuccess)
        return QVA_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess)
        return QVA_ERR_HIP;
    // the lanes' streams (default priority) and fork / join events, on the
    // current device
    while ((int)plan->lane_streams.size() < plan->lanes - 1) {
        hipStream_t x;
        if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess)
            return QVA_ERR_HIP;
        plan->lane_streams.push_back(x);
    }
    while (plan->lanes > 1 && (int)plan->lane_events.size() < plan->lanes) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return QVA_ERR_HIP;
        plan->lane_events.push_back(e);
    }
    plan->uploaded = work;
    return QVA_OK;
}

}  // extern "C"

namespace {

int batch_grad_run(qva_batch_plan plan, void* work, size_t work_bytes, void* stream, EventHook& hook)
{
    if (!plan || !work)
        return QVA_ERR_ARG;
    if (work != plan->uploaded || work_bytes < plan->total)
        return QVA_ERR_WORKSPACE;
    char* base = reinterpret_cast<char*>(work);
    BatchRoundParams R;
    R.inst = reinterpret_cast<const BatchInst*>(base + plan->off_inst);
    R.pass = reinterpret_cast<const BatchPass*>(base + plan->off_pass);
    R.items = reinterpret_cast<const BatchItem*>(base + plan->off_items);
    hipStream_t s = as_stream(stream);
    // lanes > 1 (untimed): fork the plan's lane streams from s, launch each
    // group on its lane's stream, join them back into s.  Timed calls run
    // every launch on s in plan order.
    const bool fork = plan->lanes > 1 && !hook.ev;
    if (fork) {
        if ((int)plan->lane_streams.size() != plan->lanes - 1)
            return QVA_ERR_ARG;
        if (hipEventRecord(plan->lane_events[0], s) != hipSuccess)
            return QVA_ERR_HIP;
        for (hipStream_t ls : plan->lane_streams)
            if (hipStreamWaitEvent(ls, plan->lane_events[0], 0) != hipSuccess)
                return QVA_ERR_HIP;
    }
    for (const auto& gr : plan->groups) {
        R.first = gr.first;
        const hipStream_t ls = fork && gr.lane > 0 ? plan->lane_streams[gr.lane - 1] : s;
        hook.before(s);
        const hipError_t e = launch_batch_group(R, gr.kind, gr.mode, gr.col_bits, gr.count, ls);
        hook.after(s);
        if (e != hipSuccess)
            return QVA_ERR_HIP;
    }
    if (fork) {
        for (int l = 1; l < plan->lanes; ++l) {
            if (hipEventRecord(plan->lane_events[l], plan->lane_streams[l - 1]) != hipSuccess ||
                hipStreamWaitEvent(s, plan->lane_events[l], 0) != hipSuccess)
                return QVA_ERR_HIP;
        }
    }
    return QVA_OK;
}

// Algorithmic HBM bytes per amplitude of a batched tile pass.
double batch_bytes_per_amp(int kind, int mode)
{
    if (kind == BP_FWD) {
        switch (mode) {
        case XMODE_FIRST:
            return 24.0;
        case XMODE_BOUNDARY:
            return 40.0;
        case XMODE_LAST:
            return 24.0;
        default:
            return 32.0;
        }
    }
    if (kind == BP_BWD) {
        switch (mode) {
        case GMODE_TURN:
            return 56.0;
        case GMODE_BOUND:
            return 72.0;
        case GMODE_FINAL:
            return 40.0;
        default:
            return 64.0;
        }
    }
    return kind == BP_WHOLE ? 8.0 : 0.0;  // n = 12 whole instances read q; the sums are small
}

}  // namespace

extern "C" {

int qva_batch_grad(qva_batch_plan plan, void* work, size_t work_bytes, void* stream)
{
    EventHook hook;
    return batch_grad_run(plan, work, work_bytes, stream, hook);
}

int qva_batch_grad_timed(qva_batch_plan plan, void* work, size_t work_bytes, void* const* events, int n_events,
                         void* stream)
{
    if (!events || n_events < 0)
        return QVA_ERR_ARG;
    EventHook hook;
    hook.ev = events;
    hook.n = n_events;
    return batch_grad_run(plan, work, work_bytes, stream, hook);
}

int qva_batch_launch_info(qva_batch_plan plan, int i, int* round, int64_t* workgroups, double* bytes)
{
    if (!plan || i < 0 || i >= (int)plan->groups.size())
        return QVA_ERR_ARG;
    const auto& gr = plan->groups[i];
    if (round)
        *round = gr.round;
    if (workgroups)
        *workgroups = gr.count;
    if (bytes)
        *bytes = (double)gr.count * (double)(1 << kTileBits) * batch_bytes_per_amp(gr.kind, gr.mode);
    return QVA_OK;
}

int qva_batch_sgd(qva_batch_plan plan, double lr, void* work, size_t work_bytes, void* stream)
{
    if (!plan || !work)
        return QVA_ERR_ARG;
    if (work != plan->uploaded || work_bytes < plan->total)
        return QVA_ERR_WORKSPACE;
    const BatchInst* inst = reinterpret_cast<const BatchInst*>(reinterpret_cast<char*>(work) + plan->off_inst);
    return hip_status(launch_batch_sgd(inst, (int)plan->inst.size(), 0, lr, as_stream(stream)));
}

int qva_batch_destroy(qva_batch_plan plan)
{
    delete plan;
    return QVA_OK;
}

}  // extern "C"
