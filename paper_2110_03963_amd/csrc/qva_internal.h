// qva_internal.h -- launch descriptors shared by the C ABI layer and the
// kernel translation units of libqva.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qva_device.h"

namespace qva {

// Tile geometry of the grouped passes: a tile is 2^kTileBits amplitudes,
// held as kRegs amplitudes in each of kThreads threads.
constexpr int kTileBits = 12;
constexpr int kThreads = 256;
constexpr int kRegs = 16;
// Largest qubit group handled by a strided (high) pass: the tile keeps at
// least 2^3 contiguous amplitudes (128 bytes) per row.
constexpr int kMinColBits = 3;
constexpr int kMaxHighBits = kTileBits - kMinColBits;

// Pass flags of the hypercube-mixer tile pass.
enum : int {
    XP_INIT = 1,         // start from the uniform state instead of loading psi
    XP_PHASE_PRE = 2,    // phase before the first mixer application
    XP_MIX1 = 4,         // first mixer application (angle mix1)
    XP_PHASE_MID = 8,    // phase between the two mixer applications
    XP_MIX2 = 16,        // second mixer application (angle mix2)
    XP_EXPECT = 32,      // accumulate sum |psi|^2 q and sum |psi|^2
    XP_STORE = 64,       // write psi back
    XP_FINAL_SCALE = 128, // multiply by the layer factor of mix1 (all qubits)
    XP_ZTERMS = 256      // the phase is the extended-QAOA product over Z-string terms
};

// The flag combinations the passes are compiled for.
enum : int {
    XMODE_FIRST = XP_INIT | XP_PHASE_PRE | XP_MIX1 | XP_STORE,
    XMODE_MIDDLE = XP_MIX1 | XP_STORE,
    XMODE_BOUNDARY = XP_MIX1 | XP_PHASE_MID | XP_MIX2 | XP_STORE,
    XMODE_LAST = XP_MIX1 | XP_EXPECT | XP_FINAL_SCALE,
    XMODE_LAST_STORE = XP_MIX1 | XP_EXPECT | XP_FINAL_SCALE | XP_STORE,
    XMODE_MIX_SCALE = XP_MIX1 | XP_FINAL_SCALE | XP_STORE,
    XMODE_FIRST_Z = XMODE_FIRST | XP_ZTERMS,
    XMODE_BOUNDARY_Z = XMODE_BOUNDARY | XP_ZTERMS
};

// A term of a Pauli decomposition of Q (same layout as qva_zterm):
// Sigma(j) = coef (-1)^popcount(j & support).
struct ZTerm {
    uint64_t support;
    double coef;
};

struct XPassParams {
    double2* psi;
    const double* q;
    Angle mix1, mix2, phase;  // XP_ZTERMS: phase.ptr + phase.idx is the layer's angle row
    const ZTerm* terms;       // XP_ZTERMS
    int n_terms;
    int n;        // qubits of the register
    int k;        // first target qubit of the tile's group
    int col_bits; // contiguous low index bits per tile row (0 for the low group)
    int flags;
    double2* partials;  // one (f, norm) pair per tile when XP_EXPECT
    const double* qt;   // XP_PHASE_MID without XP_ZTERMS: this group's block of the
                        // tile-ordered copy of q (qva_q_tiles), or null
};

struct SmallParams {
    double2* psi;        // in/out (read unless SM_INIT, written if SM_STORE)
    const double* q;
    const ZTerm* terms;  // extended-QAOA phases (gammas then p x n_terms), or null
    int n_terms;
    const double* gammas;
    const double* ts;
    double t_val;        // angle for SM_MIX_ONCE
    int n;
    int p;
    int flags;
    double* out_f;
    double* out_norm;
};

enum : int {
    SM_INIT = 1,
    SM_EVOLVE = 2,    // p layers with gammas/ts
    SM_MIX_ONCE = 4,  // one hypercube mixer with t_val
    SM_EXPECT = 8,
    SM_STORE = 16
};

hipError_t launch_xpass(const XPassParams& P, hipStream_t s);
// one group's block of the tile-ordered copy of q (qva_q_tiles)
hipError_t launch_qtile(const double* q, double* out, int n, int k, int col_bits, hipStream_t s);
hipError_t launch_small(const SmallParams& P, hipStream_t s);
hipError_t launch_init_uniform(double2* psi, int64_t N, hipStream_t s);
hipError_t launch_phase(double2* psi, const double* q, int64_t N, double gamma, hipStream_t s);
// Per-block partial (f, norm) over [0, N), then a fixed-order final sum.
int64_t expect_partial_count(int64_t N);
hipError_t launch_expect_partials(const double2* psi, const double* q, int64_t N,
                                  double2* partials, hipStream_t s);
hipError_t launch_final_reduce(const double2* partials, int64_t count, double* out_f,
                               double* out_norm, hipStream_t s);

// ---------------------------------------------------------------- circulant
// Where the FFT passes take lambda from.
enum : int {
    FFT_LAMBDA_NATURAL = 0,  // lambda[m], natural order (whole-state kernel only)
    FFT_LAMBDA_RING = 1,     // 2 cos(2 pi m / N), computed
    FFT_LAMBDA_COMPLETE = 2, // N - 1 for m = 0, else -1, computed
    FFT_LAMBDA_TILED = 3     // workspace copy laid out per low-group tile
};

enum : int { FP_EXPECT = 1, FP_STORE = 2 };

// Pass kinds of the circulant mixer (compile-time modes of fftpass_kernel).
enum : int {
    FMODE_FIRST = 16,           // psi_0, phase, forward transform of the top group
    FMODE_DIF = 32,             // forward transform of one group
    FMODE_DIT = 48,             // inverse transform of one group
    FMODE_DIT_SCALE = 64,       // inverse transform of the top group, times 1/N
    FMODE_LOWDIAG = 80,         // low group: forward, diag(exp(-i t lambda)), inverse
    FMODE_BOUNDARY = 96,        // inverse top group, 1/N, phase, forward top group
    FMODE_LAST = 112 | FP_EXPECT,              // inverse top group, 1/N, <Q> partials
    FMODE_LAST_STORE = 112 | FP_EXPECT | FP_STORE,
    // Bluestein (chirp-z) evolution for N not a power of two, over a padded
    // buffer of M = 2^n >= 2N - 1 amplitudes (see qva_fft.hip)
    FMODE_B_CHIRP = 128,      // chirp filter w_k (or its conjugate), forward top group
    FMODE_B_FIRST = 144,      // psi_0, phase of layer 1, conj chirp, zero pad, forward top group
    FMODE_B_BOUND_LAM = 160,  // inverse top group, exp(-i t lambda) (j < N, else 0), forward top
    FMODE_B_BOUND_Q = 176,    // inverse top group, exp(-i gamma q) / N (j < N, else 0), forward top
    FMODE_B_LAST = 192 | FP_EXPECT,            // inverse top group, <Q> over j < N
    FMODE_B_LAST_STORE = 192 | FP_EXPECT | FP_STORE,  // ... and psi_j = w_j x_j / N
    FMODE_B_STORE = 192 | FP_STORE,  // inverse top group, psi_j = w_j x_j / N only (the lone mixer)
    FMODE_LOWMUL = 208,       // low group: forward, times a complex per-tile array, inverse
    FMODE_LOWDIF_TILED = 224, // low group: forward, written per tile (times 1/M)
    FMODE_B_LOAD = 240        // the caller's psi times conj chirp, zero pad, forward top group
};

struct FftPassParams {
    double2* psi;
    const double* q;
    const double* lam;   // FFT_LAMBDA_TILED: the per-tile copy
    Angle mix1, phase;   // mix1: the diag's t (LOWDIAG); phase: gamma
    int n;
    int k;
    int col_bits;
    int flags;
    int lambda_kind;
    double2* partials;
    // Bluestein passes
    int64_t nb;           // the logical N (< 2^31); n above is log2 of the padded M
    const double2* bt;    // FMODE_LOWMUL: complex multiplier in per-tile order
    double2* out;         // FMODE_LOWDIF_TILED: its output; FMODE_B_LAST_STORE, FMODE_B_STORE: psi (nb amplitudes)
    const double2* in;    // FMODE_B_LOAD: the state to transform (nb amplitudes)
    int conj;             // FMODE_B_CHIRP: conjugate filter
    const double2* tw;    // low-group passes (LOWDIAG, LOWMUL, LOWDIF_TILED): root table W_4096^k
};

struct SmallFftParams {
    double2* psi;
    const double* q;
    const double* gammas;
    const double* ts;
    const double* lam;   // natural order, FFT_LAMBDA_NATURAL
    int lambda_kind;
    double t_val;
    int n;
    int p;
    int flags;           // SM_* flags
    double* out_f;
    double* out_norm;
};

hipError_t launch_fftpass(const FftPassParams& P, hipStream_t s);
hipError_t launch_small_fft(const SmallFftParams& P, hipStream_t s);
hipError_t launch_lambda_tiles(const double* lam, double* out, int n, hipStream_t s);
// The low-group root table tab[k] = W_4096^k = exp(-2 pi i k / 4096), k < 4096
// (kTwiddleTableBytes), read by the low-group transform passes.
constexpr size_t kTwiddleTableBytes = sizeof(double2) << kTileBits;
hipError_t launch_twiddle_table(double2* tab, hipStream_t s);

// ------------------------------------------ mixed-radix circulant (any N)
// N = A_0 A_1 ... A_{G-1} with every prime factor <= kMrMaxPrime (see
// qva_mrplan.h and qva_mixed.hip).
constexpr int kMrMaxGroups = 4;
constexpr int kMrMaxStages = 16;
constexpr int kMrMaxPrime = 31;
constexpr int kMrTileElems = 1 << kTileBits;  // amplitudes per tile (one vector)
constexpr int kMrMaxStrided = 512;            // strided groups keep >= 8 columns per row

struct MrGeom {
    int G;
    int A[kMrMaxGroups];               // group sizes, low (contiguous) first
    int64_t S[kMrMaxGroups + 1];       // S_g = A_0 ... A_{g-1}; S_G = N
    int nrad[kMrMaxGroups];
    int rad[kMrMaxGroups][kMrMaxStages];  // radices of each group's DFT stages, in stage order
    int cols[kMrMaxGroups];            // columns (independent DFTs) per tile
    int64_t tiles[kMrMaxGroups];       // tiles of each group's passes
    int tab_off[kMrMaxGroups];         // group g's roots and permutation start at entry tab_off[g]
    int tab_len;                       // sum of A_g
    int tw_off[kMrMaxGroups];          // group g's (g >= 1) inter-group twiddle table, after the roots
    int tw_len;                        // sum over g >= 1 of cols_g A_g
    double rA[kMrMaxGroups];           // 1 / A_g (the passes' integer divisions)
    int64_t U;                         // N / A_0, the low group's column count
    int lds_pad;                       // the low group's passes pad their LDS slots (mr_low_lds_cost)
};

// Pass modes of the mixed-radix passes (mrpass_kernel / mrgrad2_kernel).
enum : int {
    MR_FIRST = 1,        // psi_0, phase of layer 1, forward top group
    MR_DIF = 2,          // forward transform of one group
    MR_DIT = 3,          // inverse transform of one group
    MR_LOWDIAG = 4,      // low group: forward, diag(exp(-i t lambda)), inverse
    MR_BOUNDARY = 5,     // inverse top group, 1/N, phase, forward top group
    MR_LAST = 6,         // inverse top group, 1/N, <Q> partials
    MR_LAST_STORE = 7,   // ... and psi_p stored
    MR_SMALL = 8,        // N <= 4096: the whole evolution in one workgroup
    MR_SMALL_STORE = 9,
    MR_SMALL_MIX = 10,   // N <= 4096: the mixer alone on the caller's state, in place
    // adjoint (two vectors; DIF / DIT without inner products reuse the
    // single-vector passes once per vector)
    MRG_TURN = 16,       // inverse top of psi_p, 1/N, <Q>, chi = Q psi_p, forward top of both
    MRG_LOWDIAG = 17,    // low group forward, Im<chi^|lambda|phi^>/N, inverse diag, inverse
    MRG_BOUND = 18,      // inverse top, 1/N, Im<chi|Q|phi>, inverse phase, forward top
    MRG_FINAL = 19,      // inverse top, 1/N, Im<chi|Q|phi> (nothing written)
    MRG_SMALL = 20       // N <= 4096: forward + adjoint in one workgroup
};

struct MrPassParams {
    double2* psi;          // the state (phi in the adjoint)
    double2* chi;          // the adjoint state (MRG_*)
    const double* q;
    const double* lam;     // FFT_LAMBDA_NATURAL: lambda[m], natural order
    int lambda_kind;       // FFT_LAMBDA_RING or FFT_LAMBDA_NATURAL
    Angle t, gamma;        // the diag's t (LOWDIAG), the phase's gamma
    const double* gammas;  // MR_SMALL / MRG_SMALL: all layers
    const double* ts;
    int p;
    int64_t N;
    const MrGeom* geom;    // device copy of the geometry (written with the tables)
    int g;                 // group of the pass
    int64_t grid;          // workgroups of the launch (set by launch_mrpass)
    const double2* tab;    // per group: W_{A_g}^k, k < A_g (tab_off[g]); then per group
                           // g >= 1 W_{S_{g+1}}^(c m), c < cols_g, m < A_g at tab_len +
                           // tw_off[g] + m cols_g + c; then the digit-reversal
                           // permutation as int32 after tab_len + tw_len entries
    double2* partials;     // per-tile (f, norm)
    double* slot;          // per-tile gradient partial (MRG_LOWDIAG, MRG_BOUND, MRG_FINAL)
    double* out_f;         // MR_SMALL / MRG_SMALL
    double* out_norm;
    double* dgammas;       // MRG_SMALL
    double* dts;
    int scale_inv_n;       // MR_DIT: multiply the result by 1/N (last pass of a lone mixer)
};

// m is the host copy of *P.geom (grid sizes).
hipError_t launch_mrpass(const MrPassParams& P, const MrGeom& m, int mode, hipStream_t s);
// The geometry's device copy, then the root and permutation tables of every
// group (one workgroup per group).
hipError_t launch_mr_tables(const MrGeom& m, MrGeom* geom_dev, double2* tab, hipStream_t s);
// Bytes of the tables of geometry m.
size_t mr_table_bytes(const MrGeom& m);

// ------------------------------------------- complete-graph mixer, closed form
// Pass flags (see qva_complete.hip).
enum : int {
    CP_INIT = 1,    // start from the uniform state instead of loading psi
    CP_MIX = 2,     // psi <- e^{it} (psi + c S), c = (e^{-itN} - 1)/N, S = *sum_in
    CP_PHASE = 4,   // psi <- exp(-i gamma q) psi
    CP_SUM = 8,     // per-block sums of the output state
    CP_EXPECT = 16, // per-block sum |psi|^2 q and sum |psi|^2
    CP_STORE = 32   // write psi back
};
enum : int {
    CPMODE_FIRST = CP_INIT | CP_PHASE | CP_SUM | CP_STORE,
    CPMODE_LAYER = CP_MIX | CP_PHASE | CP_SUM | CP_STORE,
    CPMODE_LAST = CP_MIX | CP_EXPECT,
    CPMODE_LAST_STORE = CP_MIX | CP_EXPECT | CP_STORE,
    CPMODE_SUM = CP_SUM,              // the lone mixer: per-block sums of the caller's psi,
    CPMODE_MIX = CP_MIX | CP_STORE    // then psi <- e^{it} (psi + c S) in place
};

struct CompleteParams {
    double2* psi;         // N amplitudes, blocks of kCompleteChunk
    const double* q;
    const double* gammas;  // device, p
    const double* ts;      // device, p
    const double2* sum_in; // device: sum over the input state (CP_MIX)
    double2* partials;     // one per block: sums (CP_SUM) or (<Q>, norm) (CP_EXPECT)
    int64_t N;             // amplitudes (any N >= 1; the last block may be partial)
    int mix_layer;         // layer of the mixer (CP_MIX): t = ts[mix_layer], or t_val if ts is null
    double t_val;
    int phase_layer;       // layer of the phase (CP_PHASE)
    int flags;
};

constexpr int kCompleteChunk = 1 << kTileBits;  // amplitudes per block
hipError_t launch_complete(const CompleteParams& P, hipStream_t s);

// Adjoint walk with the closed-form mixer (see qva_complete.hip).
enum : int {
    GCMODE_TURN = 1,      // last mixer, <Q> partials, chi = Q psi_p, sums for dt_{p-1}
    GCMODE_BACK = 2,      // inverse mixer k, Im<chi|Q|phi>, inverse phase k, sums for dt_{k-1}
    GCMODE_BACK_LAST = 3  // inverse mixer 0, Im<chi|Q|phi> (nothing written)
};
constexpr int kCompleteParts = 8;  // doubles per block: S_phi, S_chi, Im<chi|phi>, Im<chi|Q|phi>

struct CompleteGradParams {
    double2* phi;
    double2* chi;
    const double* q;
    const double* gammas;
    const double* ts;
    const double2* sums_in;  // TURN: sum of the input phi; BACK: (S_phi, S_chi) of the input
    double* part;            // kCompleteParts per block
    double2* fpart;          // TURN: per-block (<Q>, norm)
    int64_t N;
    int layer;
    int flags;               // GCMODE_*
};
hipError_t launch_complete_grad(const CompleteGradParams& P, hipStream_t s);
// Fixed-order sums of the per-block parts: (S_phi, S_chi) -> state_out,
// sums[t_slot] = Im(conj(S_chi) S_phi) - Im<chi|phi> and sums[g_slot] = Im<chi|Q|phi>
// (a slot < 0 is skipped).
hipError_t launch_complete_gsum(const double* part, int64_t blocks, double2* state_out, double* sums,
                                int t_slot, int g_slot, hipStream_t s);

// ---------------------------------------------------------------- gradient
// Pass modes of the adjoint walk (see qva_grad.hip).
enum : int {
    GMODE_TURN = 1,    // last forward group, <Q>, chi = Q psi_p, first inverse group
    GMODE_MID = 2,     // inverse rotations of one group (hypercube)
    GMODE_BOUND = 3,   // inverse group, <chi|Q|phi>, inverse phase, inverse group
    GMODE_FINAL = 4,   // inverse of the first forward pass (accumulate only)
    GMODE_DIF = 5,     // forward transform of one group, both vectors (circulant)
    GMODE_DIT = 6,     // inverse transform of one group, both vectors
    GMODE_LOWDIAG = 7, // low group: forward, <chi^|lambda|phi^>, inverse diagonal, inverse
    GM_ZTERMS = 16,    // with GMODE_BOUND / GMODE_FINAL: extended-QAOA phase; d_j = Im(conj(chi_j) phi_j)
    GM_QTILE = 64,     // with GMODE_TURN / GMODE_BOUND / GMODE_FINAL (hypercube): q from the
                       // tile-ordered copy (GradPassParams::qt)
                       // at the phase is stored to zd for the GMODE_ZSLOT pass that follows
    GMODE_BOUND_Z = GMODE_BOUND | GM_ZTERMS,
    GMODE_FINAL_Z = GMODE_FINAL | GM_ZTERMS,
    // Bluestein adjoint (top group of the padded transform, both vectors; the
    // other passes are the forward's single-vector ones, run once per vector)
    GMODE_B_TURN = 32,   // inverse top group of psi, <Q>, chi = q x, forward top group (both)
    GMODE_B_LAM = 33,    // inverse top group, Im<chi|W|phi>, exp(+i t lambda), forward top group
    GMODE_B_Q = 34,      // inverse top group, 1/N, Im<chi|Q|phi>, exp(+i gamma q), forward top group
    GMODE_B_FINAL = 35,  // inverse top group, 1/N, Im<chi|Q|phi> (nothing written)
    GMODE_ZSLOT = 40     // per-term slots of an extended-QAOA phase from the stored d_j
};

struct GradPassParams {
    double2* phi;
    double2* chi;
    const double* q;
    const double* lam;
    Angle t1, t2, gamma;
    int n;
    int k;
    int col_bits;
    int flags;        // GMODE_*
    int lambda_kind;  // FFT_LAMBDA_*
    double* slot_t1;  // per-tile partials, or null
    double* slot_g;
    double* slot_t2;
    double2* fpart;   // per-tile (f, norm) partials (GMODE_TURN)
    const ZTerm* terms;   // GM_ZTERMS: gamma.ptr + gamma.idx is the layer's angle row
    int n_terms;
    double* slot_terms;   // GMODE_ZSLOT: term e of tile i at slot_terms[e * tiles + i]
    double* zd;           // GM_ZTERMS, GMODE_ZSLOT: d_j at the phase, indexed like psi
    int64_t nb;           // GMODE_B_*: the logical N (n above is log2 of the padded M)
    const double2* tw;    // GMODE_LOWDIAG: low-group root table W_4096^k (twiddle_table_kernel)
    const double* qt;     // GM_QTILE: this group's block of the tile-ordered copy of q
};

struct SmallGradParams {
    const double* q;
    const ZTerm* terms;  // extended-QAOA phases (gammas and dgammas p x n_terms), or null
    int n_terms;
    const double* gammas;
    const double* ts;
    const double* lam;
    int lambda_kind;
    int circulant;
    int n;
    int p;
    double* out_f;
    double* dgammas;
    double* dts;
};

hipError_t launch_gradpass(const GradPassParams& P, bool circulant, hipStream_t s);
hipError_t launch_small_grad(const SmallGradParams& P, hipStream_t s);
// Slot sums, then dts[L] = 2 sum_g sums[L G + g] and dgammas[i] = 2 sums[p G + i]
// for i < p E (E gamma slots per layer: 1, or the number of Z-string terms).
hipError_t launch_grad_reduce(const double* slots, int nslots, int64_t tiles, double* sums, int p, int G,
                              int E, double* dgammas, double* dts, hipStream_t s);

// ------------------------------------------------------ QAOAz XY passes
// One tile pass of the parity mixer: the tile's amplitudes sit in LDS, and
// each listed pair (element bits ea, eb of the tile) rotates the tile's
// {01, 10} amplitude pairs by exp(-i t (XX + YY)), in list order.
constexpr int kMaxXyOps = 24;

enum : int {
    XY_PHASE = 1,   // exp(-i gamma q) before the pairs (forward) / after their inverse (backward)
    XY_EXPECT = 2,  // (f, norm) partials of the result
    XY_STORE = 4,   // write psi back
    XY_CHI = 8      // also write chi = q psi (the turn of the adjoint walk)
};

struct XyPassParams {
    double2* psi;          // forward state; phi in the backward pass
    double2* chi;          // XY_CHI target; chi in the backward pass
    const double* q;
    const double* gammas;  // gammas[layer], ts[layer]
    const double* ts;
    int n;
    int k;                 // tile bits: [0, C) and [k, k + 12 - C)
    int C;
    int elems;             // amplitudes per tile: 4096, or N for n <= 12 (one tile)
    int flags;             // XY_*
    int layer;
    int n_ops;
    uint8_t ea[kMaxXyOps];
    uint8_t eb[kMaxXyOps];
    double2* partials;     // XY_EXPECT: one (f, norm) per tile
    double* slot_t;        // backward: per-tile Im <chi|sum of the pass's H|phi>
    double* slot_g;        // backward with XY_PHASE: per-tile Im <chi|Q|phi>
};

hipError_t launch_xypass(const XyPassParams& P, int64_t tiles, hipStream_t s);
hipError_t launch_xygrad(const XyPassParams& P, int64_t tiles, hipStream_t s);

// ---------------------------------------------------------------- batched
// Many independent hypercube-mixer instances, forward + adjoint: the passes
// of every instance are grouped into rounds (round r = pass r of every
// instance that has one) and one launch runs all tiles of a round.
enum : int {
    BP_FWD = 0,     // forward tile pass (XMODE_*)
    BP_BWD = 1,     // backward tile pass (GMODE_*)
    BP_WHOLE = 2,   // n = 12: whole forward + adjoint in one workgroup
    BP_REDUCE = 3   // per-instance fixed-order sums: f and the gradient
};

struct BatchInst {
    double2* psi;
    double2* chi;
    const double* q;
    double* gammas;
    double* ts;
    double* out_f;
    double* dgammas;
    double* dts;
    double2* fpart;   // per-tile (f, norm) partials
    double* slots;    // nslots x tiles partials
    int64_t tiles;
    int n, p, G, nslots, pass_off, npass;
};

struct BatchPass {
    int kind;       // BP_*
    int mode;       // XMODE_* or GMODE_*
    int k, col_bits;
    int t1, t2, gamma;             // layers of the angles, or -1
    int slot_t1, slot_g, slot_t2;  // slot indices, or -1
};

struct BatchItem {
    int inst;
    int pass;
    int tile;
    int pad;
};

struct BatchRoundParams {
    const BatchInst* inst;
    const BatchPass* pass;
    const BatchItem* items;
    int first;    // first item of the round
};

hipError_t launch_batch_group(const BatchRoundParams& R, int kind, int mode, int col_bits, int nitems,
                              hipStream_t s);
hipError_t launch_batch_sgd(const BatchInst* inst, int count, int max_p, double lr, hipStream_t s);

}  // namespace qva
