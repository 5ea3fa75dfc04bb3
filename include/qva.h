/*
 * qva.h -- C ABI of libqva, the MI355X (gfx950) state-vector engine for
 * quantum variational algorithms (QAOA with the hypercube mixer, QWOA with a
 * circulant mixer), after Matwiejew & Wang, "QuOp_MPI: a framework for
 * parallel simulation of quantum variational algorithms".
 *
 * The library evaluates
 *
 *     f(gamma, t) = <psi_p| Q |psi_p>,
 *     psi_p = U_W(t_p) U_Q(gamma_p) ... U_W(t_1) U_Q(gamma_1) psi_0,
 *
 * (paper Sec. 2.1 eqs. variational_generic and objective_generic; Sec. 2.3.1
 * eq. qaoa; Sec. 2.4.2 eq. qwoa), with
 *     U_Q(gamma) = diag(exp(-i gamma q_j))            (eq. phase_shift_qaoa),
 *     U_W(t)     = exp(-i t W)                         (eq. mixing_generic),
 *     psi_0      = N^(-1/2) sum_j |j>                  (eq. qaoa_initial_state),
 * and its gradient with respect to every gamma_k and t_k.
 *
 * Conventions shared by every entry point
 *   - Amplitudes are complex128, stored as interleaved (re, im) doubles: the
 *     layout of torch.complex128 / hipDoubleComplex.  Qualities q and
 *     eigenvalues lambda are float64.  All of them live in device memory.
 *   - Basis index j of an n-qubit register: bit i of j is the state of qubit i.
 *   - Every pointer named *_dev or documented "device" is a device pointer
 *     owned by the caller; the library never retains a pointer after a call
 *     returns and never allocates device memory.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default
 *     stream.  Calls only enqueue work on that stream (no host
 *     synchronisation), so results are ready after the stream is synchronised,
 *     and every call can be captured into a HIP graph.
 *   - Arguments are validated on the host before anything is enqueued; on a
 *     negative status nothing was launched.  QVA_ERR_HIP reports a failed
 *     kernel launch.
 *   - Device pointers must be 16-byte aligned for complex arrays and 8-byte
 *     aligned for double arrays (QVA_ERR_ALIGN otherwise).
 */
#ifndef QVA_H
#define QVA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double re, im;
} qva_c128;

typedef enum {
    QVA_OK = 0,
    QVA_ERR_ARG = -1,         /* null pointer, bad enum, p < 0, ...          */
    QVA_ERR_SIZE = -2,        /* N or n_qubits outside the supported range   */
    QVA_ERR_ALIGN = -3,       /* misaligned device pointer                   */
    QVA_ERR_WORKSPACE = -4,   /* workspace missing or smaller than required  */
    QVA_ERR_HIP = -5,         /* a HIP launch or runtime call failed         */
    QVA_ERR_UNSUPPORTED = -6, /* well-formed request this build cannot serve */
    QVA_ERR_SCRATCH = -7      /* qva_evolve_noalloc: the request needs more
                                 workspace than QVA_STATIC_SCRATCH_BYTES      */
} qva_status;

typedef enum {
    QVA_MIX_X = 0,         /* W = sum_i X_i, the n-cube adjacency (eq. mixing_qaoa)   */
    QVA_MIX_CIRCULANT = 1, /* W circulant, given by its eigenvalues (Sec. 3)          */
    QVA_MIX_XY = 2         /* QAOAz parity mixer: an ordered product of XY rotations
                              exp(-i t (X_a X_b + Y_a Y_b)) (eqs. parity_terms,
                              qaoaz_mixers); psi_0 is the caller's (eq. qaoaz)     */
} qva_mixer;

typedef enum {
    QVA_LAMBDA_ARRAY = 0,   /* lambda[m], m = 0..N-1, natural (DFT) order             */
    QVA_LAMBDA_RING = 1,    /* cycle graph: lambda_m = 2 cos(2 pi m / N)              */
    QVA_LAMBDA_COMPLETE = 2 /* complete graph: lambda_0 = N - 1, lambda_m = -1        */
} qva_lambda_kind;

/* One term of a Pauli decomposition of a diagonal Q (extended QAOA, eq.
 * phase_shift_qaoa_ex): the Z string on the qubits set in `support`, times
 * `coef`, i.e. Sigma(j) = coef * (-1)^popcount(j & support) on basis state j. */
typedef struct {
    uint64_t support; /* qubit mask; bits at or above n_qubits never meet a basis
                         index and are ignored (0: the identity, a global phase) */
    double coef;
} qva_zterm;

#define QVA_MAX_TERMS 1024
#define QVA_MAX_XY_PAIRS 256

/* Problem descriptor (caller-owned, read during the call only).
 *   mixer       QVA_MIX_X or QVA_MIX_CIRCULANT
 *   n_qubits    log2 N rounded up; 1 <= n_qubits <= QVA_MAX_QUBITS
 *   q           device, N doubles: the diagonal of Q (paper Sec. 2.2)
 *   lambda      device, N doubles, eigenvalues of W in natural order; read only
 *               when mixer == QVA_MIX_CIRCULANT and lambda_kind == QVA_LAMBDA_ARRAY
 *   lambda_kind a qva_lambda_kind (ignored for QVA_MIX_X)
 *   n_states    N when it is not a power of two (the solution count |S'| of a
 *               constrained QWOA, Sec. 2.4.2), else 0 (N = 2^n_qubits).  A
 *               non-power-of-two N needs 2^(n_qubits-1) < N < 2^n_qubits and a
 *               circulant mixer: the complete graph (any N), or the ring or an
 *               eigenvalue array (N < 2^31, through Bluestein's
 *               transform).  Otherwise QVA_ERR_UNSUPPORTED.
 *   terms       device, n_terms qva_zterm, or NULL.  With n_terms > 0 (mixer
 *               QVA_MIX_X only) the phase of layer k is the extended-QAOA
 *               product prod_e exp(-i gamma_{k,e} Sigma_e) (eqs.
 *               phase_shift_qaoa_ex, qaoa_ex): gammas and dgammas then hold
 *               p * n_terms values, layer-major, and q is only the observable.
 *   n_terms     0 (plain QAOA phase exp(-i gamma_k q)) or 1..QVA_MAX_TERMS;
 *               outside 0..QVA_MAX_TERMS QVA_ERR_ARG, terms NULL with
 *               n_terms > 0 QVA_ERR_ARG, terms not 8-byte aligned
 *               QVA_ERR_ALIGN, a circulant mixer QVA_ERR_UNSUPPORTED.  Batched
 *               plans (qva_batch_*) take no terms.
 *   xy_pairs    host, 2 * n_xy_pairs ints (mixer QVA_MIX_XY): factor i of the
 *               mixer is exp(-i t (X_a X_b + Y_a Y_b)) with (a, b) =
 *               (xy_pairs[2i], xy_pairs[2i+1]), qubits a != b below n_qubits;
 *               factor 0 acts first.  The parity mixer of a ring (eq.
 *               qaoaz_mixers) lists B_odd's pairs, then B_even's, then B_last.
 *               Both qubits of a pair must fit one 4096-amplitude tile:
 *               min(a, b) <= 10 or |a - b| <= 8, else QVA_ERR_UNSUPPORTED.
 *               With QVA_MIX_XY, qva_evolve and qva_grad take psi_0 from psi
 *               (a state of the constrained subspace, e.g. a Dicke state).
 *   n_xy_pairs  0..QVA_MAX_XY_PAIRS (mixer QVA_MIX_XY), else ignored; a bad
 *               count, a NULL list with pairs, or a bad qubit: QVA_ERR_ARG
 *   q_tiles     device or NULL: q in the hypercube passes' tile order, written
 *               by qva_q_tiles for this problem (a per-problem layout of the
 *               same values, kept across calls).  Read only by QVA_MIX_X
 *               without Z-string terms: by the passes that apply the phase
 *               between two groups' rotations, and by qva_grad's backward
 *               passes that read q; other mixers ignore it.
 *               Results are bit-identical with and without it.  Not 8-byte
 *               aligned: QVA_ERR_ALIGN.
 *   q_tiles_key the key qva_q_tiles returned with that copy.  A key that does
 *               not match the group split in effect for n_qubits (the copy is
 *               stale): QVA_ERR_ARG, nothing launched.  Ignored when q_tiles
 *               is NULL.                                                     */
typedef struct {
    int mixer;
    int n_qubits;
    const double *q;
    const double *lambda;
    int lambda_kind;
    int64_t n_states;
    const qva_zterm *terms;
    int n_terms;
    const int32_t *xy_pairs;
    int n_xy_pairs;
    const double *q_tiles;
    uint64_t q_tiles_key;
} qva_problem;

#define QVA_MAX_QUBITS 33

/* qva_evolve flags */
#define QVA_EVOLVE_SKIP_FINAL_STATE 1 /* psi need not hold psi_p on return */

/* Group split (tuning).  The hypercube and power-of-two transform passes
 * process the qubits in groups: the contiguous low 12, then strided groups
 * of at most 9 qubits each (a tile keeps >= 8 contiguous amplitudes per row).
 * The default is the fewest such groups with near-equal sizes.
 * qva_set_group_split sets, for n_qubits-qubit registers (13 <= n_qubits <=
 * QVA_MAX_QUBITS), the sizes of the strided groups from qubit 12 upward:
 * bits[i] in 1..9, summing to n_qubits - 12 (count = 0 restores the
 * default).  The setting is process-wide and read when a call plans its
 * launches: set it between calls, never while another thread is inside a
 * library call.  It applies to qva_evolve, qva_grad, qva_mix_x,
 * qva_mix_circulant, qva_plan and batch plans created after it.
 * QVA_ERR_SIZE for n_qubits out of range, QVA_ERR_ARG for a bad split.
 * qva_get_group_split writes the split in effect (up to max entries) and
 * returns the number of strided groups (0 for n_qubits <= 12). */
int qva_set_group_split(int n_qubits, const int *bits, int count);
int qva_get_group_split(int n_qubits, int *bits, int max);

/* The factor order of the QAOAz parity mixer of a ring of qubits (Sec.
 * 2.4.1, eqs. parity_terms and qaoaz_mixers), as qva_problem.xy_pairs takes
 * it: for the ring r_1..r_m (ring: host, m ints), B_odd's pairs
 * (r_a, r_{a+1}) for odd a < m, then B_even's (r_a, r_{a+1}) for even
 * a <= m with r_{m+1} = r_1, then B_last = (r_m, r_1) when m is odd and
 * m >= 3.  Writes the first min(count, max_pairs) pairs (2 ints each) to
 * pairs (host; may be NULL when max_pairs is 0) and returns count, the
 * number of pairs of the ring (0 for m < 2).  QVA_ERR_ARG for m < 0,
 * ring NULL with m > 0, max_pairs < 0, or pairs NULL with max_pairs > 0.
 * The qubits are not checked here; qva_evolve checks them. */
int qva_parity_ring_pairs(const int *ring, int m, int *pairs, int max_pairs);

/* Human-readable text for a status code (static storage). */
const char *qva_status_string(int status);

/* Library version string (static storage). */
const char *qva_version(void);

/* psi_j = N^(-1/2) for j < N: the equal superposition of eq.
 * qaoa_initial_state (and eq. qwoa_initial_state over N solutions).
 * psi: device, N complex.  N >= 1. */
int qva_init_uniform(qva_c128 *psi, int64_t N, void *stream);

/* psi_j <- exp(-i gamma q_j) psi_j: the phase-shift unitary of eq.
 * phase_shift_generic applied elementwise (Sec. 3).
 * psi: device, N complex, in place.  q: device, N doubles.  N >= 1. */
int qva_phase(qva_c128 *psi, const double *q, int64_t N, double gamma, void *stream);

/* psi <- exp(-i t sum_i X_i) psi on n_qubits qubits: the QAOA mixer of eq.
 * mixing_qaoa, i.e. the product over qubits of exp(-i t X_i).
 * psi: device, 2^n_qubits complex, in place. */
int qva_mix_x(qva_c128 *psi, int n_qubits, double t, void *stream);

/* psi <- F^-1 diag(exp(-i t lambda_m)) F psi: a circulant mixer exp(-i t W)
 * through its eigensystem (Sec. 3), F the unnormalised DFT
 * (F_mj = exp(-2 pi i j m / N)), F^-1 = conj(F)/N.
 * psi: device, N complex, in place.  Every N the evolution takes (the N
 * feasible solutions of a constrained QWOA, Sec. 2.4.2, need not be a power
 * of two):
 *   N = 2^k, 1 <= k <= QVA_MAX_QUBITS: any lambda_kind (radix-2 passes);
 *   QVA_LAMBDA_COMPLETE, any other 2 < N <= 2^QVA_MAX_QUBITS: the closed
 *     form e^{it}(psi + (e^{-itN} - 1)/N sum(psi)) (one sum, one update);
 *   QVA_LAMBDA_RING / QVA_LAMBDA_ARRAY, any other N < 2^31: the in-place
 *     mixed-radix transform when every prime factor of N is <= 31 (e.g. the
 *     C(m, k) portfolios, m <= 31), else Bluestein's chirp-z transform over
 *     a padded power of two M >= 2N - 1.
 * N < 2 or N > 2^QVA_MAX_QUBITS: QVA_ERR_SIZE.  Ring or array over N >= 2^31
 * not a power of two: QVA_ERR_UNSUPPORTED.
 * lambda: device, N doubles in natural order when lambda_kind ==
 * QVA_LAMBDA_ARRAY, else ignored (may be NULL).
 * work: device, 16-byte aligned, >= qva_mix_circulant_workspace_bytes(N)
 * bytes (root, twiddle and permutation tables; Bluestein's padded state and
 * two filter spectra, M complex values each; or the complete graph's block
 * sums), written by the call; NULL allowed when that is 0.  Calls that share a workspace
 * must not overlap in time. */
int qva_mix_circulant(qva_c128 *psi, const double *lambda, int lambda_kind, int64_t N,
                      double t, void *work, size_t work_bytes, void *stream);

/* Bytes of device workspace qva_mix_circulant needs for N amplitudes, enough
 * for every lambda_kind (0 when none is needed or N is not supported). */
size_t qva_mix_circulant_workspace_bytes(int64_t N);

/* Bytes of device workspace that qva_evolve (for_grad = 0) or qva_grad
 * (for_grad = 1) needs for problem P at depth p.  Returns 0 when no workspace
 * is needed or the arguments are invalid (the call itself reports which). */
size_t qva_workspace_bytes(const qva_problem *P, int p, int for_grad);

/* q rearranged for qva_problem.q_tiles.  A pass of the hypercube mixer that
 * applies the phase exp(-i gamma q) of eq. phase_shift_qaoa between two
 * groups' rotations reads q over the same 4096-amplitude tile as psi: for a
 * strided group that is 256 rows of a few contiguous entries each.  The copy
 * holds, for every qubit group g of the split in effect (block g of N
 * doubles), each tile's q as one contiguous 32 KiB run in the order the pass
 * reads it.  It is a layout of an input that stays fixed over an
 * optimisation, so it is written once per problem (one pass over q per group)
 * and reused by every later qva_evolve / qva_grad.
 * qva_q_tiles_bytes: bytes `out` needs for P: G * N * 8 with G the number of
 * groups, or 0 when P's passes would not read it (a mixer other than
 * QVA_MIX_X, Z-string terms, n_qubits <= 12) or P is invalid (P->q_tiles and
 * its key are not looked at).
 * qva_q_tiles: P->q and n_qubits as for qva_evolve (P->q_tiles is ignored);
 * out device, >= qva_q_tiles_bytes(P) bytes, 8-byte aligned, not overlapping
 * q; key (host) receives the value for qva_problem.q_tiles_key.  Errors:
 * those of P, QVA_ERR_ARG for out or key NULL, QVA_ERR_ALIGN,
 * QVA_ERR_WORKSPACE for a smaller out, QVA_ERR_UNSUPPORTED when
 * qva_q_tiles_bytes(P) is 0.  Enqueued on stream; out is ready for calls
 * enqueued after it on that stream.  A later qva_set_group_split for
 * n_qubits changes the key the calls expect: write the copy again. */
size_t qva_q_tiles_bytes(const qva_problem *P);
int qva_q_tiles(const qva_problem *P, double *out, size_t out_bytes, uint64_t *key, void *stream);

/* Bytes of device workspace that qva_expectation needs for N amplitudes. */
size_t qva_expectation_workspace_bytes(int64_t N);

/* f = sum_j |psi_j|^2 q_j (eq. objective_generic) and, if out_norm_dev is not
 * NULL, sum_j |psi_j|^2.  psi: device, N complex; q: device, N doubles;
 * out_f_dev, out_norm_dev: device doubles.  Deterministic (fixed reduction
 * order).  work: device, >= qva_expectation_workspace_bytes(N) bytes. */
int qva_expectation(const qva_c128 *psi, const double *q, int64_t N, double *out_f_dev,
                    double *out_norm_dev, void *work, size_t work_bytes, void *stream);

/* The whole p-layer evolution from psi_0 and its expectation (eqs. qaoa /
 * qwoa, objective_generic), fused into as few passes over the state as the
 * operator structure allows.
 *   gammas_dev, ts_dev  device, p doubles each (layer k uses gammas_dev[k],
 *                       ts_dev[k]; layer 0 acts first).  With Z-string terms
 *                       gammas_dev holds p * n_terms: layer k's angles at
 *                       gammas_dev[k * n_terms ...] (eq. qaoa_ex)
 *   p                   depth >= 0 (p = 0 gives f = mean(q))
 *   psi                 device, N complex; working state (holds psi_0 on entry
 *                       for QVA_MIX_XY), holds psi_p on return
 *                       unless flags has QVA_EVOLVE_SKIP_FINAL_STATE
 *   out_f_dev           device double: f.  out_norm_dev (nullable): sum |psi_p|^2
 *   work, work_bytes    device workspace >= qva_workspace_bytes(P, p, 0)      */
int qva_evolve(const qva_problem *P, const double *gammas_dev, const double *ts_dev, int p,
               qva_c128 *psi, double *out_f_dev, double *out_norm_dev, int flags, void *work,
               size_t work_bytes, void *stream);

/* Size of the library's static per-device workspace (16 MiB). */
#define QVA_STATIC_SCRATCH_BYTES ((size_t)16 << 20)

/* qva_evolve without a caller workspace, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, results and launches as qva_evolve;
 * the workspace is a QVA_STATIC_SCRATCH_BYTES array inside the library, one
 * per GPU, held until the process ends.  Nothing is allocated by the call.
 *   - A request whose qva_workspace_bytes(P, p, 0) exceeds
 *     QVA_STATIC_SCRATCH_BYTES returns QVA_ERR_SCRATCH and launches nothing
 *     (e.g. the hypercube mixer up to n_qubits = 32, the ring circulant up to
 *     2^31 states; an eigenvalue array or Bluestein's padded buffers only for
 *     small N).  Argument errors are reported as by qva_evolve.
 *   - The array belongs to the GPU of `stream` (the current device for the
 *     NULL stream); its device address is looked up once per GPU, on the
 *     first call there (QVA_ERR_HIP if that lookup fails).
 *   - All calls on one GPU share that GPU's array: calls that overlap in time
 *     on one GPU (different streams, or different host threads without
 *     ordering) race and give wrong results.  Calls on one stream are safe.
 *     Every byte the evolution reads from the array is written earlier in the
 *     same call, so contents left by a previous call never matter. */
int qva_evolve_noalloc(const qva_problem *P, const double *gammas_dev, const double *ts_dev, int p,
                       qva_c128 *psi, double *out_f_dev, double *out_norm_dev, int flags,
                       void *stream);

/* f and its gradient by the adjoint method: df/dtheta_l = 2 Im <chi_l|H_l|phi_l>
 * with phi_l the state after unitary l and chi_l = U_{l+1}^dag...U_2p^dag Q psi_p,
 * both walked back from psi_p by inverse layers (no stored intermediate
 * states).  Replaces the finite-difference gradients of the paper's Sec. 4.
 *   psi, chi            device, N complex each: working states (psi holds psi_0
 *                       on entry for QVA_MIX_XY; contents on
 *                       return unspecified)
 *   out_f_dev           device double
 *   dgammas_dev, dts_dev device, p doubles each (dgammas: p * n_terms with
 *                       Z-string terms, dgammas_dev[k * n_terms + e] =
 *                       2 Im <chi|Sigma_e|phi> at the phase of layer k)
 *   work                >= qva_workspace_bytes(P, p, 1) bytes                  */
int qva_grad(const qva_problem *P, const double *gammas_dev, const double *ts_dev, int p,
             qva_c128 *psi, qva_c128 *chi, double *out_f_dev, double *dgammas_dev,
             double *dts_dev, void *work, size_t work_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Plan introspection and per-launch timing (for cost models and profilers).
 * ---------------------------------------------------------------------- */

/* Kinds of the launches that make up a plan. */
typedef enum {
    QVA_PASS_WHOLE = 0,      /* whole state in one workgroup (n <= 12), all layers  */
    QVA_PASS_FIRST = 1,      /* psi_0, phase of layer 1, first qubit group           */
    QVA_PASS_MIDDLE = 2,     /* one qubit group of one layer                         */
    QVA_PASS_BOUNDARY = 3,   /* group of layer k, phase of layer k+1, group of k+1   */
    QVA_PASS_LAST = 4,       /* last group of the last layer + <Q> partial sums      */
    QVA_PASS_LAST_STORE = 5, /* as QVA_PASS_LAST, also writes psi_p                  */
    QVA_PASS_INIT = 6,       /* elementwise psi_0                                    */
    QVA_PASS_EXPECT = 7,     /* elementwise <Q> partial sums                         */
    QVA_PASS_REDUCE = 8,     /* fixed-order sum of the partial sums                  */
    /* circulant mixer: in-place mixed-radix FFT over qubit groups (Sec. 3) */
    QVA_PASS_FFT_FIRST = 9,     /* psi_0, phase of layer 1, forward FFT of the top group */
    QVA_PASS_FFT_DIF = 10,      /* forward FFT over one group                           */
    QVA_PASS_FFT_LOWDIAG = 11,  /* low group forward, diag(exp(-i t lambda)), inverse   */
    QVA_PASS_FFT_DIT = 12,      /* inverse FFT over one group                           */
    QVA_PASS_FFT_BOUNDARY = 13, /* inverse top group, 1/N, phase of k+1, forward top    */
    QVA_PASS_FFT_LAST = 14,     /* inverse top group, 1/N, <Q> partial sums             */
    QVA_PASS_FFT_LAST_STORE = 15, /* as QVA_PASS_FFT_LAST, also writes psi_p            */
    QVA_PASS_LAMBDA_PREP = 16,  /* lambda copied into the per-tile order of the diag    */
    /* adjoint gradient (qva_grad): two vectors (phi, chi) walked backwards */
    QVA_PASS_GRAD_WHOLE = 17,   /* forward + adjoint in one workgroup (n <= 12)         */
    QVA_PASS_GRAD_TURN = 18,    /* last forward group, <Q>, chi = Q psi, first inverse  */
    QVA_PASS_GRAD_MID = 19,     /* inverse rotations of one qubit group + <chi|X|phi>   */
    QVA_PASS_GRAD_BOUND = 20,   /* inverse group, <chi|Q|phi>, inverse phase, group     */
    QVA_PASS_GRAD_FINAL = 21,   /* inverse of the first forward pass, accumulate only   */
    QVA_PASS_GRAD_DIF = 22,     /* forward FFT of one group, both vectors               */
    QVA_PASS_GRAD_DIT = 23,     /* inverse FFT of one group, both vectors               */
    QVA_PASS_GRAD_LOWDIAG = 24, /* low group, <chi^|lambda|phi^>/N, inverse diagonal    */
    QVA_PASS_GRAD_REDUCE = 25,  /* fixed-order sums of the gradient partials            */
    /* circulant mixer of the complete graph in closed form (qva_evolve with
     * QVA_LAMBDA_COMPLETE, n > 12): W = J - I has J^2 = N J, so
     * exp(-i t W) = e^{i t} (I + (e^{-i t N} - 1)/N J) (Sec. 3 eigenvalues
     * N - 1 once and -1): one reduction plus one streaming pass per layer */
    QVA_PASS_CPL_FIRST = 26,      /* psi_0 with the phase of layer 1, written, + sums     */
    QVA_PASS_CPL_LAYER = 27,      /* mixer of layer k, phase of layer k+1, written, + sums */
    QVA_PASS_CPL_LAST = 28,       /* mixer of the last layer, <Q> partial sums            */
    QVA_PASS_CPL_LAST_STORE = 29, /* as QVA_PASS_CPL_LAST, also writes psi_p              */
    QVA_PASS_CPL_SUM = 30,        /* fixed-order sum of the state's partial sums          */
    /* qva_grad with the closed-form complete-graph mixer (n > 12) */
    QVA_PASS_GRAD_CPL_TURN = 31,  /* last mixer, <Q>, chi = Q psi_p, sums for dt_p         */
    QVA_PASS_GRAD_CPL_BACK = 32,  /* inverse mixer k, <chi|Q|phi>, inverse phase k, sums   */
    QVA_PASS_GRAD_CPL_SUM = 33,   /* fixed-order sums: state sums, dt_k and dgamma_k terms */
    /* qva_evolve with a circulant (ring or eigenvalue array) over N solutions,
     * N not a power of two: Bluestein's chirp-z form over a padded power of two
     * M >= 2N - 1 (middle groups use QVA_PASS_FFT_DIF / QVA_PASS_FFT_DIT) */
    QVA_PASS_BLU_CHIRP = 34,      /* chirp filter, forward transform of the top group     */
    QVA_PASS_BLU_TILE = 35,       /* low group forward, filter spectrum stored per tile   */
    QVA_PASS_BLU_FIRST = 36,      /* psi_0, phase of layer 1, chirp, forward top group    */
    QVA_PASS_BLU_MUL = 37,        /* low group forward, times the filter spectrum, inverse */
    QVA_PASS_BLU_LAMBDA = 38,     /* inverse top group, exp(-i t lambda), forward top     */
    QVA_PASS_BLU_PHASE = 39,      /* inverse top group, exp(-i gamma q) / N, forward top  */
    QVA_PASS_BLU_LAST = 40,       /* inverse top group, <Q> partial sums                  */
    QVA_PASS_BLU_LAST_STORE = 41, /* as QVA_PASS_BLU_LAST, also writes psi_p              */
    /* QAOAz parity mixer (QVA_MIX_XY): a layer is a few tile passes, each
     * applying the pairs whose qubits lie in its tile in order; the first
     * pass of a layer also applies the phase */
    QVA_PASS_XY = 42,             /* pairs of one layer over one tile group (+ phase)     */
    QVA_PASS_XY_LAST = 43,        /* last pass of the last layer + <Q> partial sums       */
    QVA_PASS_XY_TURN = 44,        /* as QVA_PASS_XY_LAST, also writes psi_p and Q psi_p   */
    QVA_PASS_GRAD_XY = 45,        /* inverse of one XY pass on phi and chi + inner products */
    /* adjoint through Bluestein's transform (both vectors padded to M; the
     * transform passes in between are the forward's, once per vector) */
    QVA_PASS_GRAD_BLU_TURN = 46,   /* inverse top group, <Q>, chi = Q x, forward top (both) */
    QVA_PASS_GRAD_BLU_LAMBDA = 47, /* inverse top, Im<chi|W|phi>, exp(+i t lambda), forward */
    QVA_PASS_GRAD_BLU_PHASE = 48,  /* inverse top, Im<chi|Q|phi>, exp(+i gamma q), forward  */
    QVA_PASS_GRAD_BLU_FINAL = 49,  /* inverse top group, Im<chi|Q|phi> of layer 1           */
    QVA_PASS_GRAD_ZSLOT = 50,      /* extended QAOA: per-term sums of the preceding phase
                                      pass's Im(conj(chi_j) phi_j), one tile transform each */
    QVA_PASS_TWIDDLE_PREP = 51,    /* circulant transforms: the 4096 roots W_4096^k of the
                                      low-group digits, written once per call */
    /* circulant over N solutions, N not a power of two with every prime factor
     * <= 31 (e.g. N = C(m, k) for m <= 31): the DFT of length N in place over
     * groups N = A_0 A_1 ... A_{G-1} (no padding); group_first holds the
     * group index g, group_bits its size A_g, col_bits its columns per tile */
    QVA_PASS_MR_TABLES = 52,       /* roots W_{A_g}^k and digit-reversal tables, once per call */
    QVA_PASS_MR_FIRST = 53,        /* psi_0, phase of layer 1, forward top group           */
    QVA_PASS_MR_DIF = 54,          /* forward transform of one group                       */
    QVA_PASS_MR_DIT = 55,          /* inverse transform of one group                       */
    QVA_PASS_MR_LOWDIAG = 56,      /* low group forward, diag(exp(-i t lambda)), inverse   */
    QVA_PASS_MR_BOUNDARY = 57,     /* inverse top group, 1/N, phase of k+1, forward top    */
    QVA_PASS_MR_LAST = 58,         /* inverse top group, 1/N, <Q> partial sums             */
    QVA_PASS_MR_LAST_STORE = 59,   /* as QVA_PASS_MR_LAST, also writes psi_p               */
    QVA_PASS_MR_SMALL = 60,        /* N <= 4096: the whole evolution in one workgroup      */
    QVA_PASS_GRAD_MR_TURN = 61,    /* inverse top, <Q>, chi = Q psi_p, forward top (both)   */
    QVA_PASS_GRAD_MR_DIF = 62,     /* forward transform of one group, once per vector      */
    QVA_PASS_GRAD_MR_DIT = 63,     /* inverse transform of one group, once per vector      */
    QVA_PASS_GRAD_MR_LOWDIAG = 64, /* low group, Im<chi^|lambda|phi^>/N, inverse diagonal  */
    QVA_PASS_GRAD_MR_BOUND = 65,   /* inverse top, Im<chi|Q|phi>, inverse phase, forward   */
    QVA_PASS_GRAD_MR_FINAL = 66,   /* inverse top group, Im<chi|Q|phi> of layer 1          */
    QVA_PASS_GRAD_MR_SMALL = 67    /* N <= 4096: forward + adjoint in one workgroup        */
} qva_pass_kind;

/* One launch of a plan.  `bytes` is the algorithmic HBM traffic of the
 * launch: every array element the launch must read or write, counted once
 * (16 bytes per amplitude, 8 per quality or eigenvalue). */
typedef struct {
    int kind;        /* a qva_pass_kind                                  */
    int group_first; /* first qubit of the launch's qubit group (or -1)  */
    int group_bits;  /* qubits in the group (or 0)                       */
    int col_bits;    /* contiguous low index bits per tile row            */
    int mix_layer;   /* layer (0-based) of the first mixer application, or -1 */
    int mix_layer2;  /* layer of the second mixer application, or -1; for the
                        XY passes (QVA_PASS_XY..QVA_PASS_GRAD_XY) the number of
                        pair factors the pass applies                      */
    int phase_layer; /* layer whose phase the launch applies, or -1           */
    double bytes;    /* algorithmic HBM bytes of the launch               */
} qva_pass_info;

/* Number of launches qva_evolve (for_grad = 0, with `flags` as given to it)
 * or qva_grad (for_grad = 1) enqueues for P at depth p; the first min(count,
 * max_out) launches are described in out (out may be NULL when max_out = 0).
 * Returns a negative qva_status on invalid arguments. */
int qva_plan(const qva_problem *P, int p, int for_grad, int flags, qva_pass_info *out,
             int max_out);

/* qva_evolve that also records events[2i] (hipEvent_t, passed as void*)
 * before launch i of the plan and events[2i+1] after it, for i < n_events/2.
 * Events are created and owned by the caller.  Same results as qva_evolve. */
int qva_evolve_timed(const qva_problem *P, const double *gammas_dev, const double *ts_dev, int p,
                     qva_c128 *psi, double *out_f_dev, double *out_norm_dev, int flags,
                     void *work, size_t work_bytes, void *const *events, int n_events,
                     void *stream);

/* qva_grad with per-launch events, as qva_evolve_timed. */
int qva_grad_timed(const qva_problem *P, const double *gammas_dev, const double *ts_dev, int p,
                   qva_c128 *psi, qva_c128 *chi, double *out_f_dev, double *dgammas_dev,
                   double *dts_dev, void *work, size_t work_bytes, void *const *events,
                   int n_events, void *stream);

/* ------------------------------------------------------------------------
 * Batched instances: many independent QAOA problems (hypercube mixer), f and
 * the adjoint gradient of all of them per call, plus a plain gradient step.
 * The passes of all instances are grouped into rounds (round r = pass r of
 * every instance that still has one); one call enqueues a fixed sequence of
 * launches and no host work, so it can be captured into a HIP graph together
 * with qva_batch_sgd and replayed.
 * ---------------------------------------------------------------------- */

/* One instance.  All pointers are device pointers owned by the caller and
 * must stay valid for the lifetime of the plan.  n_qubits in [12, 30],
 * p in [1, QVA_BATCH_MAX_DEPTH]. */
typedef struct {
    int n_qubits;
    int p;
    const double *q;   /* 2^n qualities                                   */
    double *gammas;    /* p angles (updated in place by qva_batch_sgd)      */
    double *ts;        /* p angles (updated in place by qva_batch_sgd)      */
    qva_c128 *psi;     /* 2^n working amplitudes                          */
    qva_c128 *chi;     /* 2^n working amplitudes (adjoint state)          */
    double *out_f;     /* 1 double: f                                     */
    double *dgammas;   /* p doubles: df/dgamma                            */
    double *dts;       /* p doubles: df/dt                                */
} qva_batch_item;

#define QVA_BATCH_MAX_DEPTH 64

/* Round alignment of the instances (load balance of the launches). */
typedef enum {
    QVA_BATCH_ALIGN_START = 0, /* every instance starts in round 0                  */
    QVA_BATCH_ALIGN_END = 1,   /* every instance finishes in the last round         */
    QVA_BATCH_ALIGN_SPREAD = 2 /* start rounds chosen to even out tiles per round   */
} qva_batch_align;

typedef struct qva_batch_plan_s *qva_batch_plan;

/* Build a plan on the host (no device work).  items: host array of count
 * instances.  Returns QVA_OK and *out, or an error (nothing allocated). */
int qva_batch_create(const qva_batch_item *items, int count, int align, qva_batch_plan *out);

#define QVA_BATCH_MAX_LANES 8

/* qva_batch_create with the instances split into `lanes` (1 ..
 * QVA_BATCH_MAX_LANES) independent sequences of rounds, balanced by tiles
 * (the batched analogue of the paper's independent sub-communicators,
 * Sec. 4).  qva_batch_grad enqueues lane 0 on the caller's stream and lane k
 * on a stream of the plan's own, forked from and joined back into the
 * caller's stream with events, so that the small launches at the end of one
 * lane's rounds overlap another lane's launches; the call still enqueues no
 * host work and can be captured into a HIP graph from the caller's stream.
 * qva_batch_upload creates those lanes - 1 streams (default priority) and
 * lanes events on the current device; qva_batch_destroy releases them.
 * qva_batch_grad_timed runs every launch on the caller's stream, in plan
 * order.  Results do not depend on the lane count.  QVA_ERR_ARG for lanes
 * out of range. */
int qva_batch_create_lanes(const qva_batch_item *items, int count, int align, int lanes,
                           qva_batch_plan *out);

/* Device workspace the plan needs (tables and per-tile partial sums). */
size_t qva_batch_workspace_bytes(qva_batch_plan plan);

/* Copy the plan's tables into `work` (device, >= qva_batch_workspace_bytes,
 * 256-byte aligned) on `stream` and wait for the copy.  Later calls must pass
 * the same workspace. */
int qva_batch_upload(qva_batch_plan plan, void *work, size_t work_bytes, void *stream);

/* f and the gradient of every instance.  Enqueues qva_batch_launches() kernel
 * launches on `stream`. */
int qva_batch_grad(qva_batch_plan plan, void *work, size_t work_bytes, void *stream);

/* qva_batch_grad with events[2i] (hipEvent_t as void*) recorded before
 * launch i and events[2i+1] after it, for i < n_events / 2 (caller-owned
 * events); same results. */
int qva_batch_grad_timed(qva_batch_plan plan, void *work, size_t work_bytes, void *const *events,
                         int n_events, void *stream);

/* Launch i of qva_batch_grad (0 <= i < qva_batch_launches): its round, its
 * workgroups (one per 4096-amplitude tile) and its algorithmic HBM bytes.
 * Any output pointer may be NULL. */
int qva_batch_launch_info(qva_batch_plan plan, int i, int *round, int64_t *workgroups, double *bytes);

/* gammas -= lr * dgammas and ts -= lr * dts for every instance. */
int qva_batch_sgd(qva_batch_plan plan, double lr, void *work, size_t work_bytes, void *stream);

/* Number of rounds and of kernel launches one qva_batch_grad enqueues, and the
 * total tile count over all rounds (for cost models). */
int qva_batch_rounds(qva_batch_plan plan);
int qva_batch_launches(qva_batch_plan plan);
int64_t qva_batch_tiles(qva_batch_plan plan);

/* Release the host plan and its lane streams and events (does not touch
 * device memory). */
int qva_batch_destroy(qva_batch_plan plan);

#ifdef __cplusplus
}
#endif

#endif /* QVA_H */
