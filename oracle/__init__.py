"""CPU oracle for the QVA state evolution -- TEST INFRASTRUCTURE ONLY.

Plain double-precision reference of what the GPU library computes.  Only the
tests, the smoke check and the benchmark's CPU-baseline leg may import it; the
product path never does.  It shares no code with the GPU library: the heavy
loops live in ``qva_oracle.c`` (built with gcc), the dense cross-check in
``dense.py`` (numpy/scipy), small helpers below (numpy).

Functions follow the paper's statement of the method:
  * initial state, eqs. qaoa_initial_state / qwoa_initial_state;
  * phase shift exp(-i gamma Q), eq. phase_shift_generic and Sec. 3;
  * hypercube mixer exp(-i t sum_i X_i), eq. mixing_qaoa;
  * circulant mixer F^-1 diag(exp(-i t lambda)) F, Sec. 3;
  * expectation <psi|Q|psi>, eq. objective_generic;
  * the layered evolution, eqs. qaoa and qwoa;
  * the extended-QAOA phase and evolution, eqs. phase_shift_qaoa_ex, qaoa_ex;
  * the QAOAz parity mixer and evolution, eqs. parity_terms, qaoaz_mixers, qaoaz.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qva_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MIX_X = 0
MIX_CIRCULANT = 1
MIX_COMPLETE = 2

_lib = None


def build(force: bool = True) -> str:
    """Compile qva_oracle.c with gcc (-O2, IEEE semantics, no fast-math,
    OpenMP over the independent loops only: results do not depend on the
    thread count)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", "-fopenmp",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    D = ctypes.c_double
    Ci = ctypes.c_int
    lib.oracle_init_uniform.argtypes = [I64, P]
    lib.oracle_phase.argtypes = [I64, P, P, D]
    lib.oracle_mix_x.argtypes = [Ci, P, D]
    lib.oracle_apply_hypercube.argtypes = [Ci, P, P]
    lib.oracle_dft.argtypes = [I64, P, P, Ci]
    lib.oracle_fft.argtypes = [I64, P, Ci]
    lib.oracle_bluestein.argtypes = [I64, P, Ci]
    lib.oracle_mix_circulant.argtypes = [I64, P, P, D]
    lib.oracle_apply_circulant.argtypes = [I64, P, P, P]
    lib.oracle_mix_complete.argtypes = [I64, P, D]
    lib.oracle_apply_complete.argtypes = [I64, P, P]
    lib.oracle_circulant_eigenvalues.argtypes = [I64, P, P, P]
    lib.oracle_expectation.argtypes = [I64, P, P, P, P]
    lib.oracle_evolve.argtypes = [Ci, I64, P, P, Ci, P, P, P, P, P]
    lib.oracle_evolve.restype = Ci
    lib.oracle_grad.argtypes = [Ci, I64, P, P, Ci, P, P, P, P, P]
    lib.oracle_grad.restype = Ci
    lib.oracle_grad_bruteforce.argtypes = [Ci, I64, P, P, Ci, P, P, P, P]
    lib.oracle_grad_bruteforce.restype = Ci
    lib.oracle_phase_terms.argtypes = [I64, P, Ci, P, P, P]
    lib.oracle_evolve_terms.argtypes = [I64, P, Ci, P, P, Ci, P, P, P, P, P]
    lib.oracle_evolve_terms.restype = Ci
    lib.oracle_grad_terms.argtypes = [I64, P, Ci, P, P, Ci, P, P, P, P, P]
    lib.oracle_grad_terms.restype = Ci
    lib.oracle_mix_xy.argtypes = [Ci, P, D, Ci, P]
    lib.oracle_parity_ring_pairs.argtypes = [Ci, P, P]
    lib.oracle_parity_ring_pairs.restype = Ci
    lib.oracle_evolve_xy.argtypes = [Ci, P, P, Ci, P, Ci, P, P, P, P, P]
    lib.oracle_evolve_xy.restype = Ci
    lib.oracle_grad_xy.argtypes = [Ci, P, P, Ci, P, Ci, P, P, P, P, P]
    lib.oracle_grad_xy.restype = Ci
    lib.oracle_set_threads.argtypes = [Ci]
    lib.oracle_get_threads.restype = Ci
    _lib = lib
    return lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _log2(N: int) -> int:
    n = int(N).bit_length() - 1
    if (1 << n) != N:
        raise ValueError(f"N={N} is not a power of two")
    return n


def set_threads(n: int) -> None:
    """Threads for the oracle's independent loops (sums stay single-threaded)."""
    _load().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


# ----------------------------------------------------------------- primitives
def init_uniform(N: int) -> np.ndarray:
    psi = np.empty(N, np.complex128)
    _load().oracle_init_uniform(N, _ptr(psi))
    return psi


def phase(psi, q, gamma: float) -> np.ndarray:
    psi = _c128(psi).copy()
    q = _f64(q)
    _load().oracle_phase(len(psi), _ptr(psi), _ptr(q), float(gamma))
    return psi


def mix_x(psi, t: float) -> np.ndarray:
    psi = _c128(psi).copy()
    _load().oracle_mix_x(_log2(len(psi)), _ptr(psi), float(t))
    return psi


def apply_hypercube(psi) -> np.ndarray:
    psi = _c128(psi)
    out = np.empty_like(psi)
    _load().oracle_apply_hypercube(_log2(len(psi)), _ptr(psi), _ptr(out))
    return out


def dft(x, sign: int = -1) -> np.ndarray:
    x = _c128(x)
    out = np.empty_like(x)
    _load().oracle_dft(len(x), _ptr(x), _ptr(out), int(sign))
    return out


def fft(x, sign: int = -1) -> np.ndarray:
    x = _c128(x).copy()
    _log2(len(x))
    _load().oracle_fft(len(x), _ptr(x), int(sign))
    return x


def mix_circulant(psi, lam, t: float) -> np.ndarray:
    psi = _c128(psi).copy()
    lam = _f64(lam)
    _load().oracle_mix_circulant(len(psi), _ptr(psi), _ptr(lam), float(t))
    return psi


def bluestein(x, sign: int = -1) -> np.ndarray:
    """sum_j x_j exp(sign 2 pi i j m / N) for any N (chirp-z over radix-2 FFTs)."""
    x = _c128(x).copy()
    _load().oracle_bluestein(len(x), _ptr(x), int(sign))
    return x


def mix_complete(psi, t: float) -> np.ndarray:
    """exp(-i t (J - I)) psi from the definition (closed form)."""
    psi = _c128(psi).copy()
    _load().oracle_mix_complete(len(psi), _ptr(psi), float(t))
    return psi


def apply_complete(psi) -> np.ndarray:
    """(J - I) psi = sum(psi) - psi."""
    psi = _c128(psi)
    out = np.empty_like(psi)
    _load().oracle_apply_complete(len(psi), _ptr(psi), _ptr(out))
    return out


def apply_circulant(psi, lam) -> np.ndarray:
    psi = _c128(psi)
    lam = _f64(lam)
    out = np.empty_like(psi)
    _load().oracle_apply_circulant(len(psi), _ptr(psi), _ptr(lam), _ptr(out))
    return out


def circulant_eigenvalues(w) -> tuple[np.ndarray, np.ndarray]:
    """(Re, Im) of lambda_m for the circulant with first row w (Sec. 3)."""
    w = _f64(w)
    re = np.empty(len(w))
    im = np.empty(len(w))
    _load().oracle_circulant_eigenvalues(len(w), _ptr(w), _ptr(re), _ptr(im))
    return re, im


def expectation(psi, q) -> tuple[float, float]:
    """(f, norm) = (sum |psi_j|^2 q_j, sum |psi_j|^2), pairwise sums."""
    psi = _c128(psi)
    q = _f64(q)
    f = ctypes.c_double()
    nrm = ctypes.c_double()
    _load().oracle_expectation(len(psi), _ptr(psi), _ptr(q), ctypes.byref(f), ctypes.byref(nrm))
    return f.value, nrm.value


# ------------------------------------------------------------ eigenvalues
def ring_lambda(N: int) -> np.ndarray:
    """Eigenvalues of the N-cycle adjacency: first row w_1 = w_{N-1} = 1, so
    lambda_m = omega^m + omega^-m = 2 cos(2 pi m / N)."""
    m = np.arange(N, dtype=np.float64)
    return 2.0 * np.cos(2.0 * math.pi * m / N)


def complete_lambda(N: int) -> np.ndarray:
    """Eigenvalues of the complete-graph adjacency (w_l = 1 for l != 0):
    lambda_0 = N - 1 and lambda_m = -1 otherwise."""
    lam = np.full(N, -1.0)
    lam[0] = N - 1.0
    return lam


def lambda_for(kind: str, N: int, lam=None) -> np.ndarray:
    if kind == "ring":
        return ring_lambda(N)
    if kind == "complete":
        return complete_lambda(N)
    if lam is None:
        raise ValueError("lambda array required")
    return _f64(lam)


# ------------------------------------------------------------- evolution
def _kind(mixer: str) -> int:
    return {"x": MIX_X, "circulant": MIX_CIRCULANT, "complete": MIX_COMPLETE}[mixer]


def evolve(mixer: str, q, gammas, ts, lam=None) -> tuple[np.ndarray, float, float]:
    """(psi_p, f, norm) for the p-layer evolution (eqs. qaoa / qwoa)."""
    q = _f64(q)
    gammas = _f64(gammas)
    ts = _f64(ts)
    if len(gammas) != len(ts):
        raise ValueError("one gamma and one t per layer")
    lam = None if lam is None else _f64(lam)
    N = len(q)
    psi = np.empty(N, np.complex128)
    f = ctypes.c_double()
    nrm = ctypes.c_double()
    rc = _load().oracle_evolve(_kind(mixer), N, _ptr(q), _ptr(lam), len(gammas), _ptr(gammas),
                               _ptr(ts), _ptr(psi), ctypes.byref(f), ctypes.byref(nrm))
    if rc:
        raise ValueError("oracle_evolve: bad arguments")
    return psi, f.value, nrm.value


def grad(mixer: str, q, gammas, ts, lam=None) -> tuple[float, np.ndarray, np.ndarray]:
    """(f, df/dgamma, df/dt) by the adjoint walk."""
    q = _f64(q)
    gammas = _f64(gammas)
    ts = _f64(ts)
    lam = None if lam is None else _f64(lam)
    p = len(gammas)
    dg = np.empty(p)
    dt = np.empty(p)
    f = ctypes.c_double()
    rc = _load().oracle_grad(_kind(mixer), len(q), _ptr(q), _ptr(lam), p, _ptr(gammas), _ptr(ts),
                             ctypes.byref(f), _ptr(dg), _ptr(dt))
    if rc:
        raise ValueError("oracle_grad: bad arguments")
    return f.value, dg, dt


def grad_bruteforce(mixer: str, q, gammas, ts, lam=None) -> tuple[np.ndarray, np.ndarray]:
    """(df/dgamma, df/dt) by differentiating each factor of the product."""
    q = _f64(q)
    gammas = _f64(gammas)
    ts = _f64(ts)
    lam = None if lam is None else _f64(lam)
    p = len(gammas)
    dg = np.empty(p)
    dt = np.empty(p)
    rc = _load().oracle_grad_bruteforce(_kind(mixer), len(q), _ptr(q), _ptr(lam), p,
                                        _ptr(gammas), _ptr(ts), _ptr(dg), _ptr(dt))
    if rc:
        raise ValueError("oracle_grad_bruteforce: bad arguments")
    return dg, dt


# ------------------------------------------------------- problem qualities
def maxcut_quality_loop(n: int, edges, weights=None, uncut: bool = False) -> np.ndarray:
    """Quality vector by a plain loop over basis states and edges (Sec. 5.1,
    eq. maxcut-cost: an edge contributes when its endpoints differ, or when
    they agree for the uncut form).  Pure Python; small n only."""
    if weights is None:
        weights = [1.0] * len(edges)
    q = np.zeros(1 << n)
    for j in range(1 << n):
        s = 0.0
        for (u, v), w in zip(edges, weights):
            differ = ((j >> u) & 1) != ((j >> v) & 1)
            if differ != uncut:
                s += w
        q[j] = s
    return q


# ------------------------------------------------------------ extended QAOA
def _terms(support, coef):
    S = np.ascontiguousarray(np.asarray(support, dtype=np.uint64))
    c = _f64(coef)
    if S.shape != c.shape:
        raise ValueError("one coefficient per term")
    return S, c


def phase_terms(psi, support, coef, gamma) -> np.ndarray:
    """psi_j <- exp(-i sum_e gamma_e c_e (-1)^popcount(j & S_e)) psi_j
    (eq. phase_shift_qaoa_ex with Z-string terms)."""
    S, c = _terms(support, coef)
    psi = _c128(psi).copy()
    _load().oracle_phase_terms(len(psi), _ptr(psi), len(S), _ptr(S), _ptr(c), _ptr(_f64(gamma)))
    return psi


def evolve_terms(q, support, coef, gammas, ts) -> tuple[np.ndarray, float, float]:
    """Extended QAOA (eq. qaoa_ex): gammas is p x n_terms; q the observable."""
    S, c = _terms(support, coef)
    q = _f64(q)
    g = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64).reshape(len(ts), len(S)))
    ts = _f64(ts)
    psi = np.empty(len(q), np.complex128)
    f = ctypes.c_double()
    nrm = ctypes.c_double()
    rc = _load().oracle_evolve_terms(len(q), _ptr(q), len(S), _ptr(S), _ptr(c), len(ts), _ptr(g), _ptr(ts),
                                     _ptr(psi), ctypes.byref(f), ctypes.byref(nrm))
    if rc:
        raise ValueError("oracle_evolve_terms: bad arguments")
    return psi, f.value, nrm.value


def grad_terms(q, support, coef, gammas, ts) -> tuple[float, np.ndarray, np.ndarray]:
    """(f, df/dgamma (p x n_terms), df/dt) by the adjoint walk."""
    S, c = _terms(support, coef)
    q = _f64(q)
    p = len(ts)
    g = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64).reshape(p, len(S)))
    ts = _f64(ts)
    dg = np.empty((p, len(S)))
    dt = np.empty(p)
    f = ctypes.c_double()
    rc = _load().oracle_grad_terms(len(q), _ptr(q), len(S), _ptr(S), _ptr(c), p, _ptr(g), _ptr(ts),
                                   ctypes.byref(f), _ptr(dg), _ptr(dt))
    if rc:
        raise ValueError("oracle_grad_terms: bad arguments")
    return f.value, dg, dt


# ------------------------------------------------------------------- QAOAz
def _pairs(pairs) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    return a


def parity_ring_pairs(ring) -> np.ndarray:
    """Factors of U_parity (eqs. parity_terms, qaoaz_mixers) for the ring of
    qubits `ring`, in the order they act: B_odd, B_even, then B_last."""
    r = np.ascontiguousarray(np.asarray(ring, dtype=np.int32))
    out = np.empty((len(r) + 1, 2), dtype=np.int32)
    c = _load().oracle_parity_ring_pairs(len(r), _ptr(r), _ptr(out))
    return out[:c].copy()


def mix_xy(psi, pairs, t: float) -> np.ndarray:
    """psi <- prod_i exp(-i t (X_a X_b + Y_a Y_b)) psi, factor 0 first."""
    psi = _c128(psi).copy()
    pr = _pairs(pairs)
    _load().oracle_mix_xy(_log2(len(psi)), _ptr(psi), float(t), len(pr), _ptr(pr))
    return psi


def evolve_xy(q, psi0, pairs, gammas, ts) -> tuple[np.ndarray, float, float]:
    """QAOAz (eq. qaoaz) from the given psi0: (psi_p, f, norm)."""
    q = _f64(q)
    psi0 = _c128(psi0)
    pr = _pairs(pairs)
    g, t = _f64(gammas), _f64(ts)
    psi = np.empty(len(q), np.complex128)
    f = ctypes.c_double()
    nrm = ctypes.c_double()
    rc = _load().oracle_evolve_xy(_log2(len(q)), _ptr(q), _ptr(psi0), len(pr), _ptr(pr), len(t), _ptr(g),
                                  _ptr(t), _ptr(psi), ctypes.byref(f), ctypes.byref(nrm))
    if rc:
        raise ValueError("oracle_evolve_xy: bad arguments")
    return psi, f.value, nrm.value


def grad_xy(q, psi0, pairs, gammas, ts) -> tuple[float, np.ndarray, np.ndarray]:
    """(f, df/dgamma, df/dt) of QAOAz by the adjoint walk."""
    q = _f64(q)
    psi0 = _c128(psi0)
    pr = _pairs(pairs)
    g, t = _f64(gammas), _f64(ts)
    p = len(t)
    dg = np.empty(p)
    dt = np.empty(p)
    f = ctypes.c_double()
    rc = _load().oracle_grad_xy(_log2(len(q)), _ptr(q), _ptr(psi0), len(pr), _ptr(pr), p, _ptr(g), _ptr(t),
                                ctypes.byref(f), _ptr(dg), _ptr(dt))
    if rc:
        raise ValueError("oracle_grad_xy: bad arguments")
    return f.value, dg, dt
