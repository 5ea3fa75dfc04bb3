"""Dense-matrix cross-check of the oracle -- TEST INFRASTRUCTURE ONLY.

For tiny systems (N <= 1024) the mixing operator W is built as a dense matrix
and exp(-i t W) is formed from its eigendecomposition (numpy.linalg.eigh):
U = V diag(exp(-i t w)) V^H.  This is an independent route to the same
definitions (paper Sec. 2.1 eq. mixing_generic, Sec. 2.3.1 eq. mixing_qaoa,
Sec. 3), sharing nothing with qva_oracle.c.
"""

from __future__ import annotations

import numpy as np

_X = np.array([[0.0, 1.0], [1.0, 0.0]])


def pauli_x_on(i: int, n: int) -> np.ndarray:
    """X acting on qubit i of n, qubit i = bit i of the basis index."""
    left = np.eye(1 << (n - 1 - i))
    right = np.eye(1 << i)
    return np.kron(left, np.kron(_X, right))


def hypercube(n: int) -> np.ndarray:
    """W_X = sum_i X_i, the n-dimensional hypercube adjacency."""
    W = np.zeros((1 << n, 1 << n))
    for i in range(n):
        W += pauli_x_on(i, n)
    return W


def circulant_from_row(w) -> np.ndarray:
    """Circulant matrix whose first row is w: C[r, c] = w[(c - r) mod N]."""
    w = np.asarray(w)
    N = len(w)
    r = np.arange(N)
    return w[(r[None, :] - r[:, None]) % N]


def expm_hermitian(W: np.ndarray, t: float) -> np.ndarray:
    """exp(-i t W) for Hermitian W by eigendecomposition."""
    w, V = np.linalg.eigh(W)
    return (V * np.exp(-1j * t * w)[None, :]) @ V.conj().T


def evolve(W: np.ndarray, q, gammas, ts) -> tuple[np.ndarray, float]:
    """psi_p and f for the alternating evolution with dense W (eqs. qaoa/qwoa)."""
    q = np.asarray(q, dtype=np.float64)
    N = len(q)
    psi = np.full(N, 1.0 / np.sqrt(N), dtype=np.complex128)
    for g, t in zip(gammas, ts):
        psi = np.exp(-1j * g * q) * psi
        psi = expm_hermitian(W, t) @ psi
    f = float(np.real(np.vdot(psi, q * psi)))
    return psi, f
