"""Quality vectors, eigenvalue vectors and parameter draws for the workloads.

The quality vector q is the diagonal of the problem's quality operator (paper,
Sec. 2.2: q_i = C(s_i) for the solution s_i encoded by basis state i).  It is an
input of the evolution, built once here and handed to both the oracle and the
GPU path.  Nothing in this module applies a unitary or reduces a state.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .graphs import erdos_renyi_edges, random_regular_edges

# One seed per benchmark workload (small QAOA, large QAOA, QWOA portfolio,
# adjoint-gradient QAOA, batched QAOA).
CONFIG_SEEDS = {"qaoa_n10": 101, "qaoa_n28": 102, "qwoa_n26": 103,
                "grad_n30": 104, "batch512": 105}

_BLOCK_BITS = 7  # q is assembled from per-byte-pair lookup tables of 2^7 x 2^7


def maxcut_qualities(n: int, edges, weights=None, *, uncut: bool = False,
                     dtype=np.float64) -> np.ndarray:
    """q_j = sum over edges (u, v) of w_uv * [bit u of j != bit v of j].

    With ``uncut=True`` the indicator is [bit u == bit v] instead (the paper's
    Example 1 quality, sum of (1 + Z_u Z_v)/2 over the edges).  Bit v of j is
    the value of vertex v.  Weights default to 1.

    Assembly: the n index bits are split into blocks of 7; an edge touches at
    most two blocks, so its contribution is a function of one 2^7 x 2^7 pair of
    block values.  Edge contributions are summed per block pair in edge order,
    and the per-pair tables are broadcast-added in a fixed order.  The result is
    deterministic for given inputs (rounding order fixed).
    """
    edges = [(int(u), int(v)) for u, v in edges]
    if weights is None:
        weights = np.ones(len(edges))
    weights = np.asarray(weights, dtype=np.float64)
    if len(weights) != len(edges):
        raise ValueError("one weight per edge")
    for u, v in edges:
        if not (0 <= u < n and 0 <= v < n) or u == v:
            raise ValueError(f"bad edge {(u, v)} for n={n}")
    N = 1 << n
    nb = (n + _BLOCK_BITS - 1) // _BLOCK_BITS
    widths = [min(_BLOCK_BITS, n - b * _BLOCK_BITS) for b in range(nb)]

    tables: dict[tuple[int, int], np.ndarray] = {}
    for (u, v), w in zip(edges, weights):
        bu, bv = u // _BLOCK_BITS, v // _BLOCK_BITS
        if bu > bv:
            u, v, bu, bv = v, u, bv, bu
        key = (bu, bv)
        su, sv = u - bu * _BLOCK_BITS, v - bv * _BLOCK_BITS
        if bu == bv:
            vals = np.arange(1 << widths[bu])
            ind = ((vals >> su) & 1) != ((vals >> sv) & 1)
            if uncut:
                ind = ~ind
            contrib = np.where(ind, w, 0.0)
            t = tables.setdefault(key, np.zeros(1 << widths[bu]))
            t += contrib
        else:
            a = (np.arange(1 << widths[bu]) >> su) & 1
            b = (np.arange(1 << widths[bv]) >> sv) & 1
            ind = a[None, :] != b[:, None]  # shape (2^wv, 2^wu): [hi, lo]
            if uncut:
                ind = ~ind
            contrib = np.where(ind, w, 0.0)
            t = tables.setdefault(key, np.zeros((1 << widths[bv], 1 << widths[bu])))
            t += contrib

    # View q as an nb-dimensional array indexed [block nb-1, ..., block 0].
    shape = tuple(1 << widths[b] for b in reversed(range(nb)))
    q = np.zeros(N, dtype=np.float64)
    qv = q.reshape(shape)
    for key in sorted(tables):
        bu, bv = key
        t = tables[key]
        idx = [None] * nb
        if bu == bv:
            idx[nb - 1 - bu] = slice(None)
            qv += t[tuple(idx)]
        else:
            # t is [block bv, block bu]; block bv is the more significant axis.
            sl = [np.newaxis] * nb
            sl[nb - 1 - bv] = slice(None)
            sl[nb - 1 - bu] = slice(None)
            qv += t[tuple(sl)]
    return q.astype(dtype, copy=False)


def maxcut_qualities_device(n: int, edges, weights, device):
    """maxcut_qualities built with torch on `device` (full-size inputs that
    are slow to build on the host).  Edge contributions are added in edge
    order, so the result is deterministic; it may differ from the host
    version in the last bit (different summation order)."""
    import torch

    j = torch.arange(1 << n, dtype=torch.int64, device=device)
    q = torch.zeros(1 << n, dtype=torch.float64, device=device)
    for (u, v), w in zip(edges, weights):
        q += (((j >> u) ^ (j >> v)) & 1).to(torch.float64) * float(w)
    del j
    return q


def ring_cut_qualities_device(n: int, device):
    """Unweighted ring MaxCut cut sizes, built with torch on `device` (for
    full-size inputs that are too slow to build on the host):
    q_j = sum_v [bit v of j != bit (v+1 mod n) of j]."""
    import torch

    q = torch.empty(1 << n, dtype=torch.float64, device=device)
    chunk = 1 << min(n, 26)  # bounded temporaries at any n
    for lo in range(0, 1 << n, chunk):
        j = torch.arange(lo, lo + chunk, dtype=torch.int64, device=device)
        acc = torch.zeros(chunk, dtype=torch.float64, device=device)
        for v in range(n):
            w = (v + 1) % n
            acc += (((j >> v) ^ (j >> w)) & 1).to(torch.float64)
        q[lo:lo + chunk] = acc
        del j, acc
    return q


def portfolio_qualities(mu: np.ndarray, sigma: np.ndarray, risk: float) -> np.ndarray:
    """q_j = mu . x - risk * x^T Sigma x with x_i = bit i of j (all 2^m subsets).

    The index is split into a low half (m_lo bits) and a high half; the cross
    term x_lo^T Sigma_lh x_hi is a small matrix product.
    """
    mu = np.asarray(mu, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    m = mu.shape[0]
    lo = m // 2
    hi = m - lo
    xl = ((np.arange(1 << lo)[:, None] >> np.arange(lo)[None, :]) & 1).astype(np.float64)
    xh = ((np.arange(1 << hi)[:, None] >> np.arange(hi)[None, :]) & 1).astype(np.float64)
    s_ll = sigma[:lo, :lo]
    s_hh = sigma[lo:, lo:]
    s_lh = sigma[:lo, lo:]
    lin_l = xl @ mu[:lo]
    lin_h = xh @ mu[lo:]
    quad_l = np.einsum("ai,ij,aj->a", xl, s_ll, xl)
    quad_h = np.einsum("ai,ij,aj->a", xh, s_hh, xh)
    cross = (xh @ s_lh.T) @ xl.T  # [hi, lo]
    q = (lin_h[:, None] + lin_l[None, :]) - risk * (
        quad_h[:, None] + quad_l[None, :] + 2.0 * cross)
    return np.ascontiguousarray(q.reshape(-1))


def draw_angles(rng: np.random.Generator, p: int, low: float = 0.0,
                high: float = math.pi) -> tuple[np.ndarray, np.ndarray]:
    """gamma[0:p] then t[0:p], each ~ U(low, high)."""
    gammas = rng.uniform(low, high, p)
    ts = rng.uniform(low, high, p)
    return gammas, ts


def random_symmetric_lambda(N: int, rng: np.random.Generator, scale: float = 2.0) -> np.ndarray:
    """A real eigenvalue vector with lambda_m = lambda_{N-m}, ~ U(-scale, scale).

    Any such vector is the spectrum of a real symmetric circulant operator.
    """
    lam = rng.uniform(-scale, scale, N)
    m = np.arange(1, N)
    lam[m] = np.maximum(lam[m], lam[N - m])  # symmetric by construction
    return lam


@dataclass
class Workload:
    """One QVA instance: mixer kind, size, q, optional lambda, parameters."""

    name: str
    mixer: str               # "x" (hypercube, N = 2^n) or "circulant"
    n: int                   # qubits (log2 N)
    q: np.ndarray
    gammas: np.ndarray
    ts: np.ndarray
    lam: np.ndarray | None = None
    lambda_kind: str = "array"   # "array", "ring" or "complete" for circulant
    edges: list = field(default_factory=list)
    weights: np.ndarray | None = None
    seed: int = 0
    supports: np.ndarray | None = None  # Z-string terms (extended QAOA); gammas then p x terms
    coefs: np.ndarray | None = None

    @property
    def N(self) -> int:
        return len(self.q) if self.q is not None else 1 << self.n

    @property
    def p(self) -> int:
        return len(self.gammas)


def qaoa_maxcut_workload(n: int, p: int, *, graph: str = "regular3", weighted: bool = True,
                         seed: int = 0, edge_prob: float = 0.5, name: str = "",
                         build_q: bool = True) -> Workload:
    """QAOA MaxCut instance: graph -> weights -> gammas -> ts from one Generator.

    With build_q=False the quality vector is left as None (build it with
    maxcut_qualities or maxcut_qualities_device from edges and weights)."""
    rng = np.random.default_rng(seed)
    if graph == "regular3":
        edges = random_regular_edges(3, n, rng)
    elif graph == "gnp":
        edges = erdos_renyi_edges(n, edge_prob, rng)
    elif graph == "ring":
        edges = [(v, (v + 1) % n) for v in range(n)]
    else:
        raise ValueError(graph)
    weights = rng.uniform(0.0, 1.0, len(edges)) if weighted else np.ones(len(edges))
    gammas, ts = draw_angles(rng, p)
    q = maxcut_qualities(n, edges, weights) if build_q else None
    return Workload(name=name or f"qaoa_maxcut_n{n}_p{p}", mixer="x", n=n, q=q,
                    gammas=gammas, ts=ts, edges=edges, weights=weights, seed=seed)


def qwoa_portfolio_workload(m: int, p: int, *, seed: int = 0, risk: float = 0.5,
                            dof: int = 30, lambda_kind: str = "ring",
                            name: str = "") -> Workload:
    """QWOA mean-variance portfolio over all 2^m subsets of m assets.

    mu ~ N(0.01, 0.02); Sigma = G^T G / dof with G (dof x m) standard normal
    (a Wishart(I, dof) draw scaled by 1/dof); then gammas, ts ~ U(0, pi).
    """
    rng = np.random.default_rng(seed)
    mu = rng.normal(0.01, 0.02, m)
    g = rng.standard_normal((dof, m))
    sigma = g.T @ g / dof
    gammas, ts = draw_angles(rng, p)
    q = portfolio_qualities(mu, sigma, risk)
    return Workload(name=name or f"qwoa_portfolio_m{m}_p{p}", mixer="circulant", n=m, q=q,
                    gammas=gammas, ts=ts, lam=None, lambda_kind=lambda_kind, seed=seed)


def qwoa_constrained_workload(m: int, k: int, p: int, *, seed: int = 0, risk: float = 0.5,
                              lambda_kind: str = "ring") -> Workload:
    """QWOA portfolio restricted to the subsets of exactly k of m assets: the
    same draws as qwoa_portfolio_workload(m, p, seed), with q kept at the
    indices of popcount k (ascending), so N = C(m, k) is not a power of two."""
    wl = qwoa_portfolio_workload(m, p, seed=seed, risk=risk, lambda_kind=lambda_kind)
    idx = np.flatnonzero(np.bitwise_count(np.arange(1 << m, dtype=np.uint64)) == k)
    return Workload(name=f"qwoa_portfolio_m{m}_k{k}_p{p}", mixer="circulant", n=int(len(idx) - 1).bit_length(),
                    q=np.ascontiguousarray(wl.q[idx]), gammas=wl.gammas, ts=wl.ts, lam=None,
                    lambda_kind=lambda_kind, seed=seed)


def maxcut_zterms(edges, weights) -> tuple[np.ndarray, np.ndarray]:
    """The non-identity terms of the MaxCut cost in the Pauli-Z basis:
    sum_e w_e [bit u != bit v] = sum_e w_e / 2 - sum_e (w_e / 2) Z_u Z_v, so one
    term per edge with support {u, v} and coefficient -w_e / 2."""
    supports = np.array([(1 << int(u)) | (1 << int(v)) for u, v in edges], dtype=np.uint64)
    coefs = -0.5 * np.asarray(weights, dtype=np.float64)
    return supports, coefs


def exqaoa_maxcut_workload(n: int, p: int, *, seed: int = 0, graph: str = "regular3",
                           build_q: bool = True) -> Workload:
    """Extended-QAOA MaxCut instance: the QAOA instance of the same seed
    (graph, weights, its per-layer gammas and ts), with the phase split into
    one term per edge; layer k starts with every term at gamma_k, plus a
    U(-0.1, 0.1) perturbation per term drawn after the QAOA draws."""
    wl = qaoa_maxcut_workload(n, p, graph=graph, seed=seed, build_q=build_q)
    supports, coefs = maxcut_zterms(wl.edges, wl.weights)
    rng = np.random.default_rng(seed + 7919)
    gammas = wl.gammas[:, None] + rng.uniform(-0.1, 0.1, (p, len(supports)))
    return Workload(name=f"exqaoa_maxcut_n{n}_p{p}", mixer="x", n=n, q=wl.q, gammas=gammas, ts=wl.ts,
                    edges=wl.edges, weights=wl.weights, seed=seed, supports=supports, coefs=coefs)


def dicke_state(n: int, k: int) -> np.ndarray:
    """|D^n_k>: equal amplitudes C(n, k)^(-1/2) on the basis states with k ones
    (a state of fixed Hamming weight, where the parity mixer keeps it)."""
    w = np.bitwise_count(np.arange(1 << n, dtype=np.uint64))
    return np.where(w == k, 1.0 / math.sqrt(math.comb(n, k)), 0.0).astype(np.complex128)


def dicke_state_device(n: int, k: int, device):
    """dicke_state built on a torch device (large n)."""
    import torch

    j = torch.arange(1 << n, dtype=torch.int64, device=device)
    w = torch.zeros_like(j)
    for b in range(n):
        w += (j >> b) & 1
    amp = (w == k).to(torch.float64) * (1.0 / math.sqrt(math.comb(n, k)))  # float64 throughout
    return amp.to(torch.complex128)


def qaoaz_portfolio_workload(m: int, k: int, p: int, *, seed: int = 0, risk: float = 0.5) -> Workload:
    """QAOAz over all 2^m subsets of the QWOA portfolio of the same seed (same
    mu, Sigma, q, gammas, ts): the parity mixer on the ring of all m qubits
    keeps the number of assets held, and psi0 = |D^m_k> starts at k of them."""
    wl = qwoa_portfolio_workload(m, p, seed=seed, risk=risk)
    return Workload(name=f"qaoaz_portfolio_m{m}_k{k}_p{p}", mixer="xy", n=m, q=wl.q, gammas=wl.gammas,
                    ts=wl.ts, seed=seed)


def batched_workloads(count: int, *, seed: int, n_range=(12, 22), p_range=(1, 8),
                      edge_prob: float = 0.4, build_q: bool = True) -> list[Workload]:
    """Independent QAOA MaxCut instances with n ~ U{n_range}, p ~ U{p_range}.

    Instance i draws its own (n, p) and then graph -> weights -> gammas -> ts
    from default_rng(seed + i).  With build_q=False q is left as None.
    """
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed + i)
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        p = int(rng.integers(p_range[0], p_range[1] + 1))
        edges = erdos_renyi_edges(n, edge_prob, rng)
        weights = rng.uniform(0.0, 1.0, len(edges))
        gammas, ts = draw_angles(rng, p)
        q = maxcut_qualities(n, edges, weights) if build_q else None
        out.append(Workload(name=f"batch{i}", mixer="x", n=n, q=q, gammas=gammas, ts=ts,
                            edges=edges, weights=weights, seed=seed + i))
    return out
