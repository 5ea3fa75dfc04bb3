"""Graph generators for MaxCut workloads (edge lists, vertex v = qubit v)."""

from __future__ import annotations

import numpy as np


def ring_edges(n: int) -> list[tuple[int, int]]:
    """Cycle C_n: edges (v, v+1 mod n), v = 0..n-1."""
    if n < 3:
        raise ValueError("a ring needs n >= 3")
    return [(v, (v + 1) % n) for v in range(n)]


def circular_ladder_edges(k: int) -> list[tuple[int, int]]:
    """Circular ladder CL_k (the graph of the paper's Example 1, k = 4).

    Vertices 0..k-1 form one cycle, k..2k-1 the other, and vertex v is joined
    to v + k by a rung.  2k vertices, 3k edges.
    """
    edges = []
    for v in range(k):
        edges.append((v, (v + 1) % k))
    for v in range(k):
        edges.append((k + v, k + (v + 1) % k))
    for v in range(k):
        edges.append((v, k + v))
    return edges


def erdos_renyi_edges(n: int, p: float, rng: np.random.Generator) -> list[tuple[int, int]]:
    """G(n, p): each pair u < v (lexicographic order) kept if rng.random() < p."""
    edges = []
    for u in range(n):
        for v in range(u + 1, n):
            if rng.random() < p:
                edges.append((u, v))
    return edges


def random_regular_edges(d: int, n: int, rng: np.random.Generator,
                         max_tries: int = 10000) -> list[tuple[int, int]]:
    """Uniform random simple d-regular graph by the pairing (configuration) model.

    n*d stubs are matched by a random permutation; a matching with a self-loop
    or a repeated edge is rejected and redrawn.
    """
    if (n * d) % 2:
        raise ValueError("n*d must be even")
    stubs = np.repeat(np.arange(n), d)
    for _ in range(max_tries):
        perm = rng.permutation(stubs)
        pairs = perm.reshape(-1, 2)
        ok = True
        seen = set()
        edges = []
        for a, b in pairs:
            a, b = int(a), int(b)
            if a == b:
                ok = False
                break
            key = (min(a, b), max(a, b))
            if key in seen:
                ok = False
                break
            seen.add(key)
            edges.append(key)
        if ok:
            edges.sort()
            return edges
    raise RuntimeError("pairing model did not produce a simple graph")
