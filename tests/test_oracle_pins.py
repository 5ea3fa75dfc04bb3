"""Pins of the CPU oracle to facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a value the
paper prints, a closed form, an invariant, a dense eigendecomposition built by
numpy, or a library routine (numpy.fft, scipy.linalg.expm, scipy.special.jv).
"""

import json
import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize
import scipy.special

import oracle
import oracle.dense as dense
from workloads import (circular_ladder_edges, erdos_renyi_edges, maxcut_qualities,
                       portfolio_qualities, random_regular_edges, ring_edges,
                       random_symmetric_lambda)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_state(rng, N):
    v = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    return v / np.linalg.norm(v)


# ------------------------------------------------------------------ paper
def _example1():
    with open(os.path.join(GOLDEN, "example1_maxcut_cl4.json")) as fh:
        return json.load(fh)


def test_example1_printed_objective(oracle_mod):
    """Sec. 5.1.1: CL_4 max-cut at depth 2 ends near f = 2.30 at x = (3.59, 6.88,
    3.95, 5.92); the optimal state 90 (q_90 = 0) is the most probable one."""
    g = _example1()
    edges = circular_ladder_edges(4)
    q = oracle.maxcut_quality_loop(8, edges, uncut=True)
    x = np.array(g["x_printed"])
    psi, f, nrm = oracle.evolve("x", q, x[0::2], x[1::2])
    assert abs(f - g["f_printed_approx"]) < 0.01
    assert q[g["optimal_state_index"]] == g["optimal_state_quality"]
    bits = [(g["optimal_state_index"] >> v) & 1 for v in range(8)]
    assert bits == g["optimal_state_bits_printed"]
    prob = np.abs(psi) ** 2
    top = np.sort(np.argsort(-prob)[:2])
    # states 90 and 165 (its complement) tie exactly by the bit-flip symmetry
    assert list(top) == [90, 165]
    assert abs(prob[90] - prob[165]) < 1e-14


def test_example1_is_a_local_minimum(oracle_mod):
    """The printed x is (to 2 decimals) a local minimum: BFGS started there
    stays within 0.01 and ends at f ~ 2.30."""
    g = _example1()
    q = oracle.maxcut_quality_loop(8, circular_ladder_edges(4), uncut=True)

    def fun(x):
        return oracle.evolve("x", q, x[0::2], x[1::2])[1]

    def jac(x):
        _, dg, dt = oracle.grad("x", q, x[0::2], x[1::2])
        out = np.empty(4)
        out[0::2] = dg
        out[1::2] = dt
        return out

    x0 = np.array(g["x_printed"])
    res = scipy.optimize.minimize(fun, x0, jac=jac, method="BFGS", tol=1e-10)
    assert np.max(np.abs(res.x - x0)) < 0.01
    assert abs(res.fun - g["f_printed_approx"]) < 0.01
    assert res.fun <= fun(x0)


def test_example1_rejects_misreadings(oracle_mod):
    """The printed pair (x, f) separates the readings: a flipped mixer sign or a
    blocked parameter order moves f far from 2.30."""
    g = _example1()
    q = oracle.maxcut_quality_loop(8, circular_ladder_edges(4), uncut=True)
    x = np.array(g["x_printed"])
    f_flip = oracle.evolve("x", q, x[0::2], -x[1::2])[1]
    f_block = oracle.evolve("x", q, x[0:2], x[2:4])[1]
    f_mixer_first = dense.evolve(dense.hypercube(8), q, [0.0], [0.0])[1]  # sanity: mean(q)
    assert abs(f_flip - 2.30) > 1.0
    assert abs(f_block - 2.30) > 1.0
    assert abs(f_mixer_first - q.mean()) < 1e-12


def test_example1_paper_graph_matches_networkx():
    nx = pytest.importorskip("networkx")
    G = nx.circular_ladder_graph(4)
    ours = {tuple(sorted(e)) for e in circular_ladder_edges(4)}
    theirs = {tuple(sorted(e)) for e in G.edges()}
    assert ours == theirs


# ------------------------------------------------------------- dense checks
@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_mix_x_matches_dense_expm(oracle_mod, n):
    rng = np.random.default_rng(n)
    psi = _rand_state(rng, 1 << n)
    W = dense.hypercube(n)
    for t in [0.0, 0.3, -1.1, 2.9, math.pi / 2]:
        ref = dense.expm_hermitian(W, t) @ psi
        ref2 = scipy.linalg.expm(-1j * t * W) @ psi
        out = oracle.mix_x(psi, t)
        assert np.max(np.abs(out - ref)) < 1e-13
        assert np.max(np.abs(out - ref2)) < 1e-12


@pytest.mark.parametrize("N", [2, 3, 5, 8, 12, 64])
def test_mix_circulant_matches_dense_expm(oracle_mod, N):
    rng = np.random.default_rng(N)
    psi = _rand_state(rng, N)
    row = rng.uniform(-1, 1, N)
    row = 0.5 * (row + row[(-np.arange(N)) % N])  # symmetric first row
    C = dense.circulant_from_row(row)
    lam_re, lam_im = oracle.circulant_eigenvalues(row)
    assert np.max(np.abs(lam_im)) < 1e-12
    for t in [0.0, 0.4, -2.0]:
        ref = dense.expm_hermitian(C, t) @ psi
        out = oracle.mix_circulant(psi, lam_re, t)
        assert np.max(np.abs(out - ref)) < 1e-13


def test_mix_circulant_fft_path_matches_dense(oracle_mod):
    """N = 8192 exercises the radix-2 FFT branch; compare with a dense
    application of the ring circulant built from its first row (N^2 too big for
    eigh, so compare with the DFT branch on the same input instead)."""
    N = 8192
    rng = np.random.default_rng(1)
    psi = _rand_state(rng, N)
    lam = oracle.ring_lambda(N)
    out = oracle.mix_circulant(psi, lam, 0.7)
    ref = np.fft.ifft(np.exp(-0.7j * lam) * np.fft.fft(psi))
    assert np.max(np.abs(out - ref)) < 1e-13


@pytest.mark.parametrize("mixer,n", [("x", 3), ("x", 6), ("circulant", 4), ("circulant", 7)])
def test_evolve_matches_dense(oracle_mod, mixer, n):
    rng = np.random.default_rng(10 + n)
    N = 1 << n
    q = rng.uniform(-1, 2, N)
    p = 3
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    if mixer == "x":
        W = dense.hypercube(n)
        lam = None
    else:
        row = np.zeros(N)
        row[1] = row[-1] = 1.0
        W = dense.circulant_from_row(row)
        lam = oracle.ring_lambda(N)
    psi, f, nrm = oracle.evolve(mixer, q, g, t, lam)
    psi_d, f_d = dense.evolve(W, q, g, t)
    assert np.max(np.abs(psi - psi_d)) < 1e-13
    assert abs(f - f_d) <= 1e-12 * np.sum(np.abs(psi_d) ** 2 * np.abs(q))
    assert abs(nrm - 1) < 1e-13


# ---------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", [1, 4, 9, 12])
def test_mix_x_on_delta_closed_form(oracle_mod, n):
    """exp(-i t sum X_i)|0> = prod_i (cos t |0> - i sin t |1>):
    amplitude of j is cos(t)^(n-|j|) (-i sin t)^|j|, |j| = popcount."""
    N = 1 << n
    psi = np.zeros(N, complex)
    psi[0] = 1
    t = 0.37
    out = oracle.mix_x(psi, t)
    pc = np.array([bin(j).count("1") for j in range(N)])
    ref = np.cos(t) ** (n - pc) * (-1j * np.sin(t)) ** pc
    assert np.max(np.abs(out - ref)) < 1e-15


@pytest.mark.parametrize("N,t", [(64, 0.9), (4096, 2.5), (16384, 3.1)])
def test_ring_circulant_on_delta_bessel(oracle_mod, N, t):
    """Ring walk from site 0: amplitude at j is sum over images d = j + mN of
    (-i)^|d| J_|d|(2t) (Jacobi-Anger expansion of exp(-2it cos k))."""
    psi = np.zeros(N, complex)
    psi[0] = 1
    out = oracle.mix_circulant(psi, oracle.ring_lambda(N), t)
    j = np.arange(N)
    ref = np.zeros(N, complex)
    for m in range(-2, 3):
        d = np.abs(j + m * N)
        mask = d < 80
        ref[mask] += (-1j) ** d[mask] * scipy.special.jv(d[mask], 2 * t)
    assert np.max(np.abs(out - ref)) < 1e-14


@pytest.mark.parametrize("N", [8, 100, 4096, 8192])
def test_complete_graph_closed_form(oracle_mod, N):
    """W = J - I: exp(-itW) psi = e^{it} (psi + (e^{-itN} - 1)/N * sum(psi))."""
    rng = np.random.default_rng(N)
    psi = _rand_state(rng, N)
    t = 0.83
    out = oracle.mix_circulant(psi, oracle.complete_lambda(N), t)
    ref = np.exp(1j * t) * (psi + (np.exp(-1j * t * N) - 1) / N * psi.sum())
    assert np.max(np.abs(out - ref)) < 1e-13


@pytest.mark.parametrize("N", [1, 2, 3, 7, 16, 33])
def test_complete_mixer_definition_matches_dense_expm(oracle_mod, N):
    """The oracle's complete-graph mixer (written from W = J - I) against a
    dense eigendecomposition of the complete graph's adjacency, and W psi
    against the dense matrix product."""
    rng = np.random.default_rng(N + 7)
    psi = _rand_state(rng, N)
    W = np.ones((N, N)) - np.eye(N)
    for t in [0.0, 0.45, -1.7, 2 * math.pi / N, 11.3]:
        ref = dense.expm_hermitian(W, t) @ psi
        assert np.max(np.abs(oracle.mix_complete(psi, t) - ref)) < 1e-13
    assert np.max(np.abs(oracle.apply_complete(psi) - W @ psi)) < 1e-14


@pytest.mark.parametrize("N", [8, 100, 4096, 8192])
def test_complete_mixer_matches_transform(oracle_mod, N):
    """The same mixer through the circulant route (Sec. 3 eigenvalues N - 1,
    -1, DFT for N <= 4096, FFT above) and numpy's expm-free closed form."""
    rng = np.random.default_rng(N)
    psi = _rand_state(rng, N)
    for t in [0.83, -0.2]:
        a = oracle.mix_complete(psi, t)
        b = oracle.mix_circulant(psi, oracle.complete_lambda(N), t)
        assert np.max(np.abs(a - b)) < 1e-13
        assert abs(np.linalg.norm(a) - 1) < 1e-14


@pytest.mark.parametrize("n,p", [(3, 2), (6, 3), (9, 4)])
def test_complete_evolve_and_gradient(oracle_mod, n, p):
    """evolve / grad with the closed-form mixer: equal to the transform route
    at small N, adjoint == brute-force differentiation, central differences."""
    rng = np.random.default_rng(40 + n)
    N = 1 << n
    q = rng.uniform(-1, 4, N)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    lam = oracle.complete_lambda(N)
    psi_a, f_a, _ = oracle.evolve("complete", q, g, t)
    psi_b, f_b, _ = oracle.evolve("circulant", q, g, t, lam)
    assert np.max(np.abs(psi_a - psi_b)) < 1e-12
    assert abs(f_a - f_b) < 1e-12 * np.max(np.abs(q))
    f, dg, dt = oracle.grad("complete", q, g, t)
    assert f == f_a
    bg, bt = oracle.grad_bruteforce("complete", q, g, t)
    _, cg, ct = oracle.grad("circulant", q, g, t, lam)
    scale = max(np.max(np.abs(dg)), np.max(np.abs(dt)))
    for ref_g, ref_t in [(bg, bt), (cg, ct)]:
        assert np.max(np.abs(dg - ref_g)) < 1e-11 * scale
        assert np.max(np.abs(dt - ref_t)) < 1e-11 * scale
    _check_complete_fd(q, g, t, dg, dt, scale, 1e-7)


def _check_complete_fd(q, g, t, dg, dt, scale, tol):
    """Central differences; f oscillates in t_k at frequency N (through
    e^{-i t N}), so the t step is taken as 1e-5 / N."""
    N, p = len(q), len(g)
    for k in range(p):
        e = np.zeros(p)
        e[k] = 1e-5
        fd_g = (oracle.evolve("complete", q, g + e, t)[1] - oracle.evolve("complete", q, g - e, t)[1]) / 2e-5
        e[k] = 1e-5 / N
        fd_t = (oracle.evolve("complete", q, g, t + e)[1] - oracle.evolve("complete", q, g, t - e)[1]) / (2e-5 / N)
        assert abs(fd_g - dg[k]) < tol * scale, (k, fd_g, dg[k])
        assert abs(fd_t - dt[k]) < tol * scale, (k, fd_t, dt[k])


def test_complete_gradient_central_differences_large(oracle_mod):
    """At N = 2^16, where the transform route loses accuracy through the
    eigenvalue N - 1, the closed-form adjoint still agrees with central
    differences of the closed-form evolution."""
    rng = np.random.default_rng(16)
    N = 1 << 16
    p = 3
    q = rng.uniform(-1, 3, N)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    _, dg, dt = oracle.grad("complete", q, g, t)
    scale = max(np.max(np.abs(dg)), np.max(np.abs(dt)))
    _check_complete_fd(q, g, t, dg, dt, scale, 1e-6)


def test_circulant_eigenvalue_formula(oracle_mod):
    """Sec. 3 eigenvalue formula vs the ring/complete closed forms and numpy's
    eigvalsh of the dense circulant."""
    for N in [3, 8, 13, 32]:
        row = np.zeros(N)
        row[1] = row[-1] = 1.0
        re, im = oracle.circulant_eigenvalues(row)
        assert np.max(np.abs(re - oracle.ring_lambda(N))) < 1e-13
        assert np.max(np.abs(im)) < 1e-13
        row = np.ones(N)
        row[0] = 0
        re, im = oracle.circulant_eigenvalues(row)
        assert np.max(np.abs(re - oracle.complete_lambda(N))) < 1e-12
        rng = np.random.default_rng(N)
        row = rng.uniform(-1, 1, N)
        row = 0.5 * (row + row[(-np.arange(N)) % N])
        re, _ = oracle.circulant_eigenvalues(row)
        ev = np.linalg.eigvalsh(dense.circulant_from_row(row))
        assert np.max(np.abs(np.sort(re) - ev)) < 1e-12


@pytest.mark.parametrize("n", [4, 5, 6, 8, 10])
def test_ring_maxcut_p1_closed_form(oracle_mod, n):
    """Unweighted ring, cut quality, p = 1:
    f = n (1/2 + 1/4 sin 4t sin 2gamma); df/dgamma = (n/2) sin 4t cos 2gamma;
    df/dt = n cos 4t sin 2gamma."""
    q = oracle.maxcut_quality_loop(n, ring_edges(n))
    for g, t in [(0.3, 0.2), (1.9, 2.7), (-0.4, 1.0)]:
        f, dg, dt = oracle.grad("x", q, [g], [t])
        assert abs(f - n * (0.5 + 0.25 * math.sin(4 * t) * math.sin(2 * g))) < 1e-13 * n
        assert abs(dg[0] - n / 2 * math.sin(4 * t) * math.cos(2 * g)) < 1e-12 * n
        assert abs(dt[0] - n * math.cos(4 * t) * math.sin(2 * g)) < 1e-12 * n


def test_weighted_triangle_free_p1_closed_form(oracle_mod):
    """Weighted triangle-free graph, p = 1, per-edge expectation
    w_uv [1/2 + 1/4 sin 4t sin(gamma w_uv) (prod_{x in N(u)\\v} cos(gamma w_ux)
    + prod_{y in N(v)\\u} cos(gamma w_vy))]."""
    rng = np.random.default_rng(7)
    n = 8
    edges = [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (5, 6), (6, 7), (7, 0), (0, 4), (2, 6)]
    # a bipartite (hence triangle-free) graph: the 8-cycle with two chords joining even vertices
    # to even vertices would create triangles only with an odd cycle of length 3; check it:
    adj = {v: set() for v in range(n)}
    for u, v in edges:
        adj[u].add(v)
        adj[v].add(u)
    assert all(not (adj[u] & adj[v]) for u, v in edges)
    w = rng.uniform(0.2, 1.0, len(edges))
    W = {}
    for (u, v), x in zip(edges, w):
        W[(u, v)] = W[(v, u)] = x
    q = oracle.maxcut_quality_loop(n, edges, w)
    g, t = 0.9, 0.35
    f = oracle.evolve("x", q, [g], [t])[1]
    ref = 0.0
    for (u, v), x in zip(edges, w):
        pu = np.prod([math.cos(g * W[(u, y)]) for y in adj[u] if y != v])
        pv = np.prod([math.cos(g * W[(v, y)]) for y in adj[v] if y != u])
        ref += x * (0.5 + 0.25 * math.sin(4 * t) * math.sin(g * x) * (pu + pv))
    assert abs(f - ref) < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3])
def test_ring_light_cone(oracle_mod, p):
    """For a ring, f/n is the same for every n >= 2p + 2 (each edge term sees
    only its distance-p neighbourhood)."""
    rng = np.random.default_rng(p)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    vals = []
    for n in range(2 * p + 2, 2 * p + 5):
        q = oracle.maxcut_quality_loop(n, ring_edges(n))
        vals.append(oracle.evolve("x", q, g, t)[1] / n)
    assert np.ptp(vals) < 1e-13


# ---------------------------------------------------------------- invariants
def test_uniform_state_is_fixed_point(oracle_mod):
    """p = 0, all gamma = 0, or all t = 0 give f = mean(q) (the uniform state is
    an eigenvector of both mixers)."""
    rng = np.random.default_rng(3)
    n = 7
    q = rng.uniform(-3, 3, 1 << n)
    assert abs(oracle.evolve("x", q, [], [])[1] - q.mean()) < 1e-14
    for mixer, lam in [("x", None), ("circulant", oracle.ring_lambda(1 << n)),
                       ("circulant", oracle.complete_lambda(1 << n))]:
        f0 = oracle.evolve(mixer, q, [0.0, 0.0], [0.4, 1.3], lam)[1]
        f1 = oracle.evolve(mixer, q, [0.5, 2.0], [0.0, 0.0], lam)[1]
        assert abs(f0 - q.mean()) < 1e-13
        assert abs(f1 - q.mean()) < 1e-13


def test_norm_preserved(oracle_mod):
    """Unitary evolution keeps the norm to ~1e-13 (the paper reports per-state
    norm deviations of that order, Sec. 6)."""
    rng = np.random.default_rng(4)
    for mixer in ["x", "circulant"]:
        n = 10
        q = rng.uniform(0, 10, 1 << n)
        lam = None if mixer == "x" else random_symmetric_lambda(1 << n, rng)
        g = rng.uniform(0, math.pi, 5)
        t = rng.uniform(0, math.pi, 5)
        _, _, nrm = oracle.evolve(mixer, q, g, t, lam)
        assert abs(nrm - 1) < 1e-13


def test_symmetries(oracle_mod):
    rng = np.random.default_rng(5)
    n = 9
    edges = erdos_renyi_edges(n, 0.5, rng)
    q = oracle.maxcut_quality_loop(n, edges)  # integer qualities
    g = rng.uniform(0, math.pi, 3)
    t = rng.uniform(0, math.pi, 3)
    psi, f, _ = oracle.evolve("x", q, g, t)
    # complex conjugation: f(-gamma, -t) = f(gamma, t)
    assert abs(oracle.evolve("x", q, -g, -t)[1] - f) < 1e-12
    # exp(-i(t+pi)X) = -exp(-itX): global sign per layer
    assert abs(oracle.evolve("x", q, g, t + math.pi)[1] - f) < 1e-12
    # integer q: gamma -> gamma + 2 pi leaves U_Q unchanged
    assert abs(oracle.evolve("x", q, g + 2 * math.pi, t)[1] - f) < 1e-12
    # max-cut is invariant under flipping every bit
    prob = np.abs(psi) ** 2
    flip = np.arange(1 << n) ^ ((1 << n) - 1)
    assert np.max(np.abs(prob - prob[flip])) < 1e-15


# ---------------------------------------------------------------------- FFT
@pytest.mark.parametrize("N", [1, 2, 4, 16, 1024, 8192])
def test_fft_matches_numpy_and_identities(oracle_mod, N):
    rng = np.random.default_rng(N)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    X = oracle.fft(x, -1)
    assert np.max(np.abs(X - np.fft.fft(x))) < 1e-11 * max(1, np.sqrt(N))
    assert np.max(np.abs(oracle.fft(X, +1) / N - x)) < 1e-14 * max(1, np.log2(N))
    assert abs(np.sum(np.abs(X) ** 2) - N * np.sum(np.abs(x) ** 2)) < 1e-12 * N * np.sum(np.abs(x) ** 2)
    d = np.zeros(N, complex)
    d[0] = 1
    assert np.max(np.abs(oracle.fft(d, -1) - 1)) < 1e-15
    if N >= 4:
        m0 = 3 % N
        e = np.exp(2j * np.pi * m0 * np.arange(N) / N)
        ref = np.zeros(N, complex)
        ref[m0] = N
        assert np.max(np.abs(oracle.fft(e, -1) - ref)) < 1e-12 * N


@pytest.mark.parametrize("N", [3, 5, 12, 1000, 4097, 5000, 65537, 100003])
def test_bluestein_matches_numpy_and_dft(oracle_mod, N):
    """Chirp-z transform for any N: against numpy.fft (both signs) and, up to
    N = 5000, against the naive DFT."""
    rng = np.random.default_rng(N)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    fwd = oracle.bluestein(x, -1)
    inv = oracle.bluestein(x, +1)
    scale = np.linalg.norm(x) * math.sqrt(N)
    assert np.max(np.abs(fwd - np.fft.fft(x))) < 1e-13 * scale
    assert np.max(np.abs(inv - N * np.fft.ifft(x))) < 1e-13 * scale
    if N <= 5000:
        assert np.max(np.abs(fwd - oracle.dft(x, -1))) < 1e-13 * scale


@pytest.mark.parametrize("N", [5000, 20011])
def test_circulant_non_power_of_two(oracle_mod, N):
    """The circulant mixer at N > 4096, N not a power of two (Bluestein route):
    ring against the closed-form DFT of numpy, and the complete graph's
    spectrum against the oracle's closed form."""
    rng = np.random.default_rng(N)
    psi = _rand_state(rng, N)
    t = 0.71
    lam = oracle.ring_lambda(N)
    ref = np.fft.ifft(np.exp(-1j * t * lam) * np.fft.fft(psi))
    out = oracle.mix_circulant(psi, lam, t)
    assert np.max(np.abs(out - ref)) < 1e-13
    out_c = oracle.mix_circulant(psi, oracle.complete_lambda(N), t)
    assert np.max(np.abs(out_c - oracle.mix_complete(psi, t))) < 1e-11
    assert abs(np.linalg.norm(out) - 1) < 1e-13


@pytest.mark.parametrize("N", [3, 12, 256])
def test_naive_dft_matches_numpy(oracle_mod, N):
    rng = np.random.default_rng(N)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    assert np.max(np.abs(oracle.dft(x, -1) - np.fft.fft(x))) < 1e-12
    assert np.max(np.abs(oracle.dft(x, +1) - N * np.fft.ifft(x))) < 1e-12


def test_expectation_pairwise_exact_on_integers(oracle_mod):
    """With dyadic amplitudes and integer q every partial sum is exact."""
    N = 1 << 16
    psi = np.full(N, 1.0 / 256.0, complex)  # |psi|^2 = 2^-16
    q = np.arange(N, dtype=float)
    f, nrm = oracle.expectation(psi, q)
    assert nrm == 1.0
    assert f == (N - 1) / 2


# ---------------------------------------------------------------- gradients
@pytest.mark.parametrize("mixer,n,p", [("x", 5, 3), ("x", 7, 2), ("circulant", 5, 3),
                                       ("circulant", 6, 4)])
def test_gradient_adjoint_vs_bruteforce_vs_fd(oracle_mod, mixer, n, p):
    rng = np.random.default_rng(100 + n + p)
    N = 1 << n
    q = rng.uniform(0, 5, N)
    lam = None if mixer == "x" else random_symmetric_lambda(N, rng)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    f, dg, dt = oracle.grad(mixer, q, g, t, lam)
    bg, bt = oracle.grad_bruteforce(mixer, q, g, t, lam)
    scale = max(np.max(np.abs(dg)), np.max(np.abs(dt)))
    assert np.max(np.abs(dg - bg)) < 1e-12 * scale
    assert np.max(np.abs(dt - bt)) < 1e-12 * scale
    h = 1e-5
    for k in range(p):
        e = np.zeros(p)
        e[k] = h
        fd_g = (oracle.evolve(mixer, q, g + e, t, lam)[1] - oracle.evolve(mixer, q, g - e, t, lam)[1]) / (2 * h)
        fd_t = (oracle.evolve(mixer, q, g, t + e, lam)[1] - oracle.evolve(mixer, q, g, t - e, lam)[1]) / (2 * h)
        assert abs(fd_g - dg[k]) < 1e-7 * scale
        assert abs(fd_t - dt[k]) < 1e-7 * scale


def test_gradient_matches_dense_derivative(oracle_mod):
    """d/dt of exp(-itW) is -iW exp(-itW): compare with a dense evaluation of
    that product rule on a tiny system."""
    rng = np.random.default_rng(9)
    n = 4
    N = 1 << n
    q = rng.uniform(0, 3, N)
    W = dense.hypercube(n)
    g = rng.uniform(0, math.pi, 2)
    t = rng.uniform(0, math.pi, 2)

    def states(dpar=None):
        psi = np.full(N, N ** -0.5, complex)
        for k in range(2):
            psi = np.exp(-1j * g[k] * q) * psi
            if dpar == ("g", k):
                psi = -1j * q * psi
            psi = dense.expm_hermitian(W, t[k]) @ psi
            if dpar == ("t", k):
                psi = -1j * (W @ psi)
        return psi

    psi = states()
    _, dg, dt = oracle.grad("x", q, g, t)
    for k in range(2):
        ref_g = 2 * np.real(np.vdot(psi, q * states(("g", k))))
        ref_t = 2 * np.real(np.vdot(psi, q * states(("t", k))))
        assert abs(dg[k] - ref_g) < 1e-12
        assert abs(dt[k] - ref_t) < 1e-12


# --------------------------------------------------- the inputs module itself
@pytest.mark.parametrize("n", [3, 6, 9, 11])
def test_workload_q_matches_plain_loop(oracle_mod, n):
    rng = np.random.default_rng(n)
    edges = erdos_renyi_edges(n, 0.5, rng)
    w = rng.uniform(0, 1, len(edges))
    a = maxcut_qualities(n, edges, w)
    b = oracle.maxcut_quality_loop(n, edges, w)
    assert np.max(np.abs(a - b)) < 1e-13
    a = maxcut_qualities(n, edges, uncut=True)
    b = oracle.maxcut_quality_loop(n, edges, uncut=True)
    assert np.array_equal(a, b)


def test_constrained_workload_selects_k_subsets():
    """The constrained QWOA inputs are the full portfolio q at the indices with
    exactly k assets, in ascending order: N = C(m, k)."""
    from workloads import qwoa_constrained_workload, qwoa_portfolio_workload
    m, k = 12, 5
    full = qwoa_portfolio_workload(m, 3, seed=9)
    sub = qwoa_constrained_workload(m, k, 3, seed=9)
    idx = [j for j in range(1 << m) if bin(j).count("1") == k]
    assert sub.N == math.comb(m, k) == len(idx)
    assert np.array_equal(sub.q, full.q[idx])
    assert np.array_equal(sub.gammas, full.gammas) and np.array_equal(sub.ts, full.ts)


def test_portfolio_q_matches_plain_loop():
    rng = np.random.default_rng(0)
    m = 9
    mu = rng.normal(0.01, 0.02, m)
    g = rng.standard_normal((30, m))
    sigma = g.T @ g / 30
    q = portfolio_qualities(mu, sigma, 0.5)
    for j in [0, 1, 5, 77, 300, 511]:
        x = np.array([(j >> i) & 1 for i in range(m)], float)
        assert abs(q[j] - (mu @ x - 0.5 * x @ sigma @ x)) < 1e-13


def test_random_regular_is_regular_and_simple():
    rng = np.random.default_rng(1)
    for n in [12, 28, 30]:
        e = random_regular_edges(3, n, rng)
        assert len(e) == 3 * n // 2
        assert len(set(e)) == len(e)
        deg = np.bincount(np.array(e).ravel(), minlength=n)
        assert np.all(deg == 3)


# ------------------------------------------------------------ extended QAOA
def _maxcut_terms(n, edges, weights):
    """q_cut = sum_e w_e (1 - Z_u Z_v) / 2 = W / 2 + sum_e (-w_e / 2) Z_u Z_v."""
    S = [(1 << u) | (1 << v) for u, v in edges]
    c = [-w / 2 for w in weights]
    return S, c


def test_extended_qaoa_equal_angles_is_qaoa(oracle_mod):
    """With every term of a layer at the same angle, U_Qext(gamma) is U_Q(gamma)
    up to a global phase (eq. phase_shift_qaoa_ex vs eq. phase_shift_qaoa), so
    f matches plain QAOA, and the per-term gradients sum to dgamma_k."""
    n, p = 8, 3
    edges = circular_ladder_edges(4)
    rng = np.random.default_rng(5)
    w = rng.uniform(0.2, 1.0, len(edges))
    q = maxcut_qualities(n, edges, w)
    S, c = _maxcut_terms(n, edges, w)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    G = np.repeat(g[:, None], len(S), axis=1)
    psi_e, f_e, _ = oracle.evolve_terms(q, S, c, G, t)
    psi_q, f_q, _ = oracle.evolve("x", q, g, t)
    assert abs(f_e - f_q) < 1e-13 * abs(f_q)
    ov = np.vdot(psi_q, psi_e)
    assert abs(abs(ov) - 1) < 1e-13
    _, dG, dT = oracle.grad_terms(q, S, c, G, t)
    _, dg, dt = oracle.grad("x", q, g, t)
    assert np.max(np.abs(dG.sum(axis=1) - dg)) < 1e-12 * np.max(np.abs(dg))
    assert np.max(np.abs(dT - dt)) < 1e-12 * np.max(np.abs(dt))


def test_extended_qaoa_phase_definition(oracle_mod):
    """The per-term phase against a direct evaluation of the Z strings on
    basis states (bits read one by one), including 1- and 3-qubit strings."""
    n = 6
    N = 1 << n
    rng = np.random.default_rng(2)
    psi = _rand_state(rng, N)
    S = [0b1, 0b11, 0b101000, 0b100110, 0b111111]
    c = [0.3, -1.1, 0.25, 0.7, -0.4]
    gam = rng.uniform(-2, 2, len(S))
    out = oracle.phase_terms(psi, S, c, gam)
    ref = psi.copy()
    for j in range(N):
        ph = 0.0
        for s, ce, ge in zip(S, c, gam):
            parity = sum((j >> b) & 1 for b in range(n) if (s >> b) & 1) % 2
            ph += ge * ce * (-1 if parity else 1)
        ref[j] *= np.exp(-1j * ph)
    assert np.max(np.abs(out - ref)) < 1e-14


@pytest.mark.parametrize("n,p", [(5, 2), (7, 3)])
def test_extended_qaoa_gradient_central_differences(oracle_mod, n, p):
    """Per-term adjoint gradient against central differences of the forward,
    and against a dense evaluation of the state at small n."""
    rng = np.random.default_rng(10 + n)
    N = 1 << n
    edges = [(i, (i + 1) % n) for i in range(n)]
    S = [(1 << u) | (1 << v) for u, v in edges] + [1 << 2, 0b10011]
    c = list(rng.uniform(-1, 1, len(S)))
    q = rng.uniform(0, 4, N)
    G = rng.uniform(0, math.pi, (p, len(S)))
    t = rng.uniform(0, math.pi, p)
    f, dG, dT = oracle.grad_terms(q, S, c, G, t)
    scale = max(np.max(np.abs(dG)), np.max(np.abs(dT)))
    h = 1e-5
    for k in range(p):
        for e in range(len(S)):
            Gp = G.copy()
            Gm = G.copy()
            Gp[k, e] += h
            Gm[k, e] -= h
            fd = (oracle.evolve_terms(q, S, c, Gp, t)[1] - oracle.evolve_terms(q, S, c, Gm, t)[1]) / (2 * h)
            assert abs(fd - dG[k, e]) < 1e-7 * scale
        tp = t.copy()
        tm = t.copy()
        tp[k] += h
        tm[k] -= h
        fd = (oracle.evolve_terms(q, S, c, G, tp)[1] - oracle.evolve_terms(q, S, c, G, tm)[1]) / (2 * h)
        assert abs(fd - dT[k]) < 1e-7 * scale
    # dense: diag phases and expm of the hypercube
    W = dense.hypercube(n)
    psi = np.full(N, N ** -0.5, dtype=complex)
    for k in range(p):
        ph = np.zeros(N)
        for s, ce, ge in zip(S, c, G[k]):
            par = np.array([bin(j & s).count("1") % 2 for j in range(N)])
            ph += ge * ce * (1 - 2 * par)
        psi = dense.expm_hermitian(W, t[k]) @ (np.exp(-1j * ph) * psi)
    assert abs(np.sum(np.abs(psi) ** 2 * q) - f) < 1e-12 * abs(f)


# ------------------------------------------------------------------ QAOAz
_PX = np.array([[0, 1], [1, 0]], dtype=complex)
_PY = np.array([[0, -1j], [1j, 0]], dtype=complex)


def _pauli_on(n, ops):
    """Dense operator of a product of single-qubit Paulis; ops maps qubit ->
    2x2 matrix; qubit i is bit i of the basis index (the last Kronecker factor
    is qubit 0)."""
    out = np.array([[1.0 + 0j]])
    for i in range(n - 1, -1, -1):
        out = np.kron(out, ops.get(i, np.eye(2)))
    return out


def _xy_dense(n, a, b):
    return _pauli_on(n, {a: _PX, b: _PX}) + _pauli_on(n, {a: _PY, b: _PY})


def _parity_B_dense(n, ring):
    """B_odd, B_even, B_last of eq. parity_terms for the ring r_1..r_m, built
    from the sums as written (a 1-based, index m + 1 read cyclically as 1)."""
    m = len(ring)
    r = lambda a: ring[(a - 1) % m]  # noqa: E731
    N = 1 << n
    B_odd = np.zeros((N, N), complex)
    B_even = np.zeros((N, N), complex)
    for a in range(1, m):
        if a % 2 == 1:
            B_odd += _xy_dense(n, r(a), r(a + 1))
    for a in range(2, m + 1, 2):
        B_even += _xy_dense(n, r(a), r(a + 1))
    B_last = _xy_dense(n, r(m), r(1)) if (m % 2 == 1 and m >= 3) else np.zeros((N, N), complex)
    return B_odd, B_even, B_last


@pytest.mark.parametrize("n,ring", [(2, [0, 1]), (3, [0, 1, 2]), (4, [0, 1, 2, 3]), (5, [0, 1, 2, 3, 4]),
                                    (6, [0, 1, 2, 3, 4, 5]), (7, [0, 1, 2, 3, 4, 5, 6]),
                                    (6, [0, 2, 4]), (6, [1, 3, 5]), (7, [6, 2, 0, 4, 1])])
def test_parity_mixer_matches_dense_expm(oracle_mod, n, ring):
    """U_parity(t) = e^{-itB_last} e^{-itB_even} e^{-itB_odd} (eq. qaoaz_mixers)
    from dense Pauli sums and scipy's expm, against the oracle's ordered
    product of pair rotations over parity_ring_pairs(ring)."""
    rng = np.random.default_rng(40 + n + len(ring))
    psi = _rand_state(rng, 1 << n)
    pairs = oracle.parity_ring_pairs(ring)
    B_odd, B_even, B_last = _parity_B_dense(n, ring)
    for t in (0.37, -1.3, 2.9):
        U = (scipy.linalg.expm(-1j * t * B_last) @ scipy.linalg.expm(-1j * t * B_even)
             @ scipy.linalg.expm(-1j * t * B_odd))
        ref = U @ psi
        out = oracle.mix_xy(psi, pairs, t)
        assert np.max(np.abs(out - ref)) < 1e-13


def test_parity_pairs_cover_the_ring(oracle_mod):
    """Every ring edge appears once for m >= 3, each B's pairs are disjoint,
    and B_last exists only for odd m."""
    for m in range(3, 12):
        ring = list(range(m))
        pairs = [tuple(x) for x in oracle.parity_ring_pairs(ring)]
        edges = sorted(tuple(sorted(e)) for e in pairs)
        assert edges == sorted(tuple(sorted((i, (i + 1) % m))) for i in range(m))
        n_odd = m // 2
        n_even = m // 2 if m % 2 == 0 else (m - 1) // 2
        for chunk in (pairs[:n_odd], pairs[n_odd:n_odd + n_even]):
            qs = [q for e in chunk for q in e]
            assert len(qs) == len(set(qs))
        assert len(pairs) == n_odd + n_even + (1 if m % 2 else 0)


def test_xy_two_qubit_closed_form(oracle_mod):
    """exp(-it(XX+YY)) on two qubits: |01> -> cos 2t |01> - i sin 2t |10>,
    |00> and |11> unchanged."""
    for t in (0.1, 0.8, -2.2):
        for j, ref in [(0, [1, 0, 0, 0]), (3, [0, 0, 0, 1]),
                       (1, [0, math.cos(2 * t), -1j * math.sin(2 * t), 0]),
                       (2, [0, -1j * math.sin(2 * t), math.cos(2 * t), 0])]:
            psi = np.zeros(4, complex)
            psi[j] = 1
            out = oracle.mix_xy(psi, [(0, 1)], t)
            assert np.max(np.abs(out - np.array(ref))) < 1e-15


def test_xy_conserves_hamming_weight(oracle_mod):
    """The parity mixer keeps the probability of every Hamming weight, and the
    evolution started in one weight stays there (the constraint of Sec. 2.4.1)."""
    n = 9
    N = 1 << n
    rng = np.random.default_rng(77)
    psi = _rand_state(rng, N)
    w = np.array([bin(j).count("1") for j in range(N)])
    pairs = oracle.parity_ring_pairs(list(range(n)))
    out = oracle.mix_xy(psi, pairs, 1.234)
    for k in range(n + 1):
        assert abs(np.sum(np.abs(out[w == k]) ** 2) - np.sum(np.abs(psi[w == k]) ** 2)) < 1e-14
    dicke = (w == 4).astype(complex) / math.sqrt(math.comb(n, 4))
    q = rng.uniform(0, 2, N)
    psi_p, f, nrm = oracle.evolve_xy(q, dicke, pairs, [0.4, 1.1], [0.9, 0.3])
    assert abs(nrm - 1) < 1e-14
    assert np.max(np.abs(psi_p[w != 4])) < 1e-15


def _xy_dense_evolve(n, q, psi0, pairs, gammas, ts, insert=None):
    """Dense evolution through the factor sequence; insert = (layer, factor)
    puts -iH of that factor right after it (factor -1: the phase)."""
    psi = psi0.astype(complex).copy()
    for k, (g, t) in enumerate(zip(gammas, ts)):
        psi = np.exp(-1j * g * q) * psi
        if insert == (k, -1):
            psi = -1j * q * psi
        for i, (a, b) in enumerate(pairs):
            H = _xy_dense(n, a, b)
            psi = scipy.linalg.expm(-1j * t * H) @ psi
            if insert == (k, i):
                psi = -1j * (H @ psi)
    return psi


@pytest.mark.parametrize("n,ring,p", [(4, [0, 1, 2, 3], 2), (5, [0, 1, 2, 3, 4], 3), (6, [0, 2, 4], 2)])
def test_xy_evolution_and_gradient_dense(oracle_mod, n, ring, p):
    """evolve_xy against a dense evolution, and grad_xy against the dense
    product rule (-iH inserted after each factor in turn) and central
    differences of the oracle's own forward."""
    rng = np.random.default_rng(90 + n + p)
    N = 1 << n
    q = rng.uniform(-1, 2, N)
    psi0 = _rand_state(rng, N)
    pairs = oracle.parity_ring_pairs(ring)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    psi_p, f, _ = oracle.evolve_xy(q, psi0, pairs, g, t)
    ref = _xy_dense_evolve(n, q, psi0, pairs, g, t)
    assert np.max(np.abs(psi_p - ref)) < 1e-13
    f_a, dg, dt = oracle.grad_xy(q, psi0, pairs, g, t)
    assert abs(f_a - f) < 1e-14
    for k in range(p):
        d = _xy_dense_evolve(n, q, psi0, pairs, g, t, insert=(k, -1))
        assert abs(2 * np.real(np.vdot(ref, q * d)) - dg[k]) < 1e-12
        s = 0.0
        for i in range(len(pairs)):
            d = _xy_dense_evolve(n, q, psi0, pairs, g, t, insert=(k, i))
            s += 2 * np.real(np.vdot(ref, q * d))
        assert abs(s - dt[k]) < 1e-12
    h = 1e-5
    scale = max(np.max(np.abs(dg)), np.max(np.abs(dt)))
    for k in range(p):
        for arr, grad_ in ((g, dg), (t, dt)):
            xp = arr.copy()
            xm = arr.copy()
            xp[k] += h
            xm[k] -= h
            if arr is g:
                fp = oracle.evolve_xy(q, psi0, pairs, xp, t)[1]
                fm = oracle.evolve_xy(q, psi0, pairs, xm, t)[1]
            else:
                fp = oracle.evolve_xy(q, psi0, pairs, g, xp)[1]
                fm = oracle.evolve_xy(q, psi0, pairs, g, xm)[1]
            assert abs((fp - fm) / (2 * h) - grad_[k]) < 1e-8 * scale


@pytest.mark.parametrize("N,kind", [(1000, "ring"), (5003, "ring"), (6000, "array"), (4099, "array")])
def test_circulant_gradient_any_n(oracle_mod, N, kind):
    """The adjoint through a circulant over N that is not a power of two (the
    naive DFT at N <= 4096, Bluestein above): against the brute-force product
    rule and central differences of the forward."""
    rng = np.random.default_rng(N + 3)
    p = 2
    q = rng.uniform(-1, 3, N)
    lam = oracle.lambda_for("ring", N) if kind == "ring" else rng.uniform(-2, 2, N)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    f, dg, dt = oracle.grad("circulant", q, g, t, lam)
    bg, bt = oracle.grad_bruteforce("circulant", q, g, t, lam)
    scale = max(np.max(np.abs(dg)), np.max(np.abs(dt)))
    assert np.max(np.abs(dg - bg)) < 1e-11 * scale
    assert np.max(np.abs(dt - bt)) < 1e-11 * scale
    h = 1e-5
    for k in range(p):
        e = np.zeros(p)
        e[k] = h
        fd_g = (oracle.evolve("circulant", q, g + e, t, lam)[1] - oracle.evolve("circulant", q, g - e, t, lam)[1]) / (2 * h)
        fd_t = (oracle.evolve("circulant", q, g, t + e, lam)[1] - oracle.evolve("circulant", q, g, t - e, lam)[1]) / (2 * h)
        assert abs(fd_g - dg[k]) < 1e-7 * scale
        assert abs(fd_t - dt[k]) < 1e-7 * scale
