"""GPU parity: circulant-mixer (QWOA) path of libqva vs the CPU oracle.

The oracle applies F^-1 diag(exp(-i t lambda)) F with its own naive DFT
(N <= 4096) or radix-2 FFT; the GPU uses the in-place mixed-radix group
passes.  Tolerances as for the hypercube path: states to 1e-12 in 2-norm,
<Q> to 1e-12 relative.  Full-size pins (N = 2^26) use closed forms: the ring
walk from a delta (Bessel functions) and the complete graph.
"""

import math

import numpy as np
import pytest
import scipy.special

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from gpu_util import f_rel_err, rand_state, state_err, to_dev  # noqa: E402
from workloads import (CONFIG_SEEDS, qwoa_portfolio_workload,  # noqa: E402
                       random_symmetric_lambda)

pytestmark = pytest.mark.gpu
qva = pytest.importorskip("paper_2110_03963_amd")

F_TOL = 1e-12
PSI_TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qva.load_library()


def _lam(kind, N, rng):
    if kind == "ring":
        return oracle.ring_lambda(N)
    if kind == "complete":
        return oracle.complete_lambda(N)
    if kind == "array":
        return random_symmetric_lambda(N, rng)
    return rng.uniform(-3, 3, N)  # "array-asym": any real spectrum (Hermitian circulant)


@pytest.mark.parametrize("n", [1, 2, 5, 10, 12, 13, 15, 17, 20, 21, 22, 23])
@pytest.mark.parametrize("kind", ["ring", "complete", "array", "array-asym"])
def test_mix_circulant(n, kind):
    rng = np.random.default_rng(100 * n + len(kind))
    N = 1 << n
    psi0 = rand_state(rng, N)
    lam = _lam(kind, N, rng)
    api_kind = "array" if kind.startswith("array") else kind
    for t in [0.37, -2.1]:
        psi = to_dev(psi0)
        qva.mix_circulant(psi, t, to_dev(lam) if api_kind == "array" else None, api_kind)
        ref = oracle.mix_complete(psi0, t) if kind == "complete" else oracle.mix_circulant(psi0, lam, t)
        assert state_err(psi.cpu().numpy(), ref) < PSI_TOL, (n, kind, t)


def _check_evolve(q, gammas, ts, kind, lam, store=True):
    prob = qva.Problem(to_dev(q), "circulant", to_dev(lam) if kind == "array" else None, kind)
    f, nrm, psi = qva.evolve(prob, gammas, ts, store=store)
    if kind == "complete":  # the oracle's closed form (definition of the mixer)
        psi_ref, f_ref, n_ref = oracle.evolve("complete", q, gammas, ts)
    else:
        psi_ref, f_ref, n_ref = oracle.evolve("circulant", q, gammas, ts, lam)
    assert f_rel_err(f.item(), f_ref, psi_ref, q) < F_TOL
    assert abs(nrm.item() - n_ref) < 1e-13
    if store:
        assert state_err(psi.cpu().numpy(), psi_ref) < PSI_TOL
    return f.item(), f_ref


@pytest.mark.parametrize("n,p", [(1, 2), (4, 3), (10, 2), (12, 3), (13, 1), (14, 2), (17, 3),
                                 (21, 2), (22, 2), (24, 1)])
@pytest.mark.parametrize("kind", ["ring", "complete", "array"])
def test_evolve_circulant(n, p, kind):
    rng = np.random.default_rng(7 * n + p)
    N = 1 << n
    q = rng.uniform(-1, 3, N)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    _check_evolve(q, g, t, kind, _lam(kind, N, rng))


@pytest.mark.parametrize("n", [8, 16])
def test_evolve_circulant_depth_zero_and_skip_state(n):
    rng = np.random.default_rng(n)
    N = 1 << n
    q = rng.uniform(-1, 1, N)
    f, _ = _check_evolve(q, [], [], "ring", oracle.ring_lambda(N))
    assert abs(f - q.mean()) < 1e-13
    _check_evolve(q, [0.4, 1.2], [2.0, 0.3], "array", random_symmetric_lambda(N, rng), store=False)


def test_qwoa_portfolio_reduced():
    """The QWOA portfolio workload (mean-variance cost, ring mixer) at m = 16."""
    wl = qwoa_portfolio_workload(16, 6, seed=CONFIG_SEEDS["qwoa_n26"], lambda_kind="ring")
    _check_evolve(wl.q, wl.gammas, wl.ts, "ring", oracle.ring_lambda(wl.N))


@pytest.mark.parametrize("n,t", [(26, 0.9), (26, 3.0), (18, 2.2)])
def test_ring_delta_bessel_full_size(n, t):
    """Ring walk from site 0 at N = 2^26: amplitude (-i)^|d| J_|d|(2t) at
    distance d (only |d| <= 60 matters; the rest is below 1e-30)."""
    N = 1 << n
    psi = torch.zeros(N, dtype=torch.complex128, device="cuda")
    psi[0] = 1.0
    qva.mix_circulant(psi, t, None, "ring")
    d = np.arange(0, 61)
    amp = (-1j) ** d * scipy.special.jv(d, 2 * t)
    out = psi.cpu().numpy()
    assert np.max(np.abs(out[:61] - amp)) < 1e-13
    assert np.max(np.abs(out[N - 60:][::-1] - amp[1:])) < 1e-13
    rest = out[61:N - 60]
    assert np.max(np.abs(rest)) < 1e-13
    assert abs(np.sum(np.abs(out) ** 2) - 1) < 1e-12


@pytest.mark.parametrize("n,p", [(13, 1), (13, 4), (15, 2), (16, 5), (19, 3)])
def test_evolve_complete_closed_form(n, p):
    """qva_evolve with the complete graph runs the closed-form passes for
    n > 12: against the oracle (transform-based) with and without the final
    state, and the same spectrum as an array (transform passes) agrees."""
    rng = np.random.default_rng(31 * n + p)
    N = 1 << n
    q = rng.uniform(-2, 5, N)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    lam = oracle.complete_lambda(N)
    f1, f_ref = _check_evolve(q, g, t, "complete", lam, store=True)
    f2, _ = _check_evolve(q, g, t, "complete", lam, store=False)
    assert f1 == f2
    # the spectrum as an array: transform passes, against the oracle's transform route
    prob_a = qva.Problem(to_dev(q), "circulant", to_dev(lam), "array")
    f_a, _, _ = qva.evolve(prob_a, g, t, store=False)
    f_tr = oracle.evolve("circulant", q, g, t, lam)[1]
    assert abs(f_a.item() - f_tr) <= F_TOL * np.mean(np.abs(q))


@pytest.mark.parametrize("N", [2, 3, 5, 1000, 4095, 4097, 100003, 3000017])
@pytest.mark.parametrize("p", [0, 1, 3])
def test_evolve_complete_any_n(N, p):
    """Complete graph on N solutions, N not a power of two (a constrained
    problem's |S'|): closed-form passes with a partial last block, against the
    oracle's closed form; state, f and norm."""
    rng = np.random.default_rng(N + 7 * p)
    q = rng.uniform(-1, 4, N)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    prob = qva.Problem(to_dev(q), "circulant", None, "complete")
    assert prob.N == N
    f, nrm, psi = qva.evolve(prob, g, t, store=True)
    psi_ref, f_ref, n_ref = oracle.evolve("complete", q, g, t)
    assert psi.numel() == N
    assert f_rel_err(f.item(), f_ref, psi_ref, q) < F_TOL
    assert abs(nrm.item() - n_ref) < 1e-13
    assert state_err(psi.cpu().numpy(), psi_ref) < PSI_TOL
    f2, _, _ = qva.evolve(prob, g, t, store=False)
    assert f2.item() == f.item()


def test_non_power_of_two_needs_circulant():
    with pytest.raises(ValueError):
        qva.Problem(to_dev(np.ones(1000)), "x")


@pytest.mark.parametrize("N", [5, 1000, 4097, 12289, 100003, 1000003])
@pytest.mark.parametrize("kind", ["ring", "array"])
@pytest.mark.parametrize("p", [1, 3])
def test_evolve_bluestein(N, kind, p):
    """Ring or eigenvalue-array circulant over N solutions, N not a power of
    two (Bluestein's chirp-z transform over a padded power of two), against
    the oracle (naive DFT up to 4096, its own chirp-z transform above)."""
    rng = np.random.default_rng(N + p + len(kind))
    q = rng.uniform(-1, 3, N)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    lam = oracle.ring_lambda(N) if kind == "ring" else random_symmetric_lambda(N, rng)
    prob = qva.Problem(to_dev(q), "circulant", to_dev(lam) if kind == "array" else None, kind)
    f, nrm, psi = qva.evolve(prob, g, t, store=True)
    psi_ref, f_ref, n_ref = oracle.evolve("circulant", q, g, t, lam)
    assert f_rel_err(f.item(), f_ref, psi_ref, q) < F_TOL
    assert abs(nrm.item() - n_ref) < 1e-12
    assert state_err(psi.cpu().numpy(), psi_ref) < PSI_TOL
    f2, _, _ = qva.evolve(prob, g, t, store=False)
    assert f2.item() == f.item()


@pytest.mark.parametrize("N", [5, 1009, 4097, 6000, 12289, 100003, 1000003])
@pytest.mark.parametrize("kind", ["ring", "array", "array-asym", "complete"])
def test_mix_circulant_any_n(N, kind):
    """qva_mix_circulant alone over N solutions, N not a power of two: the
    ring and eigenvalue arrays through Bluestein's transform where N has a
    prime factor above 31 (mixed radix otherwise), the complete graph in
    closed form for every N; against the oracle's mixer (naive DFT up to
    4096, its own chirp-z transform above) or its closed form, then -t
    restores the state."""
    rng = np.random.default_rng(3 * N + len(kind))
    psi0 = rand_state(rng, N)
    lam = _lam(kind, N, rng)
    api_kind = "array" if kind.startswith("array") else kind
    lam_dev = to_dev(lam) if api_kind == "array" else None
    t = float(rng.uniform(0.2, 3.0))
    print(f"mix_circulant any N: N={N} {kind} t={t}", flush=True)
    psi = to_dev(psi0)
    qva.mix_circulant(psi, t, lam_dev, api_kind)
    ref = oracle.mix_complete(psi0, t) if kind == "complete" else oracle.mix_circulant(psi0, lam, t)
    assert state_err(psi.cpu().numpy(), ref) < PSI_TOL
    qva.mix_circulant(psi, -t, lam_dev, api_kind)
    assert state_err(psi.cpu().numpy(), psi0) < PSI_TOL


@pytest.mark.parametrize("n", [13, 17])
def test_evolve_complete_degenerate_angles(n):
    """t = 0 and t N a multiple of 2 pi (c = 0) leave only global phases: f
    equals the value of the phases alone, i.e. mean(q); gamma = 0 everywhere
    keeps the uniform state, f = mean(q)."""
    rng = np.random.default_rng(n)
    N = 1 << n
    q = rng.uniform(0, 3, N)
    lam = oracle.complete_lambda(N)
    for g, t in [([0.4, 1.3], [0.0, 0.0]), ([0.9, 0.2, 2.0], [2 * math.pi / N, 0.0, 4 * math.pi / N]),
                 ([0.0, 0.0], [0.7, 2.2])]:
        f, f_ref = _check_evolve(q, np.array(g), np.array(t), "complete", lam)
        assert abs(f - q.mean()) < 1e-12 * abs(q.mean())


def test_complete_graph_closed_form_full_size():
    """exp(-i t (J - I)) psi = e^{it} (psi + (e^{-itN} - 1)/N sum(psi)) at N = 2^26."""
    n = 26
    N = 1 << n
    rng = np.random.default_rng(3)
    psi0 = rand_state(rng, N)
    t = 0.61
    psi = to_dev(psi0)
    qva.mix_circulant(psi, t, None, "complete")
    ref = np.exp(1j * t) * (psi0 + (np.exp(-1j * t * N) - 1) / N * psi0.sum())
    assert state_err(psi.cpu().numpy(), ref) < 1e-11
