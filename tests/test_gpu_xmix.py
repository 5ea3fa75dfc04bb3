"""GPU parity: hypercube-mixer path of libqva vs the CPU oracle.

Every comparison uses the same seeded inputs on both sides.  Tolerances:
<Q> to 1e-12 relative (|f - f_ref| / sum |psi|^2 |q|), states to 1e-12 in
2-norm (unit-norm states, ~1e-15 per operation over a few hundred
operations), sums of probabilities to 1e-13.
"""

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from gpu_util import f_rel_err, rand_state, state_err, to_dev  # noqa: E402
from workloads import (CONFIG_SEEDS, erdos_renyi_edges, maxcut_qualities,  # noqa: E402
                       qaoa_maxcut_workload, ring_edges)

pytestmark = pytest.mark.gpu

qva = pytest.importorskip("paper_2110_03963_amd")

F_TOL = 1e-12
PSI_TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qva.load_library()


@pytest.mark.parametrize("N", [1, 3, 1000, 4096, 70000])
def test_init_uniform(N):
    psi = torch.empty(N, dtype=torch.complex128, device="cuda")
    qva.init_uniform(psi)
    ref = oracle.init_uniform(N)
    assert np.array_equal(psi.cpu().numpy(), ref)


@pytest.mark.parametrize("N", [1, 7, 4096, 100001])
def test_phase(N):
    rng = np.random.default_rng(N)
    psi0 = rand_state(rng, N)
    q = rng.uniform(-20, 40, N)
    for gamma in [0.0, 0.77, -2.5]:
        psi = to_dev(psi0)
        qva.phase(psi, to_dev(q), gamma)
        ref = oracle.phase(psi0, q, gamma)
        assert np.max(np.abs(psi.cpu().numpy() - ref)) < 1e-15


@pytest.mark.parametrize("span", [4.0, 1e3, 1e7, 1e12])
def test_phase_factor_accuracy(span):
    """The phase factor exp(-i x) itself: psi = 1, gamma = 1, q = x spread over
    [-span, span] plus points next to multiples of pi/2; compared with the
    oracle's libm cexp, as complex numbers, to 1.6e-16 absolute."""
    rng = np.random.default_rng(int(np.log10(span)) + 11)
    x = rng.uniform(-span, span, 1 << 18)
    k = rng.integers(-10**6, 10**6, 1 << 12)
    near = np.nextafter(k * (np.pi / 2), np.where(rng.random(k.size) < 0.5, -np.inf, np.inf))
    x = np.concatenate([x, near, [0.0, -0.0, 1e-300, np.pi, -np.pi / 2]])
    ones = np.ones(x.size, dtype=np.complex128)
    psi = to_dev(ones)
    qva.phase(psi, to_dev(x), 1.0)
    ref = oracle.phase(ones, x, 1.0)
    assert np.max(np.abs(psi.cpu().numpy() - ref)) <= 1.6e-16


@pytest.mark.parametrize("n", [1, 2, 3, 6, 11, 12, 13, 14, 15, 17, 20, 21, 22])
def test_mix_x(n):
    rng = np.random.default_rng(n)
    psi0 = rand_state(rng, 1 << n)
    for t in [0.3, 2.2, -0.9, math.pi / 2, math.pi / 4, 0.0]:
        psi = to_dev(psi0)
        qva.mix_x(psi, t)
        ref = oracle.mix_x(psi0, t)
        assert state_err(psi.cpu().numpy(), ref) < PSI_TOL, (n, t)


@pytest.mark.parametrize("N", [1, 5, 4096, 4097, 1 << 20, 3 * 10**6])
def test_expectation(N):
    rng = np.random.default_rng(N)
    psi0 = rand_state(rng, N)
    q = rng.uniform(-1, 5, N)
    f, nrm = qva.expectation(to_dev(psi0), to_dev(q))
    f_ref, n_ref = oracle.expectation(psi0, q)
    assert f_rel_err(f.item(), f_ref, psi0, q) < F_TOL
    assert abs(nrm.item() - n_ref) < 1e-13


def _check_evolve(q, gammas, ts, store=True):
    prob = qva.Problem(to_dev(q), "x")
    f, nrm, psi = qva.evolve(prob, gammas, ts, store=store)
    psi_ref, f_ref, n_ref = oracle.evolve("x", q, gammas, ts)
    assert f_rel_err(f.item(), f_ref, psi_ref, q) < F_TOL
    assert abs(nrm.item() - n_ref) < 1e-13
    if store:
        assert state_err(psi.cpu().numpy(), psi_ref) < PSI_TOL
    return f.item(), f_ref


@pytest.mark.parametrize("n,p", [(1, 1), (2, 3), (5, 2), (10, 2), (12, 4), (13, 1), (13, 2),
                                 (14, 3), (16, 5), (20, 2), (21, 3), (22, 1), (22, 4), (24, 2)])
def test_evolve_random_q(n, p):
    rng = np.random.default_rng(1000 + 10 * n + p)
    q = rng.uniform(0, 10, 1 << n)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    _check_evolve(q, g, t)


def test_evolve_qaoa_n10_config():
    """QAOA MaxCut, n = 10, G(10, 0.5) unweighted, cut quality, p = 2."""
    wl = qaoa_maxcut_workload(10, 2, graph="gnp", weighted=False, edge_prob=0.5,
                              seed=CONFIG_SEEDS["qaoa_n10"])
    _check_evolve(wl.q, wl.gammas, wl.ts)


@pytest.mark.parametrize("n", [8, 14, 22])
def test_evolve_edge_angles(n):
    rng = np.random.default_rng(n)
    edges = erdos_renyi_edges(n, 0.4, rng)
    q = maxcut_qualities(n, edges, rng.uniform(0, 1, len(edges)))
    p = 3
    cases = [
        (np.zeros(p), rng.uniform(0, 3, p)),              # all gamma = 0
        (rng.uniform(0, 3, p), np.zeros(p)),              # all t = 0
        (rng.uniform(-3, 0, p), rng.uniform(-3, 0, p)),   # negative angles
        (np.full(p, 0.5), np.full(p, math.pi / 2)),        # cos t = 0 (pure swap)
        (np.full(p, 0.5), np.full(p, math.pi / 4)),        # |cos t| = |sin t|
        (np.full(p, 7.0), np.full(p, 11.0)),              # large angles
    ]
    for g, t in cases:
        _check_evolve(q, g, t)


@pytest.mark.parametrize("n", [3, 12, 15])
def test_evolve_depth_zero(n):
    rng = np.random.default_rng(n)
    q = rng.uniform(-2, 2, 1 << n)
    f, _ = _check_evolve(q, [], [])
    assert abs(f - np.mean(q)) < 1e-13 * np.mean(np.abs(q))


@pytest.mark.parametrize("n", [11, 16])
def test_evolve_skip_final_state(n):
    rng = np.random.default_rng(n)
    q = rng.uniform(0, 3, 1 << n)
    _check_evolve(q, [0.3, 0.5], [0.7, 1.9], store=False)


def test_evolve_repeat_is_deterministic():
    rng = np.random.default_rng(5)
    n = 18
    q = rng.uniform(0, 3, 1 << n)
    prob = qva.Problem(to_dev(q), "x")
    vals = [qva.evolve(prob, [0.3, 1.1], [0.2, 2.0])[0].item() for _ in range(3)]
    assert vals[0] == vals[1] == vals[2]


def test_ring_light_cone_max_size():
    """The largest register, n = 33 (QVA_MAX_QUBITS: 128 GiB of amplitudes,
    64 GiB of q), unweighted ring, p = 2: f/n equals the oracle's f/n at n = 6
    (light cone of radius p)."""
    from workloads import ring_cut_qualities_device

    p = 2
    rng = np.random.default_rng(33)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    n_small = 2 * p + 2
    f_small = oracle.evolve("x", oracle.maxcut_quality_loop(n_small, ring_edges(n_small)), g, t)[1]
    n = 33
    print("max size n=33", flush=True)
    q = ring_cut_qualities_device(n, "cuda")
    prob = qva.Problem(q, "x")
    psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    f, nrm, _ = qva.evolve(prob, g, t, psi=psi, store=False)
    assert abs(f.item() / n - f_small / n_small) < 1e-12 * (f_small / n_small)
    assert abs(nrm.item() - 1) < 1e-12
    del prob, q, psi
    torch.cuda.empty_cache()


def test_ring_light_cone_full_size():
    """Unweighted ring at n = 28, p = 3: f/n equals the oracle's f/n at n = 8
    (light cone of radius p; any n >= 2p + 2)."""
    p = 3
    rng = np.random.default_rng(11)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    n_small = 2 * p + 2
    f_small = oracle.evolve("x", oracle.maxcut_quality_loop(n_small, ring_edges(n_small)), g, t)[1]
    n = 28
    q = maxcut_qualities(n, ring_edges(n))
    prob = qva.Problem(to_dev(q), "x")
    f, nrm, _ = qva.evolve(prob, g, t, store=False)
    assert abs(f.item() / n - f_small / n_small) < 1e-12 * (f_small / n_small)
    assert abs(nrm.item() - 1) < 1e-12
