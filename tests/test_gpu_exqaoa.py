"""GPU parity: extended QAOA (one phase angle per Z-string term, eqs.
phase_shift_qaoa_ex and qaoa_ex) vs the CPU oracle.

Bar: f to 1e-12 relative, the final state to 1e-11 of its largest amplitude,
the adjoint gradient (p x terms angles and p mixer times) to 1e-10 of its
largest entry, all against oracle.evolve_terms / oracle.grad_terms (pinned on
the CPU against plain QAOA at equal angles, direct term evaluation, dense
states and central differences).  At the full n = 28 size, where the oracle
is too slow, the property that holds at any size: with every term of a layer
at the same angle the phase is the QAOA phase up to a global factor, so f
equals the QAOA path's f and the per-term gradients of a layer sum to its
QAOA dgamma.
"""

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from gpu_util import to_dev  # noqa: E402
from workloads import erdos_renyi_edges, exqaoa_maxcut_workload, maxcut_qualities  # noqa: E402

pytestmark = pytest.mark.gpu
qva = pytest.importorskip("paper_2110_03963_amd")

F_TOL = 1e-12
PSI_TOL = 1e-11
G_TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qva.load_library()


def _instance(n, p, seed, extra=True):
    """MaxCut on G(n, 0.3) split into one Z_u Z_v term per edge, plus (with
    extra) strings of 1, 3 and n qubits, the identity, and a support with bits
    above n; angles U(0, pi) per term and layer."""
    rng = np.random.default_rng(seed)
    edges = erdos_renyi_edges(n, 0.3, rng) if n >= 3 else [(0, 1)]
    w = rng.uniform(0.1, 1.0, len(edges))
    q = maxcut_qualities(n, edges, w)
    S = [(1 << u) | (1 << v) for u, v in edges]
    c = list(-0.5 * w)
    if extra:
        S += [1, 0b10110 & ((1 << n) - 1) or 1, (1 << n) - 1, 0, (1 << n) | 1]
        c += list(rng.uniform(-1, 1, 5))
    S = np.array(S, dtype=np.uint64)
    c = np.array(c)
    G = rng.uniform(0, math.pi, (p, len(S)))
    t = rng.uniform(0, math.pi, p)
    return q, S, c, G, t


def _problem(q, S, c):
    return qva.Problem(to_dev(q), "x", terms=(S, c))


@pytest.mark.parametrize("n,p", [(2, 1), (6, 2), (12, 3), (13, 1), (13, 3), (15, 2), (18, 2),
                                 (21, 3), (23, 2)])
def test_exqaoa_forward_parity(n, p):
    q, S, c, G, t = _instance(n, p, 100 + n)
    print(f"exqaoa forward n={n} p={p} terms={len(S)}", flush=True)
    prob = _problem(q, S, c)
    f, nrm, psi = qva.evolve(prob, G, t)
    psi_ref, f_ref, nrm_ref = oracle.evolve_terms(q, S, c, G, t)
    assert abs(f.item() - f_ref) <= F_TOL * abs(f_ref)
    assert abs(nrm.item() - 1.0) < 1e-12
    d = np.max(np.abs(psi.cpu().numpy() - psi_ref))
    assert d <= PSI_TOL * np.max(np.abs(psi_ref)), d


@pytest.mark.parametrize("n,p", [(3, 2), (8, 3), (12, 2), (13, 2), (14, 3), (17, 2), (20, 3),
                                 (22, 2)])
def test_exqaoa_grad_parity(n, p):
    q, S, c, G, t = _instance(n, p, 200 + n)
    print(f"exqaoa grad n={n} p={p} terms={len(S)}", flush=True)
    prob = _problem(q, S, c)
    f, dG, dt = qva.grad(prob, G, t)
    f_ref, rG, rt = oracle.grad_terms(q, S, c, G, t)
    assert abs(f.item() - f_ref) <= F_TOL * abs(f_ref)
    assert tuple(dG.shape) == (p, len(S))
    g = np.concatenate([dG.cpu().numpy().ravel(), dt.cpu().numpy()])
    r = np.concatenate([rG.ravel(), rt])
    err = float(np.max(np.abs(g - r)) / np.max(np.abs(r)))
    assert err < G_TOL, err


@pytest.mark.parametrize("n,E", [(13, 1), (14, 1024), (9, 1024)])
def test_exqaoa_term_counts(n, E):
    """One term and the maximum QVA_MAX_TERMS terms (random supports over all
    n qubits, repeats allowed)."""
    rng = np.random.default_rng(300 + E + n)
    p = 2
    q = rng.uniform(0, 3, 1 << n)
    S = rng.integers(0, 1 << n, E, dtype=np.uint64)
    c = rng.uniform(-1, 1, E) / math.sqrt(E)
    G = rng.uniform(0, math.pi, (p, E))
    t = rng.uniform(0, math.pi, p)
    print(f"exqaoa terms n={n} E={E}", flush=True)
    prob = _problem(q, S, c)
    f, dG, dt = qva.grad(prob, G, t)
    f_ref, rG, rt = oracle.grad_terms(q, S, c, G, t)
    assert abs(f.item() - f_ref) <= F_TOL * max(abs(f_ref), np.mean(q))
    g = np.concatenate([dG.cpu().numpy().ravel(), dt.cpu().numpy()])
    r = np.concatenate([rG.ravel(), rt])
    assert float(np.max(np.abs(g - r)) / np.max(np.abs(r))) < G_TOL
    fe, _, _ = qva.evolve(prob, G, t, store=False)
    assert abs(fe.item() - f_ref) <= F_TOL * max(abs(f_ref), np.mean(q))


def test_exqaoa_depth_zero_and_rejects():
    q, S, c, G, t = _instance(14, 1, 7)
    prob = _problem(q, S, c)
    f, _, _ = qva.evolve(prob, np.zeros((0, len(S))), [])
    assert abs(f.item() - np.mean(q)) <= 1e-13 * np.mean(q)
    with pytest.raises(ValueError):
        qva.evolve(prob, G[:, :-1], t)  # one angle short per layer
    circ = qva.Problem(to_dev(q), "circulant", lambda_kind="ring", terms=(S, c))
    with pytest.raises(RuntimeError):
        qva.evolve(circ, G, t)


def test_exqaoa_autograd():
    q, S, c, G, t = _instance(13, 2, 9)
    prob = _problem(q, S, c)
    g = torch.tensor(G, dtype=torch.float64, device="cuda", requires_grad=True)
    tt = torch.tensor(t, dtype=torch.float64, device="cuda", requires_grad=True)
    f = qva.expectation_value(prob, g, tt)
    (3.0 * f).backward()
    _, rG, rt = oracle.grad_terms(q, S, c, G, t)
    scale = max(np.max(np.abs(rG)), np.max(np.abs(rt)))
    assert g.grad.shape == g.shape
    assert np.max(np.abs(g.grad.cpu().numpy() - 3 * rG)) < 3 * G_TOL * scale
    assert np.max(np.abs(tt.grad.cpu().numpy() - 3 * rt)) < 3 * G_TOL * scale


@pytest.mark.parametrize("n,p", [(28, 3)])
def test_exqaoa_full_size_equal_angles(n, p):
    """The extended-QAOA MaxCut workload at n = 28 (3-regular, 42 edges):
    with each layer's terms at the QAOA angle gamma_k, f equals the QAOA f and
    the per-term gradients of a layer sum to the QAOA dgamma_k."""
    wl = exqaoa_maxcut_workload(n, p, seed=11)
    E = len(wl.supports)
    g_qaoa = wl.gammas.mean(axis=1)
    G = np.repeat(g_qaoa[:, None], E, axis=1)
    print(f"exqaoa full size n={n} p={p} terms={E}", flush=True)
    qd = to_dev(wl.q)
    pz = qva.Problem(qd, "x", terms=(wl.supports, wl.coefs))
    px = qva.Problem(qd, "x")
    fz, dGz, dtz = qva.grad(pz, G, wl.ts)
    fx, dgx, dtx = qva.grad(px, g_qaoa, wl.ts)
    assert abs(fz.item() - fx.item()) <= F_TOL * abs(fx.item())
    sums = dGz.sum(dim=1).cpu().numpy()
    scale = max(np.max(np.abs(dgx.cpu().numpy())), np.max(np.abs(dtx.cpu().numpy())))
    assert np.max(np.abs(sums - dgx.cpu().numpy())) < G_TOL * scale
    assert np.max(np.abs(dtz.cpu().numpy() - dtx.cpu().numpy())) < G_TOL * scale
    fe, _, _ = qva.evolve(pz, G, wl.ts, store=False)
    assert abs(fe.item() - fx.item()) <= F_TOL * abs(fx.item())
    del pz, px, qd
    torch.cuda.empty_cache()
