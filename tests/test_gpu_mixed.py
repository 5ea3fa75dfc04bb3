"""GPU parity: circulant mixers over N solutions with small prime factors
(N not a power of two, every prime factor <= 31), through the in-place
mixed-radix passes, against the CPU oracle (naive DFT for N <= 4096, its own
chirp-z transform above: an independent route).

Tolerances as for the other circulant tests: f 1e-12 relative
(|f - f_ref| / sum |psi|^2 |q|), states 1e-12 in 2-norm, gradients 1e-10
relative in the max norm.  Full-size values come from the oracle through
tests/golden/gen_full_size.py.
"""

import json
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from gpu_util import f_rel_err, rand_state, state_err, to_dev  # noqa: E402
from workloads import CONFIG_SEEDS, qwoa_constrained_workload, random_symmetric_lambda  # noqa: E402

pytestmark = pytest.mark.gpu

qva = pytest.importorskip("paper_2110_03963_amd")
_lib = qva._lib

F_TOL = 1e-12
PSI_TOL = 1e-12
G_TOL = 1e-10
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "full_size_values.json")
GOLDEN_AMP = os.path.join(os.path.dirname(__file__), "golden", "full_size_amplitudes.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qva.load_library()


def _plan_kinds(prob, p, grad=False):
    import ctypes

    lib = _lib.load()
    cnt = lib.qva_plan(prob.cstruct(), p, int(grad), 0, None, 0)
    arr = (_lib.QvaPassInfo * cnt)()
    lib.qva_plan(prob.cstruct(), p, int(grad), 0, arr, cnt)
    return [a.kind for a in arr], [(a.group_first, a.group_bits, a.col_bits) for a in arr]


def _inputs(N, p, kind, seed):
    rng = np.random.default_rng(seed)
    q = rng.uniform(-1, 3, N)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    lam = oracle.ring_lambda(N) if kind == "ring" else random_symmetric_lambda(N, rng)
    return q, g, t, lam


# one group (N <= 4096, one workgroup), two and three groups; radices up to
# 16 and the prime radices 17..31 (C(20, 10) = 2^2 11 13 17 19,
# C(24, 12) = 2^2 7 13 17 19 23); ragged tiles (columns that do not fill one);
# low groups whose last stage is a power of two after larger odd radices
# (8 19 23 7 = 24472, 29 31 512 = 460288), which run with padded LDS slots
SIZES = [6, 30, 1000, 3 * 7 * 11 * 13, 6000, 3 * 2 ** 16, 24472, 243000, 184756, 29 * 31 * 512, 2704156]


@pytest.mark.parametrize("N", SIZES)
@pytest.mark.parametrize("kind", ["ring", "array"])
@pytest.mark.parametrize("p", [1, 3])
def test_evolve_mixed_radix(N, kind, p):
    q, g, t, lam = _inputs(N, p, kind, N + 11 * p + len(kind))
    print(f"mixed evolve N={N} p={p} {kind}", flush=True)
    prob = qva.Problem(to_dev(q), "circulant", to_dev(lam) if kind == "array" else None, kind)
    kinds, _ = _plan_kinds(prob, p)
    assert 52 in kinds and not any(34 <= k <= 41 for k in kinds), kinds  # mixed radix, no Bluestein
    f, nrm, psi = qva.evolve(prob, g, t, store=True)
    psi_ref, f_ref, n_ref = oracle.evolve("circulant", q, g, t, lam)
    assert f_rel_err(f.item(), f_ref, psi_ref, q) < F_TOL
    assert abs(nrm.item() - n_ref) < 1e-12
    assert state_err(psi.cpu().numpy(), psi_ref) < PSI_TOL
    f2, _, _ = qva.evolve(prob, g, t, store=False)
    assert f2.item() == f.item()


@pytest.mark.parametrize("N,kind", [(30, "ring"), (1000, "array"), (6000, "ring"), (3 * 2 ** 16, "array"),
                                    (24472, "array"), (243000, "ring"), (184756, "array"),
                                    (29 * 31 * 512, "ring"), (2704156, "ring")])
def test_grad_mixed_radix(N, kind):
    p = 3
    q, g, t, lam = _inputs(N, p, kind, 3 * N + len(kind))
    print(f"mixed grad N={N} {kind}", flush=True)
    prob = qva.Problem(to_dev(q), "circulant", to_dev(lam) if kind == "array" else None, kind)
    f, dg, dt = qva.grad(prob, g, t)
    f_ref, rg, rt = oracle.grad("circulant", q, g, t, lam)
    assert abs(f.item() - f_ref) <= F_TOL * float(np.sum(np.abs(q))) / N * 10
    ref = np.concatenate([rg, rt])
    got = np.concatenate([dg.cpu().numpy(), dt.cpu().numpy()])
    assert np.max(np.abs(got - ref)) <= G_TOL * np.max(np.abs(ref))
    fe, _, _ = qva.evolve(prob, g, t, store=False)
    assert abs(fe.item() - f.item()) <= 1e-13 * np.mean(np.abs(q))


@pytest.mark.parametrize("N", [30, 1000, 3003, 6000, 24472, 243000, 184756, 460288, 2704156])
@pytest.mark.parametrize("kind", ["ring", "array"])
def test_mix_circulant_mixed_radix(N, kind):
    """qva_mix_circulant alone on a random state over N solutions (one, two
    and three groups; radices up to 31) against the oracle's mixer."""
    rng = np.random.default_rng(7 * N + len(kind))
    psi0 = rand_state(rng, N)
    lam = oracle.ring_lambda(N) if kind == "ring" else random_symmetric_lambda(N, rng)
    t = float(rng.uniform(0.2, 3.0))
    print(f"mix_circulant N={N} {kind}", flush=True)
    psi = to_dev(psi0)
    qva.mix_circulant(psi, t, to_dev(lam) if kind == "array" else None, kind)
    ref = oracle.mix_circulant(psi0, lam, t)
    assert state_err(psi.cpu().numpy(), ref) < PSI_TOL
    # twice in a row with -t restores the state
    qva.mix_circulant(psi, -t, to_dev(lam) if kind == "array" else None, kind)
    assert state_err(psi.cpu().numpy(), psi0) < PSI_TOL


def test_mixed_radix_mixer_and_depth_zero():
    """p = 0 gives mean(q); t = 0 or all gamma = 0 leave f at mean(q)."""
    N = 6000
    rng = np.random.default_rng(5)
    q = rng.uniform(-1, 3, N)
    prob = qva.Problem(to_dev(q), "circulant", None, "ring")
    f0, n0, _ = qva.evolve(prob, [], [])
    assert abs(f0.item() - q.mean()) <= 1e-13 * abs(q.mean())
    f1, _, _ = qva.evolve(prob, [0.0, 0.0], [0.7, 1.3], store=False)
    assert abs(f1.item() - q.mean()) <= 1e-13 * abs(q.mean())
    f2, _, _ = qva.evolve(prob, [0.4, 0.9], [0.0, 0.0], store=False)
    assert abs(f2.item() - q.mean()) <= 1e-13 * abs(q.mean())


def test_constrained_portfolio_full_size_matches_oracle():
    """C(26, 13) = 10,400,600 feasible portfolios (2^3 5^2 7 17 19 23), ring,
    p = 6: f and the oracle's psi_p at sampled indices."""
    with open(GOLDEN_AMP) as fh:
        gold = json.load(fh)
    if "qwoa_m26_k13_p6_ring_amplitudes" not in gold:
        pytest.skip("golden value not generated")
    ref = gold["qwoa_m26_k13_p6_ring_amplitudes"]
    wl = qwoa_constrained_workload(26, 13, 6, seed=CONFIG_SEEDS["qwoa_n26"], lambda_kind="ring")
    prob = qva.Problem(to_dev(wl.q), "circulant", None, "ring")
    kinds, groups = _plan_kinds(prob, 6)
    assert 52 in kinds
    f, nrm, psi = qva.evolve(prob, wl.gammas, wl.ts, store=True)
    assert abs(f.item() - ref["f"]) <= F_TOL * abs(ref["f"]) * 10
    assert abs(nrm.item() - 1.0) < 1e-12
    idx = torch.tensor(ref["index"], device="cuda")
    got = psi[idx].cpu().numpy()
    want = np.array(ref["re"]) + 1j * np.array(ref["im"])
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_smooth_n_full_size_gradient_matches_oracle():
    """N = 2^3 3^5 5^3 7^2 = 11,907,000, ring, p = 2: f and the gradient."""
    with open(GOLDEN) as fh:
        gold = json.load(fh)
    if "smooth_11907000_p2_ring_grad" not in gold:
        pytest.skip("golden value not generated")
    ref = gold["smooth_11907000_p2_ring_grad"]
    N = 2 ** 3 * 3 ** 5 * 5 ** 3 * 7 ** 2
    rng = np.random.default_rng(2029)
    q = rng.uniform(-1.0, 3.0, N)
    g = rng.uniform(0, np.pi, 2)
    t = rng.uniform(0, np.pi, 2)
    prob = qva.Problem(to_dev(q), "circulant", None, "ring")
    f, dg, dt = qva.grad(prob, g, t)
    assert abs(f.item() - ref["f"]) <= F_TOL * float(np.mean(np.abs(q))) * 10
    want = np.array(ref["dgammas"] + ref["dts"])
    got = np.concatenate([dg.cpu().numpy(), dt.cpu().numpy()])
    assert np.max(np.abs(got - want)) <= G_TOL * np.max(np.abs(want))
    fe, _, _ = qva.evolve(prob, g, t, store=False)
    assert abs(fe.item() - ref["f"]) <= F_TOL * float(np.mean(np.abs(q))) * 10
