"""GPU parity at the benchmark sizes.

* QAOA MaxCut n = 28, p = 8 (random 3-regular, weights U(0,1)) and QWOA
  portfolio N = 2^26, p = 6 (ring mixer): f against values the CPU oracle
  computed at full size (tests/golden/full_size_values.json, written by
  tests/golden/gen_full_size.py), to 1e-12 relative.
* Properties that hold at any size, checked on the same full-size inputs and
  in the launch configuration the benchmark times: f(-gamma, -t) = f(gamma, t),
  all gamma = 0 gives mean(q), |psi_j|^2 = |psi_{~j}|^2 for MaxCut, norm 1.
"""

import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import CONFIG_SEEDS, qaoa_maxcut_workload, qwoa_portfolio_workload  # noqa: E402

pytestmark = pytest.mark.gpu
qva = pytest.importorskip("paper_2110_03963_amd")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "full_size_values.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qva.load_library()


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def qaoa28():
    wl = qaoa_maxcut_workload(28, 8, graph="regular3", weighted=True, seed=CONFIG_SEEDS["qaoa_n28"])
    prob = qva.Problem(torch.from_numpy(wl.q).cuda(), "x")
    return wl, prob


def test_qaoa_n28_p8_matches_oracle(golden, qaoa28):
    wl, prob = qaoa28
    ref = golden["qaoa_n28_p8"]
    f, nrm, _ = qva.evolve(prob, wl.gammas, wl.ts, store=False)
    assert abs(f.item() - ref["f"]) < 1e-12 * abs(ref["f"])
    assert abs(nrm.item() - 1.0) < 1e-12


def test_qaoa_n28_properties(qaoa28):
    wl, prob = qaoa28
    f, _, psi = qva.evolve(prob, wl.gammas, wl.ts, store=True)
    f_neg, _, _ = qva.evolve(prob, -wl.gammas, -wl.ts, store=False)
    assert abs(f_neg.item() - f.item()) < 1e-12 * abs(f.item())
    f0, _, _ = qva.evolve(prob, np.zeros(8), wl.ts, store=False)
    assert abs(f0.item() - float(np.mean(wl.q))) < 1e-12 * float(np.mean(wl.q))
    idx = torch.randint(0, 1 << 28, (1 << 20,), device="cuda", generator=torch.Generator("cuda").manual_seed(0))
    flip = idx ^ ((1 << 28) - 1)
    a = psi[idx].abs() ** 2
    b = psi[flip].abs() ** 2
    assert torch.max(torch.abs(a - b)).item() < 1e-12 * torch.max(a).item()


def test_qwoa_n26_p6_matches_oracle(golden):
    wl = qwoa_portfolio_workload(26, 6, seed=CONFIG_SEEDS["qwoa_n26"], lambda_kind="ring")
    ref = golden["qwoa_n26_p6"]
    prob = qva.Problem(torch.from_numpy(wl.q).cuda(), "circulant", None, "ring")
    f, nrm, _ = qva.evolve(prob, wl.gammas, wl.ts, store=False)
    assert abs(f.item() - ref["f"]) < 1e-12 * abs(ref["f"])
    assert abs(nrm.item() - 1.0) < 1e-12
    # the same spectrum passed as an array takes the per-tile lambda copy path
    lam = 2.0 * torch.cos(2.0 * np.pi * torch.arange(wl.N, dtype=torch.float64, device="cuda") / wl.N)
    prob_a = qva.Problem(prob.q, "circulant", lam, "array")
    f_a, _, _ = qva.evolve(prob_a, wl.gammas, wl.ts, store=False)
    assert abs(f_a.item() - ref["f"]) < 1e-12 * abs(ref["f"])


def test_qwoa_n26_p6_complete_matches_oracle(golden):
    """Complete-graph mixer at N = 2^26: the closed-form passes against the
    oracle's closed form, and the same spectrum given as an array (so the
    transform passes run) against the oracle's transform route."""
    if "qwoa_n26_p6_complete" not in golden:
        pytest.skip("golden value not generated")
    wl = qwoa_portfolio_workload(26, 6, seed=CONFIG_SEEDS["qwoa_n26"], lambda_kind="complete")
    ref = golden["qwoa_n26_p6_complete"]
    prob = qva.Problem(torch.from_numpy(wl.q).cuda(), "circulant", None, "complete")
    f, nrm, _ = qva.evolve(prob, wl.gammas, wl.ts, store=False)
    assert abs(f.item() - ref["f"]) < 1e-12 * abs(ref["f"])
    assert abs(nrm.item() - 1.0) < 1e-12
    # as an eigenvalue array the transform passes round t (N - 1) as the
    # oracle's transform route does: compared with that route's value
    lam = torch.full((wl.N,), -1.0, dtype=torch.float64, device="cuda")
    lam[0] = wl.N - 1
    prob_a = qva.Problem(prob.q, "circulant", lam, "array")
    f_a, _, _ = qva.evolve(prob_a, wl.gammas, wl.ts, store=False)
    assert abs(f_a.item() - ref["f_transform"]) < 1e-12 * abs(ref["f_transform"])


def test_qwoa_n26_p6_complete_gradient_matches_oracle(golden):
    """Closed-form adjoint at N = 2^26, p = 6 against the oracle's gradient
    (f to 1e-12, gradient to 1e-10 relative)."""
    if "qwoa_n26_p6_complete_grad" not in golden:
        pytest.skip("golden value not generated")
    wl = qwoa_portfolio_workload(26, 6, seed=CONFIG_SEEDS["qwoa_n26"], lambda_kind="complete")
    ref = golden["qwoa_n26_p6_complete_grad"]
    prob = qva.Problem(torch.from_numpy(wl.q).cuda(), "circulant", None, "complete")
    f, dg, dt = qva.grad(prob, wl.gammas, wl.ts)
    assert abs(f.item() - ref["f"]) < 1e-12 * abs(ref["f"])
    g = np.concatenate([dg.cpu().numpy(), dt.cpu().numpy()])
    r = np.concatenate([ref["dgammas"], ref["dts"]])
    assert np.max(np.abs(g - r)) < 1e-10 * np.max(np.abs(r))
