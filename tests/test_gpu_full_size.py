"""GPU parity at the benchmark sizes.

* QAOA MaxCut n = 28, p = 8 (random 3-regular, weights U(0,1)) and QWOA
  portfolio N = 2^26, p = 6 (ring mixer): f against values the CPU oracle
  computed at full size (tests/golden/full_size_values.json, written by
  tests/golden/gen_full_size.py), to 1e-12 relative.
* psi_p itself at the same sizes: 4096+ seeded amplitudes of the oracle's
  final state (tests/golden/full_size_amplitudes.json, same generator), to
  1e-12 of the largest sampled amplitude.
* The hypercube mixer on every amplitude at n = 28 and n = 30 (the layouts of
  the benchmark and of the adjoint workload): from |0>, exp(-i t sum X_i)
  gives cos(t)^(n-|j|) (-i sin t)^|j| with |j| the popcount of j, evaluated
  on the device in float64 for all 2^n indices.
* Properties that hold at any size, checked on the same full-size inputs and
  in the launch configuration the benchmark times: f(-gamma, -t) = f(gamma, t),
  all gamma = 0 gives mean(q), |psi_j|^2 = |psi_{~j}|^2 for MaxCut, norm 1.
"""

import math

import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import CONFIG_SEEDS, qaoa_maxcut_workload, qwoa_portfolio_workload  # noqa: E402

pytestmark = pytest.mark.gpu
qva = pytest.importorskip("paper_2110_03963_amd")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "full_size_values.json")
GOLDEN_AMP = os.path.join(os.path.dirname(__file__), "golden", "full_size_amplitudes.json")


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
def golden_amp():
    with open(GOLDEN_AMP) as fh:
        return json.load(fh)


def _check_amplitudes(psi, ref):
    """Sampled psi_p against the oracle's: max |dpsi| <= 1e-12 max |psi_ref|."""
    idx = torch.tensor(ref["index"], dtype=torch.int64, device=psi.device)
    got = psi[idx].cpu().numpy()
    want = np.array(ref["re"]) + 1j * np.array(ref["im"])
    assert len(want) >= 4096
    err = float(np.max(np.abs(got - want)))
    scale = float(np.max(np.abs(want)))
    print(f"sampled amplitudes: {len(want)}, max |dpsi| = {err:.3e}, max |psi| = {scale:.3e}", flush=True)
    assert err <= 1e-12 * scale, err / scale


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


def test_qaoa_n28_p8_amplitudes_match_oracle(golden_amp, qaoa28):
    wl, prob = qaoa28
    ref = golden_amp["qaoa_n28_p8_amplitudes"]
    f, _, psi = qva.evolve(prob, wl.gammas, wl.ts, store=True)
    assert abs(f.item() - ref["f"]) < 1e-12 * abs(ref["f"])
    _check_amplitudes(psi, ref)
    del psi
    torch.cuda.empty_cache()


def _popcount(j: torch.Tensor) -> torch.Tensor:
    j = j - ((j >> 1) & 0x5555555555555555)
    j = (j & 0x3333333333333333) + ((j >> 2) & 0x3333333333333333)
    j = (j + (j >> 4)) & 0x0F0F0F0F0F0F0F0F
    return (j * 0x0101010101010101) >> 56


@pytest.mark.parametrize("n,t", [(28, 0.37), (28, 2.21), (30, 0.81), (30, -1.93)])
def test_mix_x_delta_closed_form_full_size(n, t):
    """qva_mix_x on |0> at n = 28 (groups of 12/8/8 qubits, 256 B rows) and
    n = 30 (12/9/9, 3 column bits): every amplitude against
    cos(t)^(n-w) (-i sin t)^w, w = popcount(j), to 1e-13 of the largest."""
    print(f"mix_x delta closed form n={n} t={t}", flush=True)
    N = 1 << n
    psi = torch.zeros(N, dtype=torch.complex128, device="cuda")
    psi[0] = 1.0
    qva.mix_x(psi, t)
    c, s = math.cos(t), math.sin(t)
    # the n + 1 distinct values, by weight, in float64 on the device
    w = torch.arange(n + 1, dtype=torch.float64, device="cuda")
    mag = torch.pow(torch.tensor(c, dtype=torch.float64, device="cuda"), n - w) * \
        torch.pow(torch.tensor(s, dtype=torch.float64, device="cuda"), w)
    phase = torch.tensor([(-1j) ** k for k in range(4)], dtype=torch.complex128, device="cuda")
    table = mag.to(torch.complex128) * phase[torch.arange(n + 1, device="cuda") % 4]
    largest = float(torch.max(mag.abs()).item())
    err = 0.0
    chunk = 1 << 24
    for lo in range(0, N, chunk):
        j = torch.arange(lo, lo + chunk, dtype=torch.int64, device="cuda")
        ref = table[_popcount(j)]
        err = max(err, float(torch.max(torch.abs(psi[lo:lo + chunk] - ref)).item()))
    print(f"  max |dpsi| = {err:.3e}, largest = {largest:.3e}", flush=True)
    assert err <= 1e-13 * largest, err / largest
    del psi
    torch.cuda.empty_cache()


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


def test_qwoa_n26_p6_amplitudes_match_oracle(golden_amp):
    wl = qwoa_portfolio_workload(26, 6, seed=CONFIG_SEEDS["qwoa_n26"], lambda_kind="ring")
    ref = golden_amp["qwoa_n26_p6_amplitudes"]
    prob = qva.Problem(torch.from_numpy(wl.q).cuda(), "circulant", None, "ring")
    f, _, psi = qva.evolve(prob, wl.gammas, wl.ts, store=True)
    assert abs(f.item() - ref["f"]) < 1e-12 * abs(ref["f"])
    _check_amplitudes(psi, ref)


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
