"""GPU: the tile-ordered copy of q (qva_q_tiles, qva_problem.q_tiles).

The copy holds the same q values in the order the hypercube boundary passes
read them, so an evolution or adjoint gradient that reads it must be
bit-identical to one that reads q itself.  The cases cover every tile
geometry those passes take: 3 to 11 column bits (3 with the XCD-paired
tiles), the contiguous low group of a two-group register, and splits set by
qva_set_group_split; one case is also compared with the oracle.  A split set
after the copy was written makes the calls refuse it until it is written
again.  At full size, in the configuration the benchmark times: the n = 28,
p = 8 evolution against the oracle-written f and sampled amplitudes, and the
n = 30, p = 12 adjoint bit-identical with and without the copy.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from gpu_util import to_dev  # noqa: E402

pytestmark = pytest.mark.gpu
qva = pytest.importorskip("paper_2110_03963_amd")
from paper_2110_03963_amd import _lib, autotune  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qva.load_library()


def _case(n, p, seed):
    rng = np.random.default_rng(seed)
    q = rng.standard_normal(1 << n)  # generic reals: any misplaced entry shows
    g = rng.uniform(-1.0, 1.0, p)
    t = rng.uniform(-1.0, 1.0, p)
    return q, g, t


def _same(a, b):
    return bool(torch.equal(a, b))


# (n, p, split or None): column bits of the boundary groups in the comment
CASES = [
    (13, 3, None),     # 12 + 1: C = 11, and the low group
    (15, 4, None),     # 12 + 3: C = 9
    (18, 3, None),     # 12 + 6: C = 6
    (20, 4, None),     # 12 + 8: C = 4
    (21, 3, None),     # 12 + 9: C = 3, paired tiles
    (21, 4, (2, 7)),   # C = 10 and 5
    (24, 3, None),     # 12 + 6 + 6
    (24, 4, (4, 8)),   # C = 8 and 4
    (26, 3, None),     # 12 + 7 + 7: C = 5
]


@pytest.mark.parametrize("n,p,split", CASES)
def test_q_tiles_bit_identical(n, p, split):
    print(f"q_tiles n={n} p={p} split={split}", flush=True)
    q, g, t = _case(n, p, 1000 + n + p)
    if split is not None:
        autotune.set_split(n, split)
    try:
        prob = qva.Problem(to_dev(q), "x")
        f0, nr0, psi0 = qva.evolve(prob, g, t)
        fg0, dg0, dt0 = qva.grad(prob, g, t)
        assert prob.tile_q()
        assert prob.q_tiles.numel() == (len(autotune.get_split(n)) + 1) << n
        f1, nr1, psi1 = qva.evolve(prob, g, t)
        fg1, dg1, dt1 = qva.grad(prob, g, t)
        assert _same(f0, f1) and _same(nr0, nr1)
        assert _same(psi0, psi1)
        assert _same(torch.as_tensor(fg0), torch.as_tensor(fg1))
        assert _same(dg0, dg1) and _same(dt0, dt1)
    finally:
        if split is not None:
            autotune.set_split(n, None)


def test_q_tiles_against_oracle():
    n, p = 16, 4
    q, g, t = _case(n, p, 77)
    prob = qva.Problem(to_dev(q), "x")
    assert prob.tile_q()
    f, dg, dt = qva.grad(prob, g, t)
    f_ref, rg, rt = oracle.grad("x", q, g, t)
    assert abs(float(f) - f_ref) <= 1e-12 * max(abs(f_ref), 1.0)
    r = np.concatenate([rg, rt])
    d = np.concatenate([dg.cpu().numpy(), dt.cpu().numpy()])
    assert np.max(np.abs(d - r)) <= 1e-10 * np.max(np.abs(r))


def test_q_tiles_stale_after_split():
    n, p = 20, 3
    q, g, t = _case(n, p, 5)
    prob = qva.Problem(to_dev(q), "x")
    f0, _, _ = qva.evolve(prob, g, t)
    assert prob.tile_q()
    autotune.set_split(n, (3, 5))
    try:
        with pytest.raises(_lib.QvaError) as err:
            qva.evolve(prob, g, t)
        assert err.value.status == _lib.QVA_ERR_ARG
        assert prob.tile_q()  # rewritten for the split in effect
        f1, _, _ = qva.evolve(prob, g, t)
        assert abs(float(f1) - float(f0)) <= 1e-12 * abs(float(f0))
    finally:
        autotune.set_split(n, None)
    prob.untile_q()
    f2, _, _ = qva.evolve(prob, g, t)
    assert _same(f2, f0)


def test_q_tiles_refused_after_q_changes():
    """An in-place change of q after tile_q() makes the calls raise until
    the copy is written again, which then gives the new q's result."""
    n, p = 18, 3
    q, g, t = _case(n, p, 11)
    prob = qva.Problem(to_dev(q), "x")
    assert prob.tile_q()
    prob.q.mul_(2.0)
    with pytest.raises(ValueError):
        qva.evolve(prob, g, t)
    assert prob.tile_q()
    f1, _, _ = qva.evolve(prob, g, t)
    prob.untile_q()
    f2, _, _ = qva.evolve(prob, g, t)
    assert _same(f1, f2)
    f_ref, _, _ = qva.evolve(qva.Problem(to_dev(2.0 * q), "x"), g, t)
    assert _same(f2, f_ref)


def test_q_tiles_unused_mixers():
    """No copy for circulant mixers or small registers: tile_q reports False."""
    q = np.linspace(0.0, 1.0, 1 << 14)
    assert not qva.Problem(to_dev(q), "circulant", None, "ring").tile_q()
    assert not qva.Problem(to_dev(q[:1 << 10]), "x").tile_q()


# ---------------------------------------------------------------- full size
# The benchmark times the n = 28 evolution and the n = 30 adjoint with q in
# tile order: the same launch configuration, checked here at full size.

def test_q_tiles_full_size_headline():
    import json
    import os

    from workloads import CONFIG_SEEDS, qaoa_maxcut_workload

    print("q_tiles full size: n=28 p=8", flush=True)
    gold_dir = os.path.join(os.path.dirname(__file__), "golden")
    with open(os.path.join(gold_dir, "full_size_values.json")) as fh:
        ref = json.load(fh)["qaoa_n28_p8"]
    with open(os.path.join(gold_dir, "full_size_amplitudes.json")) as fh:
        amp = json.load(fh)["qaoa_n28_p8_amplitudes"]
    wl = qaoa_maxcut_workload(28, 8, graph="regular3", weighted=True, seed=CONFIG_SEEDS["qaoa_n28"])
    prob = qva.Problem(torch.from_numpy(wl.q).cuda(), "x")
    f0, _, _ = qva.evolve(prob, wl.gammas, wl.ts, store=False)
    assert prob.tile_q()
    f1, nr1, psi = qva.evolve(prob, wl.gammas, wl.ts, store=True)
    assert _same(f0, f1)
    assert abs(f1.item() - ref["f"]) < 1e-12 * abs(ref["f"])
    assert abs(nr1.item() - 1.0) < 1e-12
    idx = torch.tensor(amp["index"], dtype=torch.int64, device=psi.device)
    got = psi[idx].cpu().numpy()
    want = np.array(amp["re"]) + 1j * np.array(amp["im"])
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    del psi, prob
    torch.cuda.empty_cache()


def test_q_tiles_full_size_adjoint():
    from workloads import CONFIG_SEEDS, maxcut_qualities_device, qaoa_maxcut_workload

    print("q_tiles full size: adjoint n=30 p=12", flush=True)
    n, p = 30, 12
    wl = qaoa_maxcut_workload(n, p, graph="regular3", weighted=True, seed=CONFIG_SEEDS["grad_n30"],
                              build_q=False)
    prob = qva.Problem(maxcut_qualities_device(n, wl.edges, wl.weights, "cuda"), "x")
    f0, dg0, dt0 = qva.grad(prob, wl.gammas, wl.ts)
    assert prob.tile_q()
    f1, dg1, dt1 = qva.grad(prob, wl.gammas, wl.ts)
    assert _same(torch.as_tensor(f0), torch.as_tensor(f1))
    assert _same(dg0, dg1) and _same(dt0, dt1)
    del prob
    torch.cuda.empty_cache()
