"""GPU parity: batched forward + adjoint over many QAOA instances.

Every instance of a batch must equal the single-instance qva_grad result
(f to 1e-12 relative, gradients to 1e-10 relative) and, for small n, the CPU
oracle.  A HIP graph that captures the batched gradient and a gradient step
is replayed several times, with eager work and synchronisation in between,
and every replay is checked against the same steps run eagerly.
"""

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from gpu_util import to_dev  # noqa: E402
from workloads import CONFIG_SEEDS, batched_workloads, maxcut_qualities_device  # noqa: E402

pytestmark = pytest.mark.gpu
qva = pytest.importorskip("paper_2110_03963_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qva.load_library()


def _rel(a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _small_batch(seed, specs):
    rng = np.random.default_rng(seed)
    qs, gs, ts, host_q = [], [], [], []
    for n, p in specs:
        q = rng.uniform(0, 4, 1 << n)
        host_q.append(q)
        qs.append(to_dev(q))
        gs.append(rng.uniform(0, math.pi, p))
        ts.append(rng.uniform(0, math.pi, p))
    return qs, gs, ts, host_q


SPECS = [(12, 1), (12, 4), (13, 1), (13, 3), (14, 2), (15, 5), (16, 1), (17, 3), (18, 2), (20, 4),
         (21, 2), (22, 3), (22, 1), (12, 2), (19, 6)]


@pytest.mark.parametrize("align", ["start", "end", "spread"])
def test_batch_matches_single_instance(align):
    qs, gs, ts, host_q = _small_batch(1, SPECS)
    b = qva.Batch(qs, gs, ts, align=align)
    b.grad()
    torch.cuda.synchronize()
    for i, (n, p) in enumerate(SPECS):
        f, dg, dt = b.instance(i)
        f1, dg1, dt1 = qva.grad(qva.Problem(qs[i], "x"), gs[i], ts[i])
        assert abs(f.item() - f1.item()) <= 1e-12 * abs(f1.item()), (i, n, p)
        g = np.concatenate([dg.cpu().numpy(), dt.cpu().numpy()])
        g1 = np.concatenate([dg1.cpu().numpy(), dt1.cpu().numpy()])
        assert _rel(g, g1) < 1e-10, (i, n, p)
        if n <= 14:
            f_ref, rg, rt = oracle.grad("x", host_q[i], gs[i], ts[i])
            assert abs(f.item() - f_ref) <= 1e-12 * abs(f_ref)
            assert _rel(g, np.concatenate([rg, rt])) < 1e-10


def test_batch_is_deterministic_and_align_independent():
    qs, gs, ts, _ = _small_batch(2, SPECS)
    res = []
    for align in ["start", "spread", "start"]:
        b = qva.Batch(qs, gs, ts, align=align)
        b.grad()
        torch.cuda.synchronize()
        res.append((b.f.cpu().numpy().copy(), b.dgammas.cpu().numpy().copy(), b.dts.cpu().numpy().copy()))
    # same plan twice: bit-identical; different alignment: same kernels per instance
    for a, c in zip(res[0], res[2]):
        assert np.array_equal(a, c)
    for a, c in zip(res[0], res[1]):
        assert np.array_equal(a, c)


def test_batch_graph_capture_replays():
    """Capture [batched gradient, gradient step] in a HIP graph; replay it four
    times with eager work and synchronisation between replays; each replay
    must equal the same step run eagerly on a second, identical batch."""
    qs, gs, ts, _ = _small_batch(3, SPECS[:9])
    lr = 0.05
    b_graph = qva.Batch(qs, gs, ts)
    b_eager = qva.Batch(qs, gs, ts)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        b_graph.grad()  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    # undo nothing: the warm-up only wrote f/gradients, not the angles
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        b_graph.grad()
        b_graph.sgd(lr)
    torch.cuda.synchronize()
    for rep in range(4):
        graph.replay()
        torch.cuda.synchronize()
        scratch = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work
        b_eager.grad()
        b_eager.sgd(lr)
        torch.cuda.synchronize()
        assert torch.isfinite(scratch)
        assert torch.equal(b_graph.f, b_eager.f), rep
        assert torch.equal(b_graph.dgammas, b_eager.dgammas), rep
        assert torch.equal(b_graph.gammas, b_eager.gammas), rep
        assert torch.equal(b_graph.ts, b_eager.ts), rep


def test_batch_sgd_step():
    qs, gs, ts, _ = _small_batch(4, SPECS[:5])
    b = qva.Batch(qs, gs, ts)
    g0 = b.gammas.clone()
    t0 = b.ts.clone()
    b.grad()
    b.sgd(0.1)
    torch.cuda.synchronize()
    assert torch.allclose(b.gammas, g0 - 0.1 * b.dgammas, rtol=0, atol=1e-15)
    assert torch.allclose(b.ts, t0 - 0.1 * b.dts, rtol=0, atol=1e-15)


def test_batch512_config_subset():
    """The batched workload: 512 instances, n ~ U{12..22}, p ~ U{1..8},
    G(n, 0.4) with weights U(0,1).  Every instance's f and gradient are
    compared with qva_grad on a sample of 40 instances (all n = 12..14 ones
    included), and the small ones also with the oracle."""
    wls = batched_workloads(512, seed=CONFIG_SEEDS["batch512"], build_q=False)
    qs = [maxcut_qualities_device(w.n, w.edges, w.weights, "cuda") for w in wls]
    b = qva.Batch(qs, [w.gammas for w in wls], [w.ts for w in wls])
    b.grad()
    torch.cuda.synchronize()
    f_all = b.f.cpu().numpy()
    assert np.all(np.isfinite(f_all))
    rng = np.random.default_rng(0)
    sample = sorted(set(rng.choice(512, 30, replace=False)) | {i for i, w in enumerate(wls) if w.n <= 13})
    for i in sample[:40]:
        w = wls[i]
        f, dg, dt = b.instance(i)
        f1, dg1, dt1 = qva.grad(qva.Problem(qs[i], "x"), w.gammas, w.ts)
        assert abs(f.item() - f1.item()) <= 1e-12 * abs(f1.item())
        g = np.concatenate([dg.cpu().numpy(), dt.cpu().numpy()])
        g1 = np.concatenate([dg1.cpu().numpy(), dt1.cpu().numpy()])
        assert _rel(g, g1) < 1e-10
        if w.n <= 13:
            f_ref, rg, rt = oracle.grad("x", qs[i].cpu().numpy(), w.gammas, w.ts)
            assert abs(f.item() - f_ref) <= 1e-12 * abs(f_ref)
            assert _rel(g, np.concatenate([rg, rt])) < 1e-10
