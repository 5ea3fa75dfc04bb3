"""qva_evolve and qva_grad captured in a HIP graph (torch.cuda.CUDAGraph).

Every path of the library only enqueues kernels on the caller's stream (no
allocation, no host synchronisation, no memset), so both calls can be captured
once and replayed.  Each case replays the graph three times, with eager calls
of the library between the replays, and requires every replay to reproduce the
eager results bit for bit (the passes sum in a fixed order).
"""

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import to_dev  # noqa: E402
from workloads import dicke_state  # noqa: E402

pytestmark = pytest.mark.gpu
qva = pytest.importorskip("paper_2110_03963_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qva.load_library()


def _case(name):
    rng = np.random.default_rng(7 * len(name) + ord(name[0]))
    p = 3
    if name == "x":
        n = 16
        prob = qva.Problem(to_dev(rng.uniform(0, 3, 1 << n)), "x")
        G = rng.uniform(0, math.pi, p)
    elif name == "ring":
        n = 17
        prob = qva.Problem(to_dev(rng.uniform(0, 3, 1 << n)), "circulant", None, "ring")
        G = rng.uniform(0, math.pi, p)
    elif name == "complete_any_n":
        N = 100003
        prob = qva.Problem(to_dev(rng.uniform(0, 3, N)), "circulant", None, "complete")
        G = rng.uniform(0, math.pi, p)
    elif name == "bluestein":
        N = 50021
        prob = qva.Problem(to_dev(rng.uniform(0, 3, N)), "circulant", to_dev(rng.uniform(-2, 2, N)), "array")
        G = rng.uniform(0, math.pi, p)
    elif name == "mixed":
        N = 243000  # 2^3 3^5 5^3: the in-place mixed-radix passes
        prob = qva.Problem(to_dev(rng.uniform(0, 3, N)), "circulant", to_dev(rng.uniform(-2, 2, N)), "array")
        G = rng.uniform(0, math.pi, p)
    elif name == "xy":
        n = 15
        prob = qva.Problem(to_dev(rng.uniform(0, 3, 1 << n)), "xy", pairs=qva.parity_ring_pairs(range(n)),
                           psi0=to_dev(dicke_state(n, 7)))
        G = rng.uniform(0, math.pi, p)
    else:  # extended QAOA
        n = 16
        S = np.array([(1 << a) | (1 << ((a + 3) % n)) for a in range(n)], dtype=np.uint64)
        prob = qva.Problem(to_dev(rng.uniform(0, 3, 1 << n)), "x", terms=(S, rng.uniform(-1, 1, n)))
        G = rng.uniform(0, math.pi, (p, n))
    T = rng.uniform(0, math.pi, p)
    return prob, torch.tensor(G, device="cuda"), torch.tensor(T, device="cuda")


@pytest.mark.parametrize("name", ["x", "ring", "complete_any_n", "bluestein", "mixed", "xy", "terms"])
def test_graph_capture_evolve_and_grad(name):
    prob, g, t = _case(name)
    p = t.numel()
    N = prob.N
    dev = prob.device
    f_ref, n_ref, _ = qva.evolve(prob, g, t, store=False)
    fg_ref, dg_ref, dt_ref = qva.grad(prob, g, t)
    f_ref, n_ref, fg_ref = f_ref.item(), n_ref.item(), fg_ref.item()
    dg_ref, dt_ref = dg_ref.clone(), dt_ref.clone()

    psi = torch.empty(N, dtype=torch.complex128, device=dev)
    psi2 = torch.empty(N, dtype=torch.complex128, device=dev)
    chi = torch.empty(N, dtype=torch.complex128, device=dev)
    ws = torch.empty(max(prob.workspace_bytes(p), 16), dtype=torch.uint8, device=dev)
    wsg = torch.empty(max(prob.workspace_bytes(p, True), 256), dtype=torch.uint8, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up outside the capture
        qva.evolve(prob, g, t, psi=psi, store=False, workspace=ws)
        qva.grad(prob, g, t, psi=psi2, chi=chi, workspace=wsg)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        f1, n1, _ = qva.evolve(prob, g, t, psi=psi, store=False, workspace=ws)
        f2, dg, dt = qva.grad(prob, g, t, psi=psi2, chi=chi, workspace=wsg)
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        assert f1.item() == f_ref and n1.item() == n_ref, (name, rep)
        assert f2.item() == fg_ref, (name, rep)
        assert torch.equal(dg, dg_ref.reshape(dg.shape)) and torch.equal(dt, dt_ref), (name, rep)
        # eager work between replays, on other buffers
        qva.evolve(prob, g, t, store=False)
        torch.cuda.synchronize()
    del graph
    torch.cuda.empty_cache()
