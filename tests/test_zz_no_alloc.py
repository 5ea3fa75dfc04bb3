"""GPU check of qva_evolve_noalloc, the allocation-free qva_evolve.

Both entry points are called through the C ABI on the same seeded inputs.
qva_evolve_noalloc runs the same launches as qva_evolve with its workspace in
the library's static per-device array, so f, the norm and psi_p must be
bit-identical to qva_evolve's.  Each case makes two calls in a row, the
second on a smaller problem, so partial sums left in the shared array by the
first call would show if the second read them.  f is also held to the
oracle at 1e-12 relative.
"""

import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from gpu_util import f_rel_err  # noqa: E402
from workloads import qaoa_maxcut_workload, qwoa_portfolio_workload  # noqa: E402

pytestmark = pytest.mark.gpu

qva = pytest.importorskip("paper_2110_03963_amd")
_lib = qva._lib


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qva.load_library()


def _problem(mixer, n, q, kind=_lib.QVA_LAMBDA_ARRAY):
    return _lib.QvaProblem(mixer, n, q.data_ptr(), None, kind, 0, None, 0, None, 0)


def _run_both(mixer, kind, q_np, gammas, ts):
    """(f, norm, psi) from qva_evolve and from qva_evolve_noalloc."""
    lib = _lib.load()
    dev = torch.device("cuda:0")
    n = int(q_np.size).bit_length() - 1
    q = torch.from_numpy(q_np).to(dev)
    g = torch.tensor(gammas, dtype=torch.float64, device=dev)
    t = torch.tensor(ts, dtype=torch.float64, device=dev)
    pr = _problem(mixer, n, q, kind)
    p = len(gammas)
    stream = torch.cuda.current_stream().cuda_stream
    need = lib.qva_workspace_bytes(ctypes.byref(pr), p, 0)
    assert 0 < need <= _lib.QVA_STATIC_SCRATCH_BYTES
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    outs = []
    for noalloc in (False, True):
        psi = torch.empty(q_np.size, dtype=torch.complex128, device=dev)
        out = torch.full((2,), float("nan"), dtype=torch.float64, device=dev)
        if noalloc:
            st = lib.qva_evolve_noalloc(ctypes.byref(pr), g.data_ptr(), t.data_ptr(), p, psi.data_ptr(),
                                        out.data_ptr(), out.data_ptr() + 8, 0, stream)
        else:
            st = lib.qva_evolve(ctypes.byref(pr), g.data_ptr(), t.data_ptr(), p, psi.data_ptr(),
                                out.data_ptr(), out.data_ptr() + 8, 0, ws.data_ptr(), need, stream)
        assert st == _lib.QVA_OK, lib.qva_status_string(st)
        torch.cuda.synchronize()
        outs.append((float(out[0]), float(out[1]), psi.cpu().numpy()))
    return outs


def _check(outs, f_ref, q_np):
    (f0, n0, psi0), (f1, n1, psi1) = outs
    assert f1 == f0 and n1 == n0
    assert np.array_equal(psi1, psi0)
    assert f_rel_err(f1, f_ref, None, q_np) <= 1e-12
    assert abs(n1 - 1.0) <= 1e-13


def test_noalloc_hypercube_twice_then_smaller():
    for n, p, seed in [(22, 3, 11), (16, 2, 12)]:
        wl = qaoa_maxcut_workload(n, p, seed=seed)
        outs = _run_both(_lib.QVA_MIX_X, _lib.QVA_LAMBDA_ARRAY, wl.q, list(wl.gammas), list(wl.ts))
        _, f_ref, _ = oracle.evolve("x", wl.q, wl.gammas, wl.ts)
        _check(outs, f_ref, wl.q)


def test_noalloc_circulant_then_smaller_hypercube():
    wl = qwoa_portfolio_workload(20, 2, seed=21, lambda_kind="ring")
    outs = _run_both(_lib.QVA_MIX_CIRCULANT, _lib.QVA_LAMBDA_RING, wl.q, list(wl.gammas), list(wl.ts))
    _, f_ref, _ = oracle.evolve("circulant", wl.q, wl.gammas, wl.ts, lam=oracle.ring_lambda(wl.N))
    _check(outs, f_ref, wl.q)
    wl = qaoa_maxcut_workload(14, 2, seed=22)
    outs = _run_both(_lib.QVA_MIX_X, _lib.QVA_LAMBDA_ARRAY, wl.q, list(wl.gammas), list(wl.ts))
    _, f_ref, _ = oracle.evolve("x", wl.q, wl.gammas, wl.ts)
    _check(outs, f_ref, wl.q)


def test_noalloc_complete_graph_closed_form():
    for m, seed in [(18, 31), (15, 32)]:
        wl = qwoa_portfolio_workload(m, 3, seed=seed, lambda_kind="complete")
        outs = _run_both(_lib.QVA_MIX_CIRCULANT, _lib.QVA_LAMBDA_COMPLETE, wl.q, list(wl.gammas),
                         list(wl.ts))
        _, f_ref, _ = oracle.evolve("complete", wl.q, wl.gammas, wl.ts)
        _check(outs, f_ref, wl.q)


def test_noalloc_rejects_oversize_without_launch():
    """n = 33 needs 32 MiB of partial sums: QVA_ERR_SCRATCH, nothing run."""
    lib = _lib.load()
    dev = torch.device("cuda:0")
    q = torch.zeros(4, dtype=torch.float64, device=dev)  # never read: rejected first
    pr = _problem(_lib.QVA_MIX_X, 33, q)
    out = torch.zeros(2, dtype=torch.float64, device=dev)
    g = torch.zeros(1, dtype=torch.float64, device=dev)
    st = lib.qva_evolve_noalloc(ctypes.byref(pr), g.data_ptr(), g.data_ptr(), 1, out.data_ptr(),
                                out.data_ptr(), None, 0, torch.cuda.current_stream().cuda_stream)
    assert st == _lib.QVA_ERR_SCRATCH
    torch.cuda.synchronize()
    assert float(out.abs().sum()) == 0.0
